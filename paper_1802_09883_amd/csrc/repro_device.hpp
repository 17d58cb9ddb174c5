// repro_device.hpp -- device-side building blocks of repro<T,L> on gfx950.
//
// Paper: Mueller, Arteaga, Hoefler, Alonso, "Reproducible Floating-Point
// Aggregation in RDBMSs" (arXiv 1802.09883).
//
// A value b is split into L integer "units" k_l on grids g_l = 2^(E_l - m),
// one per level (error-free transformation, Sec. III-B; levels W bits apart,
// Sec. III-C).  The extractor exponents sit on the fixed lattice
// E_j = B + j*W; a group's top index j* is the smallest lattice index whose
// first level can take every value of the group (the level-shift test
// |b| < 2^(W-1) ulp(S^(1)) of Alg. 2).  Units of one level add exactly, so
// their sum is independent of order.  The canonical state stores each
// level as the paper's running sum S in [1.5, 1.75) * 2^E plus a carry
// count C (Sec. III-C).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace repro {

typedef __int128 i128;
typedef unsigned __int128 u128;

// Accumulator formats.  W: 18 (float) / 40 (double) as chosen in Sec. III-C;
// m: fraction bits (ulp(x) = 2^(E-m), Sec. III-A); B = emin so that the last
// level of the lowest lattice point has the grid of the smallest subnormal;
// JMAX: largest index whose extractor 1.5*2^E is finite; CARRY = m - 2: one
// carry unit 0.25*ufp(S) measured in units of g.
template <class AT>
struct Fmt;

template <>
struct Fmt<double> {
    typedef uint64_t bits_t;
    static constexpr int m = 52, W = 40, B = -1022, JMAX = 51, BIAS = 1023, EMIN = -1022;
    static constexpr int CARRY = 50;
};

template <>
struct Fmt<float> {
    typedef uint32_t bits_t;
    static constexpr int m = 23, W = 18, B = -126, JMAX = 14, BIAS = 127, EMIN = -126;
    static constexpr int CARRY = 21;
};

constexpr uint32_t ERR_KEY = 1u, ERR_NONFINITE = 2u, ERR_RANGE = 4u;

// floor(log2 |b|) for finite nonzero b (subnormals included):
// v_frexp_exp gives e' with b = f * 2^e', |f| in [0.5, 1).
__device__ __forceinline__ int exp_of(double b) { return __builtin_amdgcn_frexp_exp(b) - 1; }
__device__ __forceinline__ int exp_of(float b) { return __builtin_amdgcn_frexp_expf(b) - 1; }

// Smallest lattice index j with |b| < 2^(W-1) * 2^(E_j - m), from e =
// floor(log2|b|): E_j >= e + m - W + 2, i.e. j = ceil((e + m - W + 2 - B)/W).
// The numerator is > -W for every finite value, so the biased division
// below is a ceiling.
template <class AT>
__device__ __forceinline__ int jreq_of_exp(int e) {
    typedef Fmt<AT> F;
    return (e + F::m - F::W + 2 - F::B + F::W - 1) / F::W;
}

__device__ __forceinline__ bool finite_val(double v) { return __builtin_isfinite(v); }
__device__ __forceinline__ bool finite_val(float v) { return __builtin_isfinite(v); }

// High 32 bits of the extractor M = 1.5 * 2^E (double) / its bits (float).
__device__ __forceinline__ uint32_t extractor_hi(double*, int E) {
    return ((uint32_t)(E + 1023) << 20) | 0x80000u;
}
__device__ __forceinline__ uint32_t extractor_hi(float*, int E) {
    return ((uint32_t)(E + 127) << 23) | 0x400000u;
}

// Units of one value at top index `top` (pre-rounded extraction).  Level l
// adds the constant extractor M_l = 1.5 * 2^E_l: |r| <= 2^(W-1) g_l keeps
// r + M_l inside M_l's binade, so the sum s is M_l + k*g_l with k the
// nearest integer to r/g_l, ties to even (M_l's significand is even) --
// the state-independent tie rule.  k is read off the bit patterns
// (s and M_l share the exponent field), s - M_l is exact (Sterbenz) and so
// is the remainder r - (s - M_l).  Requires IEEE denormals (no flush).
template <int L>
__device__ __forceinline__ void extract_units(double b, int top, long long* k) {
    typedef Fmt<double> F;
    const uint32_t h0 = extractor_hi((double*)0, F::B + top * F::W);
    double r = b;
#pragma unroll
    for (int l = 0; l < L; ++l) {
        const uint32_t mh = h0 - (uint32_t)(l * F::W) * (1u << 20);
        const double M = __hiloint2double((int)mh, 0);
        const double s = r + M;
        k[l] = (long long)((uint64_t)__double_as_longlong(s) - ((uint64_t)mh << 32));
        if (l + 1 < L) {
            const double t = s - M;
            r = r - t;
        }
    }
}

template <int L>
__device__ __forceinline__ void extract_units(float b, int top, long long* k) {
    typedef Fmt<float> F;
    const uint32_t b0 = extractor_hi((float*)0, F::B + top * F::W);
    float r = b;
#pragma unroll
    for (int l = 0; l < L; ++l) {
        const uint32_t mb = b0 - (uint32_t)(l * F::W) * (1u << 23);
        const float M = __uint_as_float(mb);
        const float s = r + M;
        k[l] = (long long)(int32_t)(__float_as_uint(s) - mb);
        if (l + 1 < L) {
            const float t = s - M;
            r = r - t;
        }
    }
}

// ---------------------------------------------------------------- states
// Canonical level: S = 1.5*2^E + lo*g with lo in [0, 2^CARRY); the level's
// exact sum is K = C * 2^CARRY + lo units of g.

__device__ __forceinline__ int state_top(double S0) {
    typedef Fmt<double> F;
    const int E = (int)((__double_as_longlong(S0) >> 52) & 0x7FF) - F::BIAS;
    return (E - F::B) / F::W;
}
__device__ __forceinline__ int state_top(float S0) {
    typedef Fmt<float> F;
    const int E = (int)((__float_as_uint(S0) >> 23) & 0xFF) - F::BIAS;
    return (E - F::B) / F::W;
}

__device__ __forceinline__ long long state_lo(double S) {
    return (long long)((uint64_t)__double_as_longlong(S) & ((1ull << Fmt<double>::CARRY) - 1));
}
__device__ __forceinline__ long long state_lo(float S) {
    return (long long)(__float_as_uint(S) & ((1u << Fmt<float>::CARRY) - 1));
}

__device__ __forceinline__ double make_S(double*, int E, long long lo) {
    const uint64_t b = ((uint64_t)(E + 1023) << 52) | (1ull << 51) | (uint64_t)lo;
    return __longlong_as_double((long long)b);
}
__device__ __forceinline__ float make_S(float*, int E, long long lo) {
    const uint32_t b = ((uint32_t)(E + 127) << 23) | (1u << 22) | (uint32_t)lo;
    return __uint_as_float(b);
}

// Normalise a level held as (hi, lo) with value hi*2^CARRY + lo (both may be
// any int64 with |lo| < 2^62): canonical C and lo' in [0, 2^CARRY).
template <class AT>
__device__ __forceinline__ void normalise(long long hi, long long lo, long long* C, long long* lo_out) {
    constexpr int c = Fmt<AT>::CARRY;
    *C = hi + (lo >> c);  // arithmetic shift: floor
    *lo_out = lo & ((1ll << c) - 1);
}

// --------------------------------------------------------- finalisation
// Nearest number of type AT to K * 2^s, ties to even, gradual underflow,
// overflow to +-Inf: the single rounding of one level's exact value.
template <class AT>
__device__ AT round_exact(i128 K, int s) {
    typedef Fmt<AT> F;
    if (K == 0) return (AT)0;
    const bool neg = K < 0;
    const u128 a = neg ? (u128)(-K) : (u128)K;
    const uint64_t ahi = (uint64_t)(a >> 64), alo = (uint64_t)a;
    const int nb = ahi ? 128 - __clzll((long long)ahi) : 64 - __clzll((long long)alo);
    int u = nb - 1 + s - F::m;
    if (u < F::EMIN - F::m) u = F::EMIN - F::m;
    const int shift = u - s;
    uint64_t q;
    if (shift <= 0) {
        q = alo;  // nb <= m+1: exact
        u = s;
    } else if (shift >= 128) {
        q = 0;
    } else {
        const u128 qq = a >> shift;
        const u128 rem = a - (qq << shift);
        const u128 half = (u128)1 << (shift - 1);
        q = (uint64_t)qq;
        if (rem > half || (rem == half && (q & 1))) q += 1;
    }
    double r = ldexp((double)q, u);  // q <= 2^(m+1): exact or +-Inf
    if (neg) r = -r;
    return (AT)r;  // float: r is a float value or beyond its range (-> Inf)
}

}  // namespace repro
