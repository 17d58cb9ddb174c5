// repro_agg.hpp -- the hot loop shared by the aggregation kernels of
// librepro (one workgroup aggregating a range of rows into per-group LDS
// bins), included by every translation unit of the library.
//
// Paper: Mueller, Arteaga, Hoefler, Alonso, "Reproducible Floating-Point
// Aggregation in RDBMSs" (arXiv 1802.09883): RSum (Sec. III-C, Alg. 2) with
// the level check per tile (as Alg. 3 does per block), pre-rounded
// extraction (Sec. III-B) and exact integer level sums.
#ifndef REPRO_AGG_HPP
#define REPRO_AGG_HPP

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "repro.h"
#include "repro_device.hpp"

namespace repro {
namespace {

constexpr int AGG_BLOCK = 1024;  // 16 waves: one workgroup per CU
constexpr int ROWS_PER_THREAD = 8;
constexpr int PREFETCH = 1;  // tiles loaded ahead of the one being processed
constexpr int AGG_TILE = AGG_BLOCK * ROWS_PER_THREAD;
constexpr int MAX_AGG_WG = 256;
// Small inputs spread over many workgroups of one tile each (load latency,
// not bandwidth, bounds them); the partials they add are few at such sizes.
constexpr int64_t MIN_ROWS_PER_WG = (int64_t)AGG_TILE;
// A bin word takes at most (rows of one workgroup) units of magnitude
// <= 2^(W-1) <= 2^39; 2^23 rows keep it below 2^62.
constexpr int64_t MAX_ROWS_PER_WG = (int64_t)1 << 23;
constexpr size_t LDS_BIN_BUDGET = 150 * 1024;  // of gfx950's 160 KiB per workgroup
constexpr size_t REPLICA_BUDGET = 32 * 1024;

__host__ __device__ inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// LDS bin replicas for G groups at L levels: few groups get several copies
// (lanes spread over them) to cut contention on the same words.
inline int replicas_for(int64_t G, int L) {
    int R = 1;
    while (R < 64 && (size_t)2 * R * G * L * 8 <= REPLICA_BUDGET) R *= 2;
    return R;
}

// LDS bytes of aggregate_range for G groups, L levels, R replicas.
inline size_t agg_lds_bytes(int64_t G, int L, int R) { return (size_t)(G + 1) * L * 8 * R + (size_t)(G + 1) * 12; }

// ----------------------------------------------------------- row loading

template <class T, int N>
struct VecT {
    typedef T type __attribute__((ext_vector_type(N)));
};

// NT: a non-temporal (streaming) load, for columns read once.
template <class T, int N, bool NT = true>
__device__ __forceinline__ void vload(const T* __restrict__ p, T* out) {
    if constexpr (N == 1) {
        out[0] = NT ? __builtin_nontemporal_load(p) : *p;
    } else {
        typedef typename VecT<T, N>::type V;
        const V x = NT ? __builtin_nontemporal_load(reinterpret_cast<const V*>(p)) : *reinterpret_cast<const V*>(p);
#pragma unroll
        for (int i = 0; i < N; ++i) out[i] = x[i];
    }
}

// Loads the ROWS_PER_THREAD rows of this thread in the tile starting at
// `base`: unit u covers rows base + off[u] + [0, VEC) with off[u] =
// (u*BLOCK + tid)*VEC, so each vector load instruction of a wave reads one
// contiguous span (the tile base is uniform, the offsets are 32-bit).  Rows
// at or beyond `end` are flagged out of range.
template <class KT, class VT, int VEC, int BLOCK, bool NT = true>
__device__ __forceinline__ uint32_t load_tile(const KT* __restrict__ keys, const VT* __restrict__ vals,
                                              int64_t base, int64_t end, KT* k, VT* v, const uint32_t* off) {
    constexpr int U = ROWS_PER_THREAD / VEC;
    const KT* kb = keys + base;
    const VT* vb = vals + base;
    uint32_t inr = 0;
    if (base + (int64_t)BLOCK * ROWS_PER_THREAD <= end) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            vload<KT, VEC, NT>(kb + off[u], k + u * VEC);
            vload<VT, VEC, NT>(vb + off[u], v + u * VEC);
        }
        inr = (1u << ROWS_PER_THREAD) - 1;
    } else {
        const uint32_t lim = (uint32_t)(end - base);
#pragma unroll
        for (int u = 0; u < U; ++u) {
#pragma unroll
            for (int e = 0; e < VEC; ++e) {
                const uint32_t row = off[u] + e;
                if (row < lim) {
                    k[u * VEC + e] = kb[row];
                    v[u * VEC + e] = vb[row];
                    inr |= 1u << (u * VEC + e);
                } else {
                    k[u * VEC + e] = 0;
                    v[u * VEC + e] = (VT)0;
                }
            }
        }
    }
    return inr;
}

__device__ __forceinline__ uint32_t wave_or(uint32_t x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x |= __shfl_xor(x, o, 64);
    return x;
}

__device__ __forceinline__ long long wave_sum64(long long x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}

// Folds the R replicas (a power of two) of every LDS bin into replica 0 by
// a tree of exact integer adds, all threads working on every round, so that
// few groups with many replicas do not leave one thread summing them in
// sequence.  Bins are [L][G+1][R] (layout below).  Call after the bins are
// final; contains barriers (R uniform).
template <int L, int BLOCK>
__device__ __forceinline__ void fold_replicas(long long* bins, int G, int R) {
    for (int h = R >> 1; h >= 1; h >>= 1) {
        const int nwords = (G + 1) * L * h;  // adds of this round
        const int sh = __builtin_ctz((unsigned)h);
        for (int i = threadIdx.x; i < nwords; i += BLOCK) {
            const int r = i & (h - 1), b = i >> sh;  // replica, bin (l, g)
            bins[(size_t)b * R + r] += bins[(size_t)b * R + r + h];
        }
        __syncthreads();
    }
}

__device__ __forceinline__ void report(uint32_t* status, uint32_t err) {
    err = wave_or(err);
    if (status && err && (threadIdx.x & 63) == 0) atomicOr(status, err);
}

// ------------------------------------------------------ the hot kernel
//
// LDS layout (G real groups plus one trash slot G that takes the rows a
// workgroup skips, so that every row has a slot and a top):
//   bins[L][G+1][R]  int64 level sums; lane r deposits into replica r % R
//                    (R > 1 only when groups are few, to spread contention).
//                    Level-major, so that the words one level-add of a wave
//                    touches (random groups) spread over all LDS banks for
//                    every L; a group-major layout with a 16- or 32-byte
//                    group stride would use only part of the banks.
//   TOP[G+1]         {top index, high word of the level-0 extractor}
//   P[G+1]           pending top, raised with ds_max while a tile is read
// A workgroup-uniform fast path applies while every group sits at the same
// top Ju ("uni"): then no per-row LDS read of the top is needed.
constexpr int RAISED_MAX = 1024;  // groups listed per synchronisation (beyond: a full scan)

struct AggShared {
    int newmax;     // largest top after a realignment
    int cnt;        // groups at newmax
    int flag[3];    // "some top was raised" per synchronisation (3 rotating slots)
    int spills[3];  // rows deposited into the spill array, per synchronisation
    int nraised[3]; // groups whose pending top rose, per synchronisation
    int raised[RAISED_MAX];  // those groups (each once), for the realignment
};

// Raises the pending top of group g to j (j > cur, the group's top since the
// last synchronisation).  The lane whose atomic max lifts P from cur lists
// the group, so every raised group is listed exactly once per interval.
__device__ __forceinline__ void raise_top(int* P, int g, int j, int cur, AggShared& sh, int slot) {
    const int old = atomicMax(&P[g], j);
    if (old == cur) {
        const int k = atomicAdd(&sh.nraised[slot], 1);
        if (k < RAISED_MAX) sh.raised[k] = g;
    }
}

__device__ __forceinline__ uint32_t extractor_hi_of(double*, int top) {
    return extractor_hi((double*)0, Fmt<double>::B + top * Fmt<double>::W);
}
__device__ __forceinline__ uint32_t extractor_hi_of(float*, int top) {
    return extractor_hi((float*)0, Fmt<float>::B + top * Fmt<float>::W);
}

// Units of one value given the extractor bits of its level 0 (see
// extract_units): the extractor of level l is 2^(l*W) smaller.
template <int L>
__device__ __forceinline__ void extract_from_hi(double b, uint32_t h0, long long* k) {
    double r = b;
#pragma unroll
    for (int l = 0; l < L; ++l) {
        const uint32_t mh = h0 - (uint32_t)(l * Fmt<double>::W) * (1u << 20);
        const double M = __hiloint2double((int)mh, 0);
        const double s = r + M;
        if (l + 1 < L) {
            const double t = s - M;
            r = r - t;
        }
        const uint64_t sb = (uint64_t)__double_as_longlong(s);
        k[l] = (long long)(((uint64_t)((uint32_t)(sb >> 32) - mh) << 32) | (sb & 0xffffffffull));
    }
}
template <int L>
__device__ __forceinline__ void extract_from_hi(float b, uint32_t b0, long long* k) {
    float r = b;
#pragma unroll
    for (int l = 0; l < L; ++l) {
        const uint32_t mb = b0 - (uint32_t)(l * Fmt<float>::W) * (1u << 23);
        const float M = __uint_as_float(mb);
        const float s = r + M;
        k[l] = (long long)(int32_t)(__float_as_uint(s) - mb);
        if (l + 1 < L) {
            const float t = s - M;
            r = r - t;
        }
    }
}

// Smallest top index able to take b (jreq_of_exp) from the raw v_frexp
// exponent f = e + 1 of a finite nonzero value, branch-free: with
// x = f + m - W + 2 - B + W - 2 in [1, 2^11], floor(x / W) equals
// (x * ceil(2^16 / W)) >> 16 for W = 40 and W = 18 on that whole range;
// one 24-bit multiply-add.
template <class AT>
__device__ __forceinline__ int jreq_raw(int f) {
    typedef Fmt<AT> F;
    constexpr int mul = (65536 + F::W - 1) / F::W;
    constexpr int add = (F::m - F::W + 2 - F::B + F::W - 2) * mul;
    return (int)((uint32_t)__mul24(f, mul) + (uint32_t)add) >> 16;
}
// Magnitude below which a value needs no top above J: |b| < 2^(W-1) *
// ulp(S) at top J (the level-shift threshold of Alg. 2), so |b| < thr
// exactly when jreq(b) <= J.  A power of two, exact in AT.
template <class AT>
__device__ __forceinline__ AT top_threshold(int J) {
    typedef Fmt<AT> F;
    return ldexp((AT)1, F::B + J * F::W - F::m + F::W - 1);
}
__device__ __forceinline__ int frexp_raw(double v) { return __builtin_amdgcn_frexp_exp(v); }
__device__ __forceinline__ int frexp_raw(float v) { return __builtin_amdgcn_frexp_expf(v); }

// Per-row classification of a tile.  A row is deposited when its key is a
// group id and its value finite and zero or inside the domain of AT; other
// rows go to the trash slot G.  Zeros require no top (j = 0).  `clean` stays true
// while no row of this lane is an error (zero values are not errors).
// With SLICE, the bins hold only groups [glo, glo + G) of Gfull groups: a
// row whose key is a valid group outside the slice is skipped (no error);
// deposited rows get bin index key - glo.
template <bool FULL, bool SLICE, class KT, class VT, class AT, int N = ROWS_PER_THREAD>
__device__ __forceinline__ void classify_rows(const KT* kc, const VT* vc, uint32_t inr, int G, int* gi, int* ji,
                                              bool& clean, int64_t glo, int64_t Gfull) {
#pragma unroll
    for (int i = 0; i < N; ++i) {
        const VT v = vc[i];
        const bool in = FULL || ((inr >> i) & 1u);
        const int64_t key = (int64_t)kc[i];
        const bool kok = (uint64_t)key < (uint64_t)(SLICE ? Gfull : (int64_t)G);
        // a valid key is below 2^31, so its offset in the slice fits 32 bits
        const bool ins = SLICE ? (kok && (uint32_t)((uint32_t)key - (uint32_t)glo) < (uint32_t)G) : kok;
        const bool fin = finite_val(v);
        const bool nz = v != (VT)0;
        const int j = jreq_raw<AT>(frexp_raw(v));
        const bool dom = j <= Fmt<AT>::JMAX;
        // zeros keep their group (their units are zero) but raise no top
        const bool use = in && ins && fin && (dom || !nz);
        clean = clean && (!in || (kok && fin && (dom || !nz)));
        gi[i] = use ? (int)(SLICE ? (uint32_t)key - (uint32_t)glo : (uint32_t)key) : G;
        ji[i] = (use && nz) ? j : 0;
    }
}

// Status bits of the error rows among this lane's rows (slow path).
template <class KT, class VT, class AT, int N = ROWS_PER_THREAD>
__device__ __forceinline__ uint32_t error_bits(const KT* kc, const VT* vc, uint32_t inr, int64_t G) {
    uint32_t e = 0;
    for (int i = 0; i < N; ++i) {
        if (!((inr >> i) & 1u)) continue;
        const VT v = vc[i];
        if ((uint64_t)(int64_t)kc[i] >= (uint64_t)G) e |= ERR_KEY;
        if (!finite_val(v))
            e |= ERR_NONFINITE;
        else if (v != (VT)0 && jreq_raw<AT>(frexp_raw(v)) > Fmt<AT>::JMAX)
            e |= ERR_RANGE;
    }
    return e;
}

// Exact add of a unit into a spill word pair {w, H} holding H * 2^64 + w
// (w unsigned): the atomic add returns the old w, from which the carry out
// of this add (-1, 0 or +1) follows; it is added to H.
__device__ __forceinline__ void spill_add(unsigned long long* w, long long k) {
    const unsigned long long old = atomicAdd(w, (unsigned long long)k);
    const unsigned long long nw = old + (unsigned long long)k;
    const long long c = (k >= 0) ? (nw < old ? 1 : 0) : (nw > old ? -1 : 0);
    if (c) atomicAdd(w + 1, (unsigned long long)c);
}

// A row whose group's bins are aligned below its required top: its units
// are extracted at its own top jr (own-window deposit) and added into the
// spill array at their absolute lattice indices jr - l.  Extraction at any
// top between jr and the group's final top gives the same units at every
// lattice index the final state keeps, so nothing has to move later.
template <class AT, int L>
__device__ __forceinline__ void spill_row(unsigned long long* __restrict__ spill, int g, AT v, int jr) {
    constexpr int NJ = Fmt<AT>::JMAX + 1;
    long long k[L];
    extract_from_hi<L>(v, extractor_hi_of((AT*)0, jr), k);
#pragma unroll
    for (int l = 0; l < L; ++l) spill_add(spill + ((size_t)g * NJ + (jr - l)) * 2, k[l]);
}

// ----------------------------------------------------------- row sources
//
// The aggregation loop reads its rows through a source, which loads a
// tile's rows into registers and turns them into "virtual rows": one per
// (row, aggregated column), each with its bin group and its value in the
// accumulator type AT.

// One value column: virtual row i is row i of the thread's rows.
template <class KT, class VT, int VEC, int BLOCK, bool NT = true>
struct SrcCol {
    static constexpr int RPT = ROWS_PER_THREAD;  // rows per thread and tile
    static constexpr int NR = RPT;               // virtual rows per thread and tile
    static constexpr int TILE = BLOCK * RPT;
    struct Buf {
        KT k[RPT];
        VT v[RPT];
    };
    const KT* keys;
    const VT* vals;
    uint32_t off[RPT / VEC];
    __device__ SrcCol(const KT* k, const VT* v) : keys(k), vals(v) {
#pragma unroll
        for (int u = 0; u < RPT / VEC; ++u) off[u] = (uint32_t)((u * BLOCK + threadIdx.x) * VEC);
    }
    __device__ __forceinline__ uint32_t load(Buf& b, int64_t base, int64_t end) const {
        return load_tile<KT, VT, VEC, BLOCK, NT>(keys, vals, base, end, b.k, b.v, off);
    }
    template <bool FULL, bool SLICE, class AT>
    __device__ __forceinline__ void classify(const Buf& b, uint32_t inr, int G, int* gi, int* ji, bool& clean,
                                             int64_t glo, int64_t Gfull) const {
        classify_rows<FULL, SLICE, KT, VT, AT>(b.k, b.v, inr, G, gi, ji, clean, glo, Gfull);
    }
    template <class AT>
    __device__ __forceinline__ uint32_t errors(const Buf& b, uint32_t inr, int64_t G) const {
        return error_bits<KT, VT, AT>(b.k, b.v, inr, G);
    }
    // Full tile, one shared top (threshold thr, see top_threshold): a row
    // whose key is a group and whose value is finite with |v| < thr goes to
    // its group; any other row sets `slow` (it needs the general path).
    template <class AT>
    __device__ __forceinline__ void classify_fast(const Buf& b, int G, AT thr, int* gi, bool& slow) const {
        const VT t = (VT)thr;  // exact, or 0 / inf beyond VT's range (then every row, resp. none, is slow)
#pragma unroll
        for (int i = 0; i < RPT; ++i) {
            const bool ok = (uint64_t)(int64_t)b.k[i] < (uint64_t)G && finite_val(b.v[i]) && fabs(b.v[i]) < t;
            gi[i] = ok ? (int)b.k[i] : G;
            slow = slow || !ok;
        }
    }
    template <class AT>
    __device__ __forceinline__ AT value(const Buf& b, int i) const {
        return (AT)b.v[i];
    }
};

// NC value columns over one key column: virtual row c * RPT + r is column
// c of row r, deposited into bin group c * Gc + key (the bins hold NC * Gc
// groups).  Column c holds floats where bit c of the column mask is set,
// doubles otherwise; floats widen exactly when AT is double.  The mask is a
// compile-time constant FMC (floats stay 4 bytes in the registers of the
// prefetched tile and widen when used), or FM_RUNTIME: then it is the
// runtime f32mask and every value widens to double as it is loaded.  Rows
// are loaded two at a time (8- or 16-byte loads); every column must be
// aligned to two of its elements and the keys to two keys.
constexpr uint32_t FM_RUNTIME = 0xffffffffu;

template <class KT, class AT, int NC, int BLOCK, uint32_t FMC = FM_RUNTIME>
struct SrcCols {
    static constexpr int RPT = 8 / NC >= 2 ? 8 / NC : 2;
    static constexpr int VEC = 2;
    static constexpr int NR = RPT * NC;
    static constexpr int TILE = BLOCK * RPT;
    static constexpr bool CT = FMC != FM_RUNTIME;
    struct Buf {
        KT k[RPT];
        double d[NC][RPT];  // double columns (every column when the mask is a runtime one)
        float f[NC][RPT];   // float columns of a compile-time mask
    };
    const KT* keys;
    const void* vals[NC];
    uint32_t f32mask;
    int Gc;  // groups per column
    uint32_t off[RPT / VEC];
    __device__ SrcCols(const KT* k, const void* const* v, uint32_t fm, int gc) : keys(k), f32mask(fm), Gc(gc) {
#pragma unroll
        for (int c = 0; c < NC; ++c) vals[c] = v[c];
#pragma unroll
        for (int u = 0; u < RPT / VEC; ++u) off[u] = (uint32_t)((u * BLOCK + threadIdx.x) * VEC);
    }
    // column c stored as float (compile-time masks only)
    static constexpr bool stored_f32(int c) { return CT && ((FMC >> c) & 1u); }
    template <class VT, class OT>
    __device__ __forceinline__ void load_col(const VT* __restrict__ vb, OT* out, bool full, uint32_t lim) const {
        if (full) {
#pragma unroll
            for (int u = 0; u < RPT / VEC; ++u) {
                VT x[VEC];
                vload<VT, VEC, true>(vb + off[u], x);
#pragma unroll
                for (int e = 0; e < VEC; ++e) out[u * VEC + e] = (OT)x[e];
            }
        } else {
#pragma unroll
            for (int u = 0; u < RPT / VEC; ++u)
#pragma unroll
                for (int e = 0; e < VEC; ++e) out[u * VEC + e] = (off[u] + e < lim) ? (OT)vb[off[u] + e] : (OT)0;
        }
    }
    __device__ __forceinline__ uint32_t load(Buf& b, int64_t base, int64_t end) const {
        const bool full = base + (int64_t)TILE <= end;
        const uint32_t lim = full ? 0u : (uint32_t)(end - base);
        const KT* kb = keys + base;
        uint32_t inr = 0;
        if (full) {
#pragma unroll
            for (int u = 0; u < RPT / VEC; ++u) vload<KT, VEC, true>(kb + off[u], b.k + u * VEC);
            inr = (1u << RPT) - 1;
        } else {
#pragma unroll
            for (int u = 0; u < RPT / VEC; ++u)
#pragma unroll
                for (int e = 0; e < VEC; ++e) {
                    const uint32_t row = off[u] + e;
                    const bool in = row < lim;
                    b.k[u * VEC + e] = in ? kb[row] : (KT)0;
                    inr |= in ? 1u << (u * VEC + e) : 0u;
                }
        }
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            if constexpr (CT) {
                if (stored_f32(c))
                    load_col<float, float>(static_cast<const float*>(vals[c]) + base, b.f[c], full, lim);
                else
                    load_col<double, double>(static_cast<const double*>(vals[c]) + base, b.d[c], full, lim);
            } else {
                if ((f32mask >> c) & 1u)
                    load_col<float, double>(static_cast<const float*>(vals[c]) + base, b.d[c], full, lim);
                else
                    load_col<double, double>(static_cast<const double*>(vals[c]) + base, b.d[c], full, lim);
            }
        }
        return inr;
    }
    template <bool FULL, bool SLICE, class AT_>
    __device__ __forceinline__ void classify(const Buf& b, uint32_t inr, int G, int* gi, int* ji, bool& clean,
                                             int64_t, int64_t) const {
        static_assert(!SLICE, "column sources have no group slices");
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            int gc[RPT], jc[RPT];
            if (stored_f32(c))
                classify_rows<FULL, false, KT, float, AT_, RPT>(b.k, b.f[c], inr, Gc, gc, jc, clean, 0, 0);
            else
                classify_rows<FULL, false, KT, double, AT_, RPT>(b.k, b.d[c], inr, Gc, gc, jc, clean, 0, 0);
#pragma unroll
            for (int r = 0; r < RPT; ++r) {
                gi[c * RPT + r] = gc[r] == Gc ? G : c * Gc + gc[r];  // skipped rows: the trash slot G = NC * Gc
                ji[c * RPT + r] = jc[r];
            }
        }
    }
    template <class AT_>
    __device__ __forceinline__ void classify_fast(const Buf& b, int G, AT_ thr, int* gi, bool& slow) const {
        const float tf = (float)thr;
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            const bool kok = (uint64_t)(int64_t)b.k[r] < (uint64_t)Gc;
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                bool ok;
                if (stored_f32(c))
                    ok = kok && finite_val(b.f[c][r]) && fabsf(b.f[c][r]) < tf;
                else
                    ok = kok && finite_val(b.d[c][r]) && fabs(b.d[c][r]) < (double)thr;
                gi[c * RPT + r] = ok ? c * Gc + (int)b.k[r] : G;
                slow = slow || !ok;
            }
        }
    }
    template <class AT_>
    __device__ __forceinline__ uint32_t errors(const Buf& b, uint32_t inr, int64_t) const {
        uint32_t e = 0;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            if (stored_f32(c))
                e |= error_bits<KT, float, AT_, RPT>(b.k, b.f[c], inr, Gc);
            else
                e |= error_bits<KT, double, AT_, RPT>(b.k, b.d[c], inr, Gc);
        }
        return e;
    }
    template <class AT_>
    __device__ __forceinline__ AT_ value(const Buf& b, int i) const {
        return stored_f32(i / RPT) ? (AT_)b.f[i / RPT][i % RPT] : (AT_)b.d[i / RPT][i % RPT];
    }
};

constexpr int EPOCH_TILES = 16;       // tiles between synchronisations in epoch mode, at first
constexpr int EPOCH_TILES_MAX = 256;  // after quiet epochs (no row spilled) the epoch doubles up to this
constexpr int QUIET_TILES = 1;   // quiet per-tile synchronisations before epoch mode

// The aggregation of rows [c0, c1) into LDS by one workgroup (the hot loop
// of both aggregation kernels).  On return the bins are aligned to every
// group's top (TOP), and the lane's status bits are returned.  EPOCH
// enables epoch mode, which needs the spill array, and the tracking of a
// top shared by all groups (few groups, whose tops settle early); without
// it every tile synchronises and rows read their group's top from LDS.
// The rows come from `src` (a row source above); G counts the bin groups.
template <class Src, class AT, int L, bool EPOCH, bool SLICE, int BLOCK>
__device__ __forceinline__ uint32_t aggregate_src(const Src& src, int64_t c0, int64_t c1, int G, int R,
                                                  unsigned char* smem, AggShared& sh,
                                                  unsigned long long* __restrict__ spill, int64_t glo, int64_t Gfull,
                                                  const int* __restrict__ seed = nullptr) {
    constexpr int TILE = Src::TILE;  // rows of one tile
    constexpr int NR = Src::NR;      // virtual rows per thread and tile
    typedef Fmt<AT> F;
    typedef typename Src::Buf Buf;
    long long* bins = reinterpret_cast<long long*>(smem);
    int2* TOP = reinterpret_cast<int2*>(bins + (size_t)(G + 1) * R * L);
    int* P = reinterpret_cast<int*>(TOP + (G + 1));

    const int tid = threadIdx.x;
    const int rep = (tid & 63) & (R - 1);
    const uint32_t gstride = (uint32_t)(R * 8);             // bytes per group in a level
    const uint32_t lstride = (uint32_t)((G + 1) * R * 8);   // bytes per level
    const uint32_t lane_off = (uint32_t)(rep * 8);
    for (int i = tid; i < (G + 1) * R * L; i += BLOCK) bins[i] = 0;
    const uint32_t h_init = extractor_hi_of((AT*)0, L - 1);
    int tmax = L - 1;  // largest seeded top of this thread's groups
    for (int i = tid; i < G; i += BLOCK) {
        int t = L - 1;
        if (EPOCH && seed) t = min(max(t, seed[i]), F::JMAX);
        TOP[i] = make_int2(t, t == L - 1 ? (int)h_init : (int)extractor_hi_of((AT*)0, t));
        P[i] = t;
        tmax = max(tmax, t);
    }
    if (tid == 0) {
        TOP[G] = make_int2(F::JMAX, (int)extractor_hi_of((AT*)0, F::JMAX));  // trash slot: never raised
        P[G] = F::JMAX;
        sh.newmax = L - 1;
        sh.cnt = (EPOCH && seed) ? 0 : G;
        for (int q = 0; q < 3; ++q) sh.flag[q] = sh.spills[q] = sh.nraised[q] = 0;
    }
    __syncthreads();

    // workgroup-uniform state
    bool uni = true;   // all groups aligned to top Ju
    int Ju = L - 1;
    uint32_t hu = h_init;
    AT thr = top_threshold<AT>(Ju);  // values below it need no top above Ju
    int sync = 0;      // synchronisations so far (selects the flag slot)
    int epoch_left = 0;  // tiles left in the current epoch (0: per-tile mode)
    int epoch_len = EPOCH_TILES;  // tiles of the current epoch
    int quiet = 0;     // consecutive per-tile synchronisations without a raise
    bool ahead = false;  // this tile's tops were raised at the previous synchronisation
    if (EPOCH && seed) {
        // seeded tops: whether they are all equal, then straight into epoch mode
        atomicMax(&sh.newmax, tmax);
        __syncthreads();
        const int nm = sh.newmax;
        int c = 0;
        for (int g = tid; g < G; g += BLOCK) c += (TOP[g].x == nm);
        if (c) atomicAdd(&sh.cnt, c);
        __syncthreads();
        uni = (sh.cnt == G);
        Ju = nm;
        hu = extractor_hi_of((AT*)0, Ju);
        thr = top_threshold<AT>(Ju);
        epoch_left = epoch_len;
    }

    // Per-tile mode: when many lanes of a wave deposit into one group (skewed
    // keys), that "hot" group (wave-uniform) is summed in registers and added
    // to its bins with one atomic per level before the next synchronisation
    // (its top, and so the units' alignment, only changes there).  Exact, so
    // the bits are the same; it spares the serialised same-address atomics.
    constexpr int HOT_MIN = 8;  // lanes of a wave on one group that make it hot
    int hot = -1;
    long long hacc[L];
#pragma unroll
    for (int l = 0; l < L; ++l) hacc[l] = 0;
    auto flush_hot = [&]() {
        if (EPOCH || hot < 0) return;  // uniform
        unsigned char* w0 = smem + __umul24((uint32_t)hot, gstride);
#pragma unroll
        for (int l = 0; l < L; ++l) {
            const long long x = wave_sum64(hacc[l]);
            if ((tid & 63) == 0 && x != 0)
                atomicAdd(reinterpret_cast<unsigned long long*>(w0 + l * lstride), (unsigned long long)x);
            hacc[l] = 0;
        }
    };

    // Synchronisation point: all deposits before it are done.  If a top was
    // raised since the last one, realign every group with P > TOP (its levels
    // move down by the rise, the lowest fall off: the level shift of Alg. 2)
    // and recompute whether all groups share one top.  Returns whether rows
    // went to the spill array since the last synchronisation.
    auto synchronise = [&](int& spilled) {
        __syncthreads();
        const int f = sh.flag[sync % 3];
        spilled = sh.spills[sync % 3];
        const int nr = sh.nraised[sync % 3];
        if (tid == 0) {  // slot (sync+2)%3 was read at the previous synchronisation
            sh.flag[(sync + 2) % 3] = 0;   // and is next written after the following one
            sh.spills[(sync + 2) % 3] = 0;
            sh.nraised[(sync + 2) % 3] = 0;
        }
        ++sync;
        if (!f) return false;
        int m = -1;  // largest realigned top (the others did not move)
        auto realign = [&](int g) {
            const int p = P[g];
            const int top = TOP[g].x;
            if (p > top) {
                const int d = p - top;
                const size_t ls = (size_t)(G + 1) * R;  // words per level
                for (int r = 0; r < R; ++r) {
                    long long* w = bins + (size_t)g * R + r;
#pragma unroll
                    for (int l = L - 1; l >= 0; --l) w[l * ls] = (l - d >= 0) ? w[(l - d) * ls] : 0;
                }
                TOP[g] = make_int2(p, (int)extractor_hi_of((AT*)0, p));
                m = max(m, p);
            }
        };
        if (nr <= RAISED_MAX) {
            for (int k = tid; k < nr; k += BLOCK) realign(sh.raised[k]);
        } else {
            for (int g = tid; g < G; g += BLOCK) realign(g);
        }
        if (!EPOCH) {
            // many groups whose tops rise at different times: no shared top
            __syncthreads();
            uni = false;
            return true;
        }
        if (tid == 0) sh.cnt = 0;
        atomicMax(&sh.newmax, m);  // newmax only grows: tops never fall
        __syncthreads();
        const int nm = sh.newmax;
        int c = 0;
        for (int g = tid; g < G; g += BLOCK) c += (TOP[g].x == nm);
        if (c) atomicAdd(&sh.cnt, c);
        __syncthreads();
        uni = (sh.cnt == G);
        Ju = nm;
        hu = extractor_hi_of((AT*)0, Ju);
        thr = top_threshold<AT>(Ju);
        return true;
    };

    uint32_t err = 0;

    // software pipeline: tiles base+TILE .. base+PREFETCH*TILE are in
    // flight (in registers) while tile `base` is processed
    Buf buf[PREFETCH + 1];
    uint32_t inr[PREFETCH + 1];
#pragma unroll
    for (int q = 0; q <= PREFETCH; ++q) inr[q] = 0;
#pragma unroll
    for (int q = 0; q < PREFETCH; ++q)
        if (c0 + (int64_t)q * TILE < c1) inr[q] = src.load(buf[q], c0 + (int64_t)q * TILE, c1);

    for (int64_t base = c0; base < c1; base += TILE) {
        const int64_t nb = base + (int64_t)PREFETCH * TILE;
        if (nb < c1)
            inr[PREFETCH] = src.load(buf[PREFETCH], nb, c1);
        else
            inr[PREFETCH] = 0;
        const Buf& bc = buf[0];
        const uint32_t inr_c = inr[0];

        int gi[NR];
        uint32_t hi_[NR];
        // Epoch mode with one top for every group, full tile: when every row
        // of the wave has a valid key and a finite value below the top's
        // threshold, its group is all it needs (no error bits, no raise);
        // otherwise the wave takes the general path below.  Waves decide
        // apart: neither path synchronises the workgroup in epoch mode.
        bool fast = false;
        if constexpr (EPOCH && !SLICE) {
            if (uni && epoch_left > 0 && base + TILE <= c1) {
                bool slow = false;
                src.template classify_fast<AT>(bc, G, thr, gi, slow);
                fast = __ballot(slow) == 0;
            }
        }
        if (!fast) {
        // classify: group (trash slot G for skipped rows) and required top
        int ji[NR];
        bool clean = true;  // no row of this lane is an error row
        if (base + TILE <= c1)
            src.template classify<true, SLICE, AT>(bc, inr_c, G, gi, ji, clean, glo, Gfull);
        else
            src.template classify<false, SLICE, AT>(bc, inr_c, G, gi, ji, clean, glo, Gfull);
        if (!clean)
            err |= src.template errors<AT>(bc, base + TILE <= c1 ? (1u << Src::RPT) - 1 : inr_c, SLICE ? Gfull : G);

        // tops of the rows' groups
        int ai[NR];
        if (uni) {
#pragma unroll
            for (int i = 0; i < NR; ++i) {
                ai[i] = Ju;
                hi_[i] = hu;
            }
        } else {
#pragma unroll
            for (int i = 0; i < NR; ++i) {
                const int2 tp = TOP[gi[i]];
                ai[i] = tp.x;
                hi_[i] = (uint32_t)tp.y;
            }
        }
        bool raise = false;
#pragma unroll
        for (int i = 0; i < NR; ++i) raise = raise || (ji[i] > ai[i]);
        if (!EPOCH && ahead) {
            // its rows' tops were raised and realigned with the previous tile
            ahead = false;
        } else if (epoch_left == 0) {
            // per-tile mode: raise the tops, synchronise, then deposit
            if (raise) {
                sh.flag[sync % 3] = 1;
#pragma unroll
                for (int i = 0; i < NR; ++i)
                    if (ji[i] > ai[i]) raise_top(P, gi[i], ji[i], ai[i], sh, sync % 3);
            }
            if (!EPOCH) {
                // look ahead: raise the tops of the prefetched tile's rows in
                // the same synchronisation, so that tile needs none
                int gn[NR], jn[NR];
                bool cn = true;
                src.template classify<false, SLICE, AT>(buf[PREFETCH], inr[PREFETCH], G, gn, jn, cn, glo, Gfull);
                bool rn = false;
#pragma unroll
                for (int i = 0; i < NR; ++i) {
                    const int cur = TOP[gn[i]].x;
                    if (jn[i] > cur) {
                        raise_top(P, gn[i], jn[i], cur, sh, sync % 3);
                        rn = true;
                    }
                }
                if (rn) sh.flag[sync % 3] = 1;
                ahead = true;
            }
            int sp;
            flush_hot();
            const bool moved = synchronise(sp);
            quiet = moved ? 0 : quiet + 1;
            if (EPOCH && quiet >= QUIET_TILES) epoch_left = epoch_len = EPOCH_TILES;
            if (moved) {
                if (uni) {
#pragma unroll
                    for (int i = 0; i < NR; ++i) hi_[i] = hu;
                } else {
#pragma unroll
                    for (int i = 0; i < NR; ++i) hi_[i] = (uint32_t)TOP[gi[i]].y;
                }
            }
        } else if (raise) {
            // epoch mode: rows above their group's top go to the spill array
            int ns = 0;
#pragma unroll
            for (int i = 0; i < NR; ++i) {
                if (ji[i] > ai[i]) {
                    raise_top(P, gi[i], ji[i], ai[i], sh, sync % 3);
                    spill_row<AT, L>(spill, gi[i], src.template value<AT>(bc, i), ji[i]);
                    gi[i] = G;  // nothing more for the bins
                    ++ns;
                }
            }
            sh.flag[sync % 3] = 1;
            atomicAdd(&sh.spills[sync % 3], ns);
        }
        }  // general path
        if (!EPOCH) {
            const int g0 = __builtin_amdgcn_readfirstlane(gi[0]);
            if (g0 != hot && g0 != G && __popcll(__ballot(gi[0] == g0)) >= HOT_MIN) {
                flush_hot();
                hot = g0;
            }
        }
        // extract and deposit
        if constexpr (EPOCH && !SLICE) {
            // branch-free: skipped rows (errors; their units are arbitrary)
            // add into the trash slot G, which is never read, so the rows'
            // extraction chains can interleave.  With one top for every group
            // the extractors are workgroup-uniform (scalar registers).
            if (uni) {
                const uint32_t hs = __builtin_amdgcn_readfirstlane(hu);
#pragma unroll
                for (int i = 0; i < NR; ++i) {
                    long long k[L];
                    extract_from_hi<L>(src.template value<AT>(bc, i), hs, k);
                    unsigned char* w = smem + __umul24((uint32_t)gi[i], gstride) + lane_off;
#pragma unroll
                    for (int l = 0; l < L; ++l)
                        atomicAdd(reinterpret_cast<unsigned long long*>(w + l * lstride), (unsigned long long)k[l]);
                }
            } else {
#pragma unroll
                for (int i = 0; i < NR; ++i) {
                    long long k[L];
                    extract_from_hi<L>(src.template value<AT>(bc, i), hi_[i], k);
                    unsigned char* w = smem + __umul24((uint32_t)gi[i], gstride) + lane_off;
#pragma unroll
                    for (int l = 0; l < L; ++l)
                        atomicAdd(reinterpret_cast<unsigned long long*>(w + l * lstride), (unsigned long long)k[l]);
                }
            }
        } else {
        // skipped rows (trash slot G: errors, and in slice mode the rows of
        // other slices) issue no LDS atomics
#pragma unroll
        for (int i = 0; i < NR; ++i) {
            long long k[L];
            extract_from_hi<L>(src.template value<AT>(bc, i), hi_[i], k);
            unsigned char* w = smem + __umul24((uint32_t)gi[i], gstride) + lane_off;
            if (!EPOCH && gi[i] == hot) {
#pragma unroll
                for (int l = 0; l < L; ++l) hacc[l] += k[l];
            } else if (gi[i] != G) {
#pragma unroll
                for (int l = 0; l < L; ++l)
                    atomicAdd(reinterpret_cast<unsigned long long*>(w + l * lstride), (unsigned long long)k[l]);
            }
        }
        }
        if (epoch_left > 0 && --epoch_left == 0) {
            int sp;
            synchronise(sp);
            // many spills: the tops are still moving, go back to per-tile mode
            // no spill: the tops have settled, synchronise half as often
            epoch_len = sp == 0 ? min(2 * epoch_len, EPOCH_TILES_MAX) : EPOCH_TILES;
            epoch_left = (sp > TILE / 16) ? 0 : epoch_len;
            quiet = 0;
        }
#pragma unroll
        for (int q = 0; q < PREFETCH; ++q) {
            buf[q] = buf[q + 1];
            inr[q] = inr[q + 1];
        }
    }
    // final synchronisation: tops include every spilled row, bins aligned
    int sp;
    flush_hot();
    synchronise(sp);
    return err;
}

// One value column (the row source SrcCol).
template <class KT, class VT, class AT, int L, int VEC, bool EPOCH, bool SLICE = false, int BLOCK = AGG_BLOCK,
          bool NT = true>
__device__ __forceinline__ uint32_t aggregate_range(const KT* __restrict__ keys, const VT* __restrict__ vals,
                                                    int64_t c0, int64_t c1, int G, int R, unsigned char* smem,
                                                    AggShared& sh, unsigned long long* __restrict__ spill,
                                                    int64_t glo = 0, int64_t Gfull = 0,
                                                    const int* __restrict__ seed = nullptr) {
    typedef SrcCol<KT, VT, VEC, BLOCK, NT> Src;
    const Src src(keys, vals);
    return aggregate_src<Src, AT, L, EPOCH, SLICE, BLOCK>(src, c0, c1, G, R, smem, sh, spill, glo, Gfull, seed);
}

// Seed tops (epoch-mode launches over many tiles): one tile per workgroup,
// spread evenly over the rows, raises seed[g] (zero-initialised) to the
// largest required top of group g among its rows.  The aggregation then
// starts every group at that top instead of its lowest one: any top between
// the lowest and the final one gives the same bits (extraction at a higher
// top and realignment agree), so only the number of synchronisations while
// tops settle changes.
template <class Src, class AT, int BLOCK>
__device__ __forceinline__ void sample_tops(const Src& src, int64_t n, int64_t tile_stride, int G, int* lt,
                                            int* __restrict__ seed) {
    constexpr int NR = Src::NR;
    for (int i = threadIdx.x; i <= G; i += BLOCK) lt[i] = 0;
    __syncthreads();
    typename Src::Buf b;
    const int64_t base = (int64_t)blockIdx.x * tile_stride;
    const uint32_t inr = src.load(b, base, n);
    int gi[NR], ji[NR];
    bool clean = true;
    src.template classify<false, false, AT>(b, inr, G, gi, ji, clean, 0, 0);
#pragma unroll
    for (int i = 0; i < NR; ++i)
        if (ji[i] > 0) atomicMax(&lt[gi[i]], ji[i]);  // error rows and zeros have ji = 0
    __syncthreads();
    for (int g = threadIdx.x; g < G; g += BLOCK)
        if (lt[g] > 0) atomicMax(&seed[g], lt[g]);
}

// Folds a workgroup's aligned LDS level sums of group g (K[l * ks], top
// `top`) and the caller's state of that group into a canonical state.
template <class AT, int L>
__device__ __forceinline__ void fold_into_state(const long long* K, int ks, int top, AT* __restrict__ S,
                                                long long* __restrict__ C, int64_t G, int64_t g) {
    typedef Fmt<AT> F;
    constexpr int c = F::CARRY;
    const int ts = state_top(S[g]);
    const int J = max(top, ts);
    long long hi[L], lo[L];
#pragma unroll
    for (int l = 0; l < L; ++l) {
        const int ls = l - (J - ts), lk = l - (J - top);
        hi[l] = (ls >= 0) ? C[(size_t)ls * G + g] : 0;
        lo[l] = (ls >= 0) ? state_lo(S[(size_t)ls * G + g]) : 0;
        long long x = 0;
#pragma unroll
        for (int q = 0; q < L; ++q) x = (q == lk) ? K[q * ks] : x;
        hi[l] += x >> c;
        lo[l] += x & ((1ll << c) - 1);
    }
#pragma unroll
    for (int l = 0; l < L; ++l) {
        long long cc, oo;
        normalise<AT>(hi[l], lo[l], &cc, &oo);
        S[(size_t)l * G + g] = make_S((AT*)0, F::B + (J - l) * F::W, oo);
        C[(size_t)l * G + g] = cc;
    }
}

// Hand-over of partial results between the workgroups of one launch (the
// last one to finish merges the others'): the words are written with
// device-scope stores, which go through to the point where every XCD sees
// them; each thread waits for its stores to complete (published) before the
// workgroup raises the arrival counter; the last workgroup reads them with
// device-scope loads.  A device-wide __threadfence() would instead write
// back the XCD's whole L2 once per workgroup, which costs microseconds each.
template <class T>
__device__ __forceinline__ void publish(T* p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T>
__device__ __forceinline__ T collect(const T* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void published() {
    __atomic_signal_fence(__ATOMIC_SEQ_CST);  // no memory access moves across
    __builtin_amdgcn_s_waitcnt(0);            // this thread's stores and atomics are complete
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// Writes the canonical state of group g from (hi, lo) level words at top J,
// and its finalised sum (equation of Sec. III-C) when `out` is given.
template <class AT, int L>
__device__ __forceinline__ void write_group(const long long* hi, const long long* lo, int J, AT* S, long long* C,
                                            int G, int g, AT* out) {
    typedef Fmt<AT> F;
    AT q[L];
#pragma unroll
    for (int l = 0; l < L; ++l) {
        long long cc, oo;
        normalise<AT>(hi[l], lo[l], &cc, &oo);
        S[(size_t)l * G + g] = make_S((AT*)0, F::B + (J - l) * F::W, oo);
        C[(size_t)l * G + g] = cc;
        if (out) {
            const i128 K = (i128)cc * ((i128)1 << F::CARRY) + (i128)oo;
            q[l] = round_exact<AT>(K, F::B + (J - l) * F::W - F::m);
        }
    }
    if (out) {
        AT acc = q[L - 1];
#pragma unroll
        for (int l = L - 2; l >= 0; --l) acc = acc + q[l];
        out[g] = acc + (AT)0;
    }
}

// Adds the level sums x[L] at top `top` to (hi, lo) words at top J >= top.
template <class AT, int L>
__device__ __forceinline__ void add_levels(const long long* x, int top, int J, long long* hi, long long* lo) {
    constexpr int c = Fmt<AT>::CARRY;
    const int d = J - top;
#pragma unroll
    for (int l = 0; l < L; ++l) {
        long long v = 0;
#pragma unroll
        for (int q = 0; q < L; ++q) v = (q == l - d) ? x[q] : v;
        hi[l] += v >> c;
        lo[l] += v & ((1ll << c) - 1);
    }
}

// Adds the spill words of one group (exact 128-bit units H * 2^64 + w per
// absolute lattice index) kept at levels J - l, l < L, to (hi, lo).
// The words are read with device-scope loads: other workgroups' atomics
// may have updated them during the same launch (see publish above).
template <class AT, int L>
__device__ __forceinline__ void add_spill(const unsigned long long* sw, int J, long long* hi, long long* lo) {
    constexpr int c = Fmt<AT>::CARRY;
#pragma unroll
    for (int l = 0; l < L; ++l) {
        const unsigned long long* w = sw + (size_t)(J - l) * 2;
        const i128 T = (i128)(long long)collect(w + 1) * ((i128)1 << 64) + (i128)collect(w);
        hi[l] += (long long)(T >> c);
        lo[l] += (long long)(T & ((1ll << c) - 1));
    }
}

// Starts (hi, lo) level words at top J from the caller's state of group g
// (C into hi, the low part of S into lo, moved down by J - top), or from
// the empty state when the job overwrites.  Returns nothing: J must already
// include the state's top (state_top_of).
template <class AT, int L>
__device__ __forceinline__ void start_from_state(const AT* S, const long long* C, int G, int g, bool use, int J,
                                                 long long* hi, long long* lo) {
#pragma unroll
    for (int l = 0; l < L; ++l) hi[l] = lo[l] = 0;
    if (!use) return;
    const int d = J - state_top(S[g]);
#pragma unroll
    for (int l = 0; l < L; ++l) {
        if (l - d >= 0) {
            hi[l] = C[(size_t)(l - d) * G + g];
            lo[l] = state_lo(S[(size_t)(l - d) * G + g]);
        }
    }
}

}  // namespace
}  // namespace repro

#endif  // REPRO_AGG_HPP
