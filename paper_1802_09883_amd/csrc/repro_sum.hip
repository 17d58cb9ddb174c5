// repro_sum.hip -- ungrouped reproducible sum into repro<T,L>, exact
// per-group counts and aggregates derived from reproducible sums (librepro,
// gfx950).
//
// Paper: Mueller, Arteaga, Hoefler, Alonso, "Reproducible Floating-Point
// Aggregation in RDBMSs" (arXiv 1802.09883).  With one group the work maps
// onto the vectorised RSum (Sec. III-D, Alg. 3): every lane keeps its own
// accumulator (a top lattice index and L exact integer level sums) and
// raises its own top when a value needs it (the level shift of Alg. 2, done
// in registers); the lanes are merged at the end like the lanes of Alg. 3,
// by realigning to the largest top and adding the level sums exactly.  No
// keys are read and no atomics or barriers sit in the loop.  The bits are
// those of repro_groupby_sum with every key 0 and one group.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "repro.h"
#include "repro_agg.hpp"
#include "repro_device.hpp"

using namespace repro;

namespace {

constexpr int SUM_BLOCK = 256;     // 4 waves
constexpr int SUM_RPT = 8;         // rows per lane and step
constexpr int SUM_STEP = SUM_BLOCK * SUM_RPT;
constexpr int SUM_MAX_WG = 1024;   // 4 workgroups per CU: half the partials of 8 for the merge, same bandwidth
constexpr int64_t SUM_MAX_ROWS_PER_LANE = 1 << 16;  // lane sums stay below 2^55

// Level words of a lane moved down by d levels (the lowest fall off).
template <int L>
__device__ __forceinline__ void shift_down(long long* acc, int d) {
#pragma unroll
    for (int l = L - 1; l >= 0; --l) {
        long long v = 0;
#pragma unroll
        for (int q = 0; q < L; ++q) v = (q == l - d) ? acc[q] : v;
        acc[l] = v;
    }
}

__device__ __forceinline__ int wave_max(int x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x = max(x, __shfl_xor(x, o, 64));
    return x;
}
__device__ __forceinline__ long long wave_add(long long x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}

// Each workgroup sums rows [b * chunk, ...) and writes its partial: top,
// then (hi, lo) per level with lo in [0, 2^CARRY) (value hi * 2^CARRY + lo).
template <class VT, class AT, int L, int VEC>
__global__ void __launch_bounds__(SUM_BLOCK) k_sum(const VT* __restrict__ vals, int64_t n, int64_t chunk,
                                                   int* __restrict__ ptop, long long* __restrict__ phi,
                                                   long long* __restrict__ plo, uint32_t* __restrict__ status) {
    typedef Fmt<AT> F;
    constexpr int c = F::CARRY;
    constexpr int U = SUM_RPT / VEC;
    __shared__ int sJ;
    __shared__ long long sH[SUM_BLOCK / 64][L], sL[SUM_BLOCK / 64][L];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t c0 = (int64_t)blockIdx.x * chunk;
    const int64_t c1 = min(n, c0 + chunk);
    int top = L - 1;
    uint32_t h = extractor_hi_of((AT*)0, top);
    long long acc[L];
#pragma unroll
    for (int l = 0; l < L; ++l) acc[l] = 0;
    uint32_t err = 0;
    for (int64_t base = c0; base < c1; base += SUM_STEP) {
        VT v[SUM_RPT];
        if (base + SUM_STEP <= c1) {
#pragma unroll
            for (int u = 0; u < U; ++u) vload<VT, VEC>(vals + base + (int64_t)(u * SUM_BLOCK + tid) * VEC, v + u * VEC);
        } else {
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int e = 0; e < VEC; ++e) {
                    const int64_t i = base + (int64_t)(u * SUM_BLOCK + tid) * VEC + e;
                    v[u * VEC + e] = (i < c1) ? vals[i] : (VT)0;
                }
        }
#pragma unroll
        for (int i = 0; i < SUM_RPT; ++i) {
            const AT b = (AT)v[i];
            const bool fin = finite_val(b);
            const int j = jreq_raw<AT>(frexp_raw(b));
            const bool nz = b != (AT)0;
            const bool dom = j <= F::JMAX;
            err |= fin ? ((nz && !dom) ? ERR_RANGE : 0u) : ERR_NONFINITE;
            const bool use = fin && nz && dom;
            if (use && j > top) {  // this lane's level shift (rare once the top settles)
                shift_down<L>(acc, j - top);
                top = j;
                h = extractor_hi_of((AT*)0, top);
            }
            long long k[L];
            extract_from_hi<L>(use ? b : (AT)0, h, k);  // 0 gives units 0
#pragma unroll
            for (int l = 0; l < L; ++l) acc[l] += k[l];
        }
    }
    // workgroup top, then every lane realigned to it
    if (tid == 0) sJ = L - 1;
    __syncthreads();
    const int wj = wave_max(top);
    if (lane == 0) atomicMax(&sJ, wj);
    __syncthreads();
    const int J = sJ;
    shift_down<L>(acc, J - top);
#pragma unroll
    for (int l = 0; l < L; ++l) {
        const long long hi = wave_add(acc[l] >> c);
        const long long lo = wave_add(acc[l] & ((1ll << c) - 1));
        if (lane == 0) {
            sH[wave][l] = hi;
            sL[wave][l] = lo;
        }
    }
    __syncthreads();
    if (tid == 0) {
#pragma unroll
        for (int l = 0; l < L; ++l) {
            long long hi = 0, lo = 0;
            for (int w = 0; w < SUM_BLOCK / 64; ++w) {
                hi += sH[w][l];
                lo += sL[w][l];
            }
            long long cc, oo;
            normalise<AT>(hi, lo, &cc, &oo);
            phi[(size_t)blockIdx.x * L + l] = cc;
            plo[(size_t)blockIdx.x * L + l] = oo;
        }
        ptop[blockIdx.x] = J;
    }
    report(status, err);
}

// One workgroup: folds every partial and the caller's state into the
// canonical state of the single group.
template <class AT, int L>
__global__ void __launch_bounds__(SUM_BLOCK) k_sum_merge(const int* __restrict__ ptop,
                                                         const long long* __restrict__ phi,
                                                         const long long* __restrict__ plo, int np,
                                                         AT* __restrict__ S, long long* __restrict__ C) {
    typedef Fmt<AT> F;
    __shared__ int sJ;
    __shared__ long long sH[SUM_BLOCK / 64][L], sL[SUM_BLOCK / 64][L];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int ts = state_top(S[0]);
    if (tid == 0) sJ = ts;
    __syncthreads();
    int m = ts;
    for (int p = tid; p < np; p += SUM_BLOCK) m = max(m, ptop[p]);
    m = wave_max(m);
    if (lane == 0) atomicMax(&sJ, m);
    __syncthreads();
    const int J = sJ;
    long long hi[L], lo[L];
#pragma unroll
    for (int l = 0; l < L; ++l) hi[l] = lo[l] = 0;
    for (int p = tid; p < np; p += SUM_BLOCK) {
        const int d = J - ptop[p];
#pragma unroll
        for (int l = 0; l < L; ++l) {
            if (l - d >= 0) {
                hi[l] += phi[(size_t)p * L + (l - d)];
                lo[l] += plo[(size_t)p * L + (l - d)];
            }
        }
    }
#pragma unroll
    for (int l = 0; l < L; ++l) {
        const long long a = wave_add(hi[l]), b = wave_add(lo[l]);
        if (lane == 0) {
            sH[wave][l] = a;
            sL[wave][l] = b;
        }
    }
    __syncthreads();
    if (tid != 0) return;
    const int ds = J - ts;
#pragma unroll
    for (int l = 0; l < L; ++l) {
        long long a = (l - ds >= 0) ? C[l - ds] : 0;
        long long b = (l - ds >= 0) ? state_lo(S[l - ds]) : 0;
        for (int w = 0; w < SUM_BLOCK / 64; ++w) {
            a += sH[w][l];
            b += sL[w][l];
        }
        long long cc, oo;
        normalise<AT>(a, b, &cc, &oo);
        S[l] = make_S((AT*)0, F::B + (J - l) * F::W, oo);
        C[l] = cc;
    }
}

struct SumPlan {
    int nwg;
    int64_t chunk;
    size_t off_hi, off_lo, ws;
};

bool sum_plan(int64_t n, int L, SumPlan* p) {
    if (n < 0 || L < 1 || L > 4) return false;
    int64_t nwg = std::min<int64_t>(SUM_MAX_WG, std::max<int64_t>(1, (n + 4 * SUM_STEP - 1) / (4 * SUM_STEP)));
    int64_t chunk = (n + nwg - 1) / nwg;
    chunk = std::max<int64_t>(SUM_STEP, (chunk + SUM_STEP - 1) / SUM_STEP * SUM_STEP);
    if (chunk / SUM_BLOCK > SUM_MAX_ROWS_PER_LANE) return false;  // n above 2^35 rows
    nwg = std::max<int64_t>(1, (n + chunk - 1) / chunk);
    p->nwg = (int)nwg;
    p->chunk = chunk;
    p->off_hi = align_up((size_t)nwg * 4, 256);
    p->off_lo = p->off_hi + align_up((size_t)nwg * L * 8, 256);
    p->ws = p->off_lo + align_up((size_t)nwg * L * 8, 256);
    return true;
}

template <class VT, class AT, int L>
int run_sum(const void* values, int64_t n, void* state, unsigned char* ws, const SumPlan& p, uint32_t* status,
            hipStream_t st) {
    const VT* v = static_cast<const VT*>(values);
    int* ptop = reinterpret_cast<int*>(ws);
    long long* phi = reinterpret_cast<long long*>(ws + p.off_hi);
    long long* plo = reinterpret_cast<long long*>(ws + p.off_lo);
    constexpr int VEC = 16 / sizeof(VT);
    if ((uintptr_t)v % 16 == 0)
        hipLaunchKernelGGL((k_sum<VT, AT, L, VEC>), dim3(p.nwg), dim3(SUM_BLOCK), 0, st, v, n, p.chunk, ptop, phi, plo,
                           status);
    else
        hipLaunchKernelGGL((k_sum<VT, AT, L, 1>), dim3(p.nwg), dim3(SUM_BLOCK), 0, st, v, n, p.chunk, ptop, phi, plo,
                           status);
    if (hipGetLastError() != hipSuccess) return REPRO_EHIP;
    AT* S = static_cast<AT*>(state);
    long long* C = reinterpret_cast<long long*>(static_cast<unsigned char*>(state) + align_up((size_t)L * sizeof(AT), 8));
    hipLaunchKernelGGL((k_sum_merge<AT, L>), dim3(1), dim3(SUM_BLOCK), 0, st, ptop, phi, plo, p.nwg, S, C);
    return hipGetLastError() == hipSuccess ? REPRO_OK : REPRO_EHIP;
}

template <class VT, class AT>
int sum_L(int L, const void* values, int64_t n, void* state, unsigned char* ws, const SumPlan& p, uint32_t* status,
          hipStream_t st) {
    switch (L) {
        case 1: return run_sum<VT, AT, 1>(values, n, state, ws, p, status, st);
        case 2: return run_sum<VT, AT, 2>(values, n, state, ws, p, status, st);
        case 3: return run_sum<VT, AT, 3>(values, n, state, ws, p, status, st);
        default: return run_sum<VT, AT, 4>(values, n, state, ws, p, status, st);
    }
}

// Exact row counts per group: an LDS histogram per workgroup for the
// groups that fit, then one integer atomic per group and workgroup (integer
// addition is exact and associative, so the counts do not depend on order).
constexpr int CNT_BLOCK = 256;
constexpr int CNT_LDS_GROUPS = 16384;

template <class KT>
__global__ void __launch_bounds__(CNT_BLOCK) k_count(const KT* __restrict__ keys, int64_t n, int64_t G,
                                                     unsigned long long* __restrict__ counts,
                                                     uint32_t* __restrict__ status) {
    __shared__ unsigned int h[CNT_LDS_GROUPS];
    const bool lds = G <= CNT_LDS_GROUPS;
    if (lds)
        for (int g = threadIdx.x; g < G; g += CNT_BLOCK) h[g] = 0;
    __syncthreads();
    uint32_t err = 0;
    for (int64_t i = (int64_t)blockIdx.x * CNT_BLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * CNT_BLOCK) {
        const int64_t k = (int64_t)keys[i];
        if ((uint64_t)k >= (uint64_t)G) {
            err |= ERR_KEY;
        } else if (lds) {
            atomicAdd(&h[k], 1u);
        } else {
            atomicAdd(&counts[k], 1ull);
        }
    }
    __syncthreads();
    if (lds)
        for (int g = threadIdx.x; g < G; g += CNT_BLOCK)
            if (h[g]) atomicAdd(&counts[g], (unsigned long long)h[g]);
    report(status, err);
}

// AVG, sample VAR and sample STDDEV of every group from its reproducible
// SUM(x), SUM(x*x) and exact COUNT, in a fixed order of IEEE operations
// (no contraction): the results are as reproducible as their inputs.
// Groups with no row give NaN for AVG; fewer than two rows give NaN for
// VAR and STDDEV.
__global__ void __launch_bounds__(256) k_derive(const double* __restrict__ sum, const double* __restrict__ sumsq,
                                                const long long* __restrict__ cnt, int64_t G,
                                                double* __restrict__ avg, double* __restrict__ var,
                                                double* __restrict__ sd) {
    for (int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x; g < G; g += (int64_t)gridDim.x * 256) {
        const double c = (double)cnt[g];  // exact below 2^53 rows
        const double s = sum[g], q = sumsq[g];
        const double m = s / c;
        const double u = q - s * m;
        const double v = u / (c - 1.0);
        if (avg) avg[g] = cnt[g] > 0 ? m : __builtin_nan("");
        if (var) var[g] = cnt[g] > 1 ? v : __builtin_nan("");
        if (sd) sd[g] = cnt[g] > 1 ? sqrt(v) : __builtin_nan("");
    }
}

}  // namespace

extern "C" {

int repro_groupby_count(const void* keys, repro_key_t kt, int64_t n, int64_t num_groups, int64_t* counts,
                        uint32_t* status, hipStream_t stream) {
    if (n < 0 || num_groups < 1 || num_groups > INT32_MAX || !counts || (kt != REPRO_I32 && kt != REPRO_I64))
        return REPRO_EINVAL;
    if (n == 0) return REPRO_OK;
    if (!keys) return REPRO_EINVAL;
    const unsigned grid = (unsigned)std::min<int64_t>(2048, (n + CNT_BLOCK * 8 - 1) / (CNT_BLOCK * 8));
    unsigned long long* c = reinterpret_cast<unsigned long long*>(counts);
    if (kt == REPRO_I32)
        hipLaunchKernelGGL(k_count<int32_t>, dim3(grid), dim3(CNT_BLOCK), 0, stream,
                           static_cast<const int32_t*>(keys), n, num_groups, c, status);
    else
        hipLaunchKernelGGL(k_count<int64_t>, dim3(grid), dim3(CNT_BLOCK), 0, stream,
                           static_cast<const int64_t*>(keys), n, num_groups, c, status);
    return hipGetLastError() == hipSuccess ? REPRO_OK : REPRO_EHIP;
}

int repro_derive_stats(const double* sum, const double* sumsq, const int64_t* count, int64_t num_groups, double* avg,
                       double* var_samp, double* stddev_samp, hipStream_t stream) {
    if (!sum || !sumsq || !count || num_groups < 1 || num_groups > INT32_MAX) return REPRO_EINVAL;
    const unsigned grid = (unsigned)std::min<int64_t>(4096, (num_groups + 255) / 256);
    hipLaunchKernelGGL(k_derive, dim3(grid), dim3(256), 0, stream, sum, sumsq,
                       reinterpret_cast<const long long*>(count), num_groups, avg, var_samp, stddev_samp);
    return hipGetLastError() == hipSuccess ? REPRO_OK : REPRO_EHIP;
}

size_t repro_sum_workspace_bytes(int64_t n, int L) {
    SumPlan p;
    return sum_plan(n, L, &p) ? p.ws : 0;
}

int repro_sum(const void* values, repro_scalar_t vt, int64_t n, repro_scalar_t T, int L, void* state,
              void* workspace, size_t workspace_bytes, uint32_t* status, hipStream_t stream) {
    if (!state || (vt != REPRO_F32 && vt != REPRO_F64) || (T != REPRO_F32 && T != REPRO_F64)) return REPRO_EINVAL;
    if (vt == REPRO_F64 && T == REPRO_F32) return REPRO_EINVAL;  // narrowing is not exact
    SumPlan p;
    if (!sum_plan(n, L, &p)) return REPRO_EINVAL;
    if (n == 0) return REPRO_OK;
    if (!values || !workspace || workspace_bytes < p.ws || (uintptr_t)workspace % 256 != 0) return REPRO_EINVAL;
    unsigned char* ws = static_cast<unsigned char*>(workspace);
    if (vt == REPRO_F64) return sum_L<double, double>(L, values, n, state, ws, p, status, stream);
    if (T == REPRO_F64) return sum_L<float, double>(L, values, n, state, ws, p, status, stream);
    return sum_L<float, float>(L, values, n, state, ws, p, status, stream);
}

}  // extern "C"
