// repro_cols.hip -- several SUM aggregates over one GROUP BY in one pass.
//
// Paper: Mueller, Arteaga, Hoefler, Alonso, "Reproducible Floating-Point
// Aggregation in RDBMSs" (arXiv 1802.09883).  A query computes several
// aggregates per group (Sec. V-D; TPC-H Q1 of Sec. VI-E has several SUMs
// over one GROUP BY).  Each aggregate is its own repro<T,L> per group; the
// rows are the same, so the key column is read once for all of them.
//
//   k_agg_cols   the hot loop of the LDS path (aggregate_src) over a row
//                source that turns each row into one virtual row per
//                column: column c of group g goes to bin group c*G + g.  The
//                partials then merge per column exactly as for one column.
//   k_plain_cols the non-reproducible baseline over the same columns.
//
// Every result has the bits repro_groupby_sum gives on that column alone:
// the level sums are exact, so neither the shared pass nor the launch shape
// can change them.  Shapes the fused kernel does not take (T = float, too
// many groups for one workgroup's LDS, unaligned columns) run column by
// column through repro_groupby_sum.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "repro.h"
#include "repro_agg.hpp"
#include "repro_device.hpp"
#include "repro_lds.hpp"

using namespace repro;

namespace {

constexpr int COLS_FUSED_MAX = 4;  // columns per fused pass

struct ColPtrs {
    const void* p[COLS_FUSED_MAX];
};

template <class KT, int L, int NC, uint32_t FMC>
__global__ void __launch_bounds__(AGG_BLOCK) k_agg_cols(const KT* __restrict__ keys, ColPtrs vals, uint32_t f32mask,
                                                        int64_t n, int G, int R, int64_t chunk,
                                                        int* __restrict__ ptop, long long* __restrict__ pK,
                                                        unsigned long long* __restrict__ spill,
                                                        uint32_t* __restrict__ status, const int* __restrict__ seed) {
    typedef SrcCols<KT, double, NC, AGG_BLOCK, FMC> Src;
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ AggShared sh;
    const int64_t c0 = (int64_t)blockIdx.x * chunk;
    const int64_t c1 = (c0 + chunk < n) ? c0 + chunk : n;
    const int Gv = NC * G;
    const Src src(keys, vals.p, f32mask, G);
    const uint32_t err =
        aggregate_src<Src, double, L, true, false, AGG_BLOCK>(src, c0, c1, Gv, R, smem, sh, spill, 0, 0, seed);
    long long* bins = reinterpret_cast<long long*>(smem);
    const int2* TOP = reinterpret_cast<const int2*>(bins + (size_t)(Gv + 1) * R * L);
    fold_replicas<L, AGG_BLOCK>(bins, Gv, R);
    for (int g = threadIdx.x; g < Gv; g += AGG_BLOCK) {
        ptop[(size_t)blockIdx.x * Gv + g] = TOP[g].x;
#pragma unroll
        for (int l = 0; l < L; ++l) pK[((size_t)blockIdx.x * L + l) * Gv + g] = bins[((size_t)l * (Gv + 1) + g) * R];
    }
    report(status, err);
}

// Seed tops for k_agg_cols: one sampled tile per workgroup.
template <class KT, int NC, uint32_t FMC>
__global__ void __launch_bounds__(AGG_BLOCK) k_sample_cols(const KT* __restrict__ keys, ColPtrs vals,
                                                           uint32_t f32mask, int64_t n, int G, int64_t stride,
                                                           int* __restrict__ seed) {
    typedef SrcCols<KT, double, NC, AGG_BLOCK, FMC> Src;
    extern __shared__ __align__(16) unsigned char smem[];
    const Src src(keys, vals.p, f32mask, G);
    sample_tops<Src, double, AGG_BLOCK>(src, n, stride, NC * G, reinterpret_cast<int*>(smem), seed);
}

// Plain double atomics per column (LDS-privatised), the baseline.
constexpr int PLAIN_COLS_BLOCK = 256;
constexpr int PLAIN_COLS_MAX_WG = 1024;

struct ColOut {
    double* p[COLS_FUSED_MAX];
};

template <class KT, int NC>
__global__ void __launch_bounds__(PLAIN_COLS_BLOCK)
    k_plain_cols(const KT* __restrict__ keys, ColPtrs vals, uint32_t f32mask, int64_t n, int G, int64_t chunk,
                 ColOut out, uint32_t* __restrict__ status) {
    typedef SrcCols<KT, double, NC, PLAIN_COLS_BLOCK> Src;
    extern __shared__ __align__(16) unsigned char smem[];
    double* bins = reinterpret_cast<double*>(smem);
    const int tid = threadIdx.x;
    for (int i = tid; i < NC * G; i += PLAIN_COLS_BLOCK) bins[i] = 0.0;
    __syncthreads();
    const int64_t c0 = (int64_t)blockIdx.x * chunk;
    const int64_t c1 = (c0 + chunk < n) ? c0 + chunk : n;
    const Src src(keys, vals.p, f32mask, G);
    uint32_t err = 0;
    typename Src::Buf b;
    for (int64_t base = c0; base < c1; base += Src::TILE) {
        const uint32_t inr = src.load(b, base, c1);
#pragma unroll
        for (int r = 0; r < Src::RPT; ++r) {
            const bool in = (inr >> r) & 1u;
            const bool kok = (uint64_t)(int64_t)b.k[r] < (uint64_t)G;
            err |= (in && !kok) ? ERR_KEY : 0u;
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                const double v = src.template value<double>(b, c * Src::RPT + r);
                const bool fin = finite_val(v);
                err |= (in && !fin) ? ERR_NONFINITE : 0u;
                if (in && kok && fin) atomicAdd(&bins[c * G + (int)b.k[r]], v);
            }
        }
    }
    __syncthreads();
    for (int i = tid; i < NC * G; i += PLAIN_COLS_BLOCK)
        if (bins[i] != 0.0) atomicAdd(&out.p[i / G][i % G], bins[i]);
    report(status, err);
}

// ------------------------------------------------------------------ host

inline bool valid_scalar(repro_scalar_t t) { return t == REPRO_F32 || t == REPRO_F64; }
inline size_t scalar_bytes(repro_scalar_t t) { return t == REPRO_F64 ? 8 : 4; }

// Columns [c, c + nc) form one fused pass when nc >= 2 columns of G groups
// fit one workgroup's LDS together (T = double only).  Greedy from the left.
inline int fused_width(int remaining, int64_t G, repro_scalar_t T, int L) {
    if (T != REPRO_F64) return 1;
    int nc = std::min(remaining, COLS_FUSED_MAX);
    while (nc >= 2 && agg_lds_bytes((int64_t)nc * G, L, 1) > LDS_BIN_BUDGET) --nc;
    return nc >= 2 ? nc : 1;
}

inline int64_t cols_tile(int nc) {
    switch (nc) {
        case 2: return SrcCols<int32_t, double, 2, AGG_BLOCK>::TILE;
        case 3: return SrcCols<int32_t, double, 3, AGG_BLOCK>::TILE;
        default: return SrcCols<int32_t, double, 4, AGG_BLOCK>::TILE;
    }
}

inline bool cols_aligned(const void* keys, repro_key_t kt, const void* const* values, const repro_scalar_t* vts,
                         int c, int nc) {
    if ((uintptr_t)keys % (2 * (kt == REPRO_I64 ? 8 : 4)) != 0) return false;
    for (int i = c; i < c + nc; ++i)
        if ((uintptr_t)values[i] % (2 * scalar_bytes(vts[i])) != 0) return false;
    return true;
}

template <class KT, int L, int NC, uint32_t FMC>
int run_cols(const KT* keys, const void* const* values, uint32_t f32mask, int64_t n, int G, void* const* states,
             unsigned char* ws, uint32_t* status, const Plan& p, hipStream_t st) {
    const int Gv = NC * G;
    const void* fn = (const void*)k_agg_cols<KT, L, NC, FMC>;
    if (!allow_lds(fn, p.lds)) return REPRO_EHIP;
    ColPtrs vp;
    ColStates<double> cs;
    for (int c = 0; c < NC; ++c) {
        vp.p[c] = values[c];
        cs.S[c] = static_cast<double*>(states[c]);
        cs.C[c] = reinterpret_cast<long long*>(static_cast<unsigned char*>(states[c]) +
                                               align_up((size_t)G * L * sizeof(double), 8));
    }
    int* ptop = reinterpret_cast<int*>(ws);
    long long* pK = reinterpret_cast<long long*>(ws + align_up((size_t)p.nwg * Gv * 4, 256));
    unsigned long long* spill = reinterpret_cast<unsigned long long*>(ws + p.spill_off);
    int* seed = p.seed_tiles ? reinterpret_cast<int*>(ws + p.seed_off) : nullptr;
    if (p.spill_used) {
        hipLaunchKernelGGL(k_zero, dim3((unsigned)std::min<size_t>(1024, (p.zero_words + 255) / 256)), dim3(256), 0,
                           st, spill, p.zero_words);
        LAUNCH_CHECK();
    }
    if (seed) {
        hipLaunchKernelGGL((k_sample_cols<KT, NC, FMC>), dim3(p.seed_tiles), dim3(AGG_BLOCK), (size_t)(Gv + 1) * 4, st,
                           keys, vp, f32mask, n, G, p.seed_stride, seed);
        LAUNCH_CHECK();
    }
    prof_before(st);
    hipLaunchKernelGGL((k_agg_cols<KT, L, NC, FMC>), dim3(p.nwg), dim3(AGG_BLOCK), p.lds, st, keys, vp, f32mask, n, G,
                       p.R, p.chunk, ptop, pK, spill, status, seed);
    LAUNCH_CHECK();
    prof_after(st);
    return run_merge<double, L>(p, G, NC, ws, cs, st);
}

template <class KT, int L>
int dispatch_nc(int nc, const void* keys, const void* const* values, uint32_t f32mask, int64_t n, int G,
                void* const* states, unsigned char* ws, uint32_t* status, const Plan& p, hipStream_t st) {
    const KT* k = static_cast<const KT*>(keys);
    // two columns: the column types are compile-time (floats stay 4 bytes
    // while prefetched); three or four: a runtime mask
    if (nc == 2) {
        switch (f32mask) {
            case 0: return run_cols<KT, L, 2, 0u>(k, values, f32mask, n, G, states, ws, status, p, st);
            case 1: return run_cols<KT, L, 2, 1u>(k, values, f32mask, n, G, states, ws, status, p, st);
            case 2: return run_cols<KT, L, 2, 2u>(k, values, f32mask, n, G, states, ws, status, p, st);
            default: return run_cols<KT, L, 2, 3u>(k, values, f32mask, n, G, states, ws, status, p, st);
        }
    }
    switch (nc) {
        case 3: return run_cols<KT, L, 3, FM_RUNTIME>(k, values, f32mask, n, G, states, ws, status, p, st);
        case 4: return run_cols<KT, L, 4, FM_RUNTIME>(k, values, f32mask, n, G, states, ws, status, p, st);
    }
    return REPRO_EINVAL;
}

template <class KT>
int dispatch_cols_L(int L, int nc, const void* keys, const void* const* values, uint32_t f32mask, int64_t n, int G,
                    void* const* states, unsigned char* ws, uint32_t* status, const Plan& p, hipStream_t st) {
    switch (L) {
        case 1: return dispatch_nc<KT, 1>(nc, keys, values, f32mask, n, G, states, ws, status, p, st);
        case 2: return dispatch_nc<KT, 2>(nc, keys, values, f32mask, n, G, states, ws, status, p, st);
        case 3: return dispatch_nc<KT, 3>(nc, keys, values, f32mask, n, G, states, ws, status, p, st);
        case 4: return dispatch_nc<KT, 4>(nc, keys, values, f32mask, n, G, states, ws, status, p, st);
    }
    return REPRO_EINVAL;
}

bool valid_cols(int ncols, const repro_scalar_t* vts, int64_t num_groups, repro_key_t kt) {
    if (ncols < 1 || ncols > REPRO_MAX_COLS || !vts) return false;
    if (num_groups < 1 || num_groups > INT32_MAX) return false;
    if (kt != REPRO_I32 && kt != REPRO_I64) return false;
    for (int c = 0; c < ncols; ++c)
        if (!valid_scalar(vts[c])) return false;
    return true;
}

template <class KT, int NC>
int run_plain_cols(const KT* keys, const void* const* values, uint32_t f32mask, int64_t n, int G, double* const* outs,
                   uint32_t* status, hipStream_t st) {
    typedef SrcCols<KT, double, NC, PLAIN_COLS_BLOCK> Src;
    int64_t nwg = (n + 16 * Src::TILE - 1) / (16 * Src::TILE);
    nwg = std::max<int64_t>(1, std::min<int64_t>(PLAIN_COLS_MAX_WG, nwg));
    int64_t chunk = (n + nwg - 1) / nwg;
    chunk = (chunk + Src::TILE - 1) / Src::TILE * Src::TILE;
    nwg = (n + chunk - 1) / chunk;
    ColPtrs vp;
    ColOut op;
    for (int c = 0; c < NC; ++c) {
        vp.p[c] = values[c];
        op.p[c] = outs[c];
    }
    const size_t lds = (size_t)NC * G * 8;
    if (!allow_lds((const void*)k_plain_cols<KT, NC>, lds)) return REPRO_EHIP;
    hipLaunchKernelGGL((k_plain_cols<KT, NC>), dim3(nwg), dim3(PLAIN_COLS_BLOCK), lds, st, keys, vp, f32mask, n, G,
                       chunk, op, status);
    LAUNCH_CHECK();
    return REPRO_OK;
}

}  // namespace

// ============================================================== C ABI

extern "C" {

size_t repro_workspace_bytes_cols(int64_t n, int64_t num_groups, repro_key_t kt, int ncols,
                                  const repro_scalar_t* vts, repro_scalar_t T, int L) {
    if (!valid_cols(ncols, vts, num_groups, kt) || n < 0 || L < 1 || L > 4 || !valid_scalar(T)) return 0;
    size_t ws = 0;
    for (int c = 0; c < ncols;) {
        const int nc = fused_width(ncols - c, num_groups, T, L);
        if (nc >= 2) {
            Plan p;
            if (make_plan_lds(n, (int64_t)nc * num_groups, L, Fmt<double>::JMAX, cols_tile(nc), &p))
                ws = std::max(ws, p.ws);
        }
        // column by column (the fallback of a fused pass, or a lone column)
        for (int i = c; i < c + nc; ++i) {
            if (vts[i] == REPRO_F64 && T == REPRO_F32) return 0;
            const size_t w = repro_workspace_bytes(n, num_groups, kt, vts[i], T, L);
            if (w == 0 && n > 0) return 0;
            ws = std::max(ws, w);
        }
        c += nc;
    }
    return ws;
}

int repro_groupby_sum_cols(const void* keys, repro_key_t kt, int ncols, const void* const* values,
                           const repro_scalar_t* vts, int64_t n, int64_t num_groups, repro_scalar_t T, int L,
                           void* const* states, void* workspace, size_t workspace_bytes, uint32_t* status,
                           hipStream_t stream) {
    if (!valid_cols(ncols, vts, num_groups, kt) || n < 0 || L < 1 || L > 4 || !valid_scalar(T)) return REPRO_EINVAL;
    if (!states || !values) return REPRO_EINVAL;
    for (int c = 0; c < ncols; ++c) {
        if (!states[c]) return REPRO_EINVAL;
        if (vts[c] == REPRO_F64 && T == REPRO_F32) return REPRO_EINVAL;  // narrowing is not exact
        for (int d = 0; d < c; ++d)
            if (states[d] == states[c]) return REPRO_EINVAL;  // every aggregate has its own state
    }
    if (n == 0) return REPRO_OK;
    if (!keys) return REPRO_EINVAL;
    for (int c = 0; c < ncols; ++c)
        if (!values[c]) return REPRO_EINVAL;
    const size_t need = repro_workspace_bytes_cols(n, num_groups, kt, ncols, vts, T, L);
    if (need == 0) return REPRO_EINVAL;
    if (!workspace || workspace_bytes < need || (uintptr_t)workspace % 256 != 0) return REPRO_EINVAL;
    const int G = (int)num_groups;
    for (int c = 0; c < ncols;) {
        const int nc = fused_width(ncols - c, num_groups, T, L);
        Plan p;
        if (nc >= 2 && cols_aligned(keys, kt, values, vts, c, nc) &&
            make_plan_lds(n, (int64_t)nc * G, L, Fmt<double>::JMAX, cols_tile(nc), &p)) {
            uint32_t f32mask = 0;
            for (int i = 0; i < nc; ++i) f32mask |= (vts[c + i] == REPRO_F32 ? 1u : 0u) << i;
            unsigned char* ws = static_cast<unsigned char*>(workspace);
            const int rc = kt == REPRO_I32
                               ? dispatch_cols_L<int32_t>(L, nc, keys, values + c, f32mask, n, G, states + c, ws,
                                                          status, p, stream)
                               : dispatch_cols_L<int64_t>(L, nc, keys, values + c, f32mask, n, G, states + c, ws,
                                                          status, p, stream);
            if (rc != REPRO_OK) return rc;
        } else {
            for (int i = c; i < c + nc; ++i) {
                const int rc = repro_groupby_sum(keys, kt, values[i], vts[i], n, num_groups, T, L, states[i],
                                                 workspace, workspace_bytes, status, stream);
                if (rc != REPRO_OK) return rc;
            }
        }
        c += nc;
    }
    return REPRO_OK;
}

int repro_plain_groupby_sum_cols(const void* keys, repro_key_t kt, int ncols, const void* const* values,
                                 const repro_scalar_t* vts, int64_t n, int64_t num_groups, double* const* outs,
                                 uint32_t* status, hipStream_t stream) {
    if (!valid_cols(ncols, vts, num_groups, kt) || n < 0 || !outs || !values) return REPRO_EINVAL;
    for (int c = 0; c < ncols; ++c)
        if (!outs[c]) return REPRO_EINVAL;
    if (n == 0) return REPRO_OK;
    if (!keys) return REPRO_EINVAL;
    for (int c = 0; c < ncols; ++c)
        if (!values[c]) return REPRO_EINVAL;
    const int G = (int)num_groups;
    for (int c = 0; c < ncols;) {
        int nc = std::min(ncols - c, COLS_FUSED_MAX);
        while (nc >= 2 && (size_t)nc * G * 8 > LDS_BIN_BUDGET) --nc;
        if (nc >= 2 && cols_aligned(keys, kt, values, vts, c, nc)) {
            uint32_t f32mask = 0;
            for (int i = 0; i < nc; ++i) f32mask |= (vts[c + i] == REPRO_F32 ? 1u : 0u) << i;
            int rc = REPRO_EINVAL;
            if (kt == REPRO_I32) {
                const int32_t* k = static_cast<const int32_t*>(keys);
                rc = nc == 2   ? run_plain_cols<int32_t, 2>(k, values + c, f32mask, n, G, outs + c, status, stream)
                     : nc == 3 ? run_plain_cols<int32_t, 3>(k, values + c, f32mask, n, G, outs + c, status, stream)
                               : run_plain_cols<int32_t, 4>(k, values + c, f32mask, n, G, outs + c, status, stream);
            } else {
                const int64_t* k = static_cast<const int64_t*>(keys);
                rc = nc == 2   ? run_plain_cols<int64_t, 2>(k, values + c, f32mask, n, G, outs + c, status, stream)
                     : nc == 3 ? run_plain_cols<int64_t, 3>(k, values + c, f32mask, n, G, outs + c, status, stream)
                               : run_plain_cols<int64_t, 4>(k, values + c, f32mask, n, G, outs + c, status, stream);
            }
            if (rc != REPRO_OK) return rc;
        } else {
            for (int i = c; i < c + std::max(nc, 1); ++i) {
                const int rc = repro_plain_groupby_sum(keys, kt, values[i], vts[i], n, num_groups, outs[i], nullptr,
                                                       0, status, stream);
                if (rc != REPRO_OK) return rc;
            }
        }
        c += std::max(nc, 1);
    }
    return REPRO_OK;
}

}  // extern "C"
