// repro_lds.hpp -- the LDS-bin path of librepro shared by its translation
// units: the plan of a workgroup-per-chunk aggregation whose groups fit one
// workgroup's LDS, the merge of the workgroup partials into canonical
// states (operator+=(repro) of Sec. IV over all partials), and the
// profiling hooks that bracket the aggregation kernel.
#ifndef REPRO_LDS_HPP
#define REPRO_LDS_HPP

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>

#include "repro.h"
#include "repro_agg.hpp"
#include "repro_device.hpp"

namespace repro {

// HIP events around the aggregation kernel (repro_profile_arm/read).
void prof_before(hipStream_t st);
void prof_after(hipStream_t st);

namespace {

#define LAUNCH_CHECK()                                          \
    do {                                                        \
        if (hipGetLastError() != hipSuccess) return REPRO_EHIP; \
    } while (0)

// Zeroes the spill array before an aggregation pass.
__global__ void __launch_bounds__(256) k_zero(unsigned long long* __restrict__ p, size_t n) {
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) p[i] = 0;
}

// ------------------------------------------------------------- merging
//
// The workgroup partials (top, K[L]) of every group are folded into the
// caller's canonical state in two launches (operator+=(repro) over all
// partials).  Every step is exact integer arithmetic, so the split into
// blocks does not change any bit.
//
// Level 1 (k_merge_l1): block (x, y) takes groups x*64 .. x*64+63 (one per
// lane) and partials y*PB .. y*PB+PB-1 (spread over the 4 waves).  It forms
// their common top J (the largest), moves each partial's levels down by its
// distance to J and adds the level sums split as hi = sum(K >> CARRY),
// lo = sum(K & (2^CARRY - 1)) (no int64 overflow: |K| < 2^62 per partial).
// Level 2 (k_merge_l2): SL lanes per group (slices) add the level-1 results
// and the caller's state the same way; the slice sums are folded in a tree
// and the first slice writes the canonical (S, C).  The merge is bound by
// the latency of its loads, so many slices (few partials per lane) pay.
constexpr int M1_GROUPS = 64, M1_WAVES = 4;
constexpr int M2_GROUPS = 16;
// slices per group: the slice sums (SL x L x 16 groups x 2 words) stay
// within the 64 KiB of static LDS
template <int L>
constexpr int m2_slices() {
    return L <= 3 ? 64 : 32;
}
constexpr int64_t MERGE_DIRECT_MAX = 1 << 20;  // partials x groups merged by k_merge_l2 alone (one launch)
constexpr int SEED_TILES = 64;      // tiles sampled for seed tops
constexpr int SEED_MIN_TILES = 8;   // tiles per workgroup from which sampling pays

template <class AT, int L>
__global__ void __launch_bounds__(M1_GROUPS* M1_WAVES)
    k_merge_l1(const int* __restrict__ ptop, const long long* __restrict__ pK, int nparts, int PB, int G,
               int* __restrict__ qtop, long long* __restrict__ qhi, long long* __restrict__ qlo) {
    constexpr int c = Fmt<AT>::CARRY;
    __shared__ int sJ[M1_WAVES][M1_GROUPS];
    __shared__ long long sH[M1_WAVES][L][M1_GROUPS], sLo[M1_WAVES][L][M1_GROUPS];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = blockIdx.x * M1_GROUPS + lane;
    const bool gv = g < G;
    const int gg = gv ? g : 0;  // clamped: loads stay in bounds, results unused
    const int p0 = blockIdx.y * PB;
    const int p1 = min(nparts, p0 + PB);
    int J = L - 1;
    for (int p = p0 + wave; p < p1; p += M1_WAVES) J = max(J, ptop[(size_t)p * G + gg]);
    sJ[wave][lane] = J;
    __syncthreads();
#pragma unroll
    for (int w = 0; w < M1_WAVES; ++w) J = max(J, sJ[w][lane]);
    long long hi[L], lo[L];
#pragma unroll
    for (int l = 0; l < L; ++l) hi[l] = lo[l] = 0;
    for (int p = p0 + wave; p < p1; p += M1_WAVES) {
        const int d = J - ptop[(size_t)p * G + gg];
        long long x[L];
#pragma unroll
        for (int l = 0; l < L; ++l) x[l] = pK[((size_t)p * L + l) * G + gg];
#pragma unroll
        for (int l = 0; l < L; ++l) {
            // level l of the result is level l - d of this partial
            long long v = 0;
#pragma unroll
            for (int q = 0; q < L; ++q) v = (q == l - d) ? x[q] : v;
            hi[l] += v >> c;
            lo[l] += v & ((1ll << c) - 1);
        }
    }
#pragma unroll
    for (int l = 0; l < L; ++l) {
        sH[wave][l][lane] = hi[l];
        sLo[wave][l][lane] = lo[l];
    }
    __syncthreads();
    if (wave != 0 || !gv) return;
#pragma unroll
    for (int l = 0; l < L; ++l) {
        long long h = 0, o = 0;
#pragma unroll
        for (int w = 0; w < M1_WAVES; ++w) {
            h += sH[w][l][lane];
            o += sLo[w][l][lane];
        }
        qhi[((size_t)blockIdx.y * L + l) * G + g] = h;
        qlo[((size_t)blockIdx.y * L + l) * G + g] = o;
    }
    qtop[(size_t)blockIdx.y * G + g] = J;
}

// With several aggregated columns the partials hold gs = NC * G bin groups
// (column c's group g at c * G + g); blockIdx.y selects the column and so
// the state written.
template <class AT>
struct ColStates {
    AT* S[REPRO_MAX_COLS];
    long long* C[REPRO_MAX_COLS];
};

// RAW: the inputs are the workgroup partials themselves (qtop_ = their
// tops, qhi_ = their level sums K, split here as hi = K >> CARRY, lo = K &
// (2^CARRY - 1); qlo_ unused): one launch merges few partials.  spill_ is
// null when no workgroup could spill (one tile per workgroup).
template <class AT, int L, bool RAW, int SL = m2_slices<L>()>
__global__ void __launch_bounds__(M2_GROUPS* SL)
    k_merge_l2(const int* __restrict__ qtop_, const long long* __restrict__ qhi_, const long long* __restrict__ qlo_,
               int nq, int G, int gs, const unsigned long long* __restrict__ spill_, ColStates<AT> cs) {
    constexpr int NJ = Fmt<AT>::JMAX + 1;
    typedef Fmt<AT> F;
    __shared__ int sJ[SL][M2_GROUPS];
    __shared__ long long sH[SL][L][M2_GROUPS], sLo[SL][L][M2_GROUPS];
    const int col = blockIdx.y;
    AT* __restrict__ S = cs.S[col];
    long long* __restrict__ C = cs.C[col];
    const int* __restrict__ qtop = qtop_ + (size_t)col * G;
    const long long* __restrict__ qhi = qhi_ + (size_t)col * G;
    const long long* __restrict__ qlo = RAW ? nullptr : qlo_ + (size_t)col * G;
    const int lane = threadIdx.x % M2_GROUPS, sl = threadIdx.x / M2_GROUPS;
    const int g = blockIdx.x * M2_GROUPS + lane;
    const bool gv = g < G;
    const int gg = gv ? g : 0;
    const int ts = state_top(S[gg]);
    int J = ts;
#pragma unroll 4
    for (int q = sl; q < nq; q += SL) J = max(J, qtop[(size_t)q * gs + gg]);
    sJ[sl][lane] = J;
    __syncthreads();
#pragma unroll 8
    for (int w = 0; w < SL; ++w) J = max(J, sJ[w][lane]);
    long long hi[L], lo[L];
#pragma unroll
    for (int l = 0; l < L; ++l) hi[l] = lo[l] = 0;
#pragma unroll 4
    for (int q = sl; q < nq; q += SL) {
        const int d = J - qtop[(size_t)q * gs + gg];
        long long xh[L], xl[L];
#pragma unroll
        for (int l = 0; l < L; ++l) {
            if (RAW) {
                const long long x = qhi[((size_t)q * L + l) * gs + gg];
                xh[l] = x >> Fmt<AT>::CARRY;
                xl[l] = x & ((1ll << Fmt<AT>::CARRY) - 1);
            } else {
                xh[l] = qhi[((size_t)q * L + l) * gs + gg];
                xl[l] = qlo[((size_t)q * L + l) * gs + gg];
            }
        }
#pragma unroll
        for (int l = 0; l < L; ++l) {
#pragma unroll
            for (int r = 0; r < L; ++r) {
                if (r == l - d) {
                    hi[l] += xh[r];
                    lo[l] += xl[r];
                }
            }
        }
    }
#pragma unroll
    for (int l = 0; l < L; ++l) {
        sH[sl][l][lane] = hi[l];
        sLo[sl][l][lane] = lo[l];
    }
    __syncthreads();
    // tree over the slices (exact integer sums: the grouping changes no bit)
#pragma unroll
    for (int w = SL / 2; w > 0; w /= 2) {
        if (sl < w) {
#pragma unroll
            for (int l = 0; l < L; ++l) {
                sH[sl][l][lane] += sH[sl + w][l][lane];
                sLo[sl][l][lane] += sLo[sl + w][l][lane];
            }
        }
        __syncthreads();
    }
    if (sl != 0 || !gv) return;
    const int ds = J - ts;
#pragma unroll
    for (int l = 0; l < L; ++l) {
        long long h = (l - ds >= 0) ? C[(size_t)(l - ds) * G + g] : 0;
        long long o = (l - ds >= 0) ? state_lo(S[(size_t)(l - ds) * G + g]) : 0;
        h += sH[0][l][lane];
        o += sLo[0][l][lane];
        if (spill_) {  // uniform
            // spilled units at lattice index J - l: H * 2^64 + w
            const unsigned long long* sw = spill_ + (((size_t)col * G + g) * NJ + (J - l)) * 2;
            const i128 T = (i128)(long long)sw[1] * ((i128)1 << 64) + (i128)sw[0];
            h += (long long)(T >> Fmt<AT>::CARRY);
            o += (long long)(T & ((1ll << Fmt<AT>::CARRY) - 1));
        }
        hi[l] = h;
        lo[l] = o;
    }
#pragma unroll
    for (int l = 0; l < L; ++l) {
        long long cc, oo;
        normalise<AT>(hi[l], lo[l], &cc, &oo);
        S[(size_t)l * G + g] = make_S((AT*)0, F::B + (J - l) * F::W, oo);
        C[(size_t)l * G + g] = cc;
    }
}

// partials per level-1 block: enough blocks to fill the chip, at most 64
inline int merge_pb(int nwg, int G) {
    const int gx = (G + M1_GROUPS - 1) / M1_GROUPS;
    int pb = 4;
    while (pb < 64 && (int64_t)gx * ((nwg + pb - 1) / pb) > 1024) pb *= 2;
    return pb;
}

struct Plan {
    int path;       // 1: LDS bins over all groups, 2: partitioned, 3: two partitioning levels
    // path 2
    int gp_shift, F, nw;     // groups per partition 2^gp_shift, partitions, hist/scatter workgroups
    size_t lds_sc;           // scatter LDS
    int sc_ru;               // scatter rows per thread and tile
    int maxw;                // work items, upper bound
    size_t o_counts, o_rel, o_size, o_base, o_wfirst, o_items, o_nitems, o_lkey, o_lval, o_ptop, o_pK;
    size_t o_rsum, o_roff;   // per-round partition counts and offsets
    int64_t slab;            // rows per slab of the partition passes
    size_t lds_agg2;         // LDS of k_agg_part
    size_t o_l2, ws_l2;      // path 3: the one-level workspace of a super-partition, and its size
    int nwg;        // aggregate workgroups
    int64_t chunk;  // rows per workgroup (multiple of the tile)
    int R;          // LDS bin replicas
    int pb, nq;     // partials per level-1 merge block, level-1 results
    size_t spill_off, spill_words;  // spill array: G x (JMAX+1) x {w, H}
    bool spill_used;  // a workgroup takes more than one tile (epoch mode, and so spills, possible)
    size_t zero_words;  // spill array and seed tops, cleared before the launch when spill_used
    size_t seed_off;    // seed tops: int per bin group
    int seed_tiles;     // tiles sampled for them (0: no sampling)
    int64_t seed_stride;  // rows between sampled tiles
    size_t lds;     // dynamic LDS bytes
    size_t ws;      // workspace bytes
};

// Plan of the LDS path for Gv bin groups (all of them in one workgroup's
// LDS) and tiles of `tile` rows: workgroups, chunking and workspace.
// Returns false when the groups do not fit or the partials get too many.
inline bool make_plan_lds(int64_t n, int64_t Gv, int L, int jmax, int64_t tile, Plan* p) {
    memset(p, 0, sizeof(*p));
    if (agg_lds_bytes(Gv, L, 1) > LDS_BIN_BUDGET) return false;
    p->path = 1;
    p->R = replicas_for(Gv, L);
    p->lds = agg_lds_bytes(Gv, L, p->R);
    const int64_t min_rows = tile;  // small inputs: one tile per workgroup (latency-bound)
    int64_t nwg = (n + min_rows - 1) / min_rows;
    if (nwg > MAX_AGG_WG) nwg = MAX_AGG_WG;
    if (nwg < (n + MAX_ROWS_PER_WG - 1) / MAX_ROWS_PER_WG) nwg = (n + MAX_ROWS_PER_WG - 1) / MAX_ROWS_PER_WG;
    if (nwg < 1) nwg = 1;
    int64_t chunk = (n + nwg - 1) / nwg;
    chunk = (chunk + tile - 1) / tile * tile;
    if (chunk < tile) chunk = tile;
    nwg = (n + chunk - 1) / chunk;
    if (nwg < 1) nwg = 1;
    if (nwg > 4096) return false;  // keeps the merge's int64 carry sums exact
    p->nwg = (int)nwg;
    p->chunk = chunk;
    p->pb = merge_pb(p->nwg, (int)Gv);
    p->nq = (p->nwg + p->pb - 1) / p->pb;
    size_t ws = 0;
    ws += align_up((size_t)nwg * Gv * 4, 256);          // partial tops
    ws += align_up((size_t)nwg * Gv * L * 8, 256);      // partial K
    ws += align_up((size_t)p->nq * Gv * 4, 256);        // level-1 tops
    ws += 2 * align_up((size_t)p->nq * Gv * L * 8, 256);  // level-1 hi, lo
    p->spill_off = ws;
    p->spill_words = (size_t)Gv * (jmax + 1) * 2;
    // epoch mode starts after a workgroup's first tile: with one tile per
    // workgroup no row can spill, and the array is neither cleared nor read
    p->spill_used = chunk > tile;
    ws += align_up(p->spill_words * 8, 256);
    // seed tops (one int per bin group), cleared together with the spill
    // array; sampled when every workgroup streams many tiles
    p->seed_off = ws;
    ws += align_up((size_t)Gv * 4, 256);
    p->zero_words = (ws - p->spill_off) / 8;
    const int64_t ntiles = (n + tile - 1) / tile;
    p->seed_tiles = (chunk >= SEED_MIN_TILES * tile) ? (int)std::min<int64_t>(SEED_TILES, ntiles) : 0;
    p->seed_stride = p->seed_tiles ? (ntiles / p->seed_tiles) * tile : 0;
    p->ws = ws;
    return true;
}

// Merges the partials of a planned LDS-path launch over nc columns of G
// groups each (nc * G bin groups) into the columns' states.
template <class AT, int L>
int run_merge(const Plan& p, int G, int nc, unsigned char* ws, const ColStates<AT>& cs, hipStream_t st) {
    const int Gv = G * nc;
    int* ptop = reinterpret_cast<int*>(ws);
    long long* pK = reinterpret_cast<long long*>(ws + align_up((size_t)p.nwg * Gv * 4, 256));
    unsigned char* q = reinterpret_cast<unsigned char*>(pK) + align_up((size_t)p.nwg * Gv * L * 8, 256);
    int* qtop = reinterpret_cast<int*>(q);
    long long* qhi = reinterpret_cast<long long*>(q + align_up((size_t)p.nq * Gv * 4, 256));
    long long* qlo = reinterpret_cast<long long*>(reinterpret_cast<unsigned char*>(qhi) +
                                                  align_up((size_t)p.nq * Gv * L * 8, 256));
    const unsigned long long* spill =
        p.spill_used ? reinterpret_cast<const unsigned long long*>(ws + p.spill_off) : nullptr;
    const dim3 g2((G + M2_GROUPS - 1) / M2_GROUPS, nc);
    if ((int64_t)p.nwg * Gv <= MERGE_DIRECT_MAX) {  // few partial groups: one launch
        hipLaunchKernelGGL((k_merge_l2<AT, L, true>), g2, dim3(M2_GROUPS * m2_slices<L>()), 0, st, ptop, pK, nullptr,
                           p.nwg, G, Gv, spill, cs);
        LAUNCH_CHECK();
        return REPRO_OK;
    }
    hipLaunchKernelGGL((k_merge_l1<AT, L>), dim3((Gv + M1_GROUPS - 1) / M1_GROUPS, p.nq), dim3(M1_GROUPS * M1_WAVES),
                       0, st, ptop, pK, p.nwg, p.pb, Gv, qtop, qhi, qlo);
    LAUNCH_CHECK();
    hipLaunchKernelGGL((k_merge_l2<AT, L, false>), g2, dim3(M2_GROUPS * m2_slices<L>()), 0, st, qtop, qhi, qlo, p.nq, G,
                       Gv, spill, cs);
    LAUNCH_CHECK();
    return REPRO_OK;
}

// Dynamic LDS beyond 64 KiB must be allowed per kernel on gfx950.
inline bool allow_lds(const void* fn, size_t bytes) {
    if (bytes <= 64 * 1024) return true;
    return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) == hipSuccess;
}

}  // namespace
}  // namespace repro

#endif  // REPRO_LDS_HPP
