// repro.hip -- librepro: reproducible GroupBy-SUM into repro<T,L> for gfx950.
//
// Paper: Mueller, Arteaga, Hoefler, Alonso, "Reproducible Floating-Point
// Aggregation in RDBMSs" (arXiv 1802.09883).
//
// Hot path of repro_groupby_sum (one HBM pass over keys and values):
//   k_agg_lds    each workgroup streams a contiguous chunk of rows in tiles;
//                per tile: key -> group (identity hashing, Sec. VI-A), the
//                per-group top index (max-exponent step; Alg. 2's level
//                check done once per tile as Alg. 3 does once per block),
//                realignment of the LDS bins of groups whose top rose,
//                pre-rounded extraction into L integer units, exact int64
//                adds into per-(level, group) LDS bins.  At the end the
//                workgroup writes its partial (top, K[L]) per group.
//   k_merge_l1/l2 fold all partials into the caller's states: common top
//                per group, shift, exact integer sums in (hi, lo) carry
//                form, canonical (S, C) (carry renormalisation).
// Exact integer addition is associative, so every launch shape, chunking
// and schedule produces the same bits.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <mutex>

#include "repro.h"
#include "repro_device.hpp"
#include "repro_agg.hpp"
#include "repro_lds.hpp"

using namespace repro;

namespace repro {
namespace {
// ------------------------------------------------------------ profiling
constexpr int PROFILE_MAX = 4096;
struct ProfileSlot {
    hipEvent_t ev[2 * PROFILE_MAX];
    int created = 0, armed = 0, used = 0;
};
thread_local ProfileSlot* g_prof = nullptr;

}  // namespace

void prof_before(hipStream_t st) {
    if (g_prof && g_prof->used < g_prof->armed) (void)hipEventRecord(g_prof->ev[2 * g_prof->used], st);
}
void prof_after(hipStream_t st) {
    if (g_prof && g_prof->used < g_prof->armed) (void)hipEventRecord(g_prof->ev[2 * g_prof->used++ + 1], st);
}


}  // namespace repro

namespace {

// Low/mid cardinality: each workgroup aggregates a contiguous chunk of rows
// over all groups and writes its partial (top, K[L]) per group.
template <class KT, class VT, class AT, int L, int VEC>
__global__ void __launch_bounds__(AGG_BLOCK) k_agg_lds(const KT* __restrict__ keys, const VT* __restrict__ vals,
                                                       int64_t n, int G, int R, int64_t chunk,
                                                       int* __restrict__ ptop, long long* __restrict__ pK,
                                                       unsigned long long* __restrict__ spill,
                                                       uint32_t* __restrict__ status, const int* __restrict__ seed) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ AggShared sh;
    const int64_t c0 = (int64_t)blockIdx.x * chunk;
    const int64_t c1 = (c0 + chunk < n) ? c0 + chunk : n;
    const uint32_t err =
        aggregate_range<KT, VT, AT, L, VEC, true>(keys, vals, c0, c1, G, R, smem, sh, spill, 0, 0, seed);
    long long* bins = reinterpret_cast<long long*>(smem);
    const int2* TOP = reinterpret_cast<const int2*>(bins + (size_t)(G + 1) * R * L);
    fold_replicas<L, AGG_BLOCK>(bins, G, R);
    for (int g = threadIdx.x; g < G; g += AGG_BLOCK) {
        ptop[(size_t)blockIdx.x * G + g] = TOP[g].x;
#pragma unroll
        for (int l = 0; l < L; ++l) pK[((size_t)blockIdx.x * L + l) * G + g] = bins[((size_t)l * (G + 1) + g) * R];
    }
    report(status, err);
}


// Seed tops for k_agg_lds: one sampled tile per workgroup.
template <class KT, class VT, class AT, int VEC>
__global__ void __launch_bounds__(AGG_BLOCK) k_sample_lds(const KT* __restrict__ keys, const VT* __restrict__ vals,
                                                          int64_t n, int G, int64_t stride, int* __restrict__ seed) {
    extern __shared__ __align__(16) unsigned char smem[];
    const SrcCol<KT, VT, VEC, AGG_BLOCK> src(keys, vals);
    sample_tops<SrcCol<KT, VT, VEC, AGG_BLOCK>, AT, AGG_BLOCK>(src, n, stride, G, reinterpret_cast<int*>(smem), seed);
}

// ------------------------------------------------- high cardinality path
//
// When the groups do not fit one workgroup's LDS, the rows are first
// partitioned on the high bits of the key (ParallelPartition of Alg. 4,
// Sec. V-B) into F partitions of at most GP = 2^gp_shift groups, then every
// partition is aggregated in LDS by the same hot loop (per-tile mode: the
// groups are many and their rows few), and partitions split over several
// workgroups are merged (the merge phase of Alg. 4).  The order of rows
// inside a partition is not deterministic and needs not be: level sums are
// exact.
//
//   k_part_hist     per-slab histogram of partition ids -> counts[s][p]
//   k_part_round_scan, k_part_round_bases
//                   per partition: rows before slab s (rel[s][p] within its
//                   round, roff[k][p] before round k), size
//   k_part_plan     partition bases, chunking into work items, work table
//   k_part_scatter  (local key, value) pairs into their partition's range
//   k_agg_part      one work item = one chunk of one partition, aggregated in
//                   LDS; single-chunk partitions merge into the states
//                   directly, others write a partial per work item
//   k_merge_part    folds the partials of split partitions into the states
constexpr int PART_BLOCK = 1024;
constexpr int PART_WG = 256;                  // histogram/scatter workgroups
constexpr int64_t PART_CHUNK = 128 * 1024;    // rows per aggregation work item
constexpr int DEEP_MAX_F = 1024;              // super-partitions of the second partitioning level

struct WorkItem {
    int p;        // partition
    int nchunks;  // work items of this partition
    int first;    // its first work item
    int pad;
    long long r0, r1;  // rows in the partitioned arrays
};

// Slabs of the partition passes.  A slab is one or more of the scatter's
// tiles (RU * PART_BLOCK rows; several when the partitions are so many that
// per-tile counts would cost more than a byte per row); workgroup w of nw
// takes slabs w, w + nw, w + 2 nw, ... (round k = s / nw).  Inside a
// partition the rows are laid out round by round, and in a round workgroup
// by workgroup in XCD-major order: workgroups are dispatched round-robin
// over the 8 XCDs (XCD = w mod 8), so the runs that the workgroups of one
// XCD write into a partition in one round are adjacent and fill whole lines
// in that XCD's L2, instead of each workgroup's run ending in a partial line
// that leaves the L2 before the workgroup's next slab completes it.
constexpr int NXCD = 8;

// Workgroup at position r of the XCD-major order of nw workgroups.
__host__ __device__ inline int xcd_unrank(int r, int nw) {
    int x = 0;
    for (; x < NXCD - 1; ++x) {
        const int c = (nw - x + NXCD - 1) / NXCD;  // workgroups on XCD x
        if (r < c) break;
        r -= c;
    }
    return r * NXCD + x;
}

template <class KT>
__global__ void __launch_bounds__(PART_BLOCK) k_part_hist(const KT* __restrict__ keys, int64_t n, int64_t G,
                                                          int gp_shift, int F, int64_t slab,
                                                          int* __restrict__ counts) {
    extern __shared__ __align__(16) unsigned char smem[];
    int* h = reinterpret_cast<int*>(smem);
    const int64_t nslabs = (n + slab - 1) / slab;
    constexpr int UH = 8;  // keys in flight per thread
    for (int64_t t = blockIdx.x; t < nslabs; t += gridDim.x) {
        for (int i = threadIdx.x; i < F; i += PART_BLOCK) h[i] = 0;
        __syncthreads();
        const int64_t c0 = t * slab;
        const int64_t c1 = min(n, c0 + slab);
        for (int64_t b = c0; b < c1; b += (int64_t)UH * PART_BLOCK) {
            int64_t kk[UH];
#pragma unroll
            for (int u = 0; u < UH; ++u) {
                const int64_t i = b + u * PART_BLOCK + threadIdx.x;
                kk[u] = (i < c1) ? (int64_t)__builtin_nontemporal_load(&keys[i]) : -1;
            }
#pragma unroll
            for (int u = 0; u < UH; ++u)
                if ((uint64_t)kk[u] < (uint64_t)G) atomicAdd(&h[(int)(kk[u] >> gp_shift)], 1);
        }
        __syncthreads();
        for (int i = threadIdx.x; i < F; i += PART_BLOCK) counts[t * F + i] = h[i];
        __syncthreads();  // h is cleared for the next slab
    }
}

// Grid (ceil(F / 64), rounds), 256 threads: 64 partitions x 4 quarters of
// a round's workgroup positions (at most 64 each, nw <= 256).  Each thread
// loads its quarter's counts together, then rel[s][p] = rows of p in the
// round's earlier slabs (XCD-major order) and rsum[k][p] = rows of p in
// round k.
constexpr int RS_P = 64;
__global__ void __launch_bounds__(256) k_part_round_scan(const int* __restrict__ counts, int64_t nslabs, int nw,
                                                         int F, int* __restrict__ rel, int* __restrict__ rsum) {
    __shared__ int qsum[4][RS_P];
    const int pp = threadIdx.x % RS_P, q = threadIdx.x / RS_P;
    const int p = blockIdx.x * RS_P + pp;
    const int64_t k = blockIdx.y;
    const int per = (nw + 3) / 4;
    const int r0 = min(nw, q * per), r1 = min(nw, r0 + per);
    int c[RS_P];
    int s = 0;
#pragma unroll
    for (int j = 0; j < RS_P; ++j) {
        c[j] = 0;
        if (r0 + j < r1 && p < F) {
            const int64_t t = k * nw + xcd_unrank(r0 + j, nw);
            if (t < nslabs) c[j] = counts[t * F + p];
        }
        s += c[j];
    }
    qsum[q][pp] = s;
    __syncthreads();
    if (p >= F) return;
    int run = 0;
    for (int u = 0; u < q; ++u) run += qsum[u][pp];
#pragma unroll
    for (int j = 0; j < RS_P; ++j) {
        if (r0 + j < r1) {
            const int64_t t = k * nw + xcd_unrank(r0 + j, nw);
            if (t < nslabs) rel[t * F + p] = run;
            run += c[j];
        }
    }
    if (q == 3) rsum[k * F + p] = run;
}

// One thread per partition: roff[k][p] = rows of p before round k; size[p].
__global__ void __launch_bounds__(256) k_part_round_bases(const int* __restrict__ rsum, int64_t rounds, int F,
                                                          long long* __restrict__ roff, long long* __restrict__ size) {
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= F) return;
    long long run = 0;
    // unrolled: the loads of several rounds in flight at once
#pragma unroll 8
    for (int64_t k = 0; k < rounds; ++k) {
        roff[k * F + p] = run;
        run += rsum[k * F + p];
    }
    size[p] = run;
}

// single block: exclusive scans over the partitions (bases, work items).
// Every partition starts at a multiple of PART_ALIGN rows; the padding slots
// after its rows get local key 0 and value +0.0, which contribute nothing,
// so work items span whole aligned ranges and can use vector loads.
// The work table lists the items of split partitions (full chunks, the
// heaviest work) first and single-item partitions after them: workgroups
// are dispatched in table order, so the longest items start first and the
// end of the pass is not held up by a late large item.
constexpr int PART_ALIGN = 8;

template <class VT>
__global__ void __launch_bounds__(PART_BLOCK) k_part_plan(const long long* __restrict__ size, int F, int64_t chunk,
                                                          long long* __restrict__ base, int* __restrict__ wfirst,
                                                          WorkItem* __restrict__ items, int* __restrict__ nitems,
                                                          uint16_t* __restrict__ lkey, VT* __restrict__ lval) {
    __shared__ long long sb[PART_BLOCK];
    __shared__ int sw[PART_BLOCK], ss[PART_BLOCK];
    const int t = threadIdx.x;
    const int per = (F + PART_BLOCK - 1) / PART_BLOCK;  // partitions per thread
    const int p0 = min(F, t * per), p1 = min(F, p0 + per);
    long long rs = 0;
    int wsplit = 0, wsingle = 0;  // items of split partitions, of single-item ones
    for (int p = p0; p < p1; ++p) {
        const long long sz = (size[p] + PART_ALIGN - 1) / PART_ALIGN * PART_ALIGN;
        const int nc = (int)((sz + chunk - 1) / chunk);
        rs += sz;
        if (nc > 1)
            wsplit += nc;
        else
            wsingle += nc;
    }
    sb[t] = rs;
    sw[t] = wsplit;
    ss[t] = wsingle;
    __syncthreads();
    for (int o = 1; o < PART_BLOCK; o <<= 1) {
        const long long x = (t >= o) ? sb[t - o] : 0;
        const int y = (t >= o) ? sw[t - o] : 0;
        const int z = (t >= o) ? ss[t - o] : 0;
        __syncthreads();
        sb[t] += x;
        sw[t] += y;
        ss[t] += z;
        __syncthreads();
    }
    const int nsplit = sw[PART_BLOCK - 1];  // split items come first
    long long b = sb[t] - rs;
    int wa = sw[t] - wsplit, wb = nsplit + ss[t] - wsingle;
    for (int p = p0; p < p1; ++p) {
        const long long sz = (size[p] + PART_ALIGN - 1) / PART_ALIGN * PART_ALIGN;
        for (long long q = b + size[p]; q < b + sz; ++q) {
            lkey[q] = 0;
            lval[q] = (VT)0;
        }
        const int nc = (int)((sz + chunk - 1) / chunk);
        int& wi = (nc > 1) ? wa : wb;
        base[p] = b;
        wfirst[p] = wi;
        for (int c = 0; c < nc; ++c) {
            WorkItem it;
            it.p = p;
            it.nchunks = nc;
            it.first = wi;
            it.pad = 0;
            it.r0 = b + (long long)c * chunk;
            it.r1 = min(b + sz, it.r0 + chunk);
            items[wi + c] = it;
        }
        b += sz;
        wi += nc;
    }
    if (t == PART_BLOCK - 1) *nitems = nsplit + ss[t];
}

// Exclusive scan of cnt[0..F) into off[0..F) by one 1024-thread block
// (F <= 4096: up to 4 consecutive entries per thread, wave scans, LDS for
// the wave totals).  Returns the total.  Contains barriers.  When `base` is
// given, base[p] -= off[p] as well (by the thread that writes off[p]).
__device__ __forceinline__ int block_exclusive_scan(const int* cnt, int* off, int F, int* wsum,
                                                    long long* base = nullptr) {
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int per = (F + PART_BLOCK - 1) / PART_BLOCK;
    const int p0 = min(F, t * per), p1 = min(F, p0 + per);
    int local = 0;
    for (int p = p0; p < p1; ++p) local += cnt[p];
    int inc = local;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int x = __shfl_up(inc, o, 64);
        if (lane >= o) inc += x;
    }
    if (lane == 63) wsum[wave] = inc;
    __syncthreads();
    int before = 0, total = 0;
    for (int w = 0; w < PART_BLOCK / 64; ++w) {
        before += (w < wave) ? wsum[w] : 0;
        total += wsum[w];
    }
    int run = before + inc - local;
    for (int p = p0; p < p1; ++p) {
        off[p] = run;
        if (base) base[p] -= run;
        run += cnt[p];
    }
    __syncthreads();
    return total;
}

// Scatter of (local key, value) pairs into partitions.  The input is
// streamed with non-temporal loads.  Each tile (RU * 1024 rows) is
// counting-sorted by partition in LDS, then written out as contiguous
// per-partition runs.  A row with a valid key and an unusable value
// (NaN/Inf/out of domain) keeps its slot with value +0.0, which contributes
// nothing; its status bit is set.  The max-exponent step is left to the
// aggregation of each partition, where the partition's tops sit in LDS.
template <class KT, class VT, class AT, int RU, bool DOM = true, class LK = uint16_t>
__global__ void __launch_bounds__(PART_BLOCK)
    k_part_scatter(const KT* __restrict__ keys, const VT* __restrict__ vals, int64_t n, int64_t G, int gp_shift, int F,
                   int64_t slab, const long long* __restrict__ base, const long long* __restrict__ roff,
                   const int* __restrict__ rel, LK* __restrict__ lkey, VT* __restrict__ lval,
                   uint32_t* __restrict__ status) {
    typedef Fmt<AT> Fm;
    constexpr int SC_TILE = RU * PART_BLOCK;  // RU rows per thread and tile
    extern __shared__ __align__(16) unsigned char smem[];
    long long* cur = reinterpret_cast<long long*>(smem);         // F: next global slot
    int* cnt = reinterpret_cast<int*>(cur + F);                   // F: rows in this tile
    int* off = cnt + F;                                           // F: tile offsets
    VT* sv = reinterpret_cast<VT*>(off + F);                      // SC_TILE staged values
    LK* sk = reinterpret_cast<LK*>(sv + SC_TILE);                 // staged local keys
    uint16_t* sp = reinterpret_cast<uint16_t*>(sk + SC_TILE);     // staged partitions
    __shared__ int wsum[PART_BLOCK / 64];
    const int t = threadIdx.x;
    const int64_t nslabs = (n + slab - 1) / slab;
    const uint32_t gmask = (1u << gp_shift) - 1;
    uint32_t err = 0;
    for (int64_t sl = blockIdx.x; sl < nslabs; sl += gridDim.x) {
        const int64_t k = sl / gridDim.x;  // round
        const int64_t s1 = min(n, (sl + 1) * slab);
        for (int64_t tb = sl * slab; tb < s1; tb += SC_TILE) {
            const int64_t c1 = min(s1, tb + SC_TILE);
            for (int i = t; i < F; i += PART_BLOCK) {
                cnt[i] = 0;
                if (tb == sl * slab) cur[i] = base[i] + roff[k * F + i] + rel[sl * F + i];  // the slab's first slots
            }
            __syncthreads();
            int pi[RU], rk[RU];
            int64_t kk[RU];
            LK lk[RU];
            VT vv[RU];
            // loads first, so that the memory requests of all rows overlap
#pragma unroll
            for (int u = 0; u < RU; ++u) {
                const int64_t i = tb + u * PART_BLOCK + t;
                kk[u] = (i < c1) ? (int64_t)__builtin_nontemporal_load(&keys[i]) : -1;
                vv[u] = (i < c1) ? __builtin_nontemporal_load(&vals[i]) : (VT)0;
            }
#pragma unroll
            for (int u = 0; u < RU; ++u) {
                const int64_t i = tb + u * PART_BLOCK + t;
                pi[u] = -1;
                if (i < c1) {
                    const int64_t key = kk[u];
                    VT v = vv[u];
                    // every row's value is classified, whatever its key, so the
                    // status bits are those of the LDS path
                    if (!finite_val(v)) {
                        err |= ERR_NONFINITE;
                        v = (VT)0;
                    } else if (DOM && v != (VT)0 && jreq_raw<AT>(frexp_raw(v)) > Fm::JMAX) {
                        err |= ERR_RANGE;
                        v = (VT)0;
                    }
                    if ((uint64_t)key < (uint64_t)G) {
                        pi[u] = (int)(key >> gp_shift);
                        lk[u] = (LK)((uint32_t)key & gmask);
                        vv[u] = v;
                        rk[u] = atomicAdd(&cnt[pi[u]], 1);
                    } else {
                        err |= ERR_KEY;
                    }
                }
            }
            __syncthreads();  // all tile counts in place
            // off: the partitions' offsets in the tile; cur[p] becomes the slot of
            // the tile's first row of p minus off[p], so a staged row j of p goes
            // to slot cur[p] + j (one LDS read fewer per row when writing out)
            const int ntile = block_exclusive_scan(cnt, off, F, wsum, cur);
#pragma unroll
            for (int u = 0; u < RU; ++u) {
                if (pi[u] >= 0) {
                    const int pos = off[pi[u]] + rk[u];
                    sv[pos] = vv[u];
                    sk[pos] = lk[u];
                    sp[pos] = (uint16_t)pi[u];
                }
            }
            __syncthreads();
            // unrolled: the LDS reads of a thread's rows are in flight together
#pragma unroll
            for (int u = 0; u < RU; ++u) {
                const int j = t + u * PART_BLOCK;
                if (j < ntile) {
                    const long long slot = cur[sp[j]] + j;
                    lkey[slot] = sk[j];
                    lval[slot] = sv[j];
                }
            }
            __syncthreads();  // the staging area and counts are reused by the next tile
            if (tb + SC_TILE < s1)  // the slab's next tile follows its slots
                for (int i = t; i < F; i += PART_BLOCK) cur[i] += off[i] + cnt[i];
        }
    }
    report(status, err);
}

// One work item (a chunk of one partition): the partition's groups are
// aggregated in LDS by the same per-tile loop as the low-cardinality kernel
// (tops raised in LDS, bins realigned once per tile, no spill array).
// Partitions taken by one work item fold into the caller's states directly,
// others write a partial (top, K[L]) per group for k_merge_part.  Values in
// the partitioned array are finite and in the domain, or +0.0 (contributes
// nothing); rows of the padding have local key 0 and value +0.0.
template <class VT, class AT, int L>
__global__ void __launch_bounds__(AGG_BLOCK) k_agg_part(const uint16_t* __restrict__ lkey, const VT* __restrict__ lval,
                                                        const WorkItem* __restrict__ items,
                                                        const int* __restrict__ nitems, int64_t G, int gp_shift,
                                                        int* __restrict__ ptop, long long* __restrict__ pK,
                                                        AT* __restrict__ S, long long* __restrict__ C, int64_t gbase,
                                                        int64_t Gstride, uint32_t* __restrict__ status) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ AggShared sh;
    if ((int)blockIdx.x >= *nitems) return;  // uniform: the grid is an upper bound
    const WorkItem it = items[blockIdx.x];
    const int GP = 1 << gp_shift;
    const int64_t g0 = (int64_t)it.p << gp_shift;
    const int Gp = (int)min((int64_t)GP, G - g0);
    // [r0, r1) starts on a multiple of 8 rows (aligned partitions), so the
    // vector loads of the tiles are aligned
    constexpr int VEC = 16 / sizeof(VT);
    const uint32_t err =
        aggregate_range<uint16_t, VT, AT, L, VEC, false>(lkey, lval, it.r0, it.r1, Gp, 1, smem, sh, nullptr);
    const long long* bins = reinterpret_cast<const long long*>(smem);
    const int2* TOP = reinterpret_cast<const int2*>(bins + (size_t)(Gp + 1) * L);
    if (it.nchunks == 1) {
        for (int g = threadIdx.x; g < Gp; g += AGG_BLOCK)
            fold_into_state<AT, L>(bins + g, Gp + 1, TOP[g].x, S, C, Gstride, gbase + g0 + g);
    } else {
        for (int g = threadIdx.x; g < Gp; g += AGG_BLOCK) {
            ptop[(size_t)blockIdx.x * GP + g] = TOP[g].x;
#pragma unroll
            for (int l = 0; l < L; ++l) pK[((size_t)blockIdx.x * L + l) * GP + g] = bins[(size_t)l * (Gp + 1) + g];
        }
    }
    report(status, err);
}

// Baseline (NOT reproducible): the same partitioned pass on doubles (the
// built-in type's PartitionAndAggregate the paper compares against).  One
// work item's rows are summed into LDS doubles with atomic adds; a
// partition taken by one item adds its sums to out directly, the items of
// split partitions add theirs with global double atomics.
constexpr int PLAIN_PART_BLOCK = 1024;
template <class VT>
__global__ void __launch_bounds__(PLAIN_PART_BLOCK)
    k_agg_part_plain(const uint16_t* __restrict__ lkey, const VT* __restrict__ lval,
                     const WorkItem* __restrict__ items, const int* __restrict__ nitems, int64_t G, int gp_shift,
                     double* __restrict__ out) {
    extern __shared__ __align__(16) unsigned char smem[];
    double* bins = reinterpret_cast<double*>(smem);
    if ((int)blockIdx.x >= *nitems) return;  // uniform: the grid is an upper bound
    const WorkItem it = items[blockIdx.x];
    const int GP = 1 << gp_shift;
    const int64_t g0 = (int64_t)it.p << gp_shift;
    const int Gp = (int)min((int64_t)GP, G - g0);
    for (int g = threadIdx.x; g < Gp; g += PLAIN_PART_BLOCK) bins[g] = 0.0;
    __syncthreads();
    // [r0, r1) is a whole number of 8-row groups starting on a multiple of 8
    constexpr int VEC = 16 / sizeof(VT);
    typedef typename VecT<VT, VEC>::type V;
    typedef typename VecT<uint16_t, VEC>::type K;
    constexpr int U = 4;  // vector loads in flight per thread
    constexpr int64_t STEP = (int64_t)PLAIN_PART_BLOCK * VEC;
    for (int64_t b = it.r0; b < it.r1; b += U * STEP) {
        V x[U];
        K kk[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t r = b + u * STEP + (int64_t)threadIdx.x * VEC;
            if (r < it.r1) {
                x[u] = *reinterpret_cast<const V*>(lval + r);
                kk[u] = *reinterpret_cast<const K*>(lkey + r);
            } else {
                x[u] = (V)(VT)0;
                kk[u] = (K)(uint16_t)0;
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int e = 0; e < VEC; ++e)
                if (x[u][e] != (VT)0) atomicAdd(&bins[kk[u][e]], (double)x[u][e]);
    }
    __syncthreads();
    for (int g = threadIdx.x; g < Gp; g += PLAIN_PART_BLOCK) {
        const double b = bins[g];
        if (it.nchunks == 1)
            out[g0 + g] += b;
        else if (b != 0.0)
            atomicAdd(&out[g0 + g], b);
    }
}

// one thread per group of a split partition: fold its work items' partials
template <class AT, int L>
__global__ void __launch_bounds__(256) k_merge_part(const WorkItem* __restrict__ items, const int* __restrict__ nitems,
                                                    const int* __restrict__ wfirst, int F, int64_t G, int gp_shift,
                                                    const int* __restrict__ ptop, const long long* __restrict__ pK,
                                                    AT* __restrict__ S, long long* __restrict__ C, int64_t gbase,
                                                    int64_t Gstride) {
    typedef Fmt<AT> F_;
    constexpr int c = F_::CARRY;
    const int GP = 1 << gp_shift;
    const int p = blockIdx.y;
    const int gl = blockIdx.x * 256 + threadIdx.x;
    if (p >= F || gl >= GP) return;
    const int w0 = wfirst[p];
    if (w0 >= *nitems) return;  // empty partition (trailing)
    const WorkItem it = items[w0];
    if (it.p != p || it.nchunks < 2) return;  // empty or already folded
    if (((int64_t)p << gp_shift) + gl >= G) return;
    const int64_t g = gbase + ((int64_t)p << gp_shift) + gl;  // state index (row stride Gstride)
    const int ts = state_top(S[g]);
    int J = ts;
    // unrolled so that the loads of several work items are in flight at
    // once: the hottest partitions (skewed keys) have dozens of items
#pragma unroll 8
    for (int w = w0; w < w0 + it.nchunks; ++w) J = max(J, ptop[(size_t)w * GP + gl]);
    long long hi[L], lo[L];
#pragma unroll
    for (int l = 0; l < L; ++l) {
        const int ls = l - (J - ts);
        hi[l] = (ls >= 0) ? C[(size_t)ls * Gstride + g] : 0;
        lo[l] = (ls >= 0) ? state_lo(S[(size_t)ls * Gstride + g]) : 0;
    }
#pragma unroll 8
    for (int w = w0; w < w0 + it.nchunks; ++w) {
        const int d = J - ptop[(size_t)w * GP + gl];
        long long x[L];
#pragma unroll
        for (int l = 0; l < L; ++l) x[l] = pK[((size_t)w * L + l) * GP + gl];
#pragma unroll
        for (int l = 0; l < L; ++l) {
            long long v = 0;
#pragma unroll
            for (int q = 0; q < L; ++q) v = (q == l - d) ? x[q] : v;
            hi[l] += v >> c;
            lo[l] += v & ((1ll << c) - 1);
        }
    }
#pragma unroll
    for (int l = 0; l < L; ++l) {
        long long cc, oo;
        normalise<AT>(hi[l], lo[l], &cc, &oo);
        S[(size_t)l * Gstride + g] = make_S((AT*)0, F_::B + (J - l) * F_::W, oo);
        C[(size_t)l * Gstride + g] = cc;
    }
}

// operator+=(repro) on whole state arrays: dst[g] += src[g].
template <class AT, int L>
__global__ void __launch_bounds__(256) k_merge_states(AT* __restrict__ Sd, long long* __restrict__ Cd,
                                                      const AT* __restrict__ Ss, const long long* __restrict__ Cs,
                                                      int G) {
    typedef Fmt<AT> F;
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= G) return;
    const int td = state_top(Sd[g]), ts = state_top(Ss[g]);
    const int J = max(td, ts);
    long long hi[L], lo[L];
#pragma unroll
    for (int l = 0; l < L; ++l) {
        const int ld = l - (J - td), ls = l - (J - ts);
        hi[l] = (ld >= 0 ? Cd[(size_t)ld * G + g] : 0) + (ls >= 0 ? Cs[(size_t)ls * G + g] : 0);
        lo[l] = (ld >= 0 ? state_lo(Sd[(size_t)ld * G + g]) : 0) + (ls >= 0 ? state_lo(Ss[(size_t)ls * G + g]) : 0);
    }
#pragma unroll
    for (int l = 0; l < L; ++l) {
        long long cc, oo;
        normalise<AT>(hi[l], lo[l], &cc, &oo);
        Sd[(size_t)l * G + g] = make_S((AT*)0, F::B + (J - l) * F::W, oo);
        Cd[(size_t)l * G + g] = cc;
    }
}

template <class AT, int L>
__global__ void __launch_bounds__(256) k_state_init(AT* __restrict__ S, long long* __restrict__ C, int G) {
    typedef Fmt<AT> F;
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    // zero the padding between the S and C blocks (float states, odd G*L)
    if (g == 0 && (size_t)G * L * sizeof(AT) % 8 != 0) S[(size_t)G * L] = (AT)0;
    if (g >= G) return;
#pragma unroll
    for (int l = 0; l < L; ++l) {
        S[(size_t)l * G + g] = make_S((AT*)0, F::B + (L - 1 - l) * F::W, 0);
        C[(size_t)l * G + g] = 0;
    }
}

// Finalisation (equation of Sec. III-C): each level's exact value
// (C * 2^CARRY + lo) * 2^(E_l - m) rounded once to AT, then summed in AT
// from the last level to the first.
template <class AT, int L>
__global__ void __launch_bounds__(256) k_finalize(const AT* __restrict__ S, const long long* __restrict__ C, int G,
                                                  AT* __restrict__ out) {
    typedef Fmt<AT> F;
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= G) return;
    const int top = state_top(S[g]);
    AT q[L];
#pragma unroll
    for (int l = 0; l < L; ++l) {
        const i128 K = (i128)C[(size_t)l * G + g] * ((i128)1 << F::CARRY) + (i128)state_lo(S[(size_t)l * G + g]);
        q[l] = round_exact<AT>(K, F::B + (top - l) * F::W - F::m);
    }
    AT acc = q[L - 1];
#pragma unroll
    for (int l = L - 2; l >= 0; --l) acc = acc + q[l];
    out[g] = acc + (AT)0;
}

// --------------------------------------------------- plain FP64 baseline
// Non-reproducible reference point: LDS-privatised double atomics, then
// one global double atomic per group and workgroup.  Its own launch shape
// (4 workgroups of 256 threads per CU) streams at the full read bandwidth.
constexpr int PLAIN_BLOCK = 256;
constexpr int PLAIN_TILE = PLAIN_BLOCK * ROWS_PER_THREAD;
constexpr int PLAIN_MAX_WG = 1024;
template <class KT, class VT, int VEC>
__global__ void __launch_bounds__(PLAIN_BLOCK) k_plain_lds(const KT* __restrict__ keys, const VT* __restrict__ vals,
                                                         int64_t n, int G, int64_t chunk, double* __restrict__ out,
                                                         uint32_t* __restrict__ status) {
    extern __shared__ __align__(16) unsigned char smem[];
    double* bins = reinterpret_cast<double*>(smem);
    const int tid = threadIdx.x;
    for (int i = tid; i < G; i += PLAIN_BLOCK) bins[i] = 0.0;
    __syncthreads();
    const int64_t c0 = (int64_t)blockIdx.x * chunk;
    const int64_t c1 = (c0 + chunk < n) ? c0 + chunk : n;
    uint32_t err = 0;
    KT kc[ROWS_PER_THREAD];
    VT vc[ROWS_PER_THREAD];
    uint32_t off[ROWS_PER_THREAD / VEC];
#pragma unroll
    for (int u = 0; u < ROWS_PER_THREAD / VEC; ++u) off[u] = (uint32_t)((u * PLAIN_BLOCK + threadIdx.x) * VEC);
    for (int64_t base = c0; base < c1; base += PLAIN_TILE) {
        const uint32_t inr = load_tile<KT, VT, VEC, PLAIN_BLOCK>(keys, vals, base, c1, kc, vc, off);
#pragma unroll
        for (int i = 0; i < ROWS_PER_THREAD; ++i) {
            const bool in = (inr >> i) & 1u;
            const bool kok = (uint64_t)(int64_t)kc[i] < (uint64_t)G;
            const bool fin = finite_val(vc[i]);
            err |= (in && !kok) ? ERR_KEY : 0u;
            err |= (in && !fin) ? ERR_NONFINITE : 0u;
            if (in && kok && fin) atomicAdd(&bins[(int)kc[i]], (double)vc[i]);
        }
    }
    __syncthreads();
    for (int gg = tid; gg < G; gg += PLAIN_BLOCK)
        if (bins[gg] != 0.0) atomicAdd(&out[gg], bins[gg]);
    report(status, err);
}

template <class KT, class VT, int VEC>
__global__ void __launch_bounds__(PLAIN_BLOCK) k_plain_global(const KT* __restrict__ keys, const VT* __restrict__ vals,
                                                            int64_t n, int G, int64_t chunk, double* __restrict__ out,
                                                            uint32_t* __restrict__ status) {
    const int64_t c0 = (int64_t)blockIdx.x * chunk;
    const int64_t c1 = (c0 + chunk < n) ? c0 + chunk : n;
    uint32_t err = 0;
    KT kc[ROWS_PER_THREAD];
    VT vc[ROWS_PER_THREAD];
    uint32_t off[ROWS_PER_THREAD / VEC];
#pragma unroll
    for (int u = 0; u < ROWS_PER_THREAD / VEC; ++u) off[u] = (uint32_t)((u * PLAIN_BLOCK + threadIdx.x) * VEC);
    for (int64_t base = c0; base < c1; base += PLAIN_TILE) {
        const uint32_t inr = load_tile<KT, VT, VEC, PLAIN_BLOCK>(keys, vals, base, c1, kc, vc, off);
#pragma unroll
        for (int i = 0; i < ROWS_PER_THREAD; ++i) {
            const bool in = (inr >> i) & 1u;
            const bool kok = (uint64_t)(int64_t)kc[i] < (uint64_t)G;
            const bool fin = finite_val(vc[i]);
            err |= (in && !kok) ? ERR_KEY : 0u;
            err |= (in && !fin) ? ERR_NONFINITE : 0u;
            if (in && kok && fin) atomicAdd(&out[(int64_t)kc[i]], (double)vc[i]);
        }
    }
    report(status, err);
}

// ------------------------------------------------ read-stream ceiling
// Measurement aid: reads `words` 16-byte words once, grid-strided with four
// loads in flight per thread, and folds them into one XOR per workgroup so
// the loads are not removed.  Its rate is the read ceiling the aggregation
// kernels are held against.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
__global__ void k_read_probe(const u32x4* __restrict__ p, size_t words, unsigned long long* __restrict__ sink) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    u32x4 acc = {0u, 0u, 0u, 0u};
    for (; i + 3 * stride < words; i += 4 * stride) {
        const u32x4 a = __builtin_nontemporal_load(p + i), b = __builtin_nontemporal_load(p + i + stride);
        const u32x4 c = __builtin_nontemporal_load(p + i + 2 * stride), d = __builtin_nontemporal_load(p + i + 3 * stride);
        acc ^= a ^ b ^ c ^ d;
    }
    for (; i < words; i += stride) acc ^= p[i];
    const uint32_t any = wave_or((acc.x | acc.y | acc.z | acc.w) != 0u ? 1u : 0u);
    if (any && threadIdx.x == 0) atomicAdd(sink, 1ull);
}

__global__ void __launch_bounds__(256) k_atomic_probe(const int* __restrict__ idx, int64_t n,
                                                      unsigned long long* __restrict__ table, int64_t words) {
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) {
        const int j = idx[i];
        if ((uint64_t)(int64_t)j < (uint64_t)words) atomicAdd(&table[j], 1ull);
    }
}

// ================================================================ host

inline size_t scalar_size(repro_scalar_t t) { return t == REPRO_F64 ? 8 : 4; }

bool valid_common(int64_t G, repro_scalar_t T, int L) {
    return G >= 1 && G <= INT32_MAX && (T == REPRO_F32 || T == REPRO_F64) && L >= 1 && L <= 4;
}


// High cardinality: partition, then aggregate every partition in LDS.  A
// partition holds 2^s groups, the largest power of two up to 2^smax whose
// `gbytes` LDS bytes per group (plus one slot) fit the budget.  The plain
// baseline (L = 0) keeps one double per group and no partials.
// Rows of a slab of the partition passes: whole scatter tiles, enough of
// them that the per-slab counts and offsets (8 bytes per partition) stay
// within about a byte per row.
inline int64_t part_slab_rows(int sc_ru, int64_t F) {
    const int64_t tile = (int64_t)sc_ru * PART_BLOCK;
    const int64_t tiles = std::max<int64_t>(1, (8 * F + tile - 1) / tile);
    return tiles * tile;
}

bool make_plan_part(int64_t n, int64_t G, int L, size_t vsize, Plan* p) {
    p->path = 2;
    const size_t gbytes = L > 0 ? (size_t)8 * L + 12 : 8;
    int s = L > 0 ? 12 : 14;
    while (s > 6 && ((size_t)(1 << s) + 1) * gbytes > LDS_BIN_BUDGET) --s;
    p->gp_shift = s;
    const int64_t F = (G + (1 << s) - 1) >> s;
    if (F > 4096) return false;  // cursors, counts and offsets of all partitions in LDS
    p->sc_ru = ((size_t)F * 16 + (size_t)8 * PART_BLOCK * (vsize + 4) + 512 <= LDS_BIN_BUDGET) ? 8 : 4;
    p->lds_sc = (size_t)F * 16 + (size_t)p->sc_ru * PART_BLOCK * (vsize + 4);
    p->F = (int)F;
    int64_t nw = (n + (int64_t)PART_BLOCK * 16 - 1) / ((int64_t)PART_BLOCK * 16);
    nw = std::max<int64_t>(1, std::min<int64_t>(PART_WG, nw));
    p->nw = (int)nw;
    p->slab = part_slab_rows(p->sc_ru, F);
    const int64_t nslabs = (n + p->slab - 1) / p->slab;
    const int64_t rounds = std::max<int64_t>(1, (nslabs + nw - 1) / nw);
    if (rounds > 65535) return false;  // a grid dimension of the round scan
    const int64_t maxw = F + (n + (int64_t)PART_ALIGN * F + PART_CHUNK - 1) / PART_CHUNK;
    if (maxw > INT32_MAX / 2) return false;
    p->maxw = (int)maxw;
    p->lds_agg2 = ((size_t)(1 << s) + 1) * gbytes;  // bins, TOP and P of aggregate_range (or plain bins)
    const int GP = 1 << s;
    size_t ws = 0;
    auto take = [&](size_t bytes) { size_t o = ws; ws += align_up(bytes, 256); return o; };
    p->o_counts = take((size_t)nslabs * F * 4);
    p->o_rel = take((size_t)nslabs * F * 4);
    p->o_rsum = take((size_t)rounds * F * 4);
    p->o_roff = take((size_t)rounds * F * 8);
    p->o_size = take((size_t)F * 8);
    p->o_base = take((size_t)F * 8);
    p->o_wfirst = take((size_t)F * 4);
    p->o_items = take((size_t)maxw * sizeof(WorkItem));
    p->o_nitems = take(4);
    const size_t rows_pad = (size_t)n + (size_t)PART_ALIGN * F;  // partitions padded to 8 rows
    p->o_lkey = take(rows_pad * 2);
    p->o_lval = take(rows_pad * vsize);
    p->o_ptop = take(L > 0 ? (size_t)maxw * GP * 4 : 0);
    p->o_pK = take((size_t)maxw * GP * L * 8);
    p->ws = ws;
    return true;
}

// Two levels: super-partitions of 4096 one-level partitions each.
bool make_plan_deep(int64_t n, int64_t G, int L, size_t vsize, Plan* p) {
    Plan one;
    memset(&one, 0, sizeof(one));
    make_plan_part(1, 1, L, vsize, &one);  // the one-level partition size for L
    memset(p, 0, sizeof(*p));
    p->path = 3;
    const int sshift = one.gp_shift + 12;
    p->gp_shift = sshift;
    const int64_t F = (G + ((int64_t)1 << sshift) - 1) >> sshift;
    if (F > DEEP_MAX_F) return false;
    p->F = (int)F;
    p->sc_ru = 8;
    p->lds_sc = (size_t)F * 16 + (size_t)8 * PART_BLOCK * (vsize + 6);
    int64_t nw = (n + (int64_t)PART_BLOCK * 16 - 1) / ((int64_t)PART_BLOCK * 16);
    nw = std::max<int64_t>(1, std::min<int64_t>(PART_WG, nw));
    p->nw = (int)nw;
    p->slab = part_slab_rows(p->sc_ru, F);
    const int64_t nslabs = (n + p->slab - 1) / p->slab;
    const int64_t rounds = std::max<int64_t>(1, (nslabs + nw - 1) / nw);
    if (rounds > 65535) return false;
    size_t ws = 0;
    auto take = [&](size_t bytes) { size_t o = ws; ws += align_up(bytes, 256); return o; };
    p->o_counts = take((size_t)nslabs * F * 4);
    p->o_rel = take((size_t)nslabs * F * 4);
    p->o_rsum = take((size_t)rounds * F * 4);
    p->o_roff = take((size_t)rounds * F * 8);
    p->o_size = take((size_t)F * 8);
    p->o_base = take((size_t)F * 8);
    p->o_lkey = take((size_t)n * 4);
    p->o_lval = take((size_t)n * vsize);
    Plan two;
    memset(&two, 0, sizeof(two));
    if (!make_plan_part(n, (int64_t)1 << sshift, L, vsize, &two)) return false;
    p->ws_l2 = two.ws;  // the largest one-level workspace of a super-partition
    p->o_l2 = take(two.ws);
    p->ws = ws;
    return true;
}

bool make_plan(int64_t n, int64_t G, int L, int jmax, size_t vsize, Plan* p) {
    if (agg_lds_bytes(G, L, 1) > LDS_BIN_BUDGET) {
        memset(p, 0, sizeof(*p));
        if (make_plan_part(n, G, L, vsize, p)) return true;
        return make_plan_deep(n, G, L, vsize, p);
    }
    return make_plan_lds(n, G, L, jmax, AGG_TILE, p);
}

// gbase, Gstride: the call's groups are states' groups gbase .. gbase+G-1 of
// Gstride (the second partitioning level runs one call per super-partition).
// The histogram and the per-slab offsets of the partition passes (the
// scatter's slabs and rounds, see xcd_unrank).
template <class KT>
int partition_offsets(const KT* keys, int64_t n, int64_t G, const Plan& p, unsigned char* ws, hipStream_t st) {
    int* counts = reinterpret_cast<int*>(ws + p.o_counts);
    int* rel = reinterpret_cast<int*>(ws + p.o_rel);
    int* rsum = reinterpret_cast<int*>(ws + p.o_rsum);
    long long* roff = reinterpret_cast<long long*>(ws + p.o_roff);
    long long* size = reinterpret_cast<long long*>(ws + p.o_size);
    const int64_t nslabs = (n + p.slab - 1) / p.slab;
    const int64_t rounds = std::max<int64_t>(1, (nslabs + p.nw - 1) / p.nw);
    const size_t lds_h = (size_t)p.F * 4;
    if (!allow_lds((const void*)k_part_hist<KT>, lds_h)) return REPRO_EHIP;
    hipLaunchKernelGGL(k_part_hist<KT>, dim3(p.nw), dim3(PART_BLOCK), lds_h, st, keys, n, G, p.gp_shift, p.F, p.slab,
                       counts);
    LAUNCH_CHECK();
    hipLaunchKernelGGL(k_part_round_scan, dim3((p.F + RS_P - 1) / RS_P, (unsigned)rounds), dim3(256), 0, st, counts,
                       nslabs, p.nw, p.F, rel, rsum);
    LAUNCH_CHECK();
    hipLaunchKernelGGL(k_part_round_bases, dim3((p.F + 255) / 256), dim3(256), 0, st, rsum, rounds, p.F, roff, size);
    LAUNCH_CHECK();
    return REPRO_OK;
}

template <class KT, class VT, class AT, int L>
int run_groupby_part(const void* keys, const void* values, int64_t n, int64_t G, void* states, void* workspace,
                     uint32_t* status, const Plan& p, hipStream_t st, int64_t gbase = 0, int64_t Gstride = -1) {
    if (Gstride < 0) Gstride = G;
    unsigned char* ws = static_cast<unsigned char*>(workspace);
    const KT* k = static_cast<const KT*>(keys);
    const VT* v = static_cast<const VT*>(values);
    int* rel = reinterpret_cast<int*>(ws + p.o_rel);
    long long* roff = reinterpret_cast<long long*>(ws + p.o_roff);
    long long* size = reinterpret_cast<long long*>(ws + p.o_size);
    long long* base = reinterpret_cast<long long*>(ws + p.o_base);
    int* wfirst = reinterpret_cast<int*>(ws + p.o_wfirst);
    WorkItem* items = reinterpret_cast<WorkItem*>(ws + p.o_items);
    int* nitems = reinterpret_cast<int*>(ws + p.o_nitems);
    uint16_t* lkey = reinterpret_cast<uint16_t*>(ws + p.o_lkey);
    VT* lval = reinterpret_cast<VT*>(ws + p.o_lval);
    int* ptop = reinterpret_cast<int*>(ws + p.o_ptop);
    long long* pK = reinterpret_cast<long long*>(ws + p.o_pK);
    AT* S = static_cast<AT*>(states);
    long long* C = reinterpret_cast<long long*>(static_cast<unsigned char*>(states) +
                                                align_up((size_t)Gstride * L * sizeof(AT), 8));
    const void* scatter = p.sc_ru == 8 ? (const void*)k_part_scatter<KT, VT, AT, 8> : (const void*)k_part_scatter<KT, VT, AT, 4>;
    if (!allow_lds(scatter, p.lds_sc) ||
        !allow_lds((const void*)k_agg_part<VT, AT, L>, p.lds_agg2))
        return REPRO_EHIP;
    {
        const int rc = partition_offsets<KT>(k, n, G, p, ws, st);
        if (rc != REPRO_OK) return rc;
    }
    hipLaunchKernelGGL(k_part_plan<VT>, dim3(1), dim3(PART_BLOCK), 0, st, size, p.F, PART_CHUNK, base, wfirst, items,
                       nitems, lkey, lval);
    LAUNCH_CHECK();
    prof_before(st);
    if (p.sc_ru == 8)
        hipLaunchKernelGGL((k_part_scatter<KT, VT, AT, 8>), dim3(p.nw), dim3(PART_BLOCK), p.lds_sc, st, k, v, n, G,
                           p.gp_shift, p.F, p.slab, base, roff, rel, lkey, lval, status);
    else
        hipLaunchKernelGGL((k_part_scatter<KT, VT, AT, 4>), dim3(p.nw), dim3(PART_BLOCK), p.lds_sc, st, k, v, n, G,
                           p.gp_shift, p.F, p.slab, base, roff, rel, lkey, lval, status);
    LAUNCH_CHECK();
    prof_after(st);
    prof_before(st);
    hipLaunchKernelGGL((k_agg_part<VT, AT, L>), dim3(p.maxw), dim3(AGG_BLOCK), p.lds_agg2, st, lkey, lval, items,
                       nitems, G, p.gp_shift, ptop, pK, S, C, gbase, Gstride, status);
    LAUNCH_CHECK();
    prof_after(st);
    const int GP = 1 << p.gp_shift;
    hipLaunchKernelGGL((k_merge_part<AT, L>), dim3((GP + 255) / 256, p.F), dim3(256), 0, st, items, nitems, wfirst,
                       p.F, G, p.gp_shift, ptop, pK, S, C, gbase, Gstride);
    LAUNCH_CHECK();
    return REPRO_OK;
}

// Two partitioning levels (Alg. 4 at depth 2), for more groups than 4096
// partitions hold: rows are first scattered on the key's high bits into
// super-partitions of 2^sshift groups (local keys as uint32), then every
// non-empty super-partition runs the one-level path on its rows, into its
// range of the states.  The super-partition sizes are read back to the host
// once (the call waits for its stream there).
__global__ void k_part_bases(const long long* __restrict__ size, int F, long long* __restrict__ base) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    long long b = 0;
    for (int p = 0; p < F; ++p) {
        base[p] = b;
        b += size[p];
    }
}

template <class KT, class VT, class AT, int L>
int run_groupby_deep(const void* keys, const void* values, int64_t n, int64_t G, void* states, void* workspace,
                     uint32_t* status, const Plan& p, hipStream_t st) {
    unsigned char* ws = static_cast<unsigned char*>(workspace);
    const KT* k = static_cast<const KT*>(keys);
    const VT* v = static_cast<const VT*>(values);
    int* rel = reinterpret_cast<int*>(ws + p.o_rel);
    long long* roff = reinterpret_cast<long long*>(ws + p.o_roff);
    long long* size = reinterpret_cast<long long*>(ws + p.o_size);
    long long* base = reinterpret_cast<long long*>(ws + p.o_base);
    uint32_t* lkey = reinterpret_cast<uint32_t*>(ws + p.o_lkey);
    VT* lval = reinterpret_cast<VT*>(ws + p.o_lval);
    if (!allow_lds((const void*)k_part_scatter<KT, VT, AT, 8, true, uint32_t>, p.lds_sc))
        return REPRO_EHIP;
    {
        const int rc = partition_offsets<KT>(k, n, G, p, ws, st);
        if (rc != REPRO_OK) return rc;
    }
    hipLaunchKernelGGL(k_part_bases, dim3(1), dim3(64), 0, st, size, p.F, base);
    LAUNCH_CHECK();
    hipLaunchKernelGGL((k_part_scatter<KT, VT, AT, 8, true, uint32_t>), dim3(p.nw), dim3(PART_BLOCK), p.lds_sc, st, k,
                       v, n, G, p.gp_shift, p.F, p.slab, base, roff, rel, lkey, lval, status);
    LAUNCH_CHECK();
    long long hsize[DEEP_MAX_F];
    if (hipMemcpyAsync(hsize, size, (size_t)p.F * 8, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return REPRO_EHIP;
    unsigned char* ws2 = ws + p.o_l2;
    long long b = 0;
    for (int sp = 0; sp < p.F; ++sp) {
        const int64_t ns = hsize[sp];
        const int64_t g0 = (int64_t)sp << p.gp_shift;
        const int64_t Gs = std::min<int64_t>((int64_t)1 << p.gp_shift, G - g0);
        if (ns > 0) {
            Plan p2;
            memset(&p2, 0, sizeof(p2));
            if (!make_plan_part(ns, Gs, L, sizeof(VT), &p2) || p2.ws > p.ws_l2) return REPRO_EHIP;
            const int rc = run_groupby_part<uint32_t, VT, AT, L>(lkey + b, lval + b, ns, Gs, states, ws2, status, p2,
                                                                  st, g0, G);
            if (rc != REPRO_OK) return rc;
        }
        b += ns;
    }
    return REPRO_OK;
}

template <class KT, class VT, class AT, int L>
int run_groupby(const void* keys, const void* values, int64_t n, int64_t G64, void* states, void* workspace,
                uint32_t* status, const Plan& p, hipStream_t st) {
    if (p.path == 2) return run_groupby_part<KT, VT, AT, L>(keys, values, n, G64, states, workspace, status, p, st);
    if (p.path == 3) return run_groupby_deep<KT, VT, AT, L>(keys, values, n, G64, states, workspace, status, p, st);
    const int G = (int)G64;
    unsigned char* ws = static_cast<unsigned char*>(workspace);
    int* ptop = reinterpret_cast<int*>(ws);
    long long* pK = reinterpret_cast<long long*>(ws + align_up((size_t)p.nwg * G * 4, 256));
    const KT* k = static_cast<const KT*>(keys);
    const VT* v = static_cast<const VT*>(values);
    constexpr int VEC = 16 / sizeof(VT);
    const bool aligned = ((uintptr_t)k % (VEC * sizeof(KT)) == 0) && ((uintptr_t)v % 16 == 0);
    if (!allow_lds((const void*)k_agg_lds<KT, VT, AT, L, VEC>, p.lds) ||
        !allow_lds((const void*)k_agg_lds<KT, VT, AT, L, 1>, p.lds))
        return REPRO_EHIP;
    unsigned long long* spill = reinterpret_cast<unsigned long long*>(ws + p.spill_off);
    int* seed = p.seed_tiles ? reinterpret_cast<int*>(ws + p.seed_off) : nullptr;
    if (p.spill_used) {
        hipLaunchKernelGGL(k_zero, dim3((unsigned)std::min<size_t>(1024, (p.zero_words + 255) / 256)), dim3(256), 0,
                           st, spill, p.zero_words);
        LAUNCH_CHECK();
    }
    if (seed) {
        const size_t lds_s = (size_t)(G + 1) * 4;
        if (aligned)
            hipLaunchKernelGGL((k_sample_lds<KT, VT, AT, VEC>), dim3(p.seed_tiles), dim3(AGG_BLOCK), lds_s, st, k, v, n,
                               G, p.seed_stride, seed);
        else
            hipLaunchKernelGGL((k_sample_lds<KT, VT, AT, 1>), dim3(p.seed_tiles), dim3(AGG_BLOCK), lds_s, st, k, v, n,
                               G, p.seed_stride, seed);
        LAUNCH_CHECK();
    }
    prof_before(st);
    if (aligned)
        hipLaunchKernelGGL((k_agg_lds<KT, VT, AT, L, VEC>), dim3(p.nwg), dim3(AGG_BLOCK), p.lds, st, k, v, n, G, p.R,
                           p.chunk, ptop, pK, spill, status, seed);
    else
        hipLaunchKernelGGL((k_agg_lds<KT, VT, AT, L, 1>), dim3(p.nwg), dim3(AGG_BLOCK), p.lds, st, k, v, n, G, p.R,
                           p.chunk, ptop, pK, spill, status, seed);
    LAUNCH_CHECK();
    prof_after(st);
    ColStates<AT> cs;
    cs.S[0] = static_cast<AT*>(states);
    cs.C[0] = reinterpret_cast<long long*>(static_cast<unsigned char*>(states) + align_up((size_t)G * L * sizeof(AT), 8));
    return run_merge<AT, L>(p, G, 1, ws, cs, st);
}

template <class KT, class VT, class AT>
int dispatch_L(int L, const void* keys, const void* values, int64_t n, int64_t G, void* states, void* ws,
               uint32_t* status, const Plan& p, hipStream_t st) {
    switch (L) {
        case 1: return run_groupby<KT, VT, AT, 1>(keys, values, n, G, states, ws, status, p, st);
        case 2: return run_groupby<KT, VT, AT, 2>(keys, values, n, G, states, ws, status, p, st);
        case 3: return run_groupby<KT, VT, AT, 3>(keys, values, n, G, states, ws, status, p, st);
        case 4: return run_groupby<KT, VT, AT, 4>(keys, values, n, G, states, ws, status, p, st);
    }
    return REPRO_EINVAL;
}

template <class KT>
int dispatch_types(repro_scalar_t vt, repro_scalar_t T, int L, const void* keys, const void* values, int64_t n, int64_t G,
                   void* states, void* ws, uint32_t* status, const Plan& p, hipStream_t st) {
    if (T == REPRO_F64 && vt == REPRO_F64)
        return dispatch_L<KT, double, double>(L, keys, values, n, G, states, ws, status, p, st);
    if (T == REPRO_F64 && vt == REPRO_F32)
        return dispatch_L<KT, float, double>(L, keys, values, n, G, states, ws, status, p, st);
    if (T == REPRO_F32 && vt == REPRO_F32)
        return dispatch_L<KT, float, float>(L, keys, values, n, G, states, ws, status, p, st);
    return REPRO_EINVAL;
}

template <class AT>
AT* S_of(void* states) { return static_cast<AT*>(states); }

template <class AT>
long long* C_of(void* states, int G, int L) {
    return reinterpret_cast<long long*>(static_cast<unsigned char*>(states) + align_up((size_t)G * L * sizeof(AT), 8));
}

template <class AT, int L>
int run_state_op(int op, void* a, const void* b, int G, hipStream_t st) {
    const dim3 blk(256), grd((G + 255) / 256);
    if (op == 0) {
        hipLaunchKernelGGL((k_state_init<AT, L>), grd, blk, 0, st, S_of<AT>(a), C_of<AT>(a, G, L), G);
    } else if (op == 1) {
        void* bb = const_cast<void*>(b);
        hipLaunchKernelGGL((k_merge_states<AT, L>), grd, blk, 0, st, S_of<AT>(a), C_of<AT>(a, G, L),
                           (const AT*)S_of<AT>(bb), (const long long*)C_of<AT>(bb, G, L), G);
    } else {
        void* aa = const_cast<void*>(b);  // states
        hipLaunchKernelGGL((k_finalize<AT, L>), grd, blk, 0, st, (const AT*)S_of<AT>(aa),
                           (const long long*)C_of<AT>(aa, G, L), G, static_cast<AT*>(a));
    }
    LAUNCH_CHECK();
    return REPRO_OK;
}

template <class AT>
int state_op_L(int op, int L, void* a, const void* b, int G, hipStream_t st) {
    switch (L) {
        case 1: return run_state_op<AT, 1>(op, a, b, G, st);
        case 2: return run_state_op<AT, 2>(op, a, b, G, st);
        case 3: return run_state_op<AT, 3>(op, a, b, G, st);
        case 4: return run_state_op<AT, 4>(op, a, b, G, st);
    }
    return REPRO_EINVAL;
}

int state_op(int op, repro_scalar_t T, int L, void* a, const void* b, int64_t G, hipStream_t st) {
    if (!valid_common(G, T, L) || !a || !b) return REPRO_EINVAL;
    return T == REPRO_F64 ? state_op_L<double>(op, L, a, b, (int)G, st) : state_op_L<float>(op, L, a, b, (int)G, st);
}

// Plan of the partitioned baseline, or false (then global atomics).
bool make_plan_plain(int64_t n, int64_t G, size_t vsize, Plan* p) {
    memset(p, 0, sizeof(*p));
    if ((size_t)G * 8 <= LDS_BIN_BUDGET) return false;
    return make_plan_part(n, G, 0, vsize, p);
}

template <class KT, class VT>
int run_plain_part(const void* keys, const void* values, int64_t n, int64_t G, double* out, void* workspace,
                   uint32_t* status, const Plan& p, hipStream_t st) {
    unsigned char* ws = static_cast<unsigned char*>(workspace);
    const KT* k = static_cast<const KT*>(keys);
    const VT* v = static_cast<const VT*>(values);
    int* rel = reinterpret_cast<int*>(ws + p.o_rel);
    long long* roff = reinterpret_cast<long long*>(ws + p.o_roff);
    long long* size = reinterpret_cast<long long*>(ws + p.o_size);
    long long* base = reinterpret_cast<long long*>(ws + p.o_base);
    int* wfirst = reinterpret_cast<int*>(ws + p.o_wfirst);
    WorkItem* items = reinterpret_cast<WorkItem*>(ws + p.o_items);
    int* nitems = reinterpret_cast<int*>(ws + p.o_nitems);
    uint16_t* lkey = reinterpret_cast<uint16_t*>(ws + p.o_lkey);
    VT* lval = reinterpret_cast<VT*>(ws + p.o_lval);
    const void* scatter = p.sc_ru == 8 ? (const void*)k_part_scatter<KT, VT, double, 8, false>
                                       : (const void*)k_part_scatter<KT, VT, double, 4, false>;
    if (!allow_lds(scatter, p.lds_sc) ||
        !allow_lds((const void*)k_agg_part_plain<VT>, p.lds_agg2))
        return REPRO_EHIP;
    {
        const int rc = partition_offsets<KT>(k, n, G, p, ws, st);
        if (rc != REPRO_OK) return rc;
    }
    hipLaunchKernelGGL(k_part_plan<VT>, dim3(1), dim3(PART_BLOCK), 0, st, size, p.F, PART_CHUNK, base, wfirst, items,
                       nitems, lkey, lval);
    LAUNCH_CHECK();
    if (p.sc_ru == 8)
        hipLaunchKernelGGL((k_part_scatter<KT, VT, double, 8, false>), dim3(p.nw), dim3(PART_BLOCK), p.lds_sc, st, k, v,
                           n, G, p.gp_shift, p.F, p.slab, base, roff, rel, lkey, lval, status);
    else
        hipLaunchKernelGGL((k_part_scatter<KT, VT, double, 4, false>), dim3(p.nw), dim3(PART_BLOCK), p.lds_sc, st, k, v,
                           n, G, p.gp_shift, p.F, p.slab, base, roff, rel, lkey, lval, status);
    LAUNCH_CHECK();
    hipLaunchKernelGGL((k_agg_part_plain<VT>), dim3(p.maxw), dim3(PLAIN_PART_BLOCK), p.lds_agg2, st, lkey, lval, items,
                       nitems, G, p.gp_shift, out);
    LAUNCH_CHECK();
    return REPRO_OK;
}

template <class KT, class VT>
int run_plain(const void* keys, const void* values, int64_t n, int G, double* out, void* workspace,
              size_t workspace_bytes, uint32_t* status, hipStream_t st) {
    Plan pp;
    if (make_plan_plain(n, G, sizeof(VT), &pp) && workspace && workspace_bytes >= pp.ws)
        return run_plain_part<KT, VT>(keys, values, n, G, out, workspace, status, pp, st);
    const KT* k = static_cast<const KT*>(keys);
    const VT* v = static_cast<const VT*>(values);
    int64_t nwg = (n + 16 * PLAIN_TILE - 1) / (16 * PLAIN_TILE);
    if (nwg > PLAIN_MAX_WG) nwg = PLAIN_MAX_WG;
    if (nwg < 1) nwg = 1;
    int64_t chunk = (n + nwg - 1) / nwg;
    chunk = (chunk + PLAIN_TILE - 1) / PLAIN_TILE * PLAIN_TILE;
    nwg = (n + chunk - 1) / chunk;
    constexpr int VEC = 16 / sizeof(VT);
    const bool aligned = ((uintptr_t)k % (VEC * sizeof(KT)) == 0) && ((uintptr_t)v % 16 == 0);
    if ((size_t)G * 8 <= LDS_BIN_BUDGET) {
        const size_t lds = (size_t)G * 8;
        if (aligned)
            hipLaunchKernelGGL((k_plain_lds<KT, VT, VEC>), dim3(nwg), dim3(PLAIN_BLOCK), lds, st, k, v, n, G, chunk, out,
                               status);
        else
            hipLaunchKernelGGL((k_plain_lds<KT, VT, 1>), dim3(nwg), dim3(PLAIN_BLOCK), lds, st, k, v, n, G, chunk, out,
                               status);
    } else {
        if (aligned)
            hipLaunchKernelGGL((k_plain_global<KT, VT, VEC>), dim3(nwg), dim3(PLAIN_BLOCK), 0, st, k, v, n, G, chunk,
                               out, status);
        else
            hipLaunchKernelGGL((k_plain_global<KT, VT, 1>), dim3(nwg), dim3(PLAIN_BLOCK), 0, st, k, v, n, G, chunk, out,
                               status);
    }
    LAUNCH_CHECK();
    return REPRO_OK;
}

}  // namespace

// ------------------------------------------- allocation-free entry point
//
// repro_groupby_sum_noalloc runs the planned kernels of repro_groupby_sum on
// this static device array instead of a caller workspace.  In host code the
// name `scratch` is only a host-side stand-in: the array's device address is
// looked up once per device with hipGetSymbolAddress and that pointer is
// what the kernels get.
static __device__ __align__(256) unsigned char scratch[REPRO_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};

// Device address of the current device's copy of `scratch`.
int scratch_of_current_device(void** out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= NOALLOC_MAX_DEVICES) return REPRO_EHIP;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return REPRO_EHIP;
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return REPRO_OK;
}
}  // namespace

// ============================================================== C ABI

extern "C" {

size_t repro_state_bytes(int64_t num_groups, repro_scalar_t T, int L) {
    if (!valid_common(num_groups, T, L)) return 0;
    return align_up((size_t)num_groups * L * scalar_size(T), 8) + (size_t)num_groups * L * 8;
}

size_t repro_workspace_bytes(int64_t n, int64_t num_groups, repro_key_t kt, repro_scalar_t vt, repro_scalar_t T,
                             int L) {
    (void)kt;
    if (vt != REPRO_F32 && vt != REPRO_F64) return 0;
    Plan p;
    if (!valid_common(num_groups, T, L) || n < 0) return 0;
    if (!make_plan(n, num_groups, L, T == REPRO_F64 ? Fmt<double>::JMAX : Fmt<float>::JMAX, scalar_size(vt), &p))
        return 0;
    return p.ws;
}

int repro_state_init(void* states, int64_t num_groups, repro_scalar_t T, int L, hipStream_t stream) {
    return state_op(0, T, L, states, states, num_groups, stream);
}

int repro_groupby_sum(const void* keys, repro_key_t kt, const void* values, repro_scalar_t vt, int64_t n,
                      int64_t num_groups, repro_scalar_t T, int L, void* states, void* workspace,
                      size_t workspace_bytes, uint32_t* status, hipStream_t stream) {
    if (!valid_common(num_groups, T, L) || n < 0 || !states) return REPRO_EINVAL;
    if (kt != REPRO_I32 && kt != REPRO_I64) return REPRO_EINVAL;
    if (vt != REPRO_F32 && vt != REPRO_F64) return REPRO_EINVAL;
    if (vt == REPRO_F64 && T == REPRO_F32) return REPRO_EINVAL;  // narrowing is not exact
    if (n == 0) return REPRO_OK;
    if (!keys || !values) return REPRO_EINVAL;
    Plan p;
    if (!make_plan(n, num_groups, L, T == REPRO_F64 ? Fmt<double>::JMAX : Fmt<float>::JMAX, scalar_size(vt), &p))
        return REPRO_EINVAL;
    if (p.ws > 0 && (!workspace || workspace_bytes < p.ws || (uintptr_t)workspace % 256 != 0)) return REPRO_EINVAL;
    const int64_t G = num_groups;
    if (kt == REPRO_I32)
        return dispatch_types<int32_t>(vt, T, L, keys, values, n, G, states, workspace, status, p, stream);
    return dispatch_types<int64_t>(vt, T, L, keys, values, n, G, states, workspace, status, p, stream);
}

int repro_merge(void* dst, const void* src, int64_t num_groups, repro_scalar_t T, int L, hipStream_t stream) {
    if (dst == src) return REPRO_EINVAL;
    return state_op(1, T, L, dst, src, num_groups, stream);
}

int repro_finalize(const void* states, int64_t num_groups, repro_scalar_t T, int L, void* out, hipStream_t stream) {
    if (!out) return REPRO_EINVAL;
    return state_op(2, T, L, out, states, num_groups, stream);
}

size_t repro_plain_workspace_bytes(int64_t n, int64_t num_groups, repro_key_t kt, repro_scalar_t vt) {
    (void)kt;
    if (num_groups < 1 || num_groups > INT32_MAX || n < 0 || (vt != REPRO_F32 && vt != REPRO_F64)) return 0;
    Plan p;
    return make_plan_plain(n, num_groups, scalar_size(vt), &p) ? p.ws : 0;
}

int repro_plain_groupby_sum(const void* keys, repro_key_t kt, const void* values, repro_scalar_t vt, int64_t n,
                            int64_t num_groups, double* out, void* workspace, size_t workspace_bytes,
                            uint32_t* status, hipStream_t stream) {
    if (num_groups < 1 || num_groups > INT32_MAX || n < 0 || !out) return REPRO_EINVAL;
    if ((kt != REPRO_I32 && kt != REPRO_I64) || (vt != REPRO_F32 && vt != REPRO_F64)) return REPRO_EINVAL;
    if (workspace && (uintptr_t)workspace % 256 != 0) return REPRO_EINVAL;
    if (n == 0) return REPRO_OK;
    if (!keys || !values) return REPRO_EINVAL;
    const int G = (int)num_groups;
    void* ws = workspace;
    const size_t wb = workspace_bytes;
    if (kt == REPRO_I32)
        return vt == REPRO_F64 ? run_plain<int32_t, double>(keys, values, n, G, out, ws, wb, status, stream)
                               : run_plain<int32_t, float>(keys, values, n, G, out, ws, wb, status, stream);
    return vt == REPRO_F64 ? run_plain<int64_t, double>(keys, values, n, G, out, ws, wb, status, stream)
                           : run_plain<int64_t, float>(keys, values, n, G, out, ws, wb, status, stream);
}

int repro_profile_arm(int max_launches) {
    if (max_launches < 1 || max_launches > PROFILE_MAX) return REPRO_EINVAL;
    if (!g_prof) g_prof = new ProfileSlot();
    while (g_prof->created < 2 * max_launches) {
        if (hipEventCreate(&g_prof->ev[g_prof->created]) != hipSuccess) return REPRO_EHIP;
        ++g_prof->created;
    }
    g_prof->armed = max_launches;
    g_prof->used = 0;
    return REPRO_OK;
}

int repro_profile_read(float* ms, int cap, int* count) {
    if (!ms || !count || cap < 0 || !g_prof) return REPRO_EINVAL;
    int k = g_prof->used < cap ? g_prof->used : cap;
    for (int i = 0; i < k; ++i) {
        if (hipEventSynchronize(g_prof->ev[2 * i + 1]) != hipSuccess) return REPRO_EHIP;
        if (hipEventElapsedTime(&ms[i], g_prof->ev[2 * i], g_prof->ev[2 * i + 1]) != hipSuccess) return REPRO_EHIP;
    }
    *count = k;
    g_prof->armed = g_prof->used = 0;
    return REPRO_OK;
}

int repro_read_probe(const void* data, size_t bytes, int workgroups, int threads, unsigned long long* sink,
                     hipStream_t stream) {
    if (!data || !sink || (uintptr_t)data % 16 != 0 || bytes % 16 != 0 || workgroups < 1 || threads < 64 ||
        threads > 1024 || threads % 64 != 0)
        return REPRO_EINVAL;
    hipLaunchKernelGGL(k_read_probe, dim3(workgroups), dim3(threads), 0, stream, static_cast<const u32x4*>(data),
                       bytes / 16, sink);
    LAUNCH_CHECK();
    return REPRO_OK;
}

int repro_atomic_probe(const int32_t* idx, int64_t n, unsigned long long* table, int64_t table_words,
                       int workgroups, hipStream_t stream) {
    if (n < 0 || table_words < 1 || workgroups < 1 || (n > 0 && (!idx || !table))) return REPRO_EINVAL;
    if (n == 0) return REPRO_OK;
    hipLaunchKernelGGL(k_atomic_probe, dim3(workgroups), dim3(256), 0, stream, idx, n, table, table_words);
    LAUNCH_CHECK();
    return REPRO_OK;
}

const char* repro_version(void) { return "librepro 0.1 (gfx950)"; }

int repro_groupby_sum_noalloc(const void* keys, repro_key_t kt, const void* values, repro_scalar_t vt, int64_t n,
                              int64_t num_groups, repro_scalar_t T, int L, void* states, uint32_t* status,
                              hipStream_t stream) {
    if (!valid_common(num_groups, T, L) || n < 0 || !states) return REPRO_EINVAL;
    if (kt != REPRO_I32 && kt != REPRO_I64) return REPRO_EINVAL;
    if (vt != REPRO_F32 && vt != REPRO_F64) return REPRO_EINVAL;
    if (vt == REPRO_F64 && T == REPRO_F32) return REPRO_EINVAL;
    if (n == 0) return REPRO_OK;
    Plan p;
    if (!make_plan(n, num_groups, L, T == REPRO_F64 ? Fmt<double>::JMAX : Fmt<float>::JMAX, scalar_size(vt), &p))
        return REPRO_EINVAL;
    if (p.ws > REPRO_NOALLOC_SCRATCH_BYTES) return REPRO_EINVAL;
    void* ws = nullptr;
    const int rc = scratch_of_current_device(&ws);
    if (rc != REPRO_OK) return rc;
    return repro_groupby_sum(keys, kt, values, vt, n, num_groups, T, L, states, ws, REPRO_NOALLOC_SCRATCH_BYTES,
                             status, stream);
}

}  // extern "C"
