// repro_batch.hip -- many independent GroupBy-SUM jobs in one persistent
// launch (librepro, gfx950).
//
// Paper: Mueller, Arteaga, Hoefler, Alonso, "Reproducible Floating-Point
// Aggregation in RDBMSs" (arXiv 1802.09883).  Every job is the GroupBy-SUM
// of Sec. II-A into repro<T,L> (Sec. IV); its pieces are combined with
// operator+=(repro) (the merge phase of Alg. 4), whose exact integer
// arithmetic makes the bits independent of how the batch is cut and
// scheduled.
//
// Work items are (job, row chunk, group slice).  A persistent grid of
// 512-thread workgroups takes items from a queue (one atomic counter) in
// the order of a host-made table, largest items first.  An item aggregates
// its chunk's rows of its slice's groups in LDS with the shared per-tile
// loop (aggregate_range in slice mode), then either folds them straight
// into the job's states (the job's only chunk) or writes a partial; the
// last item of a (job, slice) to finish -- a device-scope counter -- folds
// all partials of that slice into the states and, when asked, finalises.
// A job whose groups exceed one workgroup's LDS is, by default, not read
// once per slice: one item per chunk sorts the chunk's rows by slice into
// a copy in the workspace (a counting sort: slice counts, then positions),
// then aggregates each slice from its own rows -- the chunk-local form of
// the partitioning step of Alg. 4.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "repro.h"
#include "repro_agg.hpp"
#include "repro_device.hpp"
#include "repro_batch_internal.hpp"

using namespace repro;

namespace {

constexpr int64_t BATCH_DEFAULT_CHUNK = 128 * 1024;
constexpr int BATCH_MAX_CHUNKS = 1024;   // per job; chunks grow to stay below
constexpr int BATCH_BLOCK = 512;         // 8 waves: room for 256 VGPRs per lane, no spills
constexpr int BATCH_MAX_WG = 512;        // persistent workgroups: as many as fit (one or two per CU)

// Device record of a job (built by the planner).
struct BatchJob {
    const void* keys;
    const void* vals;
    void* states;
    void* out;
    long long n;
    long long chunk;      // rows per chunk (multiple of the tile)
    long long part_off;   // byte offset of this job's partials in the partial area
    long long spill_off;  // byte offset of its spill array in the spill area (epoch mode), or -1
    long long scr_off;    // sorted jobs: first row of its sorted copies in the scratch area, else -1
    int G, L, accumulate, vec;
    int nslices, gs, R;   // slices, groups per slice (the last may be smaller), LDS replicas
    int nchunks;
    int done_off;         // first completion counter of this job (one per slice)
    int gshift;           // sorted jobs: gs = 2^gshift
    int scr_stride;       // sorted jobs: scratch rows per chunk (its rows and the slices' alignment)
    int pad;
};

// slice -1: a sorted item (every slice of the chunk)
struct BatchItem {
    int job, chunk, slice, pad;
};

constexpr int SORT_MAX_SLICES = 64;  // slices of a sorted job (LDS counters)
constexpr int SORT_ALIGN = 8;        // each slice's rows start on a multiple of 8 (vector loads)

// Workspace: [head][jobs][items][counters | spill arrays][partials]; the
// counters and spill words (zeroed by k_batch_reset) are one contiguous
// range.  Offsets are in the head.
struct BatchHead {
    int next;  // queue position (reset by k_batch_reset)
    int nitems;
    int njobs;
    int ncounters;
    long long off_jobs, off_items, off_counters, off_spill, off_partials;
    long long zero_words;  // 8-byte words from off_counters that k_batch_reset clears
    int merge;             // 0: the last item of a (job, slice) merges; 1: a merge launch after the batch
    int nunits;            // merge launch: work units (256 groups of one split job each)
    long long off_units;
    long long off_scr_keys, off_scr_vals;  // sorted copies: local keys (uint16), values
};

// A work unit of the merge launch: groups g0 .. g0+255 of a split job.
struct MergeUnit {
    int job, g0;
};
constexpr int MERGE_UNIT = 256;

struct BatchLayout {
    size_t jobs, items, units, counters, spill, partials, scr_keys, scr_vals, total;
};

inline BatchLayout batch_layout(int njobs, int64_t nitems, int64_t nunits, int64_t ncounters, size_t spill_bytes,
                                size_t partial_bytes, int64_t scr_rows, size_t vsz) {
    BatchLayout b;
    b.jobs = 256;
    b.items = b.jobs + align_up((size_t)njobs * sizeof(BatchJob), 256);
    b.units = b.items + align_up((size_t)nitems * sizeof(BatchItem), 256);
    b.counters = b.units + align_up((size_t)nunits * sizeof(MergeUnit), 256);
    b.spill = b.counters + align_up((size_t)ncounters * 4, 256);
    b.partials = b.spill + align_up(spill_bytes, 256);
    b.scr_keys = b.partials + align_up(partial_bytes, 256);
    b.scr_vals = b.scr_keys + align_up((size_t)scr_rows * 2, 256);
    b.total = b.scr_vals + align_up((size_t)scr_rows * vsz, 256);
    return b;
}

// bytes of one (slice, chunk) partial: top[gs] int32, then K[L][gs] int64
__host__ __device__ inline size_t partial_bytes(int gs, int L) { return align_up((size_t)gs * 4, 8) + (size_t)gs * L * 8; }

template <class AT>
__device__ __forceinline__ AT* S_ptr(void* st) {
    return static_cast<AT*>(st);
}
template <class AT>
__device__ __forceinline__ long long* C_ptr(void* st, int G, int L) {
    return reinterpret_cast<long long*>(static_cast<unsigned char*>(st) + align_up((size_t)G * L * sizeof(AT), 8));
}

template <class AT>
__device__ __forceinline__ int state_top_of(const AT* S, int g, bool use, int L) {
    return use ? state_top(S[g]) : L - 1;
}

// After the aggregation of one (chunk, slice) in LDS (bins and tops of Gs
// groups, R replicas): fold them straight into the states (the job's only
// chunk) or publish a partial; the last chunk of the slice to finish folds
// the slice (merge schedule 0).
template <class AT, int L, bool EPOCH>
__device__ void finish_slice(const BatchJob& jb, int chunk, int slice, int Gs, int64_t glo, int R,
                             unsigned char* partials, int* counters, unsigned long long* spill, unsigned char* smem,
                             int* s_last, int merge) {
    constexpr int NJ = Fmt<AT>::JMAX + 1;
    const int tid = threadIdx.x;
    long long* bins = reinterpret_cast<long long*>(smem);
    const int2* TOP = reinterpret_cast<const int2*>(bins + (size_t)(Gs + 1) * R * L);
    fold_replicas<L, BATCH_BLOCK>(bins, Gs, R);
    AT* S = S_ptr<AT>(jb.states);
    long long* C = C_ptr<AT>(jb.states, jb.G, L);
    AT* out = static_cast<AT*>(jb.out);
    auto level_sums = [&](int g, long long* x) {
#pragma unroll
        for (int l = 0; l < L; ++l) x[l] = bins[((size_t)l * (Gs + 1) + g) * R];
    };
    if (jb.nchunks == 1) {
        if (EPOCH) {  // this workgroup's spill atomics, read back below
            published();
            __syncthreads();
        }
        for (int g = tid; g < Gs; g += BATCH_BLOCK) {
            const int gg = (int)glo + g;
            long long x[L], hi[L], lo[L];
            level_sums(g, x);
            const int J = max(TOP[g].x, state_top_of(S, gg, jb.accumulate, L));
            start_from_state<AT, L>(S, C, jb.G, gg, jb.accumulate, J, hi, lo);
            add_levels<AT, L>(x, TOP[g].x, J, hi, lo);
            if (EPOCH) add_spill<AT, L>(spill + (size_t)g * NJ * 2, J, hi, lo);
            write_group<AT, L>(hi, lo, J, S, C, jb.G, gg, out);
        }
        __syncthreads();  // LDS is reused by the next item
        return;
    }
    // publish this chunk's partial of the slice
    const size_t pbytes = partial_bytes(jb.gs, L);
    unsigned char* part0 = partials + jb.part_off + (size_t)slice * jb.nchunks * pbytes;
    {
        unsigned char* pp = part0 + (size_t)chunk * pbytes;
        int* ptop = reinterpret_cast<int*>(pp);
        long long* pK = reinterpret_cast<long long*>(pp + align_up((size_t)jb.gs * 4, 8));
        for (int g = tid; g < Gs; g += BATCH_BLOCK) {
            long long x[L];
            level_sums(g, x);
            publish(&ptop[g], TOP[g].x);
#pragma unroll
            for (int l = 0; l < L; ++l) publish(&pK[(size_t)l * jb.gs + g], x[l]);
        }
    }
    if (merge) {  // the merge launch after the batch folds the partials
        __syncthreads();  // LDS is reused by the next item
        return;
    }
    published();  // this thread's partial words (and spill atomics) complete before the count
    __syncthreads();
    if (tid == 0) *s_last = (atomicAdd(&counters[jb.done_off + slice], 1) == jb.nchunks - 1);
    __syncthreads();
    if (*s_last) {
        for (int g = tid; g < Gs; g += BATCH_BLOCK) {
            const int gg = (int)glo + g;
            long long hi[L], lo[L];
            int J = state_top_of(S, gg, jb.accumulate, L);
            // unrolled: the loads of several chunks' partials in flight at once
#pragma unroll 4
            for (int c = 0; c < jb.nchunks; ++c)
                J = max(J, collect(reinterpret_cast<const int*>(part0 + (size_t)c * pbytes) + g));
            start_from_state<AT, L>(S, C, jb.G, gg, jb.accumulate, J, hi, lo);
#pragma unroll 4
            for (int c = 0; c < jb.nchunks; ++c) {
                const unsigned char* pp = part0 + (size_t)c * pbytes;
                const long long* pK = reinterpret_cast<const long long*>(pp + align_up((size_t)jb.gs * 4, 8));
                long long x[L];
#pragma unroll
                for (int l = 0; l < L; ++l) x[l] = collect(&pK[(size_t)l * jb.gs + g]);
                add_levels<AT, L>(x, collect(reinterpret_cast<const int*>(pp) + g), J, hi, lo);
            }
            if (EPOCH) add_spill<AT, L>(spill + (size_t)g * NJ * 2, J, hi, lo);
            write_group<AT, L>(hi, lo, J, S, C, jb.G, gg, out);
        }
    }
    __syncthreads();
}

// One (chunk, slice) item: aggregate, then fold or publish.  Returns the
// lane's status bits.  SLICE: the job is cut into group slices (the rows of
// other slices are skipped); a job in one slice takes the unsliced loop.
template <class KT, class VT, class AT, int L, int VEC, bool EPOCH, bool SLICE>
__device__ __attribute__((noinline)) uint32_t run_item(const BatchJob& jb, const BatchItem& bi, unsigned char* partials, int* counters,
                             unsigned long long* spill_area, unsigned char* smem, AggShared& sh, int* s_last,
                             int merge) {
    const int64_t r0 = (int64_t)bi.chunk * jb.chunk;
    const int64_t r1 = min((int64_t)jb.n, r0 + jb.chunk);
    const int64_t glo = (int64_t)bi.slice * jb.gs;
    const int Gs = (int)min((int64_t)jb.gs, (int64_t)jb.G - glo);
    // epoch mode (unsliced jobs): rows above a frozen top go to the job's spill array
    unsigned long long* spill = EPOCH ? spill_area + jb.spill_off / 8 : nullptr;
    // temporal loads: the items of one chunk's group slices read the same rows
    const uint32_t err = aggregate_range<KT, VT, AT, L, VEC, EPOCH, SLICE, BATCH_BLOCK, false>(
        static_cast<const KT*>(jb.keys), static_cast<const VT*>(jb.vals), r0, r1, Gs, jb.R, smem, sh, spill, glo,
        jb.G);
    finish_slice<AT, L, EPOCH>(jb, bi.chunk, bi.slice, Gs, glo, jb.R, partials, counters, spill, smem, s_last, merge);
    return err;
}

// A sorted item: every slice of one chunk.  A counting pass takes the rows
// per slice, a second pass writes each row's local key (key - slice start)
// and value to its slice's range of the chunk's scratch rows (a row with an
// unusable value keeps its slot with value +0.0, which contributes nothing;
// rows with invalid keys are dropped; both set their status bits, as every
// path does), then each slice is aggregated from its own rows.  Rows land
// in a slice's range in no fixed order: the level sums are exact.  The
// scratch rows of a chunk belong to this item alone, and the barrier after
// the second pass makes its stores visible to the whole workgroup (one CU).
//
// Atomics of many lanes on one LDS address serialise, so the counting pass
// spreads its counters over SORT_REP replicas (replica = thread index mod
// SORT_REP, stride SORT_REP_STRIDE words).  The second pass takes positions
// from one cursor per slice, so the rows of a wave's store instruction fall
// into few runs (spreading the cursors as well scattered the stores, and a
// wave-level ranking by ballots was slower than the serialised atomics).
// The counters live in the bin area of LDS, which the passes do not use.
constexpr int SORT_REP = 16;
constexpr int SORT_REP_STRIDE = SORT_MAX_SLICES + 1;  // odd: replicas of a slice in different banks

template <class KT, class VT, class AT, int L>
__device__ __attribute__((noinline)) uint32_t run_sorted(const BatchJob& jb, const BatchItem& bi,
                                                         unsigned char* partials, int* counters, uint16_t* scr_keys,
                                                         VT* scr_vals, unsigned char* smem, AggShared& sh,
                                                         int* s_last, int merge, int* s_cnt, int* s_off) {
    typedef Fmt<AT> Fm;
    // rows in flight per thread (no barrier inside either pass: the waves
    // overlap their loads); a workgroup keeps 64-96 KiB of loads in flight
    constexpr int UC = 32, U = 16;
    constexpr int NREP = SORT_REP * SORT_REP_STRIDE;
    const int tid = threadIdx.x;
    const int64_t r0 = (int64_t)bi.chunk * jb.chunk;
    const int64_t r1 = min((int64_t)jb.n, r0 + jb.chunk);
    const KT* keys = static_cast<const KT*>(jb.keys);
    const VT* vals = static_cast<const VT*>(jb.vals);
    const uint64_t G = (uint64_t)jb.G;
    const int sh_g = jb.gshift;
    const int ns = jb.nslices;
    const uint32_t gmask = (uint32_t)jb.gs - 1;
    uint16_t* lk = scr_keys + jb.scr_off + (int64_t)bi.chunk * jb.scr_stride;
    VT* lv = scr_vals + jb.scr_off + (int64_t)bi.chunk * jb.scr_stride;
    int* rcnt = reinterpret_cast<int*>(smem);  // [SORT_REP][SORT_REP_STRIDE]
    int* cur = rcnt + NREP;                    // [SORT_MAX_SLICES]: next row of each slice
    int* my_cnt = rcnt + (tid % SORT_REP) * SORT_REP_STRIDE;
    for (int k = tid; k < NREP; k += BATCH_BLOCK) rcnt[k] = 0;
    __syncthreads();
    // rows per (replica, slice) (temporal loads: the keys are read again below)
    for (int64_t b = r0; b < r1; b += (int64_t)UC * BATCH_BLOCK) {
        KT kk[UC];
#pragma unroll
        for (int u = 0; u < UC; ++u) {
            const int64_t i = b + u * BATCH_BLOCK + tid;
            kk[u] = i < r1 ? keys[i] : (KT)-1;
        }
#pragma unroll
        for (int u = 0; u < UC; ++u)
            if ((uint64_t)(int64_t)kk[u] < G) atomicAdd(&my_cnt[(int)((uint64_t)(int64_t)kk[u] >> sh_g)], 1);
    }
    __syncthreads();
    for (int s = tid; s < ns; s += BATCH_BLOCK) {
        int c = 0;
        for (int r = 0; r < SORT_REP; ++r) c += rcnt[r * SORT_REP_STRIDE + s];
        s_cnt[s] = c;
    }
    __syncthreads();
    if (tid == 0) {  // at most SORT_MAX_SLICES: a serial scan; slices start on multiples of SORT_ALIGN
        int o = 0;
        for (int s = 0; s < ns; ++s) {
            s_off[s] = o;
            o += (s_cnt[s] + SORT_ALIGN - 1) / SORT_ALIGN * SORT_ALIGN;
        }
    }
    __syncthreads();
    for (int k = tid; k < ns; k += BATCH_BLOCK) cur[k] = s_off[k];
    __syncthreads();
    uint32_t err = 0;
    for (int64_t b = r0; b < r1; b += (int64_t)U * BATCH_BLOCK) {
        KT kk[U];
        VT vv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t i = b + u * BATCH_BLOCK + tid;
            kk[u] = i < r1 ? keys[i] : (KT)0;
            vv[u] = i < r1 ? __builtin_nontemporal_load(&vals[i]) : (VT)0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t i = b + u * BATCH_BLOCK + tid;
            int sl = -1;  // slice of the row, -1: no row or an invalid key
            VT v = vv[u];
            const uint64_t key = (uint64_t)(int64_t)kk[u];
            if (i < r1) {
                if (!finite_val(v)) {
                    err |= ERR_NONFINITE;
                    v = (VT)0;
                } else if (v != (VT)0 && jreq_raw<AT>(frexp_raw(v)) > Fm::JMAX) {
                    err |= ERR_RANGE;
                    v = (VT)0;
                }
                if (key < G)
                    sl = (int)(key >> sh_g);
                else
                    err |= ERR_KEY;
            }
            const int pos = sl >= 0 ? atomicAdd(&cur[sl], 1) : 0;
            if (sl >= 0) {
                lk[pos] = (uint16_t)((uint32_t)key & gmask);
                lv[pos] = v;
            }
        }
    }
    __syncthreads();  // the sorted rows are complete; the bin area is free again
    constexpr int VEC = 16 / sizeof(VT);
    for (int s = 0; s < ns; ++s) {
        const int64_t glo = (int64_t)s << sh_g;
        const int Gs = (int)min((int64_t)jb.gs, (int64_t)jb.G - glo);
        const int64_t c0 = s_off[s];
        // per-tile mode, no spill array; the values are finite and in the domain, or +0.0
        aggregate_range<uint16_t, VT, AT, L, VEC, false, false, BATCH_BLOCK, false>(lk, lv, c0, c0 + s_cnt[s], Gs, 1,
                                                                                     smem, sh, nullptr, 0, 0);
        finish_slice<AT, L, false>(jb, bi.chunk, s, Gs, glo, 1, partials, counters, nullptr, smem, s_last, merge);
    }
    return err;
}

template <class KT, class VT, class AT, int L>
__device__ __forceinline__ uint32_t run_item_vec(const BatchJob& jb, const BatchItem& bi, unsigned char* partials,
                                                 int* counters, unsigned long long* spill, unsigned char* smem,
                                                 AggShared& sh, int* s_last, int merge) {
    constexpr int VEC = 16 / sizeof(VT);
    // epoch mode (a spill array) only for jobs in one slice
    if (jb.spill_off >= 0) {
        if (jb.vec)
            return run_item<KT, VT, AT, L, VEC, true, false>(jb, bi, partials, counters, spill, smem, sh, s_last, merge);
        return run_item<KT, VT, AT, L, 1, true, false>(jb, bi, partials, counters, spill, smem, sh, s_last, merge);
    }
    if (jb.nslices == 1) {
        if (jb.vec)
            return run_item<KT, VT, AT, L, VEC, false, false>(jb, bi, partials, counters, spill, smem, sh, s_last, merge);
        return run_item<KT, VT, AT, L, 1, false, false>(jb, bi, partials, counters, spill, smem, sh, s_last, merge);
    }
    if (jb.vec)
        return run_item<KT, VT, AT, L, VEC, false, true>(jb, bi, partials, counters, spill, smem, sh, s_last, merge);
    return run_item<KT, VT, AT, L, 1, false, true>(jb, bi, partials, counters, spill, smem, sh, s_last, merge);
}

template <class KT, class VT, class AT>
__device__ __forceinline__ uint32_t run_sorted_any(const BatchJob& jb, const BatchItem& bi, unsigned char* partials,
                                                   int* counters, uint16_t* scr_keys, VT* scr_vals,
                                                   unsigned char* smem, AggShared& sh, int* s_last, int merge,
                                                   int* s_cnt, int* s_off) {
    switch (jb.L) {
        case 1: return run_sorted<KT, VT, AT, 1>(jb, bi, partials, counters, scr_keys, scr_vals, smem, sh, s_last, merge, s_cnt, s_off);
        case 2: return run_sorted<KT, VT, AT, 2>(jb, bi, partials, counters, scr_keys, scr_vals, smem, sh, s_last, merge, s_cnt, s_off);
        case 3: return run_sorted<KT, VT, AT, 3>(jb, bi, partials, counters, scr_keys, scr_vals, smem, sh, s_last, merge, s_cnt, s_off);
        default: return run_sorted<KT, VT, AT, 4>(jb, bi, partials, counters, scr_keys, scr_vals, smem, sh, s_last, merge, s_cnt, s_off);
    }
}

// The merge launch (merge schedule 1): one 256-thread block per unit, one
// thread per group of a split job: the group's chunk partials, the caller's
// state (or the empty one) and the spill words fold into canonical states
// and the finalised sum, exactly as the last item does under schedule 0.
template <class AT, int L>
__device__ __forceinline__ void merge_group(const BatchJob& jb, int g, const unsigned char* partials,
                                            const unsigned long long* spill_area) {
    constexpr int NJ = Fmt<AT>::JMAX + 1;
    const int slice = g / jb.gs, gl = g - slice * jb.gs;
    const size_t pbytes = partial_bytes(jb.gs, L);
    const unsigned char* part0 = partials + jb.part_off + (size_t)slice * jb.nchunks * pbytes;
    AT* S = S_ptr<AT>(jb.states);
    long long* C = C_ptr<AT>(jb.states, jb.G, L);
    long long hi[L], lo[L];
    int J = state_top_of(S, g, jb.accumulate, L);
#pragma unroll 4
    for (int c = 0; c < jb.nchunks; ++c) J = max(J, reinterpret_cast<const int*>(part0 + (size_t)c * pbytes)[gl]);
    start_from_state<AT, L>(S, C, jb.G, g, jb.accumulate, J, hi, lo);
#pragma unroll 4
    for (int c = 0; c < jb.nchunks; ++c) {
        const unsigned char* pp = part0 + (size_t)c * pbytes;
        const long long* pK = reinterpret_cast<const long long*>(pp + align_up((size_t)jb.gs * 4, 8));
        long long x[L];
#pragma unroll
        for (int l = 0; l < L; ++l) x[l] = pK[(size_t)l * jb.gs + gl];
        add_levels<AT, L>(x, reinterpret_cast<const int*>(pp)[gl], J, hi, lo);
    }
    if (jb.spill_off >= 0) add_spill<AT, L>(spill_area + jb.spill_off / 8 + (size_t)gl * NJ * 2, J, hi, lo);
    write_group<AT, L>(hi, lo, J, S, C, jb.G, g, static_cast<AT*>(jb.out));
}

template <class AT>
__global__ void __launch_bounds__(MERGE_UNIT) k_batch_merge(const unsigned char* __restrict__ ws) {
    const BatchHead* hd = reinterpret_cast<const BatchHead*>(ws);
    if ((int)blockIdx.x >= hd->nunits) return;
    const MergeUnit u = reinterpret_cast<const MergeUnit*>(ws + hd->off_units)[blockIdx.x];
    const BatchJob jb = reinterpret_cast<const BatchJob*>(ws + hd->off_jobs)[u.job];
    const int g = u.g0 + (int)threadIdx.x;
    if (g >= jb.G) return;
    const unsigned char* partials = ws + hd->off_partials;
    const unsigned long long* spill = reinterpret_cast<const unsigned long long*>(ws + hd->off_spill);
    switch (jb.L) {
        case 1: merge_group<AT, 1>(jb, g, partials, spill); break;
        case 2: merge_group<AT, 2>(jb, g, partials, spill); break;
        case 3: merge_group<AT, 3>(jb, g, partials, spill); break;
        default: merge_group<AT, 4>(jb, g, partials, spill); break;
    }
}

// Zeroes the queue position and the completion counters (a kernel, so that
// the launch can be captured into a graph without memset nodes).
__global__ void __launch_bounds__(256) k_batch_reset(unsigned char* __restrict__ ws) {
    BatchHead* hd = reinterpret_cast<BatchHead*>(ws);
    unsigned long long* z = reinterpret_cast<unsigned long long*>(ws + hd->off_counters);
    const long long nz = hd->zero_words;
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < nz; i += (long long)gridDim.x * 256) z[i] = 0;
    if (blockIdx.x == 0 && threadIdx.x == 0) hd->next = 0;
}

// The persistent kernel: every workgroup takes items until the queue is
// empty (each loop iteration advances the shared position by one, so every
// workgroup reaches the exit).
template <class KT, class VT, class AT>
__global__ void __launch_bounds__(BATCH_BLOCK) k_batch(unsigned char* __restrict__ ws, uint32_t* __restrict__ status) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ AggShared sh;
    __shared__ int s_item, s_last;
    __shared__ int s_cnt[SORT_MAX_SLICES], s_off[SORT_MAX_SLICES];
    BatchHead* hd = reinterpret_cast<BatchHead*>(ws);
    const BatchJob* jobs = reinterpret_cast<const BatchJob*>(ws + hd->off_jobs);
    const BatchItem* items = reinterpret_cast<const BatchItem*>(ws + hd->off_items);
    int* counters = reinterpret_cast<int*>(ws + hd->off_counters);
    unsigned long long* spill = reinterpret_cast<unsigned long long*>(ws + hd->off_spill);
    unsigned char* partials = ws + hd->off_partials;
    uint16_t* scr_keys = reinterpret_cast<uint16_t*>(ws + hd->off_scr_keys);
    VT* scr_vals = reinterpret_cast<VT*>(ws + hd->off_scr_vals);
    const int nitems = hd->nitems;
    const int merge = hd->merge;
    uint32_t err = 0;
    for (;;) {
        if (threadIdx.x == 0) s_item = atomicAdd(&hd->next, 1);
        __syncthreads();
        const int it = __builtin_amdgcn_readfirstlane(s_item);  // uniform: job records load as scalars
        __syncthreads();  // every thread has read s_item before it changes
        if (it >= nitems) break;
        const BatchItem bi = items[it];
        const BatchJob jb = jobs[bi.job];
        if (bi.slice < 0) {
            err |= run_sorted_any<KT, VT, AT>(jb, bi, partials, counters, scr_keys, scr_vals, smem, sh, &s_last, merge,
                                              s_cnt, s_off);
            continue;
        }
        switch (jb.L) {
            case 1: err |= run_item_vec<KT, VT, AT, 1>(jb, bi, partials, counters, spill, smem, sh, &s_last, merge); break;
            case 2: err |= run_item_vec<KT, VT, AT, 2>(jb, bi, partials, counters, spill, smem, sh, &s_last, merge); break;
            case 3: err |= run_item_vec<KT, VT, AT, 3>(jb, bi, partials, counters, spill, smem, sh, &s_last, merge); break;
            default: err |= run_item_vec<KT, VT, AT, 4>(jb, bi, partials, counters, spill, smem, sh, &s_last, merge); break;
        }
    }
    report(status, err);
}

// ---------------------------------------------------------------- host

inline size_t scalar_bytes(repro_scalar_t t) { return t == REPRO_F64 ? 8 : 4; }

struct HostPlan {
    std::vector<BatchJob> jobs;
    std::vector<BatchItem> items;
    std::vector<MergeUnit> units;  // merge schedule 1
    int merge = 0;
    int64_t ncounters = 0;
    size_t spill_bytes = 0;
    size_t partial_bytes = 0;
    int64_t scr_rows = 0;  // sorted copies of the chunks of sorted jobs
    size_t lds = 0;
    BatchLayout lay{};
};

bool valid_types(repro_key_t kt, repro_scalar_t vt, repro_scalar_t T) {
    if (kt != REPRO_I32 && kt != REPRO_I64) return false;
    if (vt != REPRO_F32 && vt != REPRO_F64) return false;
    if (T != REPRO_F32 && T != REPRO_F64) return false;
    return !(vt == REPRO_F64 && T == REPRO_F32);  // narrowing is not exact
}

// Largest slice (groups) whose LDS bins fit, under the configured cap.
int slice_cap(int L, int cap_cfg) {
    int g = (int)(LDS_BIN_BUDGET / (size_t)(8 * L + 12)) - 1;
    while (g > 1 && agg_lds_bytes(g, L, 1) > LDS_BIN_BUDGET) --g;
    if (cap_cfg > 0 && cap_cfg < g) g = cap_cfg;
    return g;
}

bool make_batch_plan(const repro_batch_job* jobs, int njobs, repro_key_t kt, repro_scalar_t vt, repro_scalar_t T,
                     const repro_batch_config* cfg, HostPlan* hp) {
    if (njobs < 0 || (njobs > 0 && !jobs) || !valid_types(kt, vt, T)) return false;
    int64_t chunk_cfg = (cfg && cfg->chunk_rows > 0) ? cfg->chunk_rows : BATCH_DEFAULT_CHUNK;
    chunk_cfg = (chunk_cfg + AGG_TILE - 1) / AGG_TILE * AGG_TILE;
    const int cap_cfg = cfg ? cfg->max_slice_groups : 0;
    const int order = cfg ? cfg->order : 0;
    if (order != 0 && order != 1) return false;
    const int merge = cfg ? cfg->merge : 0;
    if (merge != 0 && merge != 1) return false;
    const int split = cfg ? cfg->split : 0;
    if (split != 0 && split != 1) return false;
    hp->merge = merge;
    hp->units.clear();
    const size_t ksz = kt == REPRO_I64 ? 8 : 4, vsz = scalar_bytes(vt);
    hp->jobs.resize(njobs);
    hp->items.clear();
    hp->ncounters = 0;
    hp->spill_bytes = 0;
    hp->partial_bytes = 0;
    hp->scr_rows = 0;
    const int NJ = (T == REPRO_F64 ? 51 : 14) + 1;  // lattice indices of the accumulator format
    hp->lds = 0;
    std::vector<int64_t> cost;
    for (int j = 0; j < njobs; ++j) {
        const repro_batch_job& u = jobs[j];
        if (u.n < 0 || u.n > INT32_MAX || u.num_groups < 1 || u.num_groups > INT32_MAX || u.L < 1 || u.L > 4 ||
            !u.states || (u.n > 0 && (!u.keys || !u.values)) || (u.accumulate != 0 && u.accumulate != 1))
            return false;
        BatchJob& b = hp->jobs[j];
        memset(&b, 0, sizeof(b));
        b.keys = u.keys;
        b.vals = u.values;
        b.states = u.states;
        b.out = u.out;
        b.n = u.n;
        b.G = (int)u.num_groups;
        b.L = u.L;
        b.accumulate = u.accumulate;
        b.vec = ((uintptr_t)u.keys % (16 / vsz * ksz) == 0) && ((uintptr_t)u.values % 16 == 0);
        const int cap = slice_cap(u.L, cap_cfg);
        b.nslices = (int)((u.num_groups + cap - 1) / cap);
        b.gs = (int)((u.num_groups + b.nslices - 1) / b.nslices);
        b.scr_off = -1;
        bool sorted = false;
        if (split == 0 && b.nslices > 1) {
            // sorted: slices of 2^gshift groups (the largest power of two
            // that fits), at most SORT_MAX_SLICES of them
            int gshift = 0;
            while ((2 << gshift) <= cap) ++gshift;
            const int64_t ns = (u.num_groups + ((int64_t)1 << gshift) - 1) >> gshift;
            if (ns <= SORT_MAX_SLICES) {
                sorted = true;
                b.nslices = (int)ns;
                b.gs = 1 << gshift;
                b.gshift = gshift;
            }
        }
        b.R = b.nslices == 1 ? replicas_for(b.gs, u.L) : 1;
        hp->lds = std::max(hp->lds, agg_lds_bytes(b.gs, u.L, b.R));
        // chunks: the configured size, larger when the job would need too many;
        // at most 2^23 rows each (bin words stay below 2^62)
        int64_t chunk = chunk_cfg;
        const int64_t need = (u.n + BATCH_MAX_CHUNKS - 1) / BATCH_MAX_CHUNKS;
        if (chunk < need) chunk = (need + AGG_TILE - 1) / AGG_TILE * AGG_TILE;
        if (chunk > MAX_ROWS_PER_WG) chunk = MAX_ROWS_PER_WG;
        b.chunk = chunk;
        // a job without rows still gets one item per slice: it writes the
        // (empty, or unchanged) states and the finalised sums
        b.nchunks = u.n > 0 ? (int)((u.n + chunk - 1) / chunk) : 1;
        // epoch mode for jobs in one slice whose items span several tiles: a
        // spill array of NJ exact 128-bit words per group
        b.spill_off = -1;
        if (b.nslices == 1 && std::min<int64_t>(u.n, chunk) >= 4 * (int64_t)AGG_TILE) {
            b.spill_off = (long long)hp->spill_bytes;
            hp->spill_bytes += (size_t)b.gs * NJ * 16;
        }
        if (b.nchunks > 1) {
            if (merge)
                for (int g0 = 0; g0 < b.G; g0 += MERGE_UNIT) hp->units.push_back(MergeUnit{j, g0});
            b.done_off = (int)hp->ncounters;
            hp->ncounters += b.nslices;
            b.part_off = (long long)hp->partial_bytes;
            hp->partial_bytes += align_up((size_t)b.nslices * b.nchunks * partial_bytes(b.gs, u.L), 256);
        }
        if (sorted) {
            // one item per chunk; its scratch rows: the chunk's rows plus the
            // slices' alignment
            b.scr_stride = (int)(align_up((size_t)std::min<int64_t>(chunk, u.n), SORT_ALIGN) +
                                 (size_t)SORT_ALIGN * b.nslices);
            b.scr_off = hp->scr_rows;
            hp->scr_rows += (int64_t)b.nchunks * b.scr_stride;
            // the slice counters use the bin area during the passes
            hp->lds = std::max(hp->lds, (SORT_REP * SORT_REP_STRIDE + SORT_MAX_SLICES) * sizeof(int));
            for (int c = 0; c < b.nchunks; ++c) {
                hp->items.push_back(BatchItem{j, c, -1, 0});
                // two passes over the chunk, then its slices' rows once more
                // and a partial per slice: measured at about 5-6 times the
                // time per row of an unsliced item (the weight orders the queue)
                cost.push_back(6 * std::min<int64_t>(chunk, u.n - (int64_t)c * chunk));
            }
            continue;
        }
        for (int c = 0; c < b.nchunks; ++c)
            for (int s = 0; s < b.nslices; ++s) {
                hp->items.push_back(BatchItem{j, c, s, 0});
                cost.push_back(std::min<int64_t>(chunk, u.n - (int64_t)c * chunk));
            }
    }
    if (hp->items.size() > (size_t)INT32_MAX / 2 || hp->ncounters > INT32_MAX / 2 ||
        hp->units.size() > (size_t)INT32_MAX / 2)
        return false;
    if (order == 0) {
        // largest first; the slices of one chunk stay together (they read the same rows)
        std::vector<int> idx(hp->items.size());
        for (size_t i = 0; i < idx.size(); ++i) idx[i] = (int)i;
        std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return cost[a] > cost[b]; });
        std::vector<BatchItem> sorted(idx.size());
        for (size_t i = 0; i < idx.size(); ++i) sorted[i] = hp->items[idx[i]];
        hp->items.swap(sorted);
    }
    hp->lay = batch_layout(njobs, (int64_t)hp->items.size(), (int64_t)hp->units.size(), hp->ncounters,
                           hp->spill_bytes, hp->partial_bytes, hp->scr_rows, vsz);
    return true;
}

template <class KT, class VT, class AT>
const void* batch_kernel() {
    return reinterpret_cast<const void*>(k_batch<KT, VT, AT>);
}

const void* pick_kernel(int kt, int vt, int T) {
    if (kt == REPRO_I32) {
        if (vt == REPRO_F32) return T == REPRO_F32 ? batch_kernel<int32_t, float, float>() : batch_kernel<int32_t, float, double>();
        return batch_kernel<int32_t, double, double>();
    }
    if (vt == REPRO_F32) return T == REPRO_F32 ? batch_kernel<int64_t, float, float>() : batch_kernel<int64_t, float, double>();
    return batch_kernel<int64_t, double, double>();
}

int launch_plan(const repro_batch_plan* p, uint32_t* status, hipStream_t st) {
    unsigned char* ws = static_cast<unsigned char*>(p->workspace);
    hipLaunchKernelGGL(k_batch_reset, dim3(1024), dim3(256), 0, st, ws);
    if (hipGetLastError() != hipSuccess) return REPRO_EHIP;
    if (p->items == 0) return REPRO_OK;
    const void* fn = pick_kernel(p->kt, p->vt, p->T);  // its LDS limit was raised by the prepare call
    void* args[] = {&ws, &status};
    if (hipLaunchKernel(fn, dim3(p->grid), dim3(BATCH_BLOCK), args, (size_t)p->lds_bytes, st) != hipSuccess)
        return REPRO_EHIP;
    const int nunits = p->reserved[0];  // merge schedule 1: the merge launch
    if (nunits > 0) {
        if (p->T == REPRO_F64)
            hipLaunchKernelGGL(k_batch_merge<double>, dim3(nunits), dim3(MERGE_UNIT), 0, st, ws);
        else
            hipLaunchKernelGGL(k_batch_merge<float>, dim3(nunits), dim3(MERGE_UNIT), 0, st, ws);
        if (hipGetLastError() != hipSuccess) return REPRO_EHIP;
    }
    return REPRO_OK;
}

}  // namespace

namespace repro {
namespace batchx {

bool plan_sizes(const repro_batch_job* jobs, int njobs, repro_key_t kt, repro_scalar_t vt, repro_scalar_t T,
                const repro_batch_config* cfg, size_t* workspace_bytes, size_t* image_bytes) {
    HostPlan hp;
    if (!make_batch_plan(jobs, njobs, kt, vt, T, cfg, &hp)) return false;
    *workspace_bytes = hp.lay.total;
    *image_bytes = hp.lay.counters;
    return true;
}

int plan_into(const repro_batch_job* jobs, int njobs, repro_key_t kt, repro_scalar_t vt, repro_scalar_t T,
              const repro_batch_config* cfg, void* image, size_t image_cap, void* workspace, size_t workspace_bytes,
              repro_batch_plan* plan) {
    if (!plan) return REPRO_EINVAL;
    HostPlan hp;
    if (!make_batch_plan(jobs, njobs, kt, vt, T, cfg, &hp)) return REPRO_EINVAL;
    if (!workspace || workspace_bytes < hp.lay.total || (uintptr_t)workspace % 256 != 0) return REPRO_EINVAL;
    if (!image || image_cap < hp.lay.counters) return REPRO_EINVAL;
    // the plan image: head, jobs, items (counters, spill words and partials
    // are device-only, cleared or written by the kernels)
    unsigned char* img = static_cast<unsigned char*>(image);
    memset(img, 0, hp.lay.counters);
    BatchHead hd;
    memset(&hd, 0, sizeof(hd));
    hd.nitems = (int)hp.items.size();
    hd.njobs = njobs;
    hd.ncounters = (int)hp.ncounters;
    hd.off_jobs = (long long)hp.lay.jobs;
    hd.off_items = (long long)hp.lay.items;
    hd.off_counters = (long long)hp.lay.counters;
    hd.off_spill = (long long)hp.lay.spill;
    hd.off_partials = (long long)hp.lay.partials;
    hd.zero_words = (long long)((hp.lay.partials - hp.lay.counters) / 8);
    hd.merge = hp.merge;
    hd.nunits = (int)hp.units.size();
    hd.off_units = (long long)hp.lay.units;
    hd.off_scr_keys = (long long)hp.lay.scr_keys;
    hd.off_scr_vals = (long long)hp.lay.scr_vals;
    memcpy(img, &hd, sizeof(hd));
    if (njobs) memcpy(img + hp.lay.jobs, hp.jobs.data(), hp.jobs.size() * sizeof(BatchJob));
    if (!hp.items.empty()) memcpy(img + hp.lay.items, hp.items.data(), hp.items.size() * sizeof(BatchItem));
    if (!hp.units.empty()) memcpy(img + hp.lay.units, hp.units.data(), hp.units.size() * sizeof(MergeUnit));
    // dynamic LDS beyond 64 KiB must be allowed per kernel; done here, on the
    // host and outside any graph capture of the launches
    if (hp.lds > 64 * 1024 && hipFuncSetAttribute(pick_kernel(kt, vt, T), hipFuncAttributeMaxDynamicSharedMemorySize,
                                                  (int)hp.lds) != hipSuccess)
        return REPRO_EHIP;
    memset(plan, 0, sizeof(*plan));
    plan->workspace = workspace;
    plan->items = (int64_t)hp.items.size();
    plan->grid = (int)std::min<int64_t>(BATCH_MAX_WG, std::max<int64_t>(1, plan->items));
    plan->lds_bytes = (int)hp.lds;
    plan->kt = kt;
    plan->vt = vt;
    plan->T = T;
    plan->reserved[0] = (int)hp.units.size();  // units of the merge launch (merge schedule 1)
    return REPRO_OK;
}

int launch(const repro_batch_plan* plan, uint32_t* status, hipStream_t stream) { return launch_plan(plan, status, stream); }

int slice_limit(int L) { return slice_cap(L, 0); }

}  // namespace batchx
}  // namespace repro

extern "C" {

size_t repro_batch_workspace_bytes(const repro_batch_job* jobs, int njobs, repro_key_t kt, repro_scalar_t vt,
                                   repro_scalar_t T, const repro_batch_config* cfg) {
    HostPlan hp;
    if (!make_batch_plan(jobs, njobs, kt, vt, T, cfg, &hp)) return 0;
    return hp.lay.total;
}

int repro_batch_prepare(const repro_batch_job* jobs, int njobs, repro_key_t kt, repro_scalar_t vt, repro_scalar_t T,
                        const repro_batch_config* cfg, void* workspace, size_t workspace_bytes,
                        repro_batch_plan* plan, hipStream_t stream) {
    size_t total = 0, image = 0;
    if (!repro::batchx::plan_sizes(jobs, njobs, kt, vt, T, cfg, &total, &image)) return REPRO_EINVAL;
    std::vector<unsigned char> img(image);
    int rc = repro::batchx::plan_into(jobs, njobs, kt, vt, T, cfg, img.data(), img.size(), workspace, workspace_bytes,
                                      plan);
    if (rc != REPRO_OK) return rc;
    if (hipMemcpyAsync(workspace, img.data(), img.size(), hipMemcpyHostToDevice, stream) != hipSuccess)
        return REPRO_EHIP;
    if (hipStreamSynchronize(stream) != hipSuccess) return REPRO_EHIP;
    return REPRO_OK;
}

int repro_batch_launch(const repro_batch_plan* plan, uint32_t* status, hipStream_t stream) {
    if (!plan || !plan->workspace || plan->items < 0 || !valid_types((repro_key_t)plan->kt, (repro_scalar_t)plan->vt,
                                                                      (repro_scalar_t)plan->T))
        return REPRO_EINVAL;
    return launch_plan(plan, status, stream);
}

int repro_batch_tune(const repro_batch_job* jobs, int njobs, repro_key_t kt, repro_scalar_t vt, repro_scalar_t T,
                     void* workspace, size_t workspace_bytes, repro_batch_config* best, float* best_ms,
                     hipStream_t stream) {
    if (!best) return REPRO_EINVAL;
    // chunk sizes: the binding sizes the workspace over these same candidates
    const int64_t chunks[] = {65536, 131072, 262144, 524288, 1048576, 2097152};
    const int caps[] = {0, 1024};
    const int orders[] = {0, 1};
    const int merges[] = {0, 1};
    const int splits[] = {0, 1};
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return REPRO_EHIP;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return REPRO_EHIP;
    }
    float best_t = -1.0f;
    int rc = REPRO_OK;
    for (int64_t ch : chunks)
        for (int cap : caps)
            for (int ord : orders)
                for (int mg : merges)
                    for (int sp : splits) {
                repro_batch_config c{ch, cap, ord, mg, sp};
                if (repro_batch_workspace_bytes(jobs, njobs, kt, vt, T, &c) > workspace_bytes) continue;
                repro_batch_plan p;
                rc = repro_batch_prepare(jobs, njobs, kt, vt, T, &c, workspace, workspace_bytes, &p, stream);
                if (rc != REPRO_OK) goto done;
                if ((rc = launch_plan(&p, nullptr, stream)) != REPRO_OK) goto done;  // warm-up
                if (hipEventRecord(e0, stream) != hipSuccess) { rc = REPRO_EHIP; goto done; }
                for (int r = 0; r < 2; ++r)
                    if ((rc = launch_plan(&p, nullptr, stream)) != REPRO_OK) goto done;
                if (hipEventRecord(e1, stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
                    rc = REPRO_EHIP;
                    goto done;
                }
                float ms = 0;
                if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) { rc = REPRO_EHIP; goto done; }
                ms *= 0.5f;
                if (best_t < 0 || ms < best_t) {
                    best_t = ms;
                    *best = c;
                }
            }
done:
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != REPRO_OK) return rc;
    if (best_t < 0) return REPRO_EINVAL;  // no candidate fits the workspace
    if (best_ms) *best_ms = best_t;
    return REPRO_OK;
}

}  // extern "C"
