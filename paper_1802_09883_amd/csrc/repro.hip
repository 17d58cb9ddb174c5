// repro.hip -- librepro: reproducible GroupBy-SUM into repro<T,L> for gfx950.
//
// Paper: Mueller, Arteaga, Hoefler, Alonso, "Reproducible Floating-Point
// Aggregation in RDBMSs" (arXiv 1802.09883).
//
// Hot path of repro_groupby_sum (one HBM pass over keys and values):
//   k_agg_lds    each workgroup streams a contiguous chunk of rows in tiles;
//                per tile: key -> group (identity hashing, Sec. VI-A), the
//                per-group top index (max-exponent step; Alg. 1's level
//                check done once per tile as Alg. 2 does once per block),
//                realignment of the LDS bins of groups whose top rose,
//                pre-rounded extraction into L integer units, exact int64
//                adds into per-(level, group) LDS bins.  At the end the
//                workgroup writes its partial (top, K[L]) per group.
//   k_merge_l1   reduces blocks of partials: common top per group, shift,
//                exact integer sums split into (hi, lo) carry form.
//   k_merge_l2   folds the reduced partials into the caller's states and
//                writes canonical (S, C) (carry renormalisation).
// Exact integer addition is associative, so every launch shape, chunking
// and schedule produces the same bits.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include "repro.h"
#include "repro_device.hpp"

using namespace repro;

namespace {

constexpr int AGG_BLOCK = 256;
constexpr int ROWS_PER_THREAD = 8;
constexpr int AGG_TILE = AGG_BLOCK * ROWS_PER_THREAD;
constexpr int MAX_AGG_WG = 1024;
constexpr int64_t MIN_ROWS_PER_WG = 16 * (int64_t)AGG_TILE;
// A bin word takes at most (rows of one workgroup) units of magnitude
// <= 2^(W-1) <= 2^39; 2^23 rows keep it below 2^62.
constexpr int64_t MAX_ROWS_PER_WG = (int64_t)1 << 23;
constexpr size_t LDS_BIN_BUDGET = 64 * 1024;
constexpr size_t REPLICA_BUDGET = 32 * 1024;
constexpr int MERGE_GROUPS = 64;     // groups per merge block (one per lane)
constexpr int MERGE_WAVES = 4;
constexpr int MERGE_PARTS = 32;      // partials reduced per level-1 block

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// ----------------------------------------------------------- row loading

template <class T, int N>
struct VecT {
    typedef T type __attribute__((ext_vector_type(N)));
};

template <class T, int N>
__device__ __forceinline__ void vload(const T* __restrict__ p, T* out) {
    if constexpr (N == 1) {
        out[0] = *p;
    } else {
        typedef typename VecT<T, N>::type V;
        const V x = *reinterpret_cast<const V*>(p);
#pragma unroll
        for (int i = 0; i < N; ++i) out[i] = x[i];
    }
}

// Loads the ROWS_PER_THREAD rows of this thread in the tile starting at
// `base`: unit u covers rows base + (u*BLOCK + tid)*VEC + [0, VEC), so each
// vector load instruction of a wave reads one contiguous span.  Rows at or
// beyond `end` are flagged out of range.
template <class KT, class VT, int VEC, int BLOCK>
__device__ __forceinline__ uint32_t load_tile(const KT* __restrict__ keys, const VT* __restrict__ vals,
                                              int64_t base, int64_t end, KT* k, VT* v) {
    constexpr int U = ROWS_PER_THREAD / VEC;
    const int tid = threadIdx.x;
    uint32_t inr = 0;
    if (base + (int64_t)BLOCK * ROWS_PER_THREAD <= end) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t row = base + ((int64_t)u * BLOCK + tid) * VEC;
            vload<KT, VEC>(keys + row, k + u * VEC);
            vload<VT, VEC>(vals + row, v + u * VEC);
        }
        inr = (1u << ROWS_PER_THREAD) - 1;
    } else {
#pragma unroll
        for (int u = 0; u < U; ++u) {
#pragma unroll
            for (int e = 0; e < VEC; ++e) {
                const int64_t row = base + ((int64_t)u * BLOCK + tid) * VEC + e;
                if (row < end) {
                    k[u * VEC + e] = keys[row];
                    v[u * VEC + e] = vals[row];
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

__device__ __forceinline__ void report(uint32_t* status, uint32_t err) {
    err = wave_or(err);
    if (status && err && (threadIdx.x & 63) == 0) atomicOr(status, err);
}

// ------------------------------------------------------ the hot kernel
//
// LDS: A[G] (top each group's bins are aligned to), P[G] (pending top,
// raised with ds_max during a tile), bins[L][G][R] int64 (R replicas, lane
// r uses replica lane % R to spread contention when groups are few).
template <class KT, class VT, class AT, int L, int VEC>
__global__ void __launch_bounds__(AGG_BLOCK) k_agg_lds(const KT* __restrict__ keys, const VT* __restrict__ vals,
                                                       int64_t n, int G, int R, int64_t chunk,
                                                       int* __restrict__ ptop, long long* __restrict__ pK,
                                                       uint32_t* __restrict__ status) {
    typedef Fmt<AT> F;
    extern __shared__ __align__(16) unsigned char smem[];
    long long* bins = reinterpret_cast<long long*>(smem);
    int* A = reinterpret_cast<int*>(bins + (size_t)L * G * R);
    int* P = A + G;

    const int tid = threadIdx.x;
    const int rep = (tid & 63) & (R - 1);
    for (int i = tid; i < L * G * R; i += AGG_BLOCK) bins[i] = 0;
    for (int i = tid; i < G; i += AGG_BLOCK) {
        A[i] = L - 1;
        P[i] = L - 1;
    }
    __syncthreads();

    const int64_t c0 = (int64_t)blockIdx.x * chunk;
    const int64_t c1 = (c0 + chunk < n) ? c0 + chunk : n;
    uint32_t err = 0;

    KT kc[ROWS_PER_THREAD], kn[ROWS_PER_THREAD];
    VT vc[ROWS_PER_THREAD], vn[ROWS_PER_THREAD];
    uint32_t inr_c = 0, inr_n = 0;
    if (c0 < c1) inr_c = load_tile<KT, VT, VEC, AGG_BLOCK>(keys, vals, c0, c1, kc, vc);

    for (int64_t base = c0; base < c1; base += AGG_TILE) {
        // prefetch the next tile while this one is processed
        const int64_t nb = base + AGG_TILE;
        if (nb < c1) inr_n = load_tile<KT, VT, VEC, AGG_BLOCK>(keys, vals, nb, c1, kn, vn);

        int g[ROWS_PER_THREAD], a[ROWS_PER_THREAD];
        uint32_t ok = 0, first = 0;
        int raise = 0;
#pragma unroll
        for (int i = 0; i < ROWS_PER_THREAD; ++i) {
            const bool in = (inr_c >> i) & 1u;
            const VT v = vc[i];
            const bool kok = (uint64_t)(int64_t)kc[i] < (uint64_t)G;
            const bool fin = finite_val(v);
            const int j = jreq_of_exp<AT>(exp_of(v));
            const bool dom = j <= F::JMAX;
            err |= (in && !kok) ? ERR_KEY : 0u;
            err |= (in && !fin) ? ERR_NONFINITE : 0u;
            err |= (in && fin && v != (VT)0 && !dom) ? ERR_RANGE : 0u;
            const bool use = in && kok && fin && dom && v != (VT)0;
            g[i] = use ? (int)kc[i] : 0;
            a[i] = 0;
            if (use) {
                ok |= 1u << i;
                a[i] = A[g[i]];
                if (j > a[i]) {
                    raise = 1;
                    const int old = atomicMax(&P[g[i]], j);
                    if (old == a[i]) first |= 1u << i;  // first raiser realigns
                }
            }
        }
        if (__syncthreads_or(raise)) {
            // realign: move each raised group's levels down by the rise;
            // the lowest ones fall off (the level shift of Alg. 1)
#pragma unroll
            for (int i = 0; i < ROWS_PER_THREAD; ++i) {
                if ((first >> i) & 1u) {
                    const int gg = g[i];
                    const int d = P[gg] - A[gg];
                    for (int r = 0; r < R; ++r) {
#pragma unroll
                        for (int l = L - 1; l >= 0; --l) {
                            const long long x = (l - d >= 0) ? bins[((size_t)(l - d) * G + gg) * R + r] : 0;
                            bins[((size_t)l * G + gg) * R + r] = x;
                        }
                    }
                    A[gg] = P[gg];
                }
            }
            __syncthreads();
#pragma unroll
            for (int i = 0; i < ROWS_PER_THREAD; ++i)
                if ((ok >> i) & 1u) a[i] = A[g[i]];
        }
#pragma unroll
        for (int i = 0; i < ROWS_PER_THREAD; ++i) {
            if ((ok >> i) & 1u) {
                long long k[L];
                extract_units<L>((AT)vc[i], a[i], k);
#pragma unroll
                for (int l = 0; l < L; ++l)
                    atomicAdd(reinterpret_cast<unsigned long long*>(&bins[((size_t)l * G + g[i]) * R + rep]),
                              (unsigned long long)k[l]);
            }
        }
#pragma unroll
        for (int i = 0; i < ROWS_PER_THREAD; ++i) {
            kc[i] = kn[i];
            vc[i] = vn[i];
        }
        inr_c = inr_n;
    }
    __syncthreads();
    for (int gg = tid; gg < G; gg += AGG_BLOCK) {
        ptop[(size_t)blockIdx.x * G + gg] = A[gg];
#pragma unroll
        for (int l = 0; l < L; ++l) {
            long long s = 0;
            for (int r = 0; r < R; ++r) s += bins[((size_t)l * G + gg) * R + r];
            pK[((size_t)blockIdx.x * L + l) * G + gg] = s;
        }
    }
    report(status, err);
}

// ------------------------------------------------------------- merging
//
// Level 1: block (bx, by) reduces partials [by*MERGE_PARTS, ...) for groups
// bx*64 + lane.  Output per (by, g): common top and, per level, the exact
// sum split as hi = sum(K >> CARRY), lo = sum(K & mask) (no overflow for up
// to 2^13 partials).
template <class AT, int L>
__global__ void __launch_bounds__(MERGE_GROUPS* MERGE_WAVES)
    k_merge_l1(const int* __restrict__ ptop, const long long* __restrict__ pK, int nparts, int G,
               int* __restrict__ qtop, long long* __restrict__ qhi, long long* __restrict__ qlo) {
    constexpr int c = Fmt<AT>::CARRY;
    __shared__ int sJ[MERGE_WAVES][MERGE_GROUPS];
    __shared__ long long sH[MERGE_WAVES][L][MERGE_GROUPS], sL[MERGE_WAVES][L][MERGE_GROUPS];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = blockIdx.x * MERGE_GROUPS + lane;
    const bool gv = g < G;
    const int p0 = blockIdx.y * MERGE_PARTS;
    const int p1 = min(nparts, p0 + MERGE_PARTS);
    int J = L - 1;
    if (gv)
        for (int p = p0 + wave; p < p1; p += MERGE_WAVES) J = max(J, ptop[(size_t)p * G + g]);
    sJ[wave][lane] = J;
    __syncthreads();
#pragma unroll
    for (int w = 0; w < MERGE_WAVES; ++w) J = max(J, sJ[w][lane]);
    long long hi[L], lo[L];
#pragma unroll
    for (int l = 0; l < L; ++l) hi[l] = lo[l] = 0;
    if (gv) {
        for (int p = p0 + wave; p < p1; p += MERGE_WAVES) {
            const int d = J - ptop[(size_t)p * G + g];
#pragma unroll
            for (int l = 0; l < L; ++l) {
                if (l - d >= 0) {
                    const long long x = pK[((size_t)p * L + (l - d)) * G + g];
                    hi[l] += x >> c;
                    lo[l] += x & ((1ll << c) - 1);
                }
            }
        }
    }
#pragma unroll
    for (int l = 0; l < L; ++l) {
        sH[wave][l][lane] = hi[l];
        sL[wave][l][lane] = lo[l];
    }
    __syncthreads();
    if (wave == 0 && gv) {
#pragma unroll
        for (int l = 0; l < L; ++l) {
            long long h = 0, o = 0;
#pragma unroll
            for (int w = 0; w < MERGE_WAVES; ++w) {
                h += sH[w][l][lane];
                o += sL[w][l][lane];
            }
            qhi[((size_t)blockIdx.y * L + l) * G + g] = h;
            qlo[((size_t)blockIdx.y * L + l) * G + g] = o;
        }
        qtop[(size_t)blockIdx.y * G + g] = J;
    }
}

// Level 2: one thread per group folds the reduced partials (hi, lo form, or
// raw K when RAW) into the caller's canonical state and renormalises.
template <class AT, int L, bool RAW>
__global__ void __launch_bounds__(256)
    k_merge_l2(const int* __restrict__ qtop, const long long* __restrict__ qhi, const long long* __restrict__ qlo,
               int nparts, int G, AT* __restrict__ S, long long* __restrict__ C) {
    typedef Fmt<AT> F;
    constexpr int c = F::CARRY;
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= G) return;
    const int ts = state_top(S[g]);
    int J = ts;
    for (int p = 0; p < nparts; ++p) J = max(J, qtop[(size_t)p * G + g]);
    long long hi[L], lo[L];
    const int ds = J - ts;
#pragma unroll
    for (int l = 0; l < L; ++l) {
        hi[l] = (l - ds >= 0) ? C[(size_t)(l - ds) * G + g] : 0;
        lo[l] = (l - ds >= 0) ? state_lo(S[(size_t)(l - ds) * G + g]) : 0;
    }
    for (int p = 0; p < nparts; ++p) {
        const int d = J - qtop[(size_t)p * G + g];
#pragma unroll
        for (int l = 0; l < L; ++l) {
            if (l - d >= 0) {
                if (RAW) {
                    const long long x = qhi[((size_t)p * L + (l - d)) * G + g];
                    hi[l] += x >> c;
                    lo[l] += x & ((1ll << c) - 1);
                } else {
                    hi[l] += qhi[((size_t)p * L + (l - d)) * G + g];
                    lo[l] += qlo[((size_t)p * L + (l - d)) * G + g];
                }
            }
        }
    }
#pragma unroll
    for (int l = 0; l < L; ++l) {
        long long cc, oo;
        normalise<AT>(hi[l], lo[l], &cc, &oo);
        S[(size_t)l * G + g] = make_S((AT*)0, F::B + (J - l) * F::W, oo);
        C[(size_t)l * G + g] = cc;
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
// one global double atomic per group and workgroup.
template <class KT, class VT, int VEC>
__global__ void __launch_bounds__(AGG_BLOCK) k_plain_lds(const KT* __restrict__ keys, const VT* __restrict__ vals,
                                                         int64_t n, int G, int64_t chunk, double* __restrict__ out,
                                                         uint32_t* __restrict__ status) {
    extern __shared__ __align__(16) unsigned char smem[];
    double* bins = reinterpret_cast<double*>(smem);
    const int tid = threadIdx.x;
    for (int i = tid; i < G; i += AGG_BLOCK) bins[i] = 0.0;
    __syncthreads();
    const int64_t c0 = (int64_t)blockIdx.x * chunk;
    const int64_t c1 = (c0 + chunk < n) ? c0 + chunk : n;
    uint32_t err = 0;
    KT kc[ROWS_PER_THREAD];
    VT vc[ROWS_PER_THREAD];
    for (int64_t base = c0; base < c1; base += AGG_TILE) {
        const uint32_t inr = load_tile<KT, VT, VEC, AGG_BLOCK>(keys, vals, base, c1, kc, vc);
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
    for (int gg = tid; gg < G; gg += AGG_BLOCK)
        if (bins[gg] != 0.0) atomicAdd(&out[gg], bins[gg]);
    report(status, err);
}

template <class KT, class VT, int VEC>
__global__ void __launch_bounds__(AGG_BLOCK) k_plain_global(const KT* __restrict__ keys, const VT* __restrict__ vals,
                                                            int64_t n, int G, int64_t chunk, double* __restrict__ out,
                                                            uint32_t* __restrict__ status) {
    const int64_t c0 = (int64_t)blockIdx.x * chunk;
    const int64_t c1 = (c0 + chunk < n) ? c0 + chunk : n;
    uint32_t err = 0;
    KT kc[ROWS_PER_THREAD];
    VT vc[ROWS_PER_THREAD];
    for (int64_t base = c0; base < c1; base += AGG_TILE) {
        const uint32_t inr = load_tile<KT, VT, VEC, AGG_BLOCK>(keys, vals, base, c1, kc, vc);
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

// ================================================================ host

// ------------------------------------------------------------ profiling
constexpr int PROFILE_MAX = 4096;
struct ProfileSlot {
    hipEvent_t ev[2 * PROFILE_MAX];
    int created = 0, armed = 0, used = 0;
};
thread_local ProfileSlot* g_prof = nullptr;

inline void prof_before(hipStream_t st) {
    if (g_prof && g_prof->used < g_prof->armed) (void)hipEventRecord(g_prof->ev[2 * g_prof->used], st);
}
inline void prof_after(hipStream_t st) {
    if (g_prof && g_prof->used < g_prof->armed) (void)hipEventRecord(g_prof->ev[2 * g_prof->used++ + 1], st);
}

struct Plan {
    int path;       // 1: LDS bins
    int nwg;        // aggregate workgroups
    int64_t chunk;  // rows per workgroup (multiple of the tile)
    int R;          // LDS bin replicas
    size_t lds;     // dynamic LDS bytes
    int n_l1;       // level-1 merge blocks along the partial axis (0: skip)
    size_t ws;      // workspace bytes
};

inline size_t scalar_size(repro_scalar_t t) { return t == REPRO_F64 ? 8 : 4; }

bool valid_common(int64_t G, repro_scalar_t T, int L) {
    return G >= 1 && G <= INT32_MAX && (T == REPRO_F32 || T == REPRO_F64) && L >= 1 && L <= 4;
}

int replicas_for(int64_t G, int L) {
    int R = 1;
    while (R < 64 && (size_t)2 * R * G * L * 8 <= REPLICA_BUDGET) R *= 2;
    return R;
}

bool make_plan(int64_t n, int64_t G, int L, Plan* p) {
    memset(p, 0, sizeof(*p));
    const size_t lds1 = (size_t)G * L * 8 + (size_t)G * 8;
    if (lds1 > LDS_BIN_BUDGET) return false;  // high cardinality: not on this path
    p->path = 1;
    p->R = replicas_for(G, L);
    p->lds = (size_t)G * L * 8 * p->R + (size_t)G * 8;
    int64_t nwg = (n + MIN_ROWS_PER_WG - 1) / MIN_ROWS_PER_WG;
    if (nwg > MAX_AGG_WG) nwg = MAX_AGG_WG;
    if (nwg < (n + MAX_ROWS_PER_WG - 1) / MAX_ROWS_PER_WG) nwg = (n + MAX_ROWS_PER_WG - 1) / MAX_ROWS_PER_WG;
    if (nwg < 1) nwg = 1;
    int64_t chunk = (n + nwg - 1) / nwg;
    chunk = (chunk + AGG_TILE - 1) / AGG_TILE * AGG_TILE;
    if (chunk < AGG_TILE) chunk = AGG_TILE;
    nwg = (n + chunk - 1) / chunk;
    if (nwg < 1) nwg = 1;
    if (nwg > INT32_MAX / 2) return false;
    p->nwg = (int)nwg;
    p->chunk = chunk;
    p->n_l1 = nwg > MERGE_PARTS ? (int)((nwg + MERGE_PARTS - 1) / MERGE_PARTS) : 0;
    size_t ws = 0;
    ws += align_up((size_t)nwg * G * 4, 256);          // partial tops
    ws += align_up((size_t)nwg * G * L * 8, 256);      // partial K
    if (p->n_l1) {
        ws += align_up((size_t)p->n_l1 * G * 4, 256);      // reduced tops
        ws += 2 * align_up((size_t)p->n_l1 * G * L * 8, 256);  // reduced hi, lo
    }
    p->ws = ws;
    return true;
}

#define LAUNCH_CHECK()                                  \
    do {                                                \
        if (hipGetLastError() != hipSuccess) return REPRO_EHIP; \
    } while (0)

template <class AT, int L>
int run_merge(const Plan& p, int G, unsigned char* ws, AT* S, long long* C, hipStream_t st) {
    int* ptop = reinterpret_cast<int*>(ws);
    long long* pK = reinterpret_cast<long long*>(ws + align_up((size_t)p.nwg * G * 4, 256));
    const dim3 b2(256), g2((G + 255) / 256);
    if (p.n_l1 == 0) {
        hipLaunchKernelGGL((k_merge_l2<AT, L, true>), g2, b2, 0, st, ptop, pK, (const long long*)nullptr, p.nwg, G, S,
                           C);
        LAUNCH_CHECK();
        return REPRO_OK;
    }
    unsigned char* q = ws + align_up((size_t)p.nwg * G * 4, 256) + align_up((size_t)p.nwg * G * L * 8, 256);
    int* qtop = reinterpret_cast<int*>(q);
    long long* qhi = reinterpret_cast<long long*>(q + align_up((size_t)p.n_l1 * G * 4, 256));
    long long* qlo = reinterpret_cast<long long*>(reinterpret_cast<unsigned char*>(qhi) +
                                                  align_up((size_t)p.n_l1 * G * L * 8, 256));
    const dim3 b1(MERGE_GROUPS * MERGE_WAVES), g1((G + MERGE_GROUPS - 1) / MERGE_GROUPS, p.n_l1);
    hipLaunchKernelGGL((k_merge_l1<AT, L>), g1, b1, 0, st, ptop, pK, p.nwg, G, qtop, qhi, qlo);
    LAUNCH_CHECK();
    hipLaunchKernelGGL((k_merge_l2<AT, L, false>), g2, b2, 0, st, qtop, qhi, qlo, p.n_l1, G, S, C);
    LAUNCH_CHECK();
    return REPRO_OK;
}

template <class KT, class VT, class AT, int L>
int run_groupby(const void* keys, const void* values, int64_t n, int G, void* states, void* workspace,
                uint32_t* status, const Plan& p, hipStream_t st) {
    unsigned char* ws = static_cast<unsigned char*>(workspace);
    int* ptop = reinterpret_cast<int*>(ws);
    long long* pK = reinterpret_cast<long long*>(ws + align_up((size_t)p.nwg * G * 4, 256));
    const KT* k = static_cast<const KT*>(keys);
    const VT* v = static_cast<const VT*>(values);
    constexpr int VEC = 16 / sizeof(VT);
    const bool aligned = ((uintptr_t)k % (VEC * sizeof(KT)) == 0) && ((uintptr_t)v % 16 == 0);
    prof_before(st);
    if (aligned)
        hipLaunchKernelGGL((k_agg_lds<KT, VT, AT, L, VEC>), dim3(p.nwg), dim3(AGG_BLOCK), p.lds, st, k, v, n, G, p.R,
                           p.chunk, ptop, pK, status);
    else
        hipLaunchKernelGGL((k_agg_lds<KT, VT, AT, L, 1>), dim3(p.nwg), dim3(AGG_BLOCK), p.lds, st, k, v, n, G, p.R,
                           p.chunk, ptop, pK, status);
    LAUNCH_CHECK();
    prof_after(st);
    AT* S = static_cast<AT*>(states);
    long long* C = reinterpret_cast<long long*>(static_cast<unsigned char*>(states) +
                                                align_up((size_t)G * L * sizeof(AT), 8));
    return run_merge<AT, L>(p, G, ws, S, C, st);
}

template <class KT, class VT, class AT>
int dispatch_L(int L, const void* keys, const void* values, int64_t n, int G, void* states, void* ws,
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
int dispatch_types(repro_scalar_t vt, repro_scalar_t T, int L, const void* keys, const void* values, int64_t n, int G,
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

template <class KT, class VT>
int run_plain(const void* keys, const void* values, int64_t n, int G, double* out, uint32_t* status, hipStream_t st) {
    const KT* k = static_cast<const KT*>(keys);
    const VT* v = static_cast<const VT*>(values);
    int64_t nwg = (n + MIN_ROWS_PER_WG - 1) / MIN_ROWS_PER_WG;
    if (nwg > MAX_AGG_WG) nwg = MAX_AGG_WG;
    if (nwg < 1) nwg = 1;
    int64_t chunk = (n + nwg - 1) / nwg;
    chunk = (chunk + AGG_TILE - 1) / AGG_TILE * AGG_TILE;
    nwg = (n + chunk - 1) / chunk;
    constexpr int VEC = 16 / sizeof(VT);
    const bool aligned = ((uintptr_t)k % (VEC * sizeof(KT)) == 0) && ((uintptr_t)v % 16 == 0);
    if ((size_t)G * 8 <= LDS_BIN_BUDGET) {
        const size_t lds = (size_t)G * 8;
        if (aligned)
            hipLaunchKernelGGL((k_plain_lds<KT, VT, VEC>), dim3(nwg), dim3(AGG_BLOCK), lds, st, k, v, n, G, chunk, out,
                               status);
        else
            hipLaunchKernelGGL((k_plain_lds<KT, VT, 1>), dim3(nwg), dim3(AGG_BLOCK), lds, st, k, v, n, G, chunk, out,
                               status);
    } else {
        if (aligned)
            hipLaunchKernelGGL((k_plain_global<KT, VT, VEC>), dim3(nwg), dim3(AGG_BLOCK), 0, st, k, v, n, G, chunk,
                               out, status);
        else
            hipLaunchKernelGGL((k_plain_global<KT, VT, 1>), dim3(nwg), dim3(AGG_BLOCK), 0, st, k, v, n, G, chunk, out,
                               status);
    }
    LAUNCH_CHECK();
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
    (void)vt;
    Plan p;
    if (!valid_common(num_groups, T, L) || n < 0) return 0;
    if (!make_plan(n, num_groups, L, &p)) return 0;
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
    if (!make_plan(n, num_groups, L, &p)) return REPRO_EINVAL;
    if (p.ws > 0 && (!workspace || workspace_bytes < p.ws || (uintptr_t)workspace % 256 != 0)) return REPRO_EINVAL;
    const int G = (int)num_groups;
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

int repro_plain_groupby_sum(const void* keys, repro_key_t kt, const void* values, repro_scalar_t vt, int64_t n,
                            int64_t num_groups, double* out, uint32_t* status, hipStream_t stream) {
    if (num_groups < 1 || num_groups > INT32_MAX || n < 0 || !out) return REPRO_EINVAL;
    if ((kt != REPRO_I32 && kt != REPRO_I64) || (vt != REPRO_F32 && vt != REPRO_F64)) return REPRO_EINVAL;
    if (n == 0) return REPRO_OK;
    if (!keys || !values) return REPRO_EINVAL;
    const int G = (int)num_groups;
    if (kt == REPRO_I32)
        return vt == REPRO_F64 ? run_plain<int32_t, double>(keys, values, n, G, out, status, stream)
                               : run_plain<int32_t, float>(keys, values, n, G, out, status, stream);
    return vt == REPRO_F64 ? run_plain<int64_t, double>(keys, values, n, G, out, status, stream)
                           : run_plain<int64_t, float>(keys, values, n, G, out, status, stream);
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

const char* repro_version(void) { return "librepro 0.1 (gfx950)"; }

}  // extern "C"
