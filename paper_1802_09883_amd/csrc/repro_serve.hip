// repro_serve.hip -- request loop for reproducible GroupBy-SUM queries
// (librepro, gfx950).
//
// Paper: Mueller, Arteaga, Hoefler, Alonso, "Reproducible Floating-Point
// Aggregation in RDBMSs" (arXiv 1802.09883).  A query is a GroupBy with
// several RSum(expression, L) aggregates (Sec. V-D); its states are resumable
// (Alg. 2 loads and stores them), so they stay resident in device memory and
// take the query's rows chunk by chunk; exact level sums make the result
// independent of the chunking and of whatever else runs on the device.
//
// Host side: a FIFO of submitted queries, a fixed set of slots (one stream
// each) and a first-fit allocator over a caller-owned device arena.  A query
// is admitted when a slot is free and its memory fits; its whole pipeline is
// then enqueued on its slot's stream (state initialisation, product columns,
// one repro_groupby_sum per chunk and aggregate, finalisation, an event).
// Polling retires queries whose event completed and admits the next ones.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <deque>
#include <iterator>
#include <map>
#include <vector>

#include "repro.h"
#include "repro_batch_internal.hpp"

namespace {

constexpr int64_t SERVE_DEFAULT_CHUNK = 16ll << 20;
constexpr int64_t SERVE_BATCH_CHUNK = 512 * 1024;  // rows per batch item (the tuned size on the batch workload)
constexpr size_t SERVE_IMAGE_BYTES = 64 * 1024;    // pinned plan image per slot
constexpr size_t SERVE_ALIGN = 256;

inline size_t up(size_t x) { return (x + SERVE_ALIGN - 1) / SERVE_ALIGN * SERVE_ALIGN; }

// out[i] = a[i] * b[i] in double precision, one IEEE rounding (the build
// disables contraction); float inputs widen exactly first.
template <class TA, class TB>
__global__ void __launch_bounds__(256) k_mul(const TA* __restrict__ a, const TB* __restrict__ b,
                                             double* __restrict__ out, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        out[i] = (double)a[i] * (double)b[i];
}

template <class TA, class TB>
int launch_mul(const void* a, const void* b, int64_t n, double* out, hipStream_t st) {
    const int64_t blocks = std::min<int64_t>(4096, (n + 255) / 256);
    hipLaunchKernelGGL((k_mul<TA, TB>), dim3((unsigned)blocks), dim3(256), 0, st, static_cast<const TA*>(a),
                       static_cast<const TB*>(b), out, n);
    return hipGetLastError() == hipSuccess ? REPRO_OK : REPRO_EHIP;
}

// First-fit allocator over [0, size) with coalescing; offsets 256-aligned.
class Arena {
   public:
    void init(size_t size) {
        free_.clear();
        if (size) free_[0] = size;
    }
    bool alloc(size_t bytes, size_t* off) {
        bytes = up(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes;
                const size_t at = it->first + bytes;
                free_.erase(it);
                if (rest) free_[at] = rest;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        bytes = up(bytes);
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }

   private:
    std::map<size_t, size_t> free_;
};

// Arena layout of one admitted query.
struct QueryLayout {
    size_t state_bytes, ws_bytes, total, image_bytes;
    size_t off_state[REPRO_MAX_AGGS], off_prod[REPRO_MAX_AGGS], off_ws;
    int64_t chunk;
    bool batch;  // aggregates as jobs of one batch launch
};

// The batch jobs of a query's aggregates; `prod` gives the product columns
// (arena addresses, or stand-ins while only sizing).
void query_jobs(const repro_query* q, void* const* states, const double* const* prod, repro_batch_job* jobs) {
    for (int a = 0; a < q->naggs; ++a) {
        repro_batch_job& j = jobs[a];
        memset(&j, 0, sizeof(j));
        j.keys = q->keys;
        j.values = q->agg_b[a] >= 0 ? (const void*)prod[a] : (const void*)q->cols[q->agg_a[a]];
        j.n = q->n;
        j.num_groups = q->num_groups;
        j.L = q->L;
        j.accumulate = 0;
        j.states = states[a];
        j.out = q->out[a];
    }
}

bool valid_query(const repro_query* q) {
    if (!q || q->n < 0 || q->num_groups < 1 || q->num_groups > INT32_MAX || q->L < 1 || q->L > 4 || q->naggs < 1 ||
        q->naggs > REPRO_MAX_AGGS)
        return false;
    if (q->n > 0 && !q->keys) return false;
    for (int a = 0; a < q->naggs; ++a) {
        const int ca = q->agg_a[a], cb = q->agg_b[a];
        if (ca < 0 || ca >= REPRO_MAX_COLS || cb >= REPRO_MAX_COLS || !q->out[a]) return false;
        if (q->n > 0 && (!q->cols[ca] || (cb >= 0 && !q->cols[cb]))) return false;
    }
    return true;
}

bool layout_query(const repro_query* q, int64_t chunk_cfg, bool batch_path, QueryLayout* ly) {
    if (!valid_query(q)) return false;
    memset(ly, 0, sizeof(*ly));
    ly->chunk = chunk_cfg > 0 ? chunk_cfg : SERVE_DEFAULT_CHUNK;
    ly->state_bytes = repro_state_bytes(q->num_groups, REPRO_F64, q->L);
    if (ly->state_bytes == 0) return false;
    ly->batch = false;
    if (batch_path && q->n > 0 && q->num_groups <= repro::batchx::slice_limit(q->L)) {
        // the aggregates as batch jobs, sized with stand-in addresses
        repro_batch_job jobs[REPRO_MAX_AGGS];
        void* st[REPRO_MAX_AGGS];
        const double* pr[REPRO_MAX_AGGS];
        for (int a = 0; a < q->naggs; ++a) {
            st[a] = reinterpret_cast<void*>((uintptr_t)SERVE_ALIGN * (a + 1));
            pr[a] = reinterpret_cast<const double*>((uintptr_t)SERVE_ALIGN * (a + 9));
        }
        query_jobs(q, st, pr, jobs);
        const repro_batch_config cfg{SERVE_BATCH_CHUNK, 0, 0};
        size_t wsb = 0, img = 0;
        if (repro::batchx::plan_sizes(jobs, q->naggs, REPRO_I32, REPRO_F64, REPRO_F64, &cfg, &wsb, &img) &&
            img <= SERVE_IMAGE_BYTES) {
            ly->batch = true;
            ly->ws_bytes = wsb;
            ly->image_bytes = img;
        }
    }
    if (!ly->batch && q->n > 0) {
        ly->ws_bytes = repro_workspace_bytes(std::min<int64_t>(q->n, ly->chunk), q->num_groups, REPRO_I32, REPRO_F64,
                                             REPRO_F64, q->L);
        if (ly->ws_bytes == 0) return false;  // no plan for these sizes: refused at submission
    }
    size_t off = 0;
    for (int a = 0; a < q->naggs; ++a) {
        ly->off_state[a] = off;
        off += up(ly->state_bytes);
    }
    for (int a = 0; a < q->naggs; ++a) {
        ly->off_prod[a] = off;
        if (q->agg_b[a] >= 0) off += up((size_t)q->n * 8);
    }
    ly->off_ws = off;
    off += up(ly->ws_bytes);
    ly->total = off;
    return true;
}

struct Pending {
    int64_t ticket;
    repro_query q;
    int bypassed = 0;  // later queries admitted ahead of this one
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    void* image = nullptr;  // pinned host memory: the batch plan of the slot's query
    bool busy = false;
    int64_t ticket = -1;
    size_t off = 0, bytes = 0;
};

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

}  // namespace

struct repro_server {
    unsigned char* arena = nullptr;
    size_t arena_bytes = 0;
    int64_t chunk = SERVE_DEFAULT_CHUNK;
    bool batch_path = true;
    int query_wg = 0;
    int max_bypass = 0;
    Arena alloc;
    std::vector<Slot> slots;
    std::deque<Pending> queue;
    int64_t next_ticket = 0;
};

namespace {

// Enqueues an admitted query's whole pipeline on its slot's stream.
int enqueue_query(repro_server* s, Slot& sl, const repro_query& q, const QueryLayout& ly) {
    hipStream_t st = sl.stream;
    unsigned char* base = s->arena + sl.off;
    const int64_t G = q.num_groups;
    const double* vals[REPRO_MAX_AGGS];
    for (int a = 0; a < q.naggs; ++a) {
        if (!ly.batch && repro_state_init(base + ly.off_state[a], G, REPRO_F64, q.L, st) != REPRO_OK)
            return REPRO_EHIP;
        vals[a] = q.cols[q.agg_a[a]];
        if (q.agg_b[a] >= 0 && q.n > 0) {
            double* prod = reinterpret_cast<double*>(base + ly.off_prod[a]);
            if (launch_mul<double, double>(q.cols[q.agg_a[a]], q.cols[q.agg_b[a]], q.n, prod, st) != REPRO_OK)
                return REPRO_EHIP;
            vals[a] = prod;
        }
    }
    if (ly.batch) {
        // one batch launch: a job per aggregate, states overwritten, sums finalised
        repro_batch_job jobs[REPRO_MAX_AGGS];
        void* states[REPRO_MAX_AGGS];
        for (int a = 0; a < q.naggs; ++a) states[a] = base + ly.off_state[a];
        query_jobs(&q, states, vals, jobs);
        const repro_batch_config cfg{SERVE_BATCH_CHUNK, 0, 0};
        repro_batch_plan plan;
        int rc = repro::batchx::plan_into(jobs, q.naggs, REPRO_I32, REPRO_F64, REPRO_F64, &cfg, sl.image,
                                          SERVE_IMAGE_BYTES, base + ly.off_ws, ly.ws_bytes, &plan);
        if (rc != REPRO_OK) return rc;
        if (s->query_wg > 0 && plan.grid > s->query_wg) plan.grid = s->query_wg;  // share the CUs between slots
        if (hipMemcpyAsync(base + ly.off_ws, sl.image, ly.image_bytes, hipMemcpyHostToDevice, st) != hipSuccess)
            return REPRO_EHIP;
        if ((rc = repro::batchx::launch(&plan, q.status, st)) != REPRO_OK) return rc;
        return hipEventRecord(sl.done, st) == hipSuccess ? REPRO_OK : REPRO_EHIP;
    }
    for (int64_t r0 = 0; r0 < q.n; r0 += ly.chunk) {
        const int64_t m = std::min<int64_t>(ly.chunk, q.n - r0);
        for (int a = 0; a < q.naggs; ++a) {
            const int rc = repro_groupby_sum(q.keys + r0, REPRO_I32, vals[a] + r0, REPRO_F64, m, G, REPRO_F64, q.L,
                                             base + ly.off_state[a], base + ly.off_ws, ly.ws_bytes, q.status, st);
            if (rc != REPRO_OK) return rc;
        }
    }
    for (int a = 0; a < q.naggs; ++a)
        if (repro_finalize(base + ly.off_state[a], G, REPRO_F64, q.L, q.out[a], st) != REPRO_OK) return REPRO_EHIP;
    if (hipEventRecord(sl.done, st) != hipSuccess) return REPRO_EHIP;
    return REPRO_OK;
}

}  // namespace

extern "C" {

int repro_mul(const void* a, repro_scalar_t at, const void* b, repro_scalar_t bt, int64_t n, double* out,
              hipStream_t stream) {
    if (n < 0 || (at != REPRO_F32 && at != REPRO_F64) || (bt != REPRO_F32 && bt != REPRO_F64)) return REPRO_EINVAL;
    if (n == 0) return REPRO_OK;
    if (!a || !b || !out) return REPRO_EINVAL;
    if (at == REPRO_F64)
        return bt == REPRO_F64 ? launch_mul<double, double>(a, b, n, out, stream)
                               : launch_mul<double, float>(a, b, n, out, stream);
    return bt == REPRO_F64 ? launch_mul<float, double>(a, b, n, out, stream)
                           : launch_mul<float, float>(a, b, n, out, stream);
}

size_t repro_query_bytes(const repro_query* q, const repro_server_config* cfg) {
    QueryLayout ly;
    if (!layout_query(q, cfg ? cfg->chunk_rows : 0, !(cfg && cfg->no_batch_path), &ly)) return 0;
    return ly.total;
}

double repro_server_clock(void) { return now_s(); }

int repro_server_create(void* arena, size_t arena_bytes, const repro_server_config* cfg, repro_server** srv) {
    if (!srv || !arena || (uintptr_t)arena % SERVE_ALIGN != 0 || arena_bytes < SERVE_ALIGN) return REPRO_EINVAL;
    const int nslots = cfg ? cfg->slots : 4;
    if (nslots < 1 || nslots > 64 ||
        (cfg && (cfg->chunk_rows < 0 || cfg->query_workgroups < 0 || cfg->max_bypass < 0)))
        return REPRO_EINVAL;
    repro_server* s = new repro_server();
    s->arena = static_cast<unsigned char*>(arena);
    s->arena_bytes = arena_bytes / SERVE_ALIGN * SERVE_ALIGN;
    s->chunk = (cfg && cfg->chunk_rows > 0) ? cfg->chunk_rows : SERVE_DEFAULT_CHUNK;
    s->batch_path = !(cfg && cfg->no_batch_path);
    s->query_wg = cfg ? cfg->query_workgroups : 0;
    s->max_bypass = cfg ? cfg->max_bypass : 0;
    s->alloc.init(s->arena_bytes);
    s->slots.resize(nslots);
    for (Slot& sl : s->slots) {
        if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess ||
            hipHostMalloc(&sl.image, SERVE_IMAGE_BYTES, hipHostMallocDefault) != hipSuccess) {
            repro_server_destroy(s);
            return REPRO_EHIP;
        }
    }
    *srv = s;
    return REPRO_OK;
}

int repro_server_submit(repro_server* s, const repro_query* q, int64_t* ticket) {
    if (!s) return REPRO_EINVAL;
    QueryLayout ly;
    if (!layout_query(q, s->chunk, s->batch_path, &ly) || up(ly.total) > s->arena_bytes) return REPRO_EINVAL;
    Pending p;
    p.ticket = s->next_ticket++;
    p.q = *q;
    s->queue.push_back(p);
    if (ticket) *ticket = p.ticket;
    return REPRO_OK;
}

int repro_server_poll(repro_server* s, int64_t* tickets, double* times, int cap, int* ndone, int* nqueued,
                      int* nrunning, int64_t* dropped) {
    if (!s || cap < 0) return REPRO_EINVAL;
    int rc = REPRO_OK;
    int done = 0;
    if (dropped) *dropped = -1;
    // retire: a finished query is reported and its slot freed only while
    // there is room in the caller's arrays; the others stay busy and are
    // reported by a later poll
    for (Slot& sl : s->slots) {
        if (!sl.busy || done >= cap) continue;
        const hipError_t e = hipEventQuery(sl.done);
        if (e == hipErrorNotReady) continue;
        if (e != hipSuccess) {
            rc = REPRO_EHIP;
            break;
        }
        if (tickets) tickets[done] = sl.ticket;
        if (times) times[done] = now_s();
        ++done;
        s->alloc.release(sl.off, sl.bytes);
        sl.busy = false;
        sl.ticket = -1;
    }
    // admit in arrival order while a slot is free: the first queued query
    // whose memory fits; one that does not fit is passed by later ones at
    // most max_bypass times, then admission waits for it (no starvation)
    while (rc == REPRO_OK && !s->queue.empty()) {
        Slot* free_slot = nullptr;
        for (Slot& sl : s->slots)
            if (!sl.busy) {
                free_slot = &sl;
                break;
            }
        if (!free_slot) break;
        auto pick = s->queue.end();
        QueryLayout ly;
        size_t off = 0;
        for (auto it = s->queue.begin(); it != s->queue.end(); ++it) {
            if (!layout_query(&it->q, s->chunk, s->batch_path, &ly)) {  // validated at submission: cannot happen
                rc = REPRO_EINVAL;
                break;
            }
            if (s->alloc.alloc(ly.total, &off)) {
                pick = it;
                break;
            }
            if (it->bypassed >= s->max_bypass) break;  // aged: wait for its memory
        }
        if (pick == s->queue.end()) break;
        for (auto it = s->queue.begin(); it != pick; ++it) ++it->bypassed;
        free_slot->busy = true;
        free_slot->ticket = pick->ticket;
        free_slot->off = off;
        free_slot->bytes = ly.total;
        const repro_query q = pick->q;
        s->queue.erase(pick);
        if (enqueue_query(s, *free_slot, q, ly) != REPRO_OK) {
            // drop the query: let what was enqueued finish before its memory
            // and slot are reused, report its ticket and stop admitting
            (void)hipStreamSynchronize(free_slot->stream);
            s->alloc.release(free_slot->off, free_slot->bytes);
            if (dropped) *dropped = free_slot->ticket;
            free_slot->busy = false;
            free_slot->ticket = -1;
            rc = REPRO_EHIP;
        }
    }
    if (ndone) *ndone = done;
    if (nqueued) *nqueued = (int)s->queue.size();
    if (nrunning) {
        int r = 0;
        for (const Slot& sl : s->slots) r += sl.busy;
        *nrunning = r;
    }
    return rc;
}

int repro_server_destroy(repro_server* s) {
    if (!s) return REPRO_EINVAL;
    int rc = REPRO_OK;
    for (Slot& sl : s->slots) {
        if (sl.stream) {
            if (hipStreamSynchronize(sl.stream) != hipSuccess) rc = REPRO_EHIP;
            (void)hipStreamDestroy(sl.stream);
        }
        if (sl.done) (void)hipEventDestroy(sl.done);
        if (sl.image) (void)hipHostFree(sl.image);
    }
    delete s;
    return rc;
}

}  // extern "C"
