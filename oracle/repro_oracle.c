/*
 * repro_oracle.c -- CPU oracle for reproducible GroupBy-SUM into repro<T,L>.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or constant with the HIP library: every constant below is
 * restated here from the paper.
 *
 * It is deliberately plain and slow: two passes over the rows (the
 * "maximum absolute value first" scheme the paper mentions in Sec. III-B as
 * the obvious alternative to on-the-fly level shifting), exact integer level
 * sums in __int128, and the canonical state written out at the end.
 *
 * Paper: Mueller, Arteaga, Hoefler, Alonso, "Reproducible Floating-Point
 * Aggregation in RDBMSs" (arXiv 1802.09883).  Sections cited below:
 *   Sec. II-B   floating-point numbers, ufp/ulp
 *   Sec. III-B  error-free transformation (EFT)
 *   Sec. III-C  RSum, Alg. 2 (levels, extractors, carry bits, finalisation
 *               equation)
 *   Sec. IV     the repro<ScalarT,L> type and its operator+=(repro)
 *
 * Readings taken where the paper is silent or ambiguous (each one is listed
 * with its justification in the design notes of the repository):
 *   (R1) a level shift is needed when |b| >= 2^(W-1) * ulp(S^(1)) (Alg. 2);
 *   (R2) the contribution at a level is round-half-even of r / g, the same
 *        for every state (extracting with the constant 1.5*2^E);
 *   (R3) extractor exponents sit on a fixed lattice E_j = B + j*W with
 *        j >= L-1, B = emin of the format;
 *   (R5) carry counts are int64 and states are kept canonical;
 *   (R6) finalisation rounds each level once, then adds the levels from the
 *        last to the first;
 *   (R7) NaN/Inf and out-of-domain values are skipped with a status bit;
 *   (R8) keys are dense ids in [0, num_groups).
 *
 * Parity status: every function here is pinned by tests against the paper's
 * worked examples, closed forms, invariants and an independent exact
 * big-integer model of the one-pass algorithm (Alg. 2).  The absolute bit
 * pattern on general IEEE inputs follows from readings R1-R8.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef __int128 i128;
typedef unsigned __int128 u128;

/* status bits (same meaning as the library's device status word) */
#define ORC_ERR_KEY 1u
#define ORC_ERR_NONFINITE 2u
#define ORC_ERR_RANGE 4u

/*
 * A format: m fraction bits (ulp(x) = 2^(E-m), Sec. III-A), level spacing W
 * (Sec. III-C: W = 18 for float, 40 for double), lattice base B and the
 * largest lattice index jmax whose extractor 1.5*2^E_j is still finite;
 * emin/emax: exponent range of the format (for the final rounding).
 */
typedef struct {
    int m, W, B, jmax, emin, emax;
} orc_fmt;

static const orc_fmt FMT_DOUBLE = {52, 40, -1022, 51, -1022, 1023};
static const orc_fmt FMT_FLOAT = {23, 18, -126, 14, -126, 127};

/* ---------------------------------------------------------------- helpers */

static int64_t floor_div_i64(int64_t a, int64_t b) /* b > 0 */
{
    int64_t q = a / b;
    if ((a % b) != 0 && a < 0) q -= 1;
    return q;
}

static int ceil_div_int(int a, int b) /* b > 0 */
{
    return (int)(-floor_div_i64(-(int64_t)a, (int64_t)b));
}

/* e with |b| in [2^e, 2^(e+1)); b finite and nonzero (subnormals included) */
static int exponent_of(double b)
{
    int e;
    frexp(b, &e); /* b = f * 2^e, |f| in [0.5, 1) */
    return e - 1;
}

/* extractor exponent at lattice index j */
static int lattice_E(const orc_fmt* f, int j) { return f->B + j * f->W; }

/*
 * Smallest lattice index j whose top-level extractor can take b, i.e. the
 * smallest j with |b| < 2^(W-1) * ulp(1.5 * 2^E_j) = 2^(W-1+E_j-m)
 * (the level-shift test of Alg. 2, reading R1).  With |b| < 2^(e+1) this is
 * E_j >= e + m - W + 2.
 */
static int orc_jreq_fmt(double b, const orc_fmt* f)
{
    int e = exponent_of(b);
    return ceil_div_int(e + f->m - f->W + 2 - f->B, f->W);
}

/*
 * Extraction of one value at top index `top` (Sec. III-B/III-C): level l
 * (0 = first level) has grid g_l = 2^(E_{top-l} - m); its contribution is
 * the nearest multiple of g_l to the running remainder, ties to the even
 * multiple (reading R2); the remainder passes to the next level and the
 * last remainder is dropped.  All operations are exact in binary64: the
 * scaling is by powers of two and |r/g| < 2^(W-1).
 */
static void extract(double b, int top, int L, const orc_fmt* f, int64_t* k)
{
    double r = b;
    for (int l = 0; l < L; ++l) {
        int E = lattice_E(f, top - l);
        double q = nearbyint(ldexp(r, f->m - E)); /* default mode: half-even */
        k[l] = (int64_t)q;
        r = r - ldexp(q, E - f->m);
    }
}

/* classify one row: returns 1 if it is deposited; ORs error bits */
static int classify(int64_t key, int64_t G, double v, const orc_fmt* f, uint32_t* st, int* jr)
{
    int ok = 1;
    if (key < 0 || key >= G) {
        *st |= ORC_ERR_KEY;
        ok = 0;
    }
    if (!isfinite(v)) {
        *st |= ORC_ERR_NONFINITE;
        return 0;
    }
    if (v == 0.0) {
        *jr = -1; /* zero imposes no level and contributes nothing */
        return ok;
    }
    *jr = orc_jreq_fmt(v, f);
    if (*jr > f->jmax) {
        *st |= ORC_ERR_RANGE;
        return 0;
    }
    return ok;
}

/* --------------------------------------------------------- canonical form */

/*
 * Canonical state of one level (Sec. III-C, usable range of S and carry
 * counter C; reading R5): with D = 2^(m-2) (one carry unit 0.25*ufp(S) in
 * units of g), C = floor(K / D) and S = 1.5*2^E + (K - C*D) * g, so that S
 * lies in [1.5, 1.75) * 2^E.
 */
static int encode_level(i128 K, int E, const orc_fmt* f, double* S, int64_t* C)
{
    i128 D = (i128)1 << (f->m - 2);
    i128 q = K / D;
    if (K % D != 0 && K < 0) q -= 1;
    i128 lo = K - q * D;
    if (q > (i128)INT64_MAX || q < (i128)INT64_MIN) return -1;
    *C = (int64_t)q;
    *S = ldexp(1.5, E) + ldexp((double)(int64_t)lo, E - f->m);
    return 0;
}

static int decode_level(double S, int64_t C, int E, const orc_fmt* f, i128* K)
{
    if (!(S > 0) || exponent_of(S) != E) return -1;
    double lo = ldexp(S - ldexp(1.5, E), f->m - E); /* exact (Sterbenz) */
    if (lo < 0 || lo >= ldexp(1.0, f->m - 2)) return -1;
    *K = (i128)C * ((i128)1 << (f->m - 2)) + (i128)(int64_t)lo;
    return 0;
}

/*
 * State buffer layout (documented with the library interface): SoA,
 * S[l][g] of type T for l = 0..L-1 (level 0 is the first, largest level),
 * then, at the next multiple of 8 bytes, C[l][g] as int64.
 */
static size_t s_block_bytes(int64_t G, int T64, int L)
{
    size_t b = (size_t)G * (size_t)L * (T64 ? 8u : 4u);
    return (b + 7u) & ~(size_t)7u;
}

size_t orc_state_bytes(int64_t G, int T64, int L)
{
    return s_block_bytes(G, T64, L) + (size_t)G * (size_t)L * 8u;
}

static double get_S(const void* st, int64_t G, int T64, int l, int64_t g)
{
    if (T64) return ((const double*)st)[(int64_t)l * G + g];
    return (double)((const float*)st)[(int64_t)l * G + g];
}

static void put_S(void* st, int64_t G, int T64, int l, int64_t g, double v)
{
    if (T64)
        ((double*)st)[(int64_t)l * G + g] = v;
    else
        ((float*)st)[(int64_t)l * G + g] = (float)v; /* exact: v is representable */
}

static int64_t* C_ptr(void* st, int64_t G, int T64, int L)
{
    return (int64_t*)((char*)st + s_block_bytes(G, T64, L));
}

static const int64_t* C_cptr(const void* st, int64_t G, int T64, int L)
{
    return (const int64_t*)((const char*)st + s_block_bytes(G, T64, L));
}

static int write_group(void* st, int64_t G, int T64, int L, int64_t g, int top, const i128* K)
{
    const orc_fmt* f = T64 ? &FMT_DOUBLE : &FMT_FLOAT;
    int64_t* C = C_ptr(st, G, T64, L);
    for (int l = 0; l < L; ++l) {
        double S;
        int64_t c;
        if (encode_level(K[l], lattice_E(f, top - l), f, &S, &c)) return -1;
        put_S(st, G, T64, l, g, S);
        C[(int64_t)l * G + g] = c;
    }
    return 0;
}

static int read_group(const void* st, int64_t G, int T64, int L, int64_t g, int* top, i128* K)
{
    const orc_fmt* f = T64 ? &FMT_DOUBLE : &FMT_FLOAT;
    const int64_t* C = C_cptr(st, G, T64, L);
    double S0 = get_S(st, G, T64, 0, g);
    if (!(S0 > 0)) return -1;
    int E1 = exponent_of(S0);
    if ((E1 - f->B) % f->W != 0) return -1;
    int j = (E1 - f->B) / f->W;
    if (j < L - 1 || j > f->jmax) return -1;
    *top = j;
    for (int l = 0; l < L; ++l)
        if (decode_level(get_S(st, G, T64, l, g), C[(int64_t)l * G + g], lattice_E(f, j - l), f, &K[l]))
            return -1;
    return 0;
}

/* ----------------------------------------------------------------- API */

/* empty state: top at the lowest allowed index, all level sums zero */
int orc_state_init(void* states, int64_t G, int T64, int L)
{
    i128 K[8] = {0};
    if (L < 1 || L > 4 || G < 1) return -1;
    for (int64_t g = 0; g < G; ++g)
        if (write_group(states, G, T64, L, g, L - 1, K)) return -1;
    return 0;
}

static double load_val(const void* vals, int val64, int64_t i)
{
    return val64 ? ((const double*)vals)[i] : (double)((const float*)vals)[i];
}

static int64_t load_key(const void* keys, int key64, int64_t i)
{
    return key64 ? ((const int64_t*)keys)[i] : (int64_t)((const int32_t*)keys)[i];
}

/*
 * GroupBy-SUM of rows [0, n) from scratch into fresh canonical states.
 * Pass 1: per-group top index j* = max(L-1, max_b jreq(b)).  Pass 2: per-row
 * extraction at j*, exact integer level sums.  Then the canonical form.
 */
static int groupby_fresh(const void* keys, int key64, const void* vals, int val64, int64_t n, int64_t G,
                         int T64, int L, void* states, uint32_t* status)
{
    const orc_fmt* f = T64 ? &FMT_DOUBLE : &FMT_FLOAT;
    uint32_t st = 0;
    int* top = (int*)malloc(sizeof(int) * (size_t)G);
    i128* K = (i128*)calloc((size_t)G * (size_t)L, sizeof(i128));
    if (!top || !K) {
        free(top);
        free(K);
        return -1;
    }
    for (int64_t g = 0; g < G; ++g) top[g] = L - 1;

    for (int64_t i = 0; i < n; ++i) {
        int jr = -1;
        int64_t key = load_key(keys, key64, i);
        if (!classify(key, G, load_val(vals, val64, i), f, &st, &jr)) continue;
        if (jr > top[key]) top[key] = jr;
    }
    for (int64_t i = 0; i < n; ++i) {
        int jr = -1;
        int64_t key = load_key(keys, key64, i);
        double v = load_val(vals, val64, i);
        if (!classify(key, G, v, f, &st, &jr) || v == 0.0) continue;
        int64_t k[8];
        extract(v, top[key], L, f, k);
        for (int l = 0; l < L; ++l) K[key * L + l] += (i128)k[l];
    }
    int rc = 0;
    for (int64_t g = 0; g < G && rc == 0; ++g) rc = write_group(states, G, T64, L, g, top[g], &K[g * L]);
    free(top);
    free(K);
    if (status) *status |= st;
    return rc;
}

/*
 * operator+=(repro) (Sec. IV, and the merge step of Alg. 4): the combined
 * top is the larger one; the levels of the other state move down by the
 * difference (its lowest levels fall off), then level sums add exactly.
 */
static void merge_group(int* top_d, i128* Kd, int top_s, const i128* Ks, int L)
{
    i128 a[8], b[8];
    int J = top_d[0] > top_s ? top_d[0] : top_s;
    for (int l = 0; l < L; ++l) {
        int ld = l - (J - top_d[0]), ls = l - (J - top_s);
        a[l] = ld >= 0 ? Kd[ld] : 0;
        b[l] = ls >= 0 ? Ks[ls] : 0;
    }
    for (int l = 0; l < L; ++l) Kd[l] = a[l] + b[l];
    top_d[0] = J;
}

int orc_merge(void* dst, const void* src, int64_t G, int T64, int L)
{
    if (L < 1 || L > 4 || G < 1) return -1;
    for (int64_t g = 0; g < G; ++g) {
        int td, ts;
        i128 Kd[8], Ks[8];
        if (read_group(dst, G, T64, L, g, &td, Kd) || read_group(src, G, T64, L, g, &ts, Ks)) return -2;
        merge_group(&td, Kd, ts, Ks, L);
        if (write_group(dst, G, T64, L, g, td, Kd)) return -3;
    }
    return 0;
}

/*
 * Accumulate rows into existing canonical states (the resumable form of
 * Alg. 2: load state, add values, store state).  Defined as the merge of
 * the existing states with the states of the new rows alone.
 */
int orc_groupby_sum(const void* keys, int key64, const void* vals, int val64, int64_t n, int64_t G, int T64,
                    int L, void* states, uint32_t* status)
{
    if (L < 1 || L > 4 || G < 1 || n < 0 || (val64 && !T64)) return -1;
    void* fresh = malloc(orc_state_bytes(G, T64, L));
    if (!fresh) return -1;
    int rc = groupby_fresh(keys, key64, vals, val64, n, G, T64, L, fresh, status);
    if (rc == 0) rc = orc_merge(states, fresh, G, T64, L);
    free(fresh);
    return rc;
}

/* ------------------------------------------------------------ threaded */

typedef struct {
    const void *keys, *vals;
    int key64, val64, T64, L;
    int64_t n, G;
    void* states;
    uint32_t status;
    int rc;
} orc_job;

static void* run_job(void* p)
{
    orc_job* j = (orc_job*)p;
    j->rc = orc_state_init(j->states, j->G, j->T64, j->L);
    if (j->rc == 0) j->rc = groupby_fresh(j->keys, j->key64, j->vals, j->val64, j->n, j->G, j->T64, j->L, j->states, &j->status);
    return NULL;
}

/*
 * The same result computed on `nthreads` row chunks in parallel, then merged
 * (the thread-level parallelism of Alg. 4 with F = 1).  Bits are identical to
 * orc_groupby_sum by construction; tests check that too.
 */
int orc_groupby_sum_threads(const void* keys, int key64, const void* vals, int val64, int64_t n, int64_t G,
                            int T64, int L, void* states, uint32_t* status, int nthreads)
{
    if (nthreads < 1) nthreads = 1;
    if (L < 1 || L > 4 || G < 1 || n < 0 || (val64 && !T64)) return -1;
    orc_job* jobs = (orc_job*)calloc((size_t)nthreads, sizeof(orc_job));
    pthread_t* th = (pthread_t*)calloc((size_t)nthreads, sizeof(pthread_t));
    int rc = 0;
    if (!jobs || !th) rc = -1;
    int64_t chunk = (n + nthreads - 1) / nthreads;
    for (int t = 0; t < nthreads && rc == 0; ++t) {
        int64_t b = chunk * t, e = b + chunk;
        if (b > n) b = n;
        if (e > n) e = n;
        orc_job* j = &jobs[t];
        j->keys = (const char*)keys + b * (key64 ? 8 : 4);
        j->vals = (const char*)vals + b * (val64 ? 8 : 4);
        j->key64 = key64;
        j->val64 = val64;
        j->T64 = T64;
        j->L = L;
        j->n = e - b;
        j->G = G;
        j->states = malloc(orc_state_bytes(G, T64, L));
        if (!j->states) rc = -1;
    }
    int started = 0;
    for (int t = 0; t < nthreads && rc == 0; ++t, ++started)
        if (pthread_create(&th[t], NULL, run_job, &jobs[t])) rc = -1;
    for (int t = 0; t < started; ++t) pthread_join(th[t], NULL);
    for (int t = 0; t < nthreads && rc == 0; ++t) {
        rc = jobs[t].rc;
        if (rc == 0) rc = orc_merge(states, jobs[t].states, G, T64, L);
        if (status) *status |= jobs[t].status;
    }
    for (int t = 0; t < nthreads && jobs; ++t) free(jobs[t].states);
    free(jobs);
    free(th);
    return rc;
}

/* ------------------------------------------------------------ finalize */

static int bitlen_u128(u128 x)
{
    int n = 0;
    while (x) {
        ++n;
        x >>= 1;
    }
    return n;
}

/*
 * Round the exact value K * 2^s to the nearest number of format f (ties to
 * even), with gradual underflow below 2^emin and overflow to +-Inf: one
 * IEEE rounding (reading R6).  Returned as a double holding that number.
 */
static double round_to_fmt(i128 K, int s, const orc_fmt* f)
{
    if (K == 0) return 0.0;
    int neg = K < 0;
    u128 a = neg ? (u128)(-K) : (u128)K;
    int nb = bitlen_u128(a);
    int lead = nb - 1 + s;                  /* exponent of the leading bit */
    int u = lead - f->m;                    /* ulp exponent if normal */
    if (u < f->emin - f->m) u = f->emin - f->m; /* subnormal: fixed ulp */
    int shift = u - s;
    u128 q;
    if (shift <= 0) {
        q = a; /* exact */
        u = s;
    } else if (shift >= 128) {
        q = 0; /* far below half an ulp */
    } else {
        q = a >> shift;
        u128 rem = a - (q << shift);
        u128 half = (u128)1 << (shift - 1);
        if (rem > half || (rem == half && (q & 1))) q += 1;
    }
    double r = ldexp((double)(uint64_t)q, u); /* q <= 2^(m+1): exact */
    if (fabs(r) >= ldexp(1.0, f->emax + 1)) r = INFINITY;
    return neg ? -r : r;
}

/*
 * Finalisation (equation in Sec. III-C, reading R6): each level's exact
 * value K_l * g_l is rounded once to T, then the levels are added in T
 * from the last level to the first.  An empty group gives +0.0.
 */
int orc_finalize(const void* states, int64_t G, int T64, int L, void* out)
{
    const orc_fmt* f = T64 ? &FMT_DOUBLE : &FMT_FLOAT;
    for (int64_t g = 0; g < G; ++g) {
        int top;
        i128 K[8];
        if (read_group(states, G, T64, L, g, &top, K)) return -2;
        if (T64) {
            double acc = round_to_fmt(K[L - 1], lattice_E(f, top - (L - 1)) - f->m, f);
            for (int l = L - 2; l >= 0; --l) acc = acc + round_to_fmt(K[l], lattice_E(f, top - l) - f->m, f);
            ((double*)out)[g] = acc + 0.0; /* -0 cannot occur; keeps +0 */
        } else {
            float acc = (float)round_to_fmt(K[L - 1], lattice_E(f, top - (L - 1)) - f->m, f);
            for (int l = L - 2; l >= 0; --l) acc = acc + (float)round_to_fmt(K[l], lattice_E(f, top - l) - f->m, f);
            ((float*)out)[g] = acc + 0.0f;
        }
    }
    return 0;
}

/* ------------------------------------------------- derived aggregates */

/*
 * AVG, sample VAR and sample STDDEV of every group from its finalised
 * SUM(x), SUM(x*x) and exact COUNT: the aggregates that reduce to SUM
 * (Sec. I).  The paper fixes no formula; the one taken here is the textbook
 * sample variance (sum of squares minus sum times mean, over count - 1),
 * evaluated as one fixed sequence of IEEE binary64 operations, each rounded
 * to nearest even, with no fused multiply-add:
 *     avg = s / c;   var = (q - s * avg) / (c - 1);   sd = sqrt(var).
 * Because every input is reproducible and the sequence is fixed, so are the
 * outputs.  A group with no row has avg = NaN; fewer than two rows give
 * var = sd = NaN.  Any output pointer may be NULL.
 */
int orc_derive_stats(const double* sum, const double* sumsq, const int64_t* count, int64_t G, double* avg,
                     double* var, double* sd)
{
    if (G < 1 || !sum || !sumsq || !count) return -1;
    for (int64_t g = 0; g < G; ++g) {
        double c = (double)count[g]; /* exact below 2^53 rows */
        double s = sum[g], q = sumsq[g];
        double m = s / c;
        double p = s * m;
        double u = q - p;
        double v = u / (c - 1.0);
        if (avg) avg[g] = count[g] > 0 ? m : NAN;
        if (var) var[g] = count[g] > 1 ? v : NAN;
        if (sd) sd[g] = count[g] > 1 ? sqrt(v) : NAN; /* IEEE sqrt: correctly rounded */
    }
    return 0;
}

/* --------------------------------------------- generic-format single sum */

/*
 * Reproducible sum of one stream in an arbitrary binary format given by
 * (m, W, B, jmax, emin, emax), used for the paper's toy-format examples and
 * for IEEE formats alike.  Values are passed as binary64 numbers that are
 * representable in the format.  Outputs: the top index, the exact level sums
 * (as high/low 64-bit halves) and the finalised value in that format.  Level
 * additions in toy formats are done exactly in binary64 and rounded once to
 * the format (their exact sums are small).
 */
int orc_sum_fmt(const double* v, int64_t n, int m, int W, int B, int jmax, int emin, int emax, int L,
                int* top_out, int64_t* K_hi, uint64_t* K_lo, double* result)
{
    orc_fmt f = {m, W, B, jmax, emin, emax};
    if (L < 1 || L > 8 || W < 1 || m < 2 || W > m) return -1;
    int top = L - 1;
    for (int64_t i = 0; i < n; ++i) {
        if (!isfinite(v[i])) return -2;
        if (v[i] == 0.0) continue;
        int j = orc_jreq_fmt(v[i], &f);
        if (j > jmax) return -3;
        if (j > top) top = j;
    }
    i128 K[8] = {0};
    for (int64_t i = 0; i < n; ++i) {
        if (v[i] == 0.0) continue;
        int64_t k[8];
        extract(v[i], top, L, &f, k);
        for (int l = 0; l < L; ++l) K[l] += k[l];
    }
    double acc = round_to_fmt(K[L - 1], lattice_E(&f, top - (L - 1)) - m, &f);
    for (int l = L - 2; l >= 0; --l) {
        double q = round_to_fmt(K[l], lattice_E(&f, top - l) - m, &f);
        double ex = acc + q; /* exact for the small toy values; IEEE: fl() */
        if (m == 52 && emin == -1022)
            acc = ex;
        else {
            int e2;
            double fr = frexp(ex, &e2);
            acc = (ex == 0.0) ? 0.0 : round_to_fmt((i128)(int64_t)ldexp(fr, 60), e2 - 60, &f);
        }
    }
    *top_out = top;
    for (int l = 0; l < L; ++l) {
        K_hi[l] = (int64_t)(K[l] >> 64);
        K_lo[l] = (uint64_t)K[l];
    }
    *result = acc + 0.0;
    return 0;
}

/* one-value helpers, exported for tests */
int orc_jreq(double b, int m, int W, int B)
{
    orc_fmt f = {m, W, B, 1 << 20, -1 << 20, 1 << 20};
    return orc_jreq_fmt(b, &f);
}

void orc_extract(double b, int top, int L, int m, int W, int B, int64_t* k)
{
    orc_fmt f = {m, W, B, 1 << 20, -1 << 20, 1 << 20};
    extract(b, top, L, &f, k);
}

double orc_round(int64_t K_hi, uint64_t K_lo, int s, int m, int emin, int emax)
{
    orc_fmt f = {m, 1, emin, 0, emin, emax};
    i128 K = ((i128)K_hi << 64) | (i128)K_lo;
    return round_to_fmt(K, s, &f);
}

/* canonical (S, C) of one level with exact sum K at extractor exponent E */
int orc_encode(int64_t K_hi, uint64_t K_lo, int E, int m, double* S, int64_t* C)
{
    orc_fmt f = {m, 1, -1 << 20, 0, -1 << 20, 1 << 20};
    i128 K = ((i128)K_hi << 64) | (i128)K_lo;
    return encode_level(K, E, &f, S, C);
}
