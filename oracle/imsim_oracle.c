/*
 * CPU oracle for Monte Carlo simulation of the independent cascade (IC) and
 * linear threshold (LT) diffusion models.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no source
 * with the device path: its hash, encoders and simulators are written here
 * from their definitions, plainly and slowly, so that a reader can check them
 * against the paper by eye.
 *
 * Semantics (paper Section 2, "Diffusion Models"):
 *   IC: a node that becomes active at step t tries each out-arc (u,v) once,
 *       at step t+1, succeeding with probability p_uv.  With the coin of every
 *       (trial, arc) fixed in advance, the final active set of a trial is the
 *       set of nodes reachable from S over the arcs whose coin succeeded
 *       (Kempe-Kleinberg-Tardos live-edge view); the order of attempts cannot
 *       matter because each coin is used at most once.
 *   LT: every node v draws a threshold theta_v; in synchronous steps, v turns
 *       active when the total weight of its active in-neighbours reaches
 *       theta_v.  The run stops when a step activates nothing.
 * Frontier traversal (Section 3, "Algorithms", locality observation): only
 * out-neighbours of the nodes activated in the previous step are examined.
 *
 * Fixed-point readings (the paper states real-valued p and theta):
 *   IC threshold  thr = min(floor(p * 2^32), 2^32 - 1); thr == 2^32 - 1 means
 *                 the arc is always live; otherwise live iff coin < thr.
 *   LT weight     w = floor(w_real * 2^32) as uint64; per-node in-sum <= 2^32.
 *   LT threshold  theta = (h + 1) / 2^32 with h the 32-bit hash, so "weight at
 *                 least theta" reads  sum_fp >= h + 1,  i.e.  sum_fp > h.
 * Counter-based hash: Philox4x64 with 10 rounds (Salmon, Moraes, Dror, Shaw,
 * "Parallel Random Numbers: As Easy as 1, 2, 3", SC'11), counter
 * (id, t >> 3, 0, 0), key (rng_seed, domain); trial t takes the 32-bit half
 * (t & 1) of output word (t & 7) >> 1.  Domain 1 = IC arc coins keyed by the
 * out-CSR arc index, domain 2 = LT node thresholds keyed by node id.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { ORC_OK = 0, ORC_E_ARG = -1, ORC_E_GRAPH = -2, ORC_E_WSUM = -3, ORC_E_SEED = -4, ORC_E_OOM = -5 };

/* ------------------------------------------------------------------ hash */

/* Philox4x64-10 as published: two 64x64->128 multiplies per round, the
 * high halves xor-ed with the other counter words and the round key, the key
 * bumped by the Weyl constants between rounds. */
void orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4])
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
    uint64_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += W0;
            k1 += W1;
        }
        unsigned __int128 p0 = (unsigned __int128)M0 * x0;
        unsigned __int128 p1 = (unsigned __int128)M1 * x2;
        uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        uint64_t y0 = hi1 ^ x1 ^ k0;
        uint64_t y1 = lo1;
        uint64_t y2 = hi0 ^ x3 ^ k1;
        uint64_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

uint32_t orc_hash32(uint64_t rng_seed, uint64_t domain, uint64_t trial, uint64_t id)
{
    uint64_t ctr[4] = { id, trial >> 3, 0, 0 };
    uint64_t key[2] = { rng_seed, domain };
    uint64_t out[4];
    orc_philox4x64_10(ctr, key, out);
    uint64_t word = out[(trial & 7) >> 1];
    return (trial & 1) ? (uint32_t)(word >> 32) : (uint32_t)word;
}

/* -------------------------------------------------------------- encoders */

/* IC: thr = min(floor(p * 2^32), 2^32 - 1); p outside [0, 1] or NaN fails. */
int orc_encode_p(const double* p, int64_t m, uint32_t* thr)
{
    for (int64_t e = 0; e < m; ++e) {
        double x = p[e];
        if (!(x >= 0.0 && x <= 1.0)) return ORC_E_ARG;
        double scaled = floor(ldexp(x, 32));
        thr[e] = scaled >= 4294967295.0 ? 0xFFFFFFFFu : (uint32_t)scaled;
    }
    return ORC_OK;
}

/* LT: w = floor(w_real * 2^32) as uint64; w_real outside [0, 1] fails. */
int orc_encode_w(const double* w, int64_t m, uint64_t* w64)
{
    for (int64_t e = 0; e < m; ++e) {
        double x = w[e];
        if (!(x >= 0.0 && x <= 1.0)) return ORC_E_ARG;
        w64[e] = (uint64_t)floor(ldexp(x, 32));
    }
    return ORC_OK;
}

/* CSR sanity and, for LT, the in-weight bound sum_{u} w_uv <= 2^32 per v
 * (the paper requires the in-neighbour weights of a node to sum to at most 1). */
int orc_validate(int model, int64_t n, const int64_t* offsets, const uint32_t* indices, const uint64_t* w64)
{
    if (n < 0 || offsets[0] != 0) return ORC_E_GRAPH;
    for (int64_t u = 0; u < n; ++u)
        if (offsets[u + 1] < offsets[u]) return ORC_E_GRAPH;
    int64_t m = offsets[n];
    for (int64_t e = 0; e < m; ++e)
        if ((int64_t)indices[e] >= n) return ORC_E_GRAPH;
    if (model == 1) {
        uint64_t* in_sum = calloc((size_t)(n > 0 ? n : 1), sizeof(uint64_t));
        if (!in_sum) return ORC_E_OOM;
        int rc = ORC_OK;
        for (int64_t e = 0; e < m && rc == ORC_OK; ++e) {
            if (w64[e] > (1ULL << 32)) rc = ORC_E_WSUM;
            in_sum[indices[e]] += w64[e];
            if (in_sum[indices[e]] > (1ULL << 32)) rc = ORC_E_WSUM;
        }
        free(in_sum);
        return rc;
    }
    return ORC_OK;
}

/* ------------------------------------------------------------- one trial */

typedef struct {
    int64_t n;
    const int64_t* offsets;
    const uint32_t* indices;
    const uint32_t* thr;  /* IC */
    const uint64_t* w64;  /* LT */
    const uint32_t* seeds;
    int64_t n_seeds;
    uint64_t rng_seed;
} orc_problem;

typedef struct {
    uint32_t* stamp;   /* stamp[v] == cur  <=>  v active in the current trial */
    uint32_t* qstamp;  /* LT: v already queued for the next step */
    uint32_t* tstamp;  /* LT: acc / threshold of v valid in the current trial */
    uint64_t* acc;     /* LT: active in-weight of v, 2^-32 units */
    uint32_t* hth;     /* LT: threshold hash of v */
    uint32_t* level;   /* step at which v became active */
    uint32_t* queue;   /* nodes in activation order */
    uint32_t cur;
} orc_scratch;

static int scratch_init(orc_scratch* s, int64_t n)
{
    size_t nn = (size_t)(n > 0 ? n : 1);
    memset(s, 0, sizeof(*s));
    s->stamp = calloc(nn, sizeof(uint32_t));
    s->qstamp = calloc(nn, sizeof(uint32_t));
    s->tstamp = calloc(nn, sizeof(uint32_t));
    s->acc = calloc(nn, sizeof(uint64_t));
    s->hth = calloc(nn, sizeof(uint32_t));
    s->level = calloc(nn, sizeof(uint32_t));
    s->queue = calloc(nn, sizeof(uint32_t));
    return (s->stamp && s->qstamp && s->tstamp && s->acc && s->hth && s->level && s->queue) ? ORC_OK : ORC_E_OOM;
}

static void scratch_free(orc_scratch* s)
{
    free(s->stamp); free(s->qstamp); free(s->tstamp); free(s->acc);
    free(s->hth); free(s->level); free(s->queue);
}

/* IC trial: breadth-first cascade from the seeds; an arc e = (u, v) out of a
 * node u activated at step l is tried once, and when v is still inactive and
 * the arc's coin succeeds, v becomes active at step l + 1.  Returns the
 * number of active nodes; queue[0..count) lists them. */
static int64_t ic_trial(const orc_problem* P, orc_scratch* s, uint64_t t, uint64_t* exams)
{
    uint32_t cur = s->cur;
    int64_t head = 0, tail = 0;
    for (int64_t i = 0; i < P->n_seeds; ++i) {
        uint32_t v = P->seeds[i];
        if (s->stamp[v] != cur) {
            s->stamp[v] = cur;
            s->level[v] = 0;
            s->queue[tail++] = v;
        }
    }
    uint64_t ex = 0;
    while (head < tail) {
        uint32_t u = s->queue[head++];
        ex += (uint64_t)(P->offsets[u + 1] - P->offsets[u]);
        for (int64_t e = P->offsets[u]; e < P->offsets[u + 1]; ++e) {
            uint32_t v = P->indices[e];
            if (s->stamp[v] == cur) continue;
            uint32_t thr = P->thr[e];
            int live = (thr == 0xFFFFFFFFu) || (orc_hash32(P->rng_seed, 1, t, (uint64_t)e) < thr);
            if (live) {
                s->stamp[v] = cur;
                s->level[v] = s->level[u] + 1;
                s->queue[tail++] = v;
            }
        }
    }
    *exams = ex;
    return tail;
}

/* LT trial: synchronous steps.  Step l processes the nodes activated at
 * step l - 1 (the frontier); each out-arc (u, v) into a still inactive v
 * adds w_uv to v's active in-weight.  Because weights only accumulate, the
 * in-weight seen after the whole frontier is the sum over all active
 * in-neighbours, and v joins step l when that sum exceeds its threshold
 * hash. */
static int64_t lt_trial(const orc_problem* P, orc_scratch* s, uint64_t t, uint64_t* exams)
{
    uint32_t cur = s->cur;
    int64_t tail = 0;
    for (int64_t i = 0; i < P->n_seeds; ++i) {
        uint32_t v = P->seeds[i];
        if (s->stamp[v] != cur) {
            s->stamp[v] = cur;
            s->level[v] = 0;
            s->queue[tail++] = v;
        }
    }
    uint64_t ex = 0;
    int64_t begin = 0;
    uint32_t step = 0;
    while (begin < tail) {
        int64_t end = tail;  /* frontier = queue[begin, end) */
        ++step;
        for (int64_t i = begin; i < end; ++i) {
            uint32_t u = s->queue[i];
            ex += (uint64_t)(P->offsets[u + 1] - P->offsets[u]);
            for (int64_t e = P->offsets[u]; e < P->offsets[u + 1]; ++e) {
                uint32_t v = P->indices[e];
                if (s->stamp[v] == cur) continue;  /* already active */
                if (s->tstamp[v] != cur) {
                    s->tstamp[v] = cur;
                    s->acc[v] = 0;
                    s->hth[v] = orc_hash32(P->rng_seed, 2, t, v);
                }
                s->acc[v] += P->w64[e];
                if (s->acc[v] > (uint64_t)s->hth[v] && s->qstamp[v] != cur) {
                    s->qstamp[v] = cur;
                    s->queue[tail++] = v;
                }
            }
        }
        /* nodes queued during this step become active at its end */
        for (int64_t i = end; i < tail; ++i) {
            s->stamp[s->queue[i]] = cur;
            s->level[s->queue[i]] = step;
        }
        begin = end;
    }
    *exams = ex;
    return tail;
}

/* ------------------------------------------------------- many trials API */

/*
 * Simulate trials t in [t_begin, t_end) of one (graph, parameters, seeds,
 * rng_seed) problem.  model: 0 = IC (param = uint32 thr[m]), 1 = LT (param =
 * uint64 w[m]), both in out-CSR order.  Outputs, each optional (NULL) except
 * trial_counts:
 *   trial_counts[t - t_begin]  number of active nodes, seeds included
 *   exams[t - t_begin]         sum of out-degrees of the active nodes
 *   node_counts[v]             trials of the range in which v was active
 *                              (overwritten)
 *   active_bits[w * n + v]     bit b set iff v active in trial
 *                              t_begin + 64 w + b   (zeroed first)
 *   levels[(t - t_begin) * n + v]  activation step of v, -1 if inactive
 * n_threads <= 0 means one thread.  Trials are independent and every output
 * is an integer sum or bitwise OR over trials, so the outputs do not depend
 * on the thread count.
 */
int orc_simulate(int model, int64_t n, const int64_t* offsets, const uint32_t* indices,
                 const void* param, const uint32_t* seeds, int64_t n_seeds,
                 int64_t t_begin, int64_t t_end, uint64_t rng_seed, int n_threads,
                 uint32_t* trial_counts, uint64_t* exams, uint32_t* node_counts,
                 uint64_t* active_bits, int32_t* levels)
{
    if ((model != 0 && model != 1) || n < 0 || t_begin < 0 || t_end < t_begin || !trial_counts)
        return ORC_E_ARG;
    for (int64_t i = 0; i < n_seeds; ++i)
        if ((int64_t)seeds[i] >= n) return ORC_E_SEED;
    orc_problem P;
    P.n = n; P.offsets = offsets; P.indices = indices;
    P.thr = model == 0 ? (const uint32_t*)param : NULL;
    P.w64 = model == 1 ? (const uint64_t*)param : NULL;
    P.seeds = seeds; P.n_seeds = n_seeds; P.rng_seed = rng_seed;

    int64_t T = t_end - t_begin;
    int64_t W = (T + 63) / 64;
    if (node_counts) memset(node_counts, 0, (size_t)n * sizeof(uint32_t));
    if (active_bits) memset(active_bits, 0, (size_t)(W * n) * sizeof(uint64_t));
    if (n_threads <= 0) n_threads = 1;
    int rc_all = ORC_OK;

#pragma omp parallel num_threads(n_threads)
    {
        orc_scratch s;
        int rc = scratch_init(&s, n);
        if (rc != ORC_OK) {
#pragma omp atomic write
            rc_all = rc;
        }
#pragma omp barrier
        if (rc_all == ORC_OK) {
#pragma omp for schedule(dynamic, 1)
            for (int64_t rel = 0; rel < T; ++rel) {
                uint64_t t = (uint64_t)(t_begin + rel);
                int64_t w = rel / 64, b = rel % 64;
                s.cur += 1;
                uint64_t ex = 0;
                int64_t cnt = model == 0 ? ic_trial(&P, &s, t, &ex) : lt_trial(&P, &s, t, &ex);
                trial_counts[rel] = (uint32_t)cnt;
                if (exams) exams[rel] = ex;
                if (levels) {
                    int32_t* lv = levels + rel * n;
                    for (int64_t v = 0; v < n; ++v) lv[v] = -1;
                    for (int64_t i = 0; i < cnt; ++i) lv[s.queue[i]] = (int32_t)s.level[s.queue[i]];
                }
                for (int64_t i = 0; i < cnt; ++i) {
                    uint32_t v = s.queue[i];
                    if (node_counts) {
#pragma omp atomic update
                        node_counts[v] += 1;
                    }
                    if (active_bits) {
#pragma omp atomic update
                        active_bits[w * n + v] |= 1ULL << b;
                    }
                }
            }
        }
        scratch_free(&s);
    }
    return rc_all;
}

/* Total of the per-trial counts: the numerator of the spread estimate
 * sigma(S) = total / T (Section 2, "Influence Maximization"). */
uint64_t orc_total(const uint32_t* trial_counts, int64_t T)
{
    uint64_t s = 0;
    for (int64_t i = 0; i < T; ++i) s += trial_counts[i];
    return s;
}

int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
