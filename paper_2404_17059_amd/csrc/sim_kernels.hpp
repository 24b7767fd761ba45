// HIP kernels of the IC / LT Monte Carlo simulator for gfx950 (wave64).
//
// Trial-bit-parallel state: for trial word w (trials 64w .. 64w+63) every node
// v owns one uint64 A[w*n + v] whose bit b says "v active in trial 64w + b".
// A wavefront works on one word at a time with lane b standing for trial
// 64w + b, so a per-node mask is at once a lane mask.
//
// Two execution shapes, chosen per run by the host:
//
// * word-local ("task") kernels: one workgroup owns one 64-trial word and runs
//   that word's whole cascade, separating steps with workgroup barriers only.
//   Workgroups never wait for each other, so any launch shape is safe.  This
//   is the shape for many words with small or medium cascades.
//
// * grid-wide step kernels: one ordinary launch per IC level or LT sweep, all
//   words at once; a step that finds the run finished returns at once, so the
//   host enqueues steps in batches and waits only at the end of a batch.  This
//   is the shape for few words with huge frontiers.
//
// IC (paper Section 2; Section 3 "Algorithms": only out-neighbours of the
// nodes activated in the previous step are examined) is a level-synchronous
// push.  For an out-arc e = (u, v) of a frontier node the trials still to
// decide are mask(u) & ~A[v]; coins are drawn only for the 8-trial groups that
// contain such a trial.  New bits are OR-ed into A with atomics whose return
// value tells which bits are new.
//
// LT (Section 2): a node joins when the weight of its active in-neighbours
// exceeds its threshold.  The rule is monotone, so the final set of every trial
// is the least fixpoint above S and any order of node updates reaches it.  A
// node is evaluated by pulling: sum the in-weights of active in-neighbours per
// trial (lane = trial) and compare with the threshold hash.  The grid shape
// sweeps every node with an inactive trial until a sweep changes nothing; the
// word-local shape evaluates only the out-neighbours of the nodes that joined
// in the previous step (push-side marking, pull-side evaluation).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "philox.hpp"

namespace imsim {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;
constexpr uint32_t kChunk = 1024;     // out-arcs per grid-shape IC work item
constexpr uint32_t kMaxWords = 4096;  // grid-shape queue items carry the word in 12 bits

struct SimParams {
    int64_t n;
    uint32_t T;
    uint32_t W;
    uint64_t seed;
    // out-CSR and IC thresholds
    const int64_t* __restrict__ off;
    const uint32_t* __restrict__ idx;
    const uint32_t* __restrict__ thr;
    // in-CSR (LT): per in-arc, source node (low half) and 32-bit weight piece
    // (high half)
    const int64_t* __restrict__ in_off;
    const uint64_t* __restrict__ in_arc;
    // LT when every node's in-arc weight pieces are all equal (e.g. 1/indeg):
    // source per in-arc, and the common piece per node; the sum over active
    // in-neighbours is then (their count) * node_w[v]
    const uint32_t* __restrict__ in_src32;
    const uint32_t* __restrict__ node_w;
    int lt_uniform;
    // LT grid shape: top 16 bits of every threshold hash, [W][n][64] (or null)
    const uint16_t* __restrict__ thp;
    uint32_t thp_shift;  // the table holds hash >> thp_shift (16, or 31 in tests)
    // state
    uint64_t* A;        // [W][n]
    uint64_t* N[3];     // grid IC: next-level masks (rotating); word-local: N[0] only
    uint64_t* Q[3];     // grid IC: queues of (node, word, chunk); word-local: see below
    uint32_t* qcount;   // grid: per-step counters
    uint32_t* aux;      // word-local: per-word scratch (stamps / queue masks)
    const uint32_t* seeds;
    uint32_t n_seeds;
    uint32_t* task_counter;  // word-local: next word to take
    uint32_t* status;        // [0] max steps over words, [1] guard fired
    uint32_t cap;            // step guard
};

__device__ __forceinline__ uint64_t valid_mask(uint32_t w, uint32_t W, uint32_t T)
{
    const uint32_t tail = T & 63u;
    return (w + 1 < W || tail == 0) ? ~0ull : ((1ull << tail) - 1ull);
}

__device__ __forceinline__ uint64_t load_relaxed(const uint64_t* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint32_t load_relaxed32(const uint32_t* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint64_t atomic_or64(uint64_t* p, uint64_t v)
{
    return __hip_atomic_fetch_or(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Live mask of arc e for the trials in `todo` (bits of word w): coins are
// drawn only for 8-trial groups holding a trial of `todo`.
__device__ __forceinline__ uint64_t ic_live(uint64_t todo, uint32_t th, uint64_t e, uint32_t w, uint64_t seed)
{
    if (th == 0xFFFFFFFFu) return todo;
    uint64_t live = 0, rest = todo;
    while (rest) {
        const uint32_t g = (uint32_t)__builtin_ctzll(rest) >> 3;
        rest &= ~(0xFFull << (8 * g));
        const Block4 b = philox_block(e, (uint64_t)w * 8 + g, seed, kDomainIcArc);
        uint32_t bits = 0;
#pragma unroll
        for (uint32_t j = 0; j < 8; ++j) bits |= (block_lane(b, j) < th ? 1u : 0u) << j;
        live |= (uint64_t)bits << (8 * g);
    }
    return live & todo;
}

// One staged in-arc: the 64-bit active mask of its source split in halves (so
// lane t reads the half holding bit t) and its weight twice (so both halves
// of the wavefront read (mask half, weight) at the same relative offset).
struct ArcStage {
    uint32_t a_lo, a_hi, w_lo_half, w_hi_half;
};

__device__ __forceinline__ uint32_t uniform32(uint32_t x)
{
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)x);
}

__device__ __forceinline__ uint64_t uniform64(uint64_t x)
{
    return (uint64_t)uniform32((uint32_t)x) | ((uint64_t)uniform32((uint32_t)(x >> 32)) << 32);
}

__device__ __forceinline__ uint64_t select8(const uint64_t x[8], uint32_t j)
{
    uint64_t r = x[0];
#pragma unroll
    for (uint32_t q = 1; q < 8; ++q) r = (j == q) ? x[q] : r;
    return r;
}

// Add node J's staged arcs of chunk [c, c+64) to acc[J]: lane t adds the
// weight of every arc whose source mask has bit t set.
template <int J>
__device__ __forceinline__ void lt_accumulate_chunk(const uint64_t (&pend)[8], const uint32_t (&pre)[9], uint64_t (&acc)[8],
                                                    const uint32_t* st32, uint32_t c, uint32_t half, uint32_t bitpos)
{
    if (pend[J] == 0) return;
    const uint32_t lo = pre[J] > c ? pre[J] : c;
    const uint32_t hi = pre[J + 1] < c + 64 ? pre[J + 1] : c + 64;
    if (hi <= lo) return;
    uint64_t a = acc[J];
#pragma unroll 4
    for (uint32_t i = lo - c; i + c < hi; ++i) {
        const uint32_t h32 = st32[4 * i + half];
        const uint32_t wt = st32[4 * i + 2 + half];
        a += (uint32_t)__builtin_amdgcn_sbfe((int)h32, bitpos, 1) & wt;
    }
    acc[J] = a;
}

// Uniform-weight form: count node J's staged in-neighbours of chunk [c, c+64)
// active in lane t's trial (stage holds each source mask as two 32-bit halves).
template <int J>
__device__ __forceinline__ void lt_count_chunk(const uint64_t (&pend)[8], const uint32_t (&pre)[9], uint32_t (&cnt)[8],
                                               const uint32_t* st32, uint32_t c, uint32_t half, uint32_t bitpos)
{
    if (pend[J] == 0) return;
    // node J's arcs within [c, c+64), as absolute positions; empty when the
    // node's row ends before the chunk or starts after it
    const uint32_t lo_abs = pre[J] > c ? pre[J] : c;
    const uint32_t hi_abs = pre[J + 1] < c + 64 ? pre[J + 1] : c + 64;
    if (hi_abs <= lo_abs) return;
    const uint32_t hi = hi_abs - c;
    uint32_t a = cnt[J];
    uint32_t i = lo_abs - c;
    for (; i + 1 < hi; i += 2) {
        const uint32_t b0 = __builtin_amdgcn_ubfe(st32[2 * i + half], bitpos, 1);
        const uint32_t b1 = __builtin_amdgcn_ubfe(st32[2 * i + 2 + half], bitpos, 1);
        a = a + b0 + b1;
    }
    if (i < hi) a += __builtin_amdgcn_ubfe(st32[2 * i + half], bitpos, 1);
    cnt[J] = a;
}

// LT: evaluate up to 8 nodes of word w with one wavefront, lane = trial;
// joins are OR-ed into A and returned per node in `joined`.  Lanes 0..7 each
// describe one node: id `myv` (any value >= n for none), `pl` its trials to
// decide (inactive, and selected for evaluation; 0 to skip it), `kb`/`dg` the
// start and length of its in-arc row.
//
// The in-arcs of the evaluated nodes are concatenated and staged 64 at a time:
// lane L loads arc L of a chunk and gathers its source's mask, so 64 loads are
// in flight; the arcs of up to two chunks are fetched before the first is
// consumed.  Each chunk is written to the wavefront's LDS slots, then every
// lane walks it adding the weight of each arc whose source is active in its
// trial.
__device__ __forceinline__ void lt_eval8_core(const SimParams& P, uint32_t w, uint32_t lane, uint64_t myv, uint64_t pl,
                                              int64_t kb, uint32_t dg, uint64_t joined[8], ArcStage* stage)
{
    const uint64_t n = (uint64_t)P.n;
    uint64_t* Aw = P.A + (uint64_t)w * n;
    if (lane >= 8) {
        pl = 0;
        dg = 0;
    }
    if (pl == 0) dg = 0;
    // exclusive prefix of the in-degrees over lanes 0..7
    uint32_t incl = dg;
#pragma unroll
    for (int o = 1; o < 8; o <<= 1) {
        const uint32_t y = __shfl_up(incl, o);
        incl += lane >= (uint32_t)o ? y : 0u;
    }
    const uint32_t pre_lane = incl - dg;

    uint64_t pend[8], vsu[8];
    uint32_t pre[9];
    uint64_t any = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        joined[j] = 0;
        pend[j] = uniform64(__shfl(pl, j));
        vsu[j] = uniform64(__shfl(myv, j));
        pre[j] = uniform32(__shfl(pre_lane, j));
        any |= pend[j];
    }
    pre[8] = uniform32(__shfl(incl, 7));
    if (any == 0 || pre[8] == 0) return;  // nothing pending, or no in-weight at all

    // threshold prefixes are independent of the sums: fetch them first
    uint32_t hpre[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) hpre[j] = (P.thp && pend[j]) ? P.thp[((uint64_t)w * n + vsu[j]) * 64 + lane] : 0u;

    uint64_t acc[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) acc[j] = 0;
    const uint32_t* st32 = reinterpret_cast<const uint32_t*>(stage);
    const uint32_t half = lane >> 5, bitpos = lane & 31u;
    const uint32_t total = pre[8];
    auto arc_index = [&](uint32_t q) -> uint64_t {
        uint32_t j = 0;
#pragma unroll
        for (int jj = 1; jj < 8; ++jj) j += (q >= pre[jj]) ? 1u : 0u;
        const uint32_t pj = __shfl(pre_lane, (int)j);
        const uint64_t kbase = (uint64_t)__shfl(kb, (int)j);
        return kbase + (q - pj);
    };
    if (P.lt_uniform) {
        // in-weights of a node are all equal: count active in-neighbours
        uint32_t cnt[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) cnt[j] = 0;
        uint32_t wn_lane = 0;
        if (lane < 8 && pl) wn_lane = P.node_w[myv];
        for (uint32_t c0 = 0; c0 < total; c0 += 128) {
            const uint32_t q0 = c0 + lane, q1 = c0 + 64 + lane;
            // cross-lane reads with every lane active; only the loads are guarded
            const uint64_t k0 = arc_index(q0);
            const uint64_t k1 = arc_index(q1);
            const uint32_t s0 = q0 < total ? P.in_src32[k0] : 0u;
            const uint32_t s1 = q1 < total ? P.in_src32[k1] : 0u;
            const uint64_t a0 = q0 < total ? load_relaxed(&Aw[s0]) : 0ull;
            const uint64_t a1 = q1 < total ? load_relaxed(&Aw[s1]) : 0ull;
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const uint32_t c = c0 + 64 * q;
                if (c >= total) break;
                const uint64_t a = q ? a1 : a0;
                uint2* st2 = reinterpret_cast<uint2*>(stage);
                __builtin_amdgcn_wave_barrier();
                st2[lane] = make_uint2((uint32_t)a, (uint32_t)(a >> 32));
                __builtin_amdgcn_wave_barrier();
                lt_count_chunk<0>(pend, pre, cnt, st32, c, half, bitpos);
                lt_count_chunk<1>(pend, pre, cnt, st32, c, half, bitpos);
                lt_count_chunk<2>(pend, pre, cnt, st32, c, half, bitpos);
                lt_count_chunk<3>(pend, pre, cnt, st32, c, half, bitpos);
                lt_count_chunk<4>(pend, pre, cnt, st32, c, half, bitpos);
                lt_count_chunk<5>(pend, pre, cnt, st32, c, half, bitpos);
                lt_count_chunk<6>(pend, pre, cnt, st32, c, half, bitpos);
                lt_count_chunk<7>(pend, pre, cnt, st32, c, half, bitpos);
                __builtin_amdgcn_wave_barrier();
            }
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) acc[j] = (uint64_t)cnt[j] * (uint64_t)uniform32(__shfl(wn_lane, j));
    } else {
        for (uint32_t c0 = 0; c0 < total; c0 += 128) {
            // cross-lane reads with every lane active; only the loads are guarded
            const uint64_t k0 = arc_index(c0 + lane);
            const uint64_t k1 = arc_index(c0 + 64 + lane);
            const uint64_t arc0 = c0 + lane < total ? P.in_arc[k0] : 0ull;
            const uint64_t arc1 = c0 + 64 + lane < total ? P.in_arc[k1] : 0ull;
            const uint64_t a0 = c0 + lane < total ? load_relaxed(&Aw[(uint32_t)arc0]) : 0ull;
            const uint64_t a1 = c0 + 64 + lane < total ? load_relaxed(&Aw[(uint32_t)arc1]) : 0ull;
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const uint32_t c = c0 + 64 * q;
                if (c >= total) break;
                const uint64_t arc = q ? arc1 : arc0;
                const uint64_t a = q ? a1 : a0;
                const uint32_t wt = (uint32_t)(arc >> 32);
                __builtin_amdgcn_wave_barrier();
                stage[lane] = ArcStage{(uint32_t)a, (uint32_t)(a >> 32), wt, wt};
                __builtin_amdgcn_wave_barrier();
                lt_accumulate_chunk<0>(pend, pre, acc, st32, c, half, bitpos);
                lt_accumulate_chunk<1>(pend, pre, acc, st32, c, half, bitpos);
                lt_accumulate_chunk<2>(pend, pre, acc, st32, c, half, bitpos);
                lt_accumulate_chunk<3>(pend, pre, acc, st32, c, half, bitpos);
                lt_accumulate_chunk<4>(pend, pre, acc, st32, c, half, bitpos);
                lt_accumulate_chunk<5>(pend, pre, acc, st32, c, half, bitpos);
                lt_accumulate_chunk<6>(pend, pre, acc, st32, c, half, bitpos);
                lt_accumulate_chunk<7>(pend, pre, acc, st32, c, half, bitpos);
                __builtin_amdgcn_wave_barrier();
            }
        }
    }

    // Decide "in-weight > threshold hash" per pending trial.  With the prefix
    // table the top 16 bits settle every trial except a tie of the prefixes;
    // ties (and every trial without a table) compare with the full hash.
    uint64_t need[8], dec[8];
    uint64_t any_need = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        need[j] = 0;
        dec[j] = 0;
        if (pend[j] == 0) continue;
        if (P.thp) {
            const uint32_t hp = hpre[j];
            const uint64_t hi = acc[j] >> P.thp_shift;
            const bool pb = (pend[j] >> lane) & 1ull;
            dec[j] = __ballot(pb && hi > hp);
            need[j] = __ballot(pb && hi == hp);
        } else {
            need[j] = pend[j];
        }
        any_need |= need[j];
    }
    if (any_need) {
        // lane 8j+g draws the block of node vs[j] for trials 64w+8g .. +7 when
        // that group holds an undecided trial
        const uint32_t jj = lane >> 3, gg = lane & 7;
        uint64_t my_need = need[0];
#pragma unroll
        for (int j = 1; j < 8; ++j) my_need = (jj == (uint32_t)j) ? need[j] : my_need;
        const uint64_t my_node = __shfl(myv, (int)jj);
        Block4 blk{0, 0, 0, 0};
        if ((my_need >> (8 * gg)) & 0xFFull) blk = philox_block(my_node, (uint64_t)w * 8 + gg, P.seed, kDomainLtNode);
        const uint32_t src_off = lane >> 3;
        const uint32_t sel = (lane & 7) >> 1;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            if (need[j] == 0) continue;
            const int src = 8 * j + (int)src_off;
            const uint64_t x0 = __shfl(blk.w0, src);
            const uint64_t x1 = __shfl(blk.w1, src);
            const uint64_t x2 = __shfl(blk.w2, src);
            const uint64_t x3 = __shfl(blk.w3, src);
            const uint64_t word = sel == 0 ? x0 : sel == 1 ? x1 : sel == 2 ? x2 : x3;
            const uint32_t h = (lane & 1) ? (uint32_t)(word >> 32) : (uint32_t)word;
            dec[j] |= __ballot(((need[j] >> lane) & 1ull) && acc[j] > (uint64_t)h);
        }
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        if (dec[j] == 0) continue;
        if (lane == 0) atomic_or64(&Aw[vsu[j]], dec[j]);
        joined[j] = dec[j];
    }
}

// LT evaluation of nodes vs[0..7] (ids >= n are absent) for callers that hold
// node ids only; `mark`/`min_mark` optionally restrict it to marked nodes.
__device__ __forceinline__ void lt_eval8(const SimParams& P, uint32_t w, const uint64_t vs[8], uint32_t lane,
                                         uint64_t joined[8], ArcStage* stage, const uint32_t* mark, uint32_t min_mark)
{
    const uint64_t n = (uint64_t)P.n;
    const uint64_t vm = valid_mask(w, P.W, P.T);
    const uint64_t myv = lane < 8 ? select8(vs, lane) : ~0ull;
    const bool okv = myv < n;
    uint64_t pl = okv ? (vm & ~load_relaxed(&P.A[(uint64_t)w * n + myv])) : 0ull;
    if (okv && pl && mark && mark[(uint64_t)w * n + myv] < min_mark) pl = 0;
    const int64_t kb = pl ? P.in_off[myv] : 0;
    const uint32_t dg = pl ? (uint32_t)(P.in_off[myv + 1] - kb) : 0u;
    lt_eval8_core(P, w, lane, myv, pl, kb, dg, joined, stage);
}

// Threshold prefix table for the LT grid shape: thp[(w*n + v)*64 + b] =
// H(seed, LT, 64w + b, v) >> thp_shift (the top 16 bits for shift 16).  Lane 8j+g of a wavefront draws the block of
// node 8*item + j for trials 64w+8g .. 64w+8g+7 and stores its eight prefixes.
__global__ __launch_bounds__(kBlock) void lt_threshold_table_kernel(SimParams P, uint16_t* __restrict__ thp)
{
    const uint64_t n = (uint64_t)P.n;
    const uint64_t nb = (n + 7) / 8;
    const uint64_t items = nb * P.W;
    const uint32_t lane = threadIdx.x & 63u;
    for (uint64_t it = ((uint64_t)blockIdx.x * kBlock + threadIdx.x) >> 6; it < items; it += ((uint64_t)gridDim.x * kBlock) >> 6) {
        const uint32_t w = (uint32_t)(it / nb);
        const uint64_t v = (it % nb) * 8 + (lane >> 3);
        const uint32_t g = lane & 7;
        if (v >= n) continue;
        const Block4 b = philox_block(v, (uint64_t)w * 8 + g, P.seed, kDomainLtNode);
        const uint32_t sh = P.thp_shift;
        auto pair = [sh](uint64_t x) -> uint32_t {
            return (((uint32_t)x) >> sh) | ((((uint32_t)(x >> 32)) >> sh) << 16);
        };
        uint4 out;
        out.x = pair(b.w0);
        out.y = pair(b.w1);
        out.z = pair(b.w2);
        out.w = pair(b.w3);
        *reinterpret_cast<uint4*>(thp + ((uint64_t)w * n + v) * 64 + 8 * g) = out;
    }
}

// =========================================================== grid shape

__device__ __forceinline__ uint64_t pack_item(uint32_t v, uint32_t w, uint32_t chunk)
{
    return (uint64_t)v | ((uint64_t)w << 32) | ((uint64_t)chunk << 44);
}

__device__ __forceinline__ void grid_ic_enqueue(const SimParams& P, uint64_t* Q, uint32_t* count, uint32_t v, uint32_t w)
{
    const uint64_t deg = (uint64_t)(P.off[v + 1] - P.off[v]);
    const uint32_t nc = (uint32_t)((deg + kChunk - 1) / kChunk);
    const uint32_t pos = atomicAdd(count, nc);
    for (uint32_t c = 0; c < nc; ++c) Q[pos + c] = pack_item(v, w, c);
}

// Seeds are active in every trial; for IC, seeds with out-arcs form level 0.
__global__ __launch_bounds__(kBlock) void grid_seed_kernel(SimParams P, int model)
{
    const uint64_t pairs = (uint64_t)P.n_seeds * P.W;
    const uint64_t n = (uint64_t)P.n;
    for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < pairs; i += (uint64_t)gridDim.x * kBlock) {
        const uint32_t s = P.seeds[i / P.W];
        const uint32_t w = (uint32_t)(i % P.W);
        const uint64_t vm = valid_mask(w, P.W, P.T);
        P.A[(uint64_t)w * n + s] = vm;
        if (model == 0 && P.off[s + 1] > P.off[s]) {
            P.N[0][(uint64_t)w * n + s] = vm;
            grid_ic_enqueue(P, P.Q[0], &P.qcount[0], s, w);
        }
    }
}

// LT: mark the out-neighbours of the seeds for sweep 0 (mark value 1) in every
// word.  Threads run over the concatenated out-arcs of the seeds;
// seed_arc_pre[i] is the number of seed out-arcs before seed i.
__global__ __launch_bounds__(kBlock) void grid_lt_seed_mark_kernel(SimParams P, const uint64_t* __restrict__ seed_arc_pre)
{
    const uint64_t n = (uint64_t)P.n;
    const uint64_t total = seed_arc_pre[P.n_seeds];
    for (uint64_t q = (uint64_t)blockIdx.x * kBlock + threadIdx.x; q < total; q += (uint64_t)gridDim.x * kBlock) {
        uint32_t lo = 0, hi = P.n_seeds;  // last seed with seed_arc_pre[i] <= q
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (seed_arc_pre[mid] <= q) lo = mid; else hi = mid;
        }
        const uint32_t s = P.seeds[lo];
        const uint32_t v = P.idx[P.off[s] + (int64_t)(q - seed_arc_pre[lo])];
        for (uint32_t w = 0; w < P.W; ++w) P.aux[(uint64_t)w * n + v] = 1u;
    }
}

// IC level `lev`: clear level lev-1's masks, then expand level lev's queue.
// Masks and queues rotate over three buffers: level l reads buffer l%3, writes
// (l+1)%3 and clears (l+2)%3, which held level l-1's frontier.
__global__ __launch_bounds__(kBlock) void grid_ic_level_kernel(SimParams P, uint32_t lev)
{
    const uint32_t cnt = load_relaxed32(&P.qcount[lev]);
    const uint64_t n = (uint64_t)P.n;
    const uint64_t gtid = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    const uint64_t nthreads = (uint64_t)gridDim.x * kBlock;
    if (lev >= 1) {
        const uint32_t oc = load_relaxed32(&P.qcount[lev - 1]);
        const uint64_t* Qo = P.Q[(lev + 2) % 3];
        uint64_t* No = P.N[(lev + 2) % 3];
        for (uint64_t i = gtid; i < oc; i += nthreads) {
            const uint64_t it = Qo[i];
            if ((it >> 44) == 0) No[((it >> 32) & 0xFFFu) * n + (uint32_t)it] = 0;
        }
    }
    if (cnt == 0) return;
    if (lev + 1 >= P.cap) {
        if (gtid == 0) P.status[1] = 1;
        return;
    }
    const uint64_t* Qc = P.Q[lev % 3];
    const uint64_t* Nc = P.N[lev % 3];
    uint64_t* Nn = P.N[(lev + 1) % 3];
    uint64_t* Qn = P.Q[(lev + 1) % 3];
    uint32_t* qnext = &P.qcount[lev + 1];
    const uint32_t lane = threadIdx.x & 63u;
    for (uint64_t itx = gtid >> 6; itx < cnt; itx += nthreads >> 6) {
        const uint64_t item = Qc[itx];
        const uint32_t u = (uint32_t)item;
        const uint32_t w = (uint32_t)(item >> 32) & 0xFFFu;
        const uint32_t chunk = (uint32_t)(item >> 44);
        const uint64_t mask = load_relaxed(&Nc[(uint64_t)w * n + u]);
        const int64_t row_end = P.off[u + 1];
        const int64_t e0 = P.off[u] + (int64_t)chunk * kChunk;
        const int64_t e1 = e0 + (int64_t)kChunk < row_end ? e0 + (int64_t)kChunk : row_end;
        uint64_t* Aw = P.A + (uint64_t)w * n;
        for (int64_t e = e0 + lane; e < e1; e += 64) {
            const uint32_t v = P.idx[e];
            const uint32_t th = P.thr[e];
            if (th == 0) continue;
            const uint64_t todo = mask & ~Aw[v];
            if (todo == 0) continue;
            const uint64_t live = ic_live(todo, th, (uint64_t)e, w, P.seed);
            if (live == 0) continue;
            const uint64_t fresh = live & ~atomic_or64(&Aw[v], live);
            if (fresh == 0 || P.off[v + 1] == P.off[v]) continue;
            if (atomic_or64(&Nn[(uint64_t)w * n + v], fresh) == 0) grid_ic_enqueue(P, Qn, qnext, v, w);
        }
    }
}

// LT sweep `sw`, in place over all words.  Direction switch: a sweep "marks"
// when the previous sweep changed fewer than `tau` (node, word) pairs: every
// node that joins then stamps its out-neighbours with sw + 2 in aux.  A sweep
// that follows a marking sweep evaluates only nodes stamped >= sw + 1 (sweep 0
// follows the seed marks); any other sweep evaluates every node with an
// inactive trial.  Nodes whose in-neighbours did not change since their last
// evaluation cannot change, so both forms reach the same fixpoint.  A sweep
// that follows one without change returns at once.  qcount[sw] counts the
// (node, word) pairs that changed.
__global__ __launch_bounds__(kBlock) void grid_lt_sweep_kernel(SimParams P, uint32_t sw, uint32_t tau)
{
    __shared__ ArcStage stage[kWaves][64];
    if (sw >= 1 && load_relaxed32(&P.qcount[sw - 1]) == 0) return;
    if (sw >= P.cap) {
        if (blockIdx.x == 0 && threadIdx.x == 0) P.status[1] = 1;
        return;
    }
    // changes of sweep x (x = -1: seed pairs)
    auto changes = [&](int64_t x) -> uint32_t {
        return x < 0 ? P.n_seeds * P.W : load_relaxed32(&P.qcount[x]);
    };
    const bool marks_now = changes((int64_t)sw - 1) < tau;
    const bool marked_only = sw == 0 ? true : changes((int64_t)sw - 2) < tau;
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wave = threadIdx.x >> 6;
    const uint64_t n = (uint64_t)P.n;
    // wavefronts take blocks of 64 nodes of one word, find the 8-node batches
    // with a node to evaluate, and evaluate those
    const uint64_t nb = (n + 63) / 64;
    const uint64_t items = nb * P.W;
    const uint64_t gwave = ((uint64_t)blockIdx.x * kBlock + threadIdx.x) >> 6;
    const uint64_t nwaves = ((uint64_t)gridDim.x * kBlock) >> 6;
    uint32_t changed = 0;
    for (uint64_t it = gwave; it < items; it += nwaves) {
        const uint32_t w = (uint32_t)(it / nb);
        const uint64_t vbase = (it % nb) * 64;
        const uint64_t vm = valid_mask(w, P.W, P.T);
        const uint64_t v = vbase + lane;
        const bool inr = v < n;
        uint64_t p = inr ? (vm & ~load_relaxed(&P.A[(uint64_t)w * n + v])) : 0ull;
        const int64_t kb = inr ? P.in_off[v] : 0;
        const int64_t ke = inr ? P.in_off[v + 1] : 0;
        if (p && marked_only && P.aux[(uint64_t)w * n + v] < sw + 1) p = 0;
        const uint64_t bm = __ballot(p != 0);
        if (bm == 0) continue;
        for (uint32_t b8 = 0; b8 < 8; ++b8) {
            if (((bm >> (8 * b8)) & 0xFFull) == 0) continue;
            const int src = (int)(8 * b8 + (lane & 7));
            const uint64_t myv = __shfl(v, src);
            const uint64_t pl = __shfl(p, src);
            const int64_t kbj = __shfl(kb, src);
            const uint32_t dg = (uint32_t)(__shfl(ke, src) - kbj);
            uint64_t joined[8];
            lt_eval8_core(P, w, lane, myv, pl, kbj, dg, joined, stage[wave]);
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                if (joined[j] == 0) continue;
                ++changed;
                if (marks_now) {
                    const uint64_t vj = vbase + 8 * b8 + j;
                    uint32_t* mk = P.aux + (uint64_t)w * n;
                    for (int64_t e = P.off[vj] + lane; e < P.off[vj + 1]; e += 64) mk[P.idx[e]] = sw + 2;
                }
            }
        }
    }
    if (changed && lane == 0) atomicAdd(&P.qcount[sw], changed);
}

// ====================================================== word-local shape

// Word-local IC.  Workgroups take words from a counter.  Per word: a frontier
// list of nodes with their masks (Q[0]/Q[1] hold node ids, aux holds the
// matching masks as uint64 pairs of uint32), a scratch mask array N[0] that is
// zero between steps.  Step: every wavefront takes frontier entries and walks
// their out-arcs lane-strided; a node's first new bit of the step appends it to
// the next list (counter in LDS); after a barrier the next list picks up its
// masks from N[0] and clears them.
__global__ __launch_bounds__(kBlock) void word_ic_kernel(SimParams P, uint64_t list_cap)
{
    __shared__ uint32_t s_word;
    __shared__ uint32_t s_cnt[2];
    __shared__ uint32_t s_next_item;
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t n = (uint64_t)P.n;
    uint32_t max_steps = 0;
    bool guard = false;
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) s_word = atomicAdd(P.task_counter, 1u);
        __syncthreads();
        const uint32_t w = s_word;
        if (w >= P.W) break;
        const uint64_t vm = valid_mask(w, P.W, P.T);
        uint64_t* Aw = P.A + (uint64_t)w * n;
        uint64_t* Nw = P.N[0] + (uint64_t)w * n;
        // per-word lists: node ids in Q[0]/Q[1] (as uint32), masks in aux (as uint64)
        uint32_t* L[2] = {(uint32_t*)P.Q[0] + (uint64_t)w * list_cap, (uint32_t*)P.Q[1] + (uint64_t)w * list_cap};
        uint64_t* M[2] = {(uint64_t*)P.Q[2] + (uint64_t)w * list_cap * 2, (uint64_t*)P.Q[2] + (uint64_t)w * list_cap * 2 + list_cap};
        if (threadIdx.x == 0) {
            s_cnt[0] = 0;
            s_cnt[1] = 0;
        }
        __syncthreads();
        for (uint32_t i = threadIdx.x; i < P.n_seeds; i += kBlock) {
            const uint32_t s = P.seeds[i];
            Aw[s] = vm;
            if (P.off[s + 1] > P.off[s]) {
                const uint32_t pos = atomicAdd(&s_cnt[0], 1u);
                L[0][pos] = s;
                M[0][pos] = vm;
            }
        }
        __syncthreads();
        uint32_t cur = 0, steps = 0;
        for (;;) {
            const uint32_t cnt = s_cnt[cur];
            if (cnt == 0) break;
            if (steps + 1 >= P.cap) {
                guard = true;
                break;
            }
            ++steps;
            const uint32_t nxt = cur ^ 1u;
            if (threadIdx.x == 0) {
                s_cnt[nxt] = 0;
                s_next_item = 0;
            }
            __syncthreads();
            // wavefronts take frontier entries dynamically
            for (;;) {
                uint32_t it = 0;
                if (lane == 0) it = atomicAdd(&s_next_item, 1u);
                it = __shfl(it, 0);
                if (it >= cnt) break;
                const uint32_t u = L[cur][it];
                const uint64_t mask = M[cur][it];
                const int64_t e1 = P.off[u + 1];
                for (int64_t e = P.off[u] + lane; e < e1; e += 64) {
                    const uint32_t v = P.idx[e];
                    const uint32_t th = P.thr[e];
                    if (th == 0) continue;
                    const uint64_t todo = mask & ~Aw[v];
                    if (todo == 0) continue;
                    const uint64_t live = ic_live(todo, th, (uint64_t)e, w, P.seed);
                    if (live == 0) continue;
                    const uint64_t fresh = live & ~atomic_or64(&Aw[v], live);
                    if (fresh == 0 || P.off[v + 1] == P.off[v]) continue;
                    if (atomic_or64(&Nw[v], fresh) == 0) {
                        const uint32_t pos = atomicAdd(&s_cnt[nxt], 1u);
                        L[nxt][pos] = v;
                    }
                }
            }
            __syncthreads();
            const uint32_t nc = s_cnt[nxt];
            for (uint32_t i = threadIdx.x; i < nc; i += kBlock) {
                const uint32_t v = L[nxt][i];
                M[nxt][i] = load_relaxed(&Nw[v]);
                Nw[v] = 0;
            }
            __syncthreads();
            cur = nxt;
        }
        max_steps = steps > max_steps ? steps : max_steps;
    }
    if (threadIdx.x == 0) {
        atomicMax(&P.status[0], max_steps);
        if (guard) P.status[1] = 1;
    }
}

// Word-local LT.  Per word: the frontier list holds the nodes that joined in
// the previous step (any trial); their out-neighbours with an inactive trial
// are collected once each (stamp per node in aux) into a candidate list, then
// wavefronts evaluate candidates eight at a time; nodes that joined form the
// next frontier.
__global__ __launch_bounds__(kBlock) void word_lt_kernel(SimParams P, uint64_t list_cap)
{
    __shared__ ArcStage stage[kWaves][64];
    __shared__ uint32_t s_word;
    __shared__ uint32_t s_cnt[2];
    __shared__ uint32_t s_cand;
    __shared__ uint32_t s_next_item;
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t n = (uint64_t)P.n;
    uint32_t max_steps = 0;
    bool guard = false;
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) s_word = atomicAdd(P.task_counter, 1u);
        __syncthreads();
        const uint32_t w = s_word;
        if (w >= P.W) break;
        const uint64_t vm = valid_mask(w, P.W, P.T);
        uint64_t* Aw = P.A + (uint64_t)w * n;
        uint32_t* stamp = P.aux + (uint64_t)w * n;  // last step in which v became a candidate
        uint32_t* F[2] = {(uint32_t*)P.Q[0] + (uint64_t)w * list_cap, (uint32_t*)P.Q[1] + (uint64_t)w * list_cap};
        uint32_t* C = (uint32_t*)P.Q[2] + (uint64_t)w * list_cap;
        if (threadIdx.x == 0) {
            s_cnt[0] = 0;
            s_cnt[1] = 0;
        }
        __syncthreads();
        for (uint32_t i = threadIdx.x; i < P.n_seeds; i += kBlock) {
            const uint32_t s = P.seeds[i];
            Aw[s] = vm;
            const uint32_t pos = atomicAdd(&s_cnt[0], 1u);
            F[0][pos] = s;
        }
        __syncthreads();
        uint32_t cur = 0, steps = 0;
        for (;;) {
            const uint32_t cnt = s_cnt[cur];
            if (cnt == 0) break;
            if (steps + 1 >= P.cap) {
                guard = true;
                break;
            }
            ++steps;
            const uint32_t nxt = cur ^ 1u;
            if (threadIdx.x == 0) {
                s_cnt[nxt] = 0;
                s_cand = 0;
                s_next_item = 0;
            }
            __syncthreads();
            // push side: out-neighbours of the frontier with an inactive trial
            for (;;) {
                uint32_t it = 0;
                if (lane == 0) it = atomicAdd(&s_next_item, 1u);
                it = __shfl(it, 0);
                if (it >= cnt) break;
                const uint32_t u = F[cur][it];
                const int64_t e1 = P.off[u + 1];
                for (int64_t e = P.off[u] + lane; e < e1; e += 64) {
                    const uint32_t v = P.idx[e];
                    if ((vm & ~Aw[v]) == 0) continue;
                    if (atomicMax(&stamp[v], steps) < steps) {
                        const uint32_t pos = atomicAdd(&s_cand, 1u);
                        C[pos] = v;
                    }
                }
            }
            __syncthreads();
            if (threadIdx.x == 0) s_next_item = 0;
            __syncthreads();
            // pull side: evaluate candidates eight at a time
            const uint32_t ncand = s_cand;
            for (;;) {
                uint32_t it = 0;
                if (lane == 0) it = atomicAdd(&s_next_item, 8u);
                it = __shfl(it, 0);
                if (it >= ncand) break;
                uint64_t vs[8], joined[8];
#pragma unroll
                for (int j = 0; j < 8; ++j) vs[j] = it + j < ncand ? (uint64_t)C[it + j] : ~0ull;
                lt_eval8(P, w, vs, lane, joined, stage[threadIdx.x >> 6], nullptr, 0);
#pragma unroll
                for (int j = 0; j < 8; ++j)
                    if (joined[j] && lane == 0) {
                        const uint32_t pos = atomicAdd(&s_cnt[nxt], 1u);
                        F[nxt][pos] = (uint32_t)vs[j];
                    }
            }
            __syncthreads();
            cur = nxt;
        }
        // clear this word's stamps for the next run
        __syncthreads();
        for (uint64_t v = threadIdx.x; v < n; v += kBlock) stamp[v] = 0;
        max_steps = steps > max_steps ? steps : max_steps;
    }
    if (threadIdx.x == 0) {
        atomicMax(&P.status[0], max_steps);
        if (guard) P.status[1] = 1;
    }
}

// ============================================================ reductions

// trial_counts[64w + b] += number of nodes with bit b of A[w*n + v] set.
// Grid: (blocks over nodes, W).  Lane b counts trial 64w + b.
__global__ __launch_bounds__(kBlock) void reduce_trial_counts(const uint64_t* __restrict__ A, int64_t n, uint32_t T,
                                                              uint32_t* __restrict__ trial_counts)
{
    __shared__ uint32_t part[kWaves][64];
    const uint32_t w = blockIdx.y;
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wave = threadIdx.x >> 6;
    const uint64_t* Aw = A + (uint64_t)w * n;
    uint32_t cnt = 0;
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    for (uint64_t base = (uint64_t)blockIdx.x * kBlock + wave * 64; base < (uint64_t)n; base += stride) {
        const uint64_t v = base + lane;
        const uint64_t x = v < (uint64_t)n ? Aw[v] : 0ull;
        if (__ballot(x != 0) == 0) continue;
#pragma unroll 8
        for (uint32_t b = 0; b < 64; ++b) {
            const uint64_t bal = __ballot((x >> b) & 1ull);
            cnt += (lane == b) ? (uint32_t)__popcll(bal) : 0u;
        }
    }
    part[wave][lane] = cnt;
    __syncthreads();
    if (wave == 0) {
        uint32_t s = 0;
        for (int q = 0; q < kWaves; ++q) s += part[q][lane];
        const uint64_t t = (uint64_t)w * 64 + lane;
        if (s && t < T) atomicAdd(&trial_counts[t], s);
    }
}

// node_counts[v] = sum_w popcount(A[w*n + v]); total += sum_v node_counts[v].
__global__ __launch_bounds__(kBlock) void reduce_node_counts(const uint64_t* __restrict__ A, int64_t n, uint32_t W,
                                                             uint32_t* __restrict__ node_counts,
                                                             unsigned long long* __restrict__ total)
{
    __shared__ unsigned long long part[kWaves];
    unsigned long long sum = 0;
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    for (uint64_t v = (uint64_t)blockIdx.x * kBlock + threadIdx.x; v < (uint64_t)n; v += stride) {
        uint32_t c = 0;
        for (uint32_t w = 0; w < W; ++w) c += (uint32_t)__popcll(A[(uint64_t)w * n + v]);
        if (node_counts) node_counts[v] = c;
        sum += c;
    }
    for (int o = 32; o > 0; o >>= 1) sum += __shfl_down(sum, o);
    if ((threadIdx.x & 63u) == 0) part[threadIdx.x >> 6] = sum;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long s = 0;
        for (int q = 0; q < kWaves; ++q) s += part[q];
        if (s) atomicAdd(total, s);
    }
}

template <typename Tv>
__global__ __launch_bounds__(kBlock) void fill_kernel(Tv* __restrict__ p, uint64_t count, Tv value)
{
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < count; i += stride) p[i] = value;
}

__global__ __launch_bounds__(kBlock) void debug_hash_kernel(uint64_t seed, uint64_t domain, const uint64_t* __restrict__ trials,
                                                            const uint64_t* __restrict__ ids, uint32_t* __restrict__ out,
                                                            int64_t count)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < count) out[i] = hash32(seed, domain, trials[i], ids[i]);
}

}  // namespace imsim
