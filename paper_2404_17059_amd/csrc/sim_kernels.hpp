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
constexpr uint32_t kRowWords = 16;   // LT grid shape: words of a source row staged per pass
constexpr uint32_t kRowPitch = 17;   // LT grid shape: LDS row pitch in uint64 (odd: spreads banks)

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4a8 __attribute__((ext_vector_type(4), aligned(8)));  // 8-byte aligned

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
    // LT: weight of every out-arc (out-CSR order) in 2^-32 units, for the
    // push form of the 8-trial batch tasks
    const uint64_t* __restrict__ lt_wout;
    // LT grid shape: top 16 bits of every threshold hash, [W][n][64] (or null)
    const uint16_t* __restrict__ thp;
    uint32_t thp_shift;  // the table holds hash >> thp_shift (16, or 31 in tests)
    // LT grid shape: every threshold hash, node-major [n][W][64] (or null)
    const uint32_t* __restrict__ th32;
    // LT grid shape, equal in-weights: per (node, trial) the least number of
    // active in-arc pieces that makes the node join, k = floor(h / w_v) + 1,
    // saturated at 2^S_v - 1 (at most 127) with S_v planes for node v
    // (S_v = F(v+1) - F(v), F(v) = kinfo[2v + 1]), stored as complemented bit
    // planes: uint64 16*G*F(v) + (16g + x)*S_v + b (G = ceil(W / 16)) holds
    // NOT bit b of k for the 64 trials of word 16g + x (or null).  kinfo[2v]
    // is the low half of in_off[v]
    const uint64_t* __restrict__ kplanes;
    const uint32_t* __restrict__ kinfo;
    // LT grid shape: node batches whose in-arcs fit one 64-arc chunk (or one
    // node with more); batch b holds nodes bfirst[b] .. bfirst[b+1]-1
    const uint32_t* __restrict__ bfirst;
    uint32_t nbatch;
    // per batch: first node, node count | min(in-arc pieces, 2^24 - 1) << 8,
    // and the in-CSR position of its first piece (two halves)
    const u32x4* __restrict__ bdesc;
    // batches of one node with more than 64 in-arc pieces
    const uint32_t* __restrict__ bigb;
    uint32_t nbig;
    // state
    uint64_t* A;        // [W][n]
    uint64_t* Anm;      // LT grid shape: [n][W] (node-major)
    uint64_t* N[3];     // grid IC: next-level masks (rotating); word-local: N[0] only
    uint64_t* Q[3];     // grid IC: queues of (node, word, chunk); word-local: see below
    uint32_t* qcount;   // grid: per-step counters
    uint32_t* aux;      // word-local: per-word scratch (stamps / queue masks)
    uint32_t* nmark;    // LT grid shape: per node, the largest sweep mark of any of its words
    const uint64_t* base;  // sets form: word-major state [W][n] the sets start from, or null
    uint32_t* level_counts;  // word-local: [max_levels][T] nodes first active at each level (LT then runs synchronous steps), or null
    uint32_t max_levels;
    uint32_t w0;  // LT grid shape: global index of word 0 of this run (runs of at most 16 words)
    const uint32_t* seeds;
    uint32_t n_seeds;
    uint64_t seed_arcs;  // out-arcs of the seeds (predicts the first sweep's changes)
    uint32_t* task_counter;  // word-local: next task to take
    // sets mode: set i's nodes are set_nodes[set_off[i] .. set_off[i+1])
    const uint32_t* set_off;
    const uint32_t* set_nodes;
    uint32_t n_sets;
    uint64_t* totals;           // [n_sets] sum over trials of active nodes
    uint32_t* set_node_counts;  // [n_sets][n] or null
    uint32_t* act;              // per slot: activated nodes of the current task
    uint32_t* sstamp;           // per slot: LT candidate stamps (only grow)
    uint32_t* slot_steps;       // per slot: last LT stamp value used
    uint32_t* status;        // [0] max steps over words, [1] guard fired
    uint32_t cap;            // step guard
    // IC pull side: in-CSR (offsets in_off) over the arcs whose threshold is
    // not 0: per in-arc its source | out-CSR arc id << 32, and its threshold
    const uint64_t* __restrict__ ic_in;
    const uint32_t* __restrict__ ic_in_thr;
    // IC grid shape, direction of each level (Beamer's rule on the trial
    // words together): lvl_farcs[l] = out-arcs of the (node, word) pairs of
    // level l's frontier, lvl_full[l] = in-arcs of the pairs whose trials are
    // all active when level l starts, lvl_dir[l] = 1 push / 2 pull
    unsigned long long* lvl_farcs;
    unsigned long long* lvl_full;
    uint32_t* lvl_dir;
    uint64_t in_total;   // W * in-arcs: the pull volume of a state with nothing active
    float ic_alpha;      // push -> pull when frontier out-arcs * alpha > in-arcs of unfinished pairs
    float ic_beta;       // pull -> push when frontier pairs * beta < W * n
    int ic_dir;          // 0 = by the rule, 1 = push only, 2 = pull only
    int ic_preload;      // grid push reads a target's state before its coins (high mean arc probability)
};

// Trials of word w that exist (T trials in all); words past the last one
// (a padded state row) hold none.  W is not needed: the count comes from T.
__device__ __forceinline__ uint64_t valid_mask(uint32_t w, uint32_t W, uint32_t T)
{
    (void)W;
    const uint32_t lo = 64u * w;
    if (lo >= T) return 0ull;
    const uint32_t r = T - lo;
    return r >= 64u ? ~0ull : ((1ull << r) - 1ull);
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
// drawn only for 8-trial groups holding a trial of `todo`.  kChain picks the
// instruction schedule of the hash (same words either way): the carry-chain
// form everywhere but in the batch kernel, where the plain form measured
// faster.
template <bool kChain = true>
__device__ __forceinline__ uint64_t ic_live(uint64_t todo, uint32_t th, uint64_t e, uint32_t w, uint64_t seed)
{
    if (th == 0xFFFFFFFFu) return todo;
    uint64_t live = 0, rest = todo;
    while (rest) {
        const uint32_t g = (uint32_t)__builtin_ctzll(rest) >> 3;
        rest &= ~(0xFFull << (8 * g));
        const Block4 b = kChain ? philox_block_chain(e, (uint64_t)w * 8 + g, seed, kDomainIcArc)
                                : philox_block(e, (uint64_t)w * 8 + g, seed, kDomainIcArc);
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

// x of lane j (j may differ between lanes), as two 32-bit shuffles
__device__ __forceinline__ uint64_t shfl64(uint64_t x, uint32_t j)
{
    return (uint64_t)(uint32_t)__shfl((int)(uint32_t)x, (int)j) | ((uint64_t)(uint32_t)__shfl((int)(uint32_t)(x >> 32), (int)j) << 32);
}

__device__ __forceinline__ uint64_t uniform64(uint64_t x)
{
    return (uint64_t)uniform32((uint32_t)x) | ((uint64_t)uniform32((uint32_t)(x >> 32)) << 32);
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

// Sum for node J of a staged LT batch, word slot wl: lane t adds, over the
// node's in-arcs (positions pre[J] .. pre[J+1]-1 of the staged rows), the
// weight of each arc whose source is active in trial t.  With equal in-weights
// it counts the active sources and multiplies once by the node's weight.
template <int J>
__device__ __forceinline__ void ltg_sum_staged(const SimParams& P, const uint64_t (&pend)[8], const uint32_t (&pre)[9],
                                               const uint32_t (&wn)[8], uint64_t (&acc)[8], const uint32_t* R32,
                                               const uint32_t* WT, uint32_t wl, uint32_t half, uint32_t bitpos)
{
    if (pend[J] == 0) return;
    const uint32_t lo = pre[J], hi = pre[J + 1];
    const uint32_t* base = R32 + 2 * wl + half;
    if (P.lt_uniform) {
        uint32_t c = 0;
        uint32_t i = lo;
        for (; i + 1 < hi; i += 2) {
            const uint32_t b0 = __builtin_amdgcn_ubfe(base[2 * kRowPitch * i], bitpos, 1);
            const uint32_t b1 = __builtin_amdgcn_ubfe(base[2 * kRowPitch * (i + 1)], bitpos, 1);
            c = c + b0 + b1;
        }
        if (i < hi) c += __builtin_amdgcn_ubfe(base[2 * kRowPitch * i], bitpos, 1);
        acc[J] = (uint64_t)c * wn[J];
    } else {
        uint64_t a = 0;
        for (uint32_t i = lo; i < hi; ++i)
            a += (uint32_t)__builtin_amdgcn_sbfe((int)base[2 * kRowPitch * i], bitpos, 1) & WT[i];
        acc[J] = a;
    }
}

// Decide "in-weight > threshold hash" for the pending trials (pend[j], one
// bit per lane/trial) of up to 8 nodes vsu[j] of word w, given the exact
// sums acc[j] (this lane's trial).  With the prefix table (hpre[j] = this
// lane's threshold >> thp_shift) the prefixes settle every trial except a
// tie; ties, and every trial without a table, compare with the full hash:
// lane 8j+g draws the Philox block of node vsu[j] for trials 64w+8g .. +7 when
// that group holds an undecided trial.  Returns the join mask per node.
__device__ __forceinline__ void lt_decide(const SimParams& P, uint32_t w, uint32_t lane, const uint64_t (&vsu)[8],
                                          const uint64_t (&pend)[8], const uint64_t (&acc)[8], const uint32_t (&hpre)[8],
                                          uint64_t (&dec)[8])
{
    uint64_t need[8];
    uint64_t any_need = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        need[j] = 0;
        dec[j] = 0;
        if (pend[j] == 0) continue;
        if (P.thp) {
            const uint64_t hi = acc[j] >> P.thp_shift;
            const bool pb = (pend[j] >> lane) & 1ull;
            dec[j] = __ballot(pb && hi > hpre[j]);
            need[j] = __ballot(pb && hi == hpre[j]);
        } else {
            need[j] = pend[j];
        }
        any_need |= need[j];
    }
    if (any_need == 0) return;
    const uint32_t jj = lane >> 3, gg = lane & 7;
    uint64_t my_need = need[0], my_node = vsu[0];
#pragma unroll
    for (int j = 1; j < 8; ++j) {
        my_need = (jj == (uint32_t)j) ? need[j] : my_need;
        my_node = (jj == (uint32_t)j) ? vsu[j] : my_node;
    }
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
__device__ __forceinline__ void lt_eval8_core(const SimParams& P, uint64_t* Aw, const uint64_t* Bw, uint32_t w, uint32_t lane,
                                              uint64_t myv, uint64_t pl, int64_t kb, uint32_t dg, uint64_t joined[8],
                                              ArcStage* stage, uint64_t* defer)
{
    const uint64_t n = (uint64_t)P.n;
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
            const uint64_t a0 = q0 < total ? load_relaxed(&Aw[s0]) | (Bw ? Bw[s0] : 0ull) : 0ull;
            const uint64_t a1 = q1 < total ? load_relaxed(&Aw[s1]) | (Bw ? Bw[s1] : 0ull) : 0ull;
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
            const uint64_t a0 = c0 + lane < total ? load_relaxed(&Aw[(uint32_t)arc0]) | (Bw ? Bw[(uint32_t)arc0] : 0ull) : 0ull;
            const uint64_t a1 =
                c0 + 64 + lane < total ? load_relaxed(&Aw[(uint32_t)arc1]) | (Bw ? Bw[(uint32_t)arc1] : 0ull) : 0ull;
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

    uint64_t dec[8];
    lt_decide(P, w, lane, vsu, pend, acc, hpre, dec);
    // joins go into the state at once (in-place steps), or, for synchronous
    // steps, into `defer` until the step ends
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        if (dec[j] == 0) continue;
        if (lane == 0) {
            if (defer) defer[vsu[j]] = dec[j];
            else atomic_or64(&Aw[vsu[j]], dec[j]);
        }
        joined[j] = dec[j];
    }
}

// LT evaluation of up to 8 nodes of word w against the word's state row Aw,
// over the read-only base row Bw when given (a node is active in a trial when
// either has the bit; joins go to Aw only), in the trials of `tmask` only.
// Lane j < 8 passes node j in `myv` (ids >= n are absent; other lanes pass
// anything).  On return ids[j] is node j, joined[j] its new trials, first[j]
// set when it had no bit in Aw before and joined now.
__device__ __forceinline__ void lt_eval8(const SimParams& P, uint64_t* Aw, const uint64_t* Bw, uint32_t w, uint64_t tmask,
                                         uint64_t myv, uint32_t lane, uint64_t ids[8], uint64_t joined[8], bool first[8],
                                         ArcStage* stage, uint64_t* defer)
{
    const uint64_t n = (uint64_t)P.n;
    const uint64_t vm = valid_mask(w, P.W, P.T) & tmask;
    if (lane >= 8) myv = ~0ull;
#pragma unroll
    for (int j = 0; j < 8; ++j) ids[j] = uniform64(__shfl(myv, j));
    const bool okv = myv < n;
    const uint64_t av = okv ? load_relaxed(&Aw[myv]) : 0ull;
    const uint64_t pl = okv ? (vm & ~(av | (Bw ? Bw[myv] : 0ull))) : 0ull;
    const int64_t kb = pl ? P.in_off[myv] : 0;
    const uint32_t dg = pl ? (uint32_t)(P.in_off[myv + 1] - kb) : 0u;
    lt_eval8_core(P, Aw, Bw, w, lane, myv, pl, kb, dg, joined, stage, defer);
    const uint64_t was_empty = __ballot(okv && av == 0);
#pragma unroll
    for (int j = 0; j < 8; ++j) first[j] = joined[j] != 0 && ((was_empty >> j) & 1ull);
}

// =========================================================== grid shape

__device__ __forceinline__ uint64_t pack_item(uint32_t v, uint32_t w, uint32_t chunk)
{
    return (uint64_t)v | ((uint64_t)w << 32) | ((uint64_t)chunk << 44);
}

// Queue the chunks of frontier pair (v, w) for the next level, and add its
// out-arcs to that level's frontier volume.
__device__ __forceinline__ void grid_ic_enqueue(const SimParams& P, uint64_t* Q, uint32_t* count, uint32_t v, uint32_t w,
                                                unsigned long long* farcs)
{
    const uint64_t deg = (uint64_t)(P.off[v + 1] - P.off[v]);
    const uint32_t nc = (uint32_t)((deg + kChunk - 1) / kChunk);
    const uint32_t pos = atomicAdd(count, nc);
    for (uint32_t c = 0; c < nc; ++c) Q[pos + c] = pack_item(v, w, c);
    atomicAdd(farcs, (unsigned long long)deg);
}

// In-arcs of v on the pull side (IC in-CSR).
__device__ __forceinline__ unsigned long long ic_in_deg(const SimParams& P, uint32_t v)
{
    return (unsigned long long)(P.in_off[v + 1] - P.in_off[v]);
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
        if (model == 0) {
            if (vm) atomicAdd(&P.lvl_full[0], ic_in_deg(P, s));
            if (P.off[s + 1] > P.off[s]) {
                P.N[0][(uint64_t)w * n + s] = vm;
                grid_ic_enqueue(P, P.Q[0], &P.qcount[0], s, w, &P.lvl_farcs[0]);
            }
        }
    }
}

// Direction of IC level `lev` (every workgroup reaches the same answer from
// the same counters, which the previous level completed).  Beamer's rule with
// (node, word) pairs in place of nodes: leave push when the frontier's
// out-arcs exceed 1 / alpha of the in-arcs still to be pulled (those of pairs
// with an inactive trial), go back to push when the frontier holds fewer than
// 1 / beta of all pairs.
__device__ __forceinline__ bool grid_ic_pull(const SimParams& P, uint32_t lev, uint32_t cnt)
{
    if (P.ic_dir == 1) return false;
    if (P.ic_dir == 2) return true;
    const bool was_pull = lev > 0 && load_relaxed32(&P.lvl_dir[lev - 1]) == 2u;
    if (was_pull) return (double)cnt * (double)P.ic_beta >= (double)P.W * (double)P.n;
    const unsigned long long full = __hip_atomic_load(&P.lvl_full[lev], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const unsigned long long farcs = __hip_atomic_load(&P.lvl_farcs[lev], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const double todo = P.in_total > full ? (double)(P.in_total - full) : 0.0;
    return (double)farcs * (double)P.ic_alpha > todo;
}

// In-arcs above which a pulled pair is walked by its whole wavefront.
constexpr uint32_t kPullLaneDeg = 32;

// Pull walk of pair (v, w) by the calling lane alone: eight in-arcs per round,
// their loads issued together.  Returns the trials that joined; `pend` keeps
// the ones still pending.
template <bool kChain = true>
__device__ __forceinline__ uint64_t ic_pull_lane(const SimParams& P, const uint64_t* __restrict__ Fw, int64_t k0, int64_t k1,
                                                 uint32_t w, uint64_t& pend)
{
    uint64_t got = 0;
    for (int64_t k = k0; k < k1 && pend; k += 8) {
        uint64_t sa[8], f[8];
        uint32_t th[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            sa[j] = k + j < k1 ? P.ic_in[k + j] : 0ull;
            th[j] = k + j < k1 ? P.ic_in_thr[k + j] : 0u;
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) f[j] = k + j < k1 ? Fw[(uint32_t)sa[j]] : 0ull;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const uint64_t todo = f[j] & pend;
            if (todo == 0) continue;
            const uint64_t live = ic_live<kChain>(todo, th[j], sa[j] >> 32, w, P.seed);
            got |= live;
            pend &= ~live;
        }
    }
    return got;
}

// Pull walk of one pair by the whole wavefront (every lane calls it with the
// same arguments): 64 in-arcs per round, lane-strided, the joined trials
// OR-ed over the wavefront after each round so that the walk stops as soon as
// no trial is pending.
template <bool kChain = true>
__device__ __forceinline__ uint64_t ic_pull_wave(const SimParams& P, const uint64_t* __restrict__ Fw, int64_t k0, int64_t k1,
                                                 uint32_t w, uint64_t& pend, uint32_t lane)
{
    uint64_t got = 0;
    for (int64_t k = k0; k < k1 && pend; k += 64) {
        uint64_t mine = 0;
        if (k + lane < k1) {
            const uint64_t sa = P.ic_in[k + lane];
            const uint64_t todo = Fw[(uint32_t)sa] & pend;
            if (todo) mine = ic_live<kChain>(todo, P.ic_in_thr[k + lane], sa >> 32, w, P.seed);
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) mine |= __shfl_xor(mine, o);
        mine = uniform64(mine);
        got |= mine;
        pend &= ~mine;
    }
    return got;
}

// IC level `lev` by pulling: every (node v, word w) pair with an inactive
// trial walks v's in-arcs (u, e) and takes, for the pending trials in which u
// is in level lev's frontier, arc e's coin; it stops once every pending trial
// has joined.  A pair is written by its own lane only (pairs with more than
// kPullLaneDeg in-arcs are walked by the wavefront, then written by their
// lane).  New pairs join the next level's queue exactly as a push would put
// them there.
__device__ __forceinline__ void grid_ic_pull_level(const SimParams& P, uint32_t lev)
{
    const uint64_t n = (uint64_t)P.n;
    const uint64_t pairs = (uint64_t)P.W * n;
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t wave0 = (uint64_t)blockIdx.x * kBlock + (threadIdx.x & ~63u);
    const uint64_t nthreads = (uint64_t)gridDim.x * kBlock;
    if (wave0 >= pairs) return;
    const uint64_t* F = P.N[lev % 3];
    uint64_t* Nn = P.N[(lev + 1) % 3];
    uint64_t* Qn = P.Q[(lev + 1) % 3];
    uint32_t* qnext = &P.qcount[lev + 1];
    // (w, v) of pair i = w * n + v, advanced by nthreads without a division;
    // the loop runs the same rounds on every lane of a wavefront
    const uint64_t i0 = wave0 + lane;
    uint64_t w = i0 / n, v = i0 - w * n;
    const uint64_t dw = nthreads / n, dv = nthreads - dw * n;
    for (uint64_t base = wave0; base < pairs; base += nthreads) {
        const bool have = w < P.W;
        const uint64_t at = w * n + v;
        const uint64_t vm = have ? valid_mask((uint32_t)w, P.W, P.T) : 0ull;
        const uint64_t a = have ? P.A[at] : 0ull;
        uint64_t pend = vm & ~a;
        int64_t k0 = 0, k1 = 0;
        if (pend) {
            k0 = P.in_off[v];
            k1 = P.in_off[v + 1];
        }
        const uint64_t* Fw = F + w * n;
        uint64_t got = 0;
        const bool big = pend != 0 && (uint64_t)(k1 - k0) > kPullLaneDeg;
        if (pend && !big) got = ic_pull_lane(P, Fw, k0, k1, (uint32_t)w, pend);
        uint64_t bigs = __ballot(big);
        while (bigs) {
            const int j = __builtin_ctzll(bigs);
            bigs &= bigs - 1;
            uint64_t pj = uniform64(__shfl(pend, j));
            const uint64_t g = ic_pull_wave(P, F + uniform64(__shfl(w, j)) * n, (int64_t)uniform64((uint64_t)__shfl(k0, j)),
                                            (int64_t)uniform64((uint64_t)__shfl(k1, j)), (uint32_t)uniform64(__shfl(w, j)), pj, lane);
            if (lane == (uint32_t)j) {
                got = g;
                pend = pj;
            }
        }
        if (got) {
            P.A[at] = a | got;
            if (pend == 0) atomicAdd(&P.lvl_full[lev + 1], ic_in_deg(P, (uint32_t)v));
            if (P.off[v + 1] > P.off[v]) {
                Nn[at] = got;
                grid_ic_enqueue(P, Qn, qnext, (uint32_t)v, (uint32_t)w, &P.lvl_farcs[lev + 1]);
            }
        }
        v += dv;
        w += dw;
        if (v >= n) {
            v -= n;
            ++w;
        }
    }
}

// IC level `lev`: clear level lev-1's masks, then expand level lev's queue
// by push or pull (grid_ic_pull).
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
    const bool pull = grid_ic_pull(P, lev, cnt);
    if (gtid == 0) {
        P.lvl_dir[lev] = pull ? 2u : 1u;
        atomicAdd(&P.lvl_full[lev + 1], __hip_atomic_load(&P.lvl_full[lev], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
        // level lev + 1 adds into entry lev + 2 (the host clears entries 0, 1)
        if (lev + 2 < P.cap) {
            P.lvl_farcs[lev + 2] = 0;
            P.lvl_full[lev + 2] = 0;
        }
    }
    if (pull) {
        grid_ic_pull_level(P, lev);
        return;
    }
    const uint64_t* Qc = P.Q[lev % 3];
    const uint64_t* Nc = P.N[lev % 3];
    uint64_t* Nn = P.N[(lev + 1) % 3];
    uint64_t* Qn = P.Q[(lev + 1) % 3];
    uint32_t* qnext = &P.qcount[lev + 1];
    unsigned long long* farcs = &P.lvl_farcs[lev + 1];
    unsigned long long* full = &P.lvl_full[lev + 1];
    const uint32_t lane = threadIdx.x & 63u;
    // up to 64 items per wavefront (a wavefront's share of the level), their
    // arcs spread over the lanes (a prefix sum of the items' arc counts and,
    // per arc, a binary search for its item), so low-degree frontiers fill
    // the wavefront
    const uint64_t nwaves = nthreads >> 6;
    const uint64_t per = (cnt + nwaves - 1) / nwaves;
    const uint32_t chunkn = per >= 64 ? 64u : (uint32_t)per;
    for (uint64_t it0 = (gtid >> 6) * chunkn; it0 < cnt; it0 += nwaves * chunkn) {
        const bool have = lane < chunkn && it0 + lane < cnt;
        const uint64_t item = have ? Qc[it0 + lane] : 0ull;
        const uint32_t ui = (uint32_t)item;
        const uint32_t wi = (uint32_t)(item >> 32) & 0xFFFu;
        const uint64_t maski = have ? load_relaxed(&Nc[(uint64_t)wi * n + ui]) : 0ull;
        const int64_t row_end = have ? P.off[ui + 1] : 0;
        const int64_t e0i = have ? P.off[ui] + (int64_t)(item >> 44) * kChunk : 0;
        const uint32_t deg = have ? (uint32_t)((e0i + (int64_t)kChunk < row_end ? e0i + (int64_t)kChunk : row_end) - e0i) : 0u;
        uint32_t incl = deg;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t y = __shfl_up(incl, o);
            incl += lane >= (uint32_t)o ? y : 0u;
        }
        const uint32_t total = uniform32(__shfl(incl, 63));
        for (uint32_t base = 0; base < total; base += 64) {
            const uint32_t q = base + lane;
            uint32_t j = 0;
#pragma unroll
            for (uint32_t stp = 32; stp > 0; stp >>= 1) {
                const uint32_t im = (uint32_t)__shfl((int)incl, (int)(j + stp - 1));
                j += im <= q ? stp : 0u;
            }
            const uint32_t jc = j < 64u ? j : 63u;
            const uint32_t inc_j = (uint32_t)__shfl((int)incl, (int)jc);
            const uint32_t deg_j = (uint32_t)__shfl((int)deg, (int)jc);
            const int64_t e0_j = (int64_t)shfl64((uint64_t)e0i, jc);
            const uint64_t mask = shfl64(maski, jc);
            const uint32_t w = (uint32_t)__shfl((int)wi, (int)jc);
            if (q >= total) continue;
            const int64_t e = e0_j + (int64_t)(q - (inc_j - deg_j));
            const uint64_t vm = valid_mask(w, P.W, P.T);
            uint64_t* Aw = P.A + (uint64_t)w * n;
            const uint32_t v = P.idx[e];
            const uint32_t th = P.thr[e];
            if (th == 0) continue;
            // at a low mean arc probability the target's state is not read
            // first: coins of trials already active at v only OR known bits
            // in, and the atomic's old value tells the new ones apart, so a
            // failed coin (the common case) costs no access to v; at a high
            // one most targets of a dense cascade are already active, and
            // reading first saves their coins and atomics
            const uint64_t todo = P.ic_preload ? mask & ~Aw[v] : mask;
            if (todo == 0) continue;
            const uint64_t live = ic_live(todo, th, (uint64_t)e, w, P.seed);
            if (live == 0) continue;
            const uint64_t old = atomic_or64(&Aw[v], live);
            const uint64_t fresh = live & ~old;
            if (fresh == 0) continue;
            if (((old | live) & vm) == vm) atomicAdd(full, ic_in_deg(P, v));  // the pair's last trials joined
            if (P.off[v + 1] == P.off[v]) continue;
            if (atomic_or64(&Nn[(uint64_t)w * n + v], fresh) == 0) grid_ic_enqueue(P, Qn, qnext, v, w, farcs);
        }
    }
}

// Bits lo .. hi-1 of a 64-bit word (0 when empty).
__device__ __forceinline__ uint64_t range_of(uint32_t lo, uint32_t hi)
{
    return hi <= lo ? 0ull : (hi >= 64 ? ~0ull : ((1ull << hi) - 1ull)) & ~((1ull << lo) - 1ull);
}

// 64x64 bit transpose across a wavefront: on entry lane i holds row i, on exit
// lane t holds column t (bit i of the result = bit t of lane i's input).  Six
// rounds swap the off-diagonal blocks of side s = 32, 16, ..., 1 between lanes
// L and L ^ s.
__device__ __forceinline__ uint64_t wave_transpose64(uint64_t x, uint32_t lane)
{
    // Lanes L (bit s clear) and L ^ s swap blocks: L keeps the bits k with
    // (k & s) == 0 and takes its partner's such bits shifted up by s; the
    // partner keeps the (k & s) != 0 bits and takes L's shifted down.  Each
    // lane sends only the 32 bits its partner needs.  s = 32, 16, 8 move
    // whole bytes, packed and unpacked with v_perm_b32 (selector bytes 0-3
    // pick bytes of the second operand, 4-7 of the first).
    uint32_t lo = (uint32_t)x, hi = (uint32_t)(x >> 32);
    {
        const bool up = (lane & 32u) != 0;
        const uint32_t r = (uint32_t)__shfl_xor((int)(up ? lo : hi), 32);
        lo = up ? r : lo;
        hi = up ? hi : r;
    }
    {
        const bool up = (lane & 16u) != 0;
        const uint32_t r = (uint32_t)__shfl_xor((int)__builtin_amdgcn_perm(hi, lo, up ? 0x05040100u : 0x07060302u), 16);
        const uint32_t nlo = __builtin_amdgcn_perm(r, lo, up ? 0x03020504u : 0x05040100u);
        const uint32_t nhi = __builtin_amdgcn_perm(r, hi, up ? 0x03020706u : 0x07060100u);
        lo = nlo;
        hi = nhi;
    }
    {
        const bool up = (lane & 8u) != 0;
        const uint32_t r = (uint32_t)__shfl_xor((int)__builtin_amdgcn_perm(hi, lo, up ? 0x06040200u : 0x07050301u), 8);
        const uint32_t nlo = __builtin_amdgcn_perm(r, lo, up ? 0x03050104u : 0x05020400u);
        const uint32_t nhi = __builtin_amdgcn_perm(r, hi, up ? 0x03070106u : 0x07020600u);
        lo = nlo;
        hi = nhi;
    }
    x = (uint64_t)lo | ((uint64_t)hi << 32);
    // s = 4, 2, 1: bit blocks, the whole word exchanged
    constexpr uint64_t kHi[3] = {0xF0F0F0F0F0F0F0F0ull, 0xCCCCCCCCCCCCCCCCull, 0xAAAAAAAAAAAAAAAAull};
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        const uint32_t sft = 4u >> r;
        const uint64_t m = kHi[r];  // bit positions k with (k & sft) != 0
        const uint64_t y = __shfl_xor(x, (int)sft);
        const uint64_t upper = 0ull - (uint64_t)((lane & sft) != 0);
        const uint64_t keep = (m & upper) | (~m & ~upper);
        const uint64_t moved = ((y >> sft) & upper) | ((y << sft) & ~upper);
        x = (x & keep) | (moved & ~keep);
    }
    return x;
}

// ============================================== LT grid shape, node-major
//
// For the grid shape the LT state is kept node-major, Anm[v*W + w], so the
// masks of one source for all words share cache lines.  A wavefront takes a
// batch of up to 8 consecutive nodes whose in-arcs fit one 64-arc chunk,
// loads the mask row of every in-arc source once (16 words at a time) into
// LDS, and then evaluates the batch word by word from LDS.  Batches of one
// node with more than 64 in-arcs gather one word at a time instead.

// Seeds are active in every trial; their out-neighbours are marked (value 1)
// for sweep 0.  seed_arc_pre[i] = number of seed out-arcs before seed i.
__global__ __launch_bounds__(kBlock) void ltg_seed_kernel(SimParams P, const uint64_t* __restrict__ seed_arc_pre, int mark)
{
    const uint64_t W = P.W;
    const uint64_t gt = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    const uint64_t nt = (uint64_t)gridDim.x * kBlock;
    for (uint64_t i = gt; i < (uint64_t)P.n_seeds * W; i += nt) {
        const uint32_t s = P.seeds[i / W];
        const uint32_t w = (uint32_t)(i % W);
        P.Anm[(uint64_t)s * W + w] = valid_mask(w, P.W, P.T);
    }
    const uint64_t total = mark ? seed_arc_pre[P.n_seeds] : 0;
    for (uint64_t q = gt; q < total; q += nt) {
        uint32_t lo = 0, hi = P.n_seeds;  // last seed with seed_arc_pre[i] <= q
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (seed_arc_pre[mid] <= q) lo = mid; else hi = mid;
        }
        const uint32_t s = P.seeds[lo];
        const uint64_t v = P.idx[P.off[s] + (int64_t)(q - seed_arc_pre[lo])];
        for (uint64_t w = 0; w < W; ++w) P.aux[v * W + w] = 1u;
        P.nmark[v] = 1u;
    }
}

// Threshold table, node-major: th32[(v*W + w)*64 + b] = H(seed, LT, 64w + b, v).
// Lane 8j+g of a wavefront draws the block of node 8*item + j for trials
// 64w+8g .. 64w+8g+7 and stores its eight hashes (32 bytes).
__global__ __launch_bounds__(kBlock) void ltg_table_kernel(SimParams P, uint32_t* __restrict__ th32)
{
    const uint64_t n = (uint64_t)P.n;
    const uint64_t W = P.W;
    const uint64_t items = ((n + 7) / 8) * W;
    const uint32_t lane = threadIdx.x & 63u;
    for (uint64_t it = ((uint64_t)blockIdx.x * kBlock + threadIdx.x) >> 6; it < items; it += ((uint64_t)gridDim.x * kBlock) >> 6) {
        const uint32_t w = (uint32_t)(it % W);
        const uint64_t v = (it / W) * 8 + (lane >> 3);
        const uint32_t g = lane & 7;
        if (v >= n) continue;
        const Block4 b = philox_block(v, ((uint64_t)P.w0 + w) * 8 + g, P.seed, kDomainLtNode);
        uint4* dst = reinterpret_cast<uint4*>(th32 + (v * W + w) * 64 + 8 * g);
        dst[0] = make_uint4((uint32_t)b.w0, (uint32_t)(b.w0 >> 32), (uint32_t)b.w1, (uint32_t)(b.w1 >> 32));
        dst[1] = make_uint4((uint32_t)b.w2, (uint32_t)(b.w2 >> 32), (uint32_t)b.w3, (uint32_t)(b.w3 >> 32));
    }
}

// Count-threshold table (equal in-weights).  With c active in-arc pieces of
// weight w_v, c * w_v > h exactly when c >= floor(h / w_v) + 1, so the table
// holds k = floor(H(seed, LT, t, v) / w_v) + 1 per (node, trial), saturated at
// kmax = 2^S - 1 (at most 127), where S, the table's planes per word, is even
// and large enough that kmax exceeds every count a node evaluated from staged
// rows can reach (its in-arc pieces, at most 64): a saturated k is never met
// either way.  The sweep compares bit-sliced counts against it, so it is
// stored as complemented bit planes: for node v, word group g (G = ceil(W /
// kRowWords) groups) and word x of the group, the uint64
// ((v*G + g)*kRowWords + x)*S + b has bit t = NOT bit b of k for trial
// 64*(g*kRowWords + x) + t.
// A wavefront fills 8 nodes x one word group, eight words at a time: lane
// 8j+q draws node j's blocks for trials 8q .. 8q+7 of each word and stages
// the bytes in LDS (pitch 193 dwords per node and 3 per trial, so the byte
// writes of a wavefront and the row reads fall in distinct banks); then, node
// by node, lane t holds its trial's 8 bytes as a 64-bit row, and a 64x64 bit
// transpose turns bit b of byte x into lane 8x+b, the table's order.
__device__ __forceinline__ uint32_t kmin_of(uint32_t h, uint32_t wv, uint32_t inv, uint32_t kmax)
{
    // floor(h / wv) from inv = floor(2^32 / wv) (wv >= 2): the estimate is
    // low by at most one
    uint32_t q = wv == 1 ? h : __umulhi(h, inv);
    q += h - q * wv >= wv ? 1u : 0u;
    return wv == 0 ? kmax : (q < kmax - 1 ? q : kmax - 1) + 1;
}

constexpr uint32_t kKminNodePitch = 193;  // dwords per node in the staging area

__global__ __launch_bounds__(kBlock) void ltg_kmin_kernel(SimParams P, uint64_t* __restrict__ kplanes)
{
    __shared__ uint32_t stage[kWaves][8 * kKminNodePitch];
    const uint64_t n = (uint64_t)P.n;
    const uint32_t W = P.W;
    const uint64_t G = (W + kRowWords - 1) / kRowWords;
    const uint64_t items = ((n + 7) / 8) * G;
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t j = lane >> 3, q = lane & 7u;
    uint32_t* St = stage[threadIdx.x >> 6];
    uint8_t* Sb = reinterpret_cast<uint8_t*>(St);
    for (uint64_t it = ((uint64_t)blockIdx.x * kBlock + threadIdx.x) >> 6; it < items; it += ((uint64_t)gridDim.x * kBlock) >> 6) {
        const uint64_t grp = it % G;
        const uint64_t v0 = (it / G) * 8;
        const uint64_t v = v0 + j;
        const uint32_t wv = v < n ? P.node_w[v] : 0u;
        const uint32_t inv = wv >= 2 ? (uint32_t)(0x100000000ull / wv) : 0u;
        // this lane's node: its planes S and table block, k saturated at 2^S - 1
        const uint64_t ko = v < n ? P.kinfo[2 * v + 1] : 0u;
        const uint32_t S = v < n ? P.kinfo[2 * v + 3] - (uint32_t)ko : 0u;
        const uint32_t kmax = S >= 7 ? 127u : (1u << S) - 1u;
        for (uint32_t h8 = 0; h8 < kRowWords; h8 += 8) {
            for (uint32_t x = 0; x < 8; ++x) {
                const uint32_t w = (uint32_t)grp * kRowWords + h8 + x;
                uint32_t k[8];
                if (v < n && w < W && S > 0) {
                    const Block4 b = philox_block(v, ((uint64_t)P.w0 + w) * 8 + q, P.seed, kDomainLtNode);
#pragma unroll
                    for (uint32_t i = 0; i < 8; ++i) k[i] = kmin_of(block_lane(b, i), wv, inv, kmax);
                } else {
#pragma unroll
                    for (uint32_t i = 0; i < 8; ++i) k[i] = kmax;
                }
#pragma unroll
                for (uint32_t i = 0; i < 8; ++i) Sb[(j * kKminNodePitch + 3 * (8 * q + i)) * 4 + x] = (uint8_t)k[i];
            }
            __builtin_amdgcn_wave_barrier();
            for (uint32_t jj = 0; jj < 8; ++jj) {
                if (v0 + jj >= n) break;
                const uint32_t Sj = uniform32(__shfl(S, (int)(8 * jj)));
                if (Sj == 0) continue;  // a long row: no table
                const uint64_t kj = uniform64(__shfl(ko, (int)(8 * jj)));
                const uint32_t* src = St + jj * kKminNodePitch + 3 * lane;
                const uint64_t r = wave_transpose64((uint64_t)src[0] | ((uint64_t)src[1] << 32), lane);
                // lane 8x + b: plane b of word h8 + x
                if ((lane & 7u) < Sj)
                    kplanes[kj * kRowWords * G + (grp * kRowWords + h8 + (lane >> 3)) * Sj + (lane & 7u)] = ~r;
            }
            __builtin_amdgcn_wave_barrier();
        }
    }
}

// Bit-sliced counting: bit t of c[b] is bit b of trial t's count.  add4 adds
// four 0/1 vectors with three full adders and a carry ripple from weight 4
// (counts stay below 128).  v_bitop3_b32 evaluates any function of three
// bits: truth table 0x96 is their parity, 0xE8 their majority.
__device__ __forceinline__ uint64_t parity3(uint64_t a, uint64_t b, uint64_t c)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_bitop3_b32((uint32_t)a, (uint32_t)b, (uint32_t)c, 0x96);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_bitop3_b32((uint32_t)(a >> 32), (uint32_t)(b >> 32), (uint32_t)(c >> 32), 0x96);
    return (uint64_t)lo | ((uint64_t)hi << 32);
}

__device__ __forceinline__ uint64_t majority3(uint64_t a, uint64_t b, uint64_t c)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_bitop3_b32((uint32_t)a, (uint32_t)b, (uint32_t)c, 0xE8);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_bitop3_b32((uint32_t)(a >> 32), (uint32_t)(b >> 32), (uint32_t)(c >> 32), 0xE8);
    return (uint64_t)lo | ((uint64_t)hi << 32);
}

__device__ __forceinline__ void full_add(uint64_t a, uint64_t b, uint64_t c, uint64_t& sum, uint64_t& carry)
{
    sum = parity3(a, b, c);
    carry = majority3(a, b, c);
}

__device__ __forceinline__ void add4(uint64_t (&c)[7], uint64_t x0, uint64_t x1, uint64_t x2, uint64_t x3)
{
    uint64_t s0, y1, y2, z;
    full_add(c[0], x0, x1, s0, y1);
    full_add(s0, x2, x3, c[0], y2);
    full_add(c[1], y1, y2, c[1], z);
#pragma unroll
    for (int b = 2; b < 7; ++b) {
        const uint64_t t = c[b] & z;
        c[b] ^= z;
        z = t;
    }
}

// Trials whose count c is at least k, from the bit planes of c and of the
// 7-bit complement nk = 127 - k: c + nk + 1 = c - k + 128 carries out of bit
// 6 exactly when c >= k.
__device__ __forceinline__ uint64_t count_ge(const uint64_t (&c)[7], const uint64_t (&nk)[8])
{
    uint64_t carry = ~0ull;
#pragma unroll
    for (int b = 0; b < 7; ++b) carry = majority3(c[b], nk[b], carry);
    return carry;
}

// LT sweep `sw` over all words, in place.  Direction switch: a sweep "marks"
// when the previous sweep changed fewer than `tau` (node, word) pairs: every
// node that joins then stamps its out-neighbours with sw + 2 in aux (node-
// major, per word) and in nmark (per node, so a marked sweep can skip a batch
// after one load).  A sweep that follows a marking sweep evaluates only nodes stamped
// >= sw + 1 (sweep 0 follows the seeding, which marks the seeds' out-
// neighbours when they number fewer than tau); any other sweep evaluates
// every node with an inactive trial.  A node none of whose in-neighbours changed
// since its last evaluation cannot change, so both forms reach the same
// fixpoint.  A sweep that follows one without change returns at once.
// qcount[sw] counts the (node, word) pairs that changed.
// kMode: 0 = threshold hashes drawn in the kernel, 1 = threshold table,
// 2 = count-threshold table (equal in-weights) for batches of at most 64
// in-arc pieces, 3 = the batches of one node with a longer row, hashes drawn
// in the kernel (launched after kMode 2 in the same sweep).
template <int kMode>
__global__ __launch_bounds__(kBlock, 4) void ltg_sweep_kernel(SimParams P, uint32_t sw, uint32_t tau)
{
    // 64 staged rows, and 4 more that the count form may read (masked)
    __shared__ uint64_t rows[kWaves][68 * kRowPitch];
    __shared__ uint32_t wts[kWaves][64];
    if (sw >= 1 && load_relaxed32(&P.qcount[sw - 1]) == 0) return;
    if (sw >= P.cap) {
        if (blockIdx.x == 0 && threadIdx.x == 0) P.status[1] = 1;
        return;
    }
    // changes of sweep x; before sweep 0, the seeds' out-arcs times the words
    // stand for the pairs sweep 0 may change (x = -1) and for the seeding
    // itself (x = -2: the seeds mark their out-neighbours when that is below
    // tau, and sweep 0 then evaluates only those)
    auto changes = [&](int64_t x) -> uint64_t {
        return x < 0 ? P.seed_arcs * P.W : (uint64_t)load_relaxed32(&P.qcount[x]);
    };
    const bool marks_now = changes((int64_t)sw - 1) < tau;
    const bool marked_only = changes((int64_t)sw - 2) < tau;
    const uint32_t min_mark = sw + 1;
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wave = threadIdx.x >> 6;
    const uint64_t W = P.W;
    uint64_t* R = rows[wave];
    const uint32_t* R32 = reinterpret_cast<const uint32_t*>(rows[wave]);
    uint32_t* WT = wts[wave];
    const uint32_t half = lane >> 5, bitpos = lane & 31u;
    const uint64_t gwave = ((uint64_t)blockIdx.x * kBlock + threadIdx.x) >> 6;
    const uint64_t nwaves = ((uint64_t)gridDim.x * kBlock) >> 6;
    uint32_t changed = 0;

    // one batch, any threshold form: the in-arc pieces of the batch's nodes
    // are found from the in-CSR; long rows gather one word at a time
    auto batch_generic = [&](const uint32_t vf, const uint32_t nn) {
        const bool own = lane < nn;
        const uint64_t myv = own ? (uint64_t)vf + lane : 0ull;
        // a marked sweep skips batches none of whose nodes carries a mark
        if (marked_only && __ballot(own && P.nmark[myv] >= min_mark) == 0) return;
        const int64_t kb = own ? P.in_off[myv] : 0;
        const uint32_t dg = own ? (uint32_t)(P.in_off[myv + 1] - kb) : 0u;
        uint32_t incl = dg;
#pragma unroll
        for (int o = 1; o < 8; o <<= 1) {
            const uint32_t y = __shfl_up(incl, o);
            incl += lane >= (uint32_t)o ? y : 0u;
        }
        const uint32_t pre_lane = incl - dg;
        const uint32_t total = uniform32(__shfl(incl, 7));
        if (total == 0) return;  // no in-weight: these nodes never join
        const bool big = total > 64;  // a single node with a long in-arc row
        uint32_t wn_lane = 0;
        if (own && P.lt_uniform) wn_lane = P.node_w[myv];
        // this lane's in-arc (for the staged form): node, then row position
        uint32_t j_of = 0;
#pragma unroll
        for (int jj = 1; jj < 8; ++jj) j_of += (lane >= (uint32_t)__builtin_amdgcn_readlane((int)pre_lane, jj)) ? 1u : 0u;
        const uint32_t pj = __shfl(pre_lane, (int)j_of);
        const int64_t kbj = __shfl(kb, (int)j_of);
        const uint64_t my_arc = (uint64_t)kbj + (lane - pj);

        for (uint32_t wg = 0; wg < P.W; wg += kRowWords) {
            const uint32_t gw = P.W - wg < kRowWords ? P.W - wg : kRowWords;
            // stage the mask rows (this word group) of all in-arc sources:
            // R[i][x] = state of in-arc i's source at word wg + x
            auto stage_rows = [&]() {
                uint32_t src = 0, wt = 0;
                if (lane < total) {
                    if (P.lt_uniform) {
                        src = P.in_src32[my_arc];
                    } else {
                        const uint64_t arc = P.in_arc[my_arc];
                        src = (uint32_t)arc;
                        wt = (uint32_t)(arc >> 32);
                    }
                }
                // plain loads: a mask read stale within a sweep only delays a
                // join to the next sweep, and a sweep without joins saw the
                // state its launch started from
                uint64_t row[kRowWords];
                const uint64_t* rp = P.Anm + (uint64_t)src * W + wg;
                if ((W & 1) == 0 && gw == kRowWords) {
                    const uint4* rp4 = reinterpret_cast<const uint4*>(rp);
#pragma unroll
                    for (uint32_t x = 0; x < kRowWords / 2; ++x) {
                        const uint4 q = lane < total ? rp4[x] : make_uint4(0, 0, 0, 0);
                        row[2 * x] = (uint64_t)q.x | ((uint64_t)q.y << 32);
                        row[2 * x + 1] = (uint64_t)q.z | ((uint64_t)q.w << 32);
                    }
                } else {
#pragma unroll
                    for (uint32_t x = 0; x < kRowWords; ++x) row[x] = (lane < total && x < gw) ? rp[x] : 0ull;
                }
                __builtin_amdgcn_wave_barrier();
#pragma unroll
                for (uint32_t x = 0; x < kRowWords; ++x) R[lane * kRowPitch + x] = row[x];
                WT[lane] = wt;
                __builtin_amdgcn_wave_barrier();
            };
            // words of this group with a node to evaluate: lane 8j+x holds the
            // decidable trials of node j, word wg+x (pn0) and wg+x+8 (pn1)
            uint64_t pn0 = 0, pn1 = 0;
            uint32_t wmask = 0;
#pragma unroll
            for (uint32_t pass = 0; pass < 2; ++pass) {
                const uint32_t j = lane >> 3, wl = (lane & 7) + 8 * pass;
                uint64_t pn = 0;
                if (j < nn && wl < gw) {
                    const uint64_t v = (uint64_t)vf + j;
                    const uint32_t w = wg + wl;
                    pn = valid_mask(w, P.W, P.T) & ~load_relaxed(&P.Anm[v * W + w]);
                    if (pn && marked_only && P.aux[v * W + w] < min_mark) pn = 0;
                }
                if (pass) pn1 = pn; else pn0 = pn;
                uint64_t b = __ballot(pn != 0);
                b |= b >> 32;
                b |= b >> 16;
                b |= b >> 8;
                wmask |= (uint32_t)(b & 0xFFull) << (8 * pass);
            }
            wmask = uniform32(wmask);
            if (wmask == 0) continue;
            // pending trials of node j at word slot wl (uniform)
            auto pend_of = [&](uint32_t j, uint32_t wl) -> uint64_t {
                const uint64_t x = wl >= 8 ? pn1 : pn0;
                const int src = (int)(8 * j + (wl & 7));
                return (uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, src) |
                       ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(x >> 32), src) << 32);
            };
            if (!big) stage_rows();
            uint32_t wm = wmask;
            while (wm) {
                const uint32_t wl = (uint32_t)__builtin_ctz(wm);
                wm &= wm - 1;
                const uint32_t w = wg + wl;
                // equal in-weights: transpose the staged masks of this word so
                // that lane t holds "arc i active in trial t" as bit i; a node's
                // count is then the popcount of its arc range
                uint64_t colbits = 0;
                if (P.lt_uniform && !big)
                    colbits = wave_transpose64(lane < total ? R[lane * kRowPitch + wl] : 0ull, lane);
                constexpr bool kTable = kMode == 1;
                // nodes one at a time; with the threshold table the next node's
                // threshold is fetched while the current one is summed
                auto th_of = [&](uint32_t j) -> uint32_t {
                    return (kTable && j < nn && pend_of(j, wl)) ? P.th32[((uint64_t)(vf + j) * W + w) * 64 + lane] : 0u;
                };
                uint32_t h_next = th_of(0);
                for (uint32_t j = 0; j < nn; ++j) {
                    const uint32_t h_tab = h_next;
                    h_next = th_of(j + 1);
                    const uint64_t pend = pend_of(j, wl);
                    if (pend == 0) continue;
                    const uint64_t v = (uint64_t)vf + j;
                    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)pre_lane, (int)j);
                    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)incl, (int)j);
                    uint64_t acc = 0;
                    if (!big) {
                        const uint32_t* base = R32 + 2 * wl + half;
                        if (P.lt_uniform) {
                            const uint32_t c = (uint32_t)__popcll(colbits & range_of(lo, hi));
                            acc = (uint64_t)c * (uint32_t)__builtin_amdgcn_readlane((int)wn_lane, (int)j);
                        } else {
                            for (uint32_t i = lo; i < hi; ++i)
                                acc += (uint32_t)__builtin_amdgcn_sbfe((int)base[2 * kRowPitch * i], bitpos, 1) & WT[i];
                        }
                    } else {
                        // one node: gather this word's source masks 64 arcs at a time
                        const int64_t kb0 = uniform64((uint64_t)__shfl(kb, 0));
                        for (uint32_t c = 0; c < total; c += 64) {
                            const uint32_t q = c + lane;
                            uint32_t src = 0, wt = 0;
                            if (q < total) {
                                const uint64_t arc = P.in_arc[(uint64_t)kb0 + q];
                                src = (uint32_t)arc;
                                wt = (uint32_t)(arc >> 32);
                            }
                            const uint64_t a = q < total ? load_relaxed(&P.Anm[(uint64_t)src * W + w]) : 0ull;
                            __builtin_amdgcn_wave_barrier();
                            R[lane * kRowPitch] = a;
                            WT[lane] = wt;
                            __builtin_amdgcn_wave_barrier();
                            const uint32_t cnt = total - c < 64 ? total - c : 64;
                            for (uint32_t i = 0; i < cnt; ++i) {
                                const uint32_t h32 = R32[2 * (i * kRowPitch) + half];
                                acc += (uint32_t)__builtin_amdgcn_sbfe((int)h32, bitpos, 1) & WT[i];
                            }
                            __builtin_amdgcn_wave_barrier();
                        }
                    }
                    // this lane's trial: join when the in-weight exceeds its hash
                    uint32_t h = h_tab;
                    if (kMode != 1) {
                        const Block4 blk = philox_block(v, ((uint64_t)P.w0 + w) * 8 + (lane >> 3), P.seed, kDomainLtNode);
                        h = block_lane(blk, lane & 7);
                    }
                    const bool join = acc > (uint64_t)h;
                    const uint64_t dec = __ballot(join) & pend;
                    if (dec == 0) continue;
                    if (lane == 0) atomic_or64(&P.Anm[v * W + w], dec);
                    ++changed;
                    if (marks_now)
                        for (int64_t e = P.off[v] + lane; e < P.off[v + 1]; e += 64) {
                                const uint64_t t = P.idx[e];
                                P.aux[t * W + w] = sw + 2;
                                P.nmark[t] = sw + 2;
                            }
                }
            }
            __builtin_amdgcn_wave_barrier();
        }
    };
    if (kMode == 2) {
        // count thresholds, bit-sliced.  In a dense sweep batch descriptors
        // come two batches ahead and, over at most 16 words, the own states,
        // in-arc sources and node offsets one batch ahead, so a batch starts
        // knowing its pending trials and only lanes with pending trials load
        // threshold planes.  A marked sweep finds its batches 64 at a time.
        // The loads that depend only on the descriptor (node offsets, in-arc
        // sources, planes) are issued before any is waited on, and the source
        // rows follow: two dependent memory round trips per batch with work.
        // over at most 16 words, a batch's first loads come one batch ahead
        const bool pre = P.W <= kRowWords;
        const uint32_t x = lane & 15u;
        // a batch's in-arc source of this lane and the in-CSR offsets of its
        // nodes 0 .. nn (low halves suffice: only differences below 2^32 are
        // used), from clamped addresses
        auto src_of = [&](const u32x4 d) -> uint32_t {
            const uint32_t dtot = uniform32(d.y) >> 8;
            const uint64_t da0 = (uint64_t)uniform32(d.z) | ((uint64_t)uniform32(d.w) << 32);
            if (dtot == 0) return 0u;  // no in-arc to read (the batch is skipped)
            return P.in_src32[da0 + (lane < dtot && dtot <= 64 ? lane : 0u)];
        };
        // ... and, of the same nodes, the first threshold plane
        auto info_of = [&](const u32x4 d) -> uint2 {
            const uint32_t dvf = uniform32(d.x), dnn = uniform32(d.y) & 0xFFu;
            return reinterpret_cast<const uint2*>(P.kinfo)[(uint64_t)dvf + (lane <= dnn ? lane : dnn)];
        };
        // a batch's first loads: own states (and marks in a marked sweep) of
        // both passes, in-arc source, node offsets and first planes
        struct First {
            uint64_t own[2];
            uint32_t mk[2], src;
            uint2 info;
        };
        auto first_of = [&](const u32x4 d, First& f) {
            const uint32_t dvf = uniform32(d.x), dnn = uniform32(d.y) & 0xFFu;
            const uint32_t xc = x < P.W ? x : 0u;
#pragma unroll
            for (uint32_t p = 0; p < 2; ++p) {
                const uint32_t j = 4 * p + (lane >> 4);
                const uint64_t cell = (uint64_t)(dvf + (j < dnn ? j : 0u)) * W + xc;
                f.own[p] = P.Anm[cell];
                f.mk[p] = marked_only ? P.aux[cell] : 0u;
            }
            f.src = src_of(d);
            f.info = info_of(d);
        };
        // one batch: descriptor and (over at most 16 words) its first loads
        auto process = [&](const u32x4 dcur, const First& fc) {
            const uint32_t vf = uniform32(dcur.x);
            const uint32_t nn = uniform32(dcur.y) & 0xFFu;
            const uint32_t total = uniform32(dcur.y) >> 8;
            const uint64_t arc0 = (uint64_t)uniform32(dcur.z) | ((uint64_t)uniform32(dcur.w) << 32);
            if (total == 0) return;  // no in-weight: these nodes never join
            if (total > 64) return;  // a long row: the kMode 3 launch
            for (uint32_t wg = 0; wg < P.W; wg += kRowWords) {
                const uint32_t gw = P.W - wg < kRowWords ? P.W - wg : kRowWords;
                const uint64_t G = (W + kRowWords - 1) / kRowWords;
                const uint64_t grp = wg / kRowWords;
                const uint32_t xc = x < gw ? x : 0u;
                // own states of both passes (in pass p, lane 16i + x takes
                // node 4p + i at word wg + x), from clamped addresses with the
                // results masked afterwards
                bool live[2];
                uint64_t own[2], mk[2] = {0, 0};
#pragma unroll
                for (uint32_t p = 0; p < 2; ++p) {
                    const uint32_t j = 4 * p + (lane >> 4);
                    live[p] = j < nn && x < gw;
                    const uint64_t cell = (uint64_t)(vf + (j < nn ? j : 0u)) * W + wg + xc;
                    if (pre) {
                        own[p] = fc.own[p];
                        mk[p] = fc.mk[p];
                    } else {
                        own[p] = P.Anm[cell];
                        if (marked_only) mk[p] = P.aux[cell];
                    }
                }
                uint64_t pq[2];
                uint32_t passes = 0;
                auto pending = [&]() {
#pragma unroll
                    for (uint32_t p = 0; p < 2; ++p) {
                        const uint64_t pn = live[p] ? valid_mask(wg + x, P.W, P.T) & ~own[p] : 0ull;
                        pq[p] = marked_only && mk[p] < min_mark ? 0ull : pn;
                        passes |= (__ballot(pq[p] != 0) != 0 ? 1u : 0u) << p;
                    }
                    passes = uniform32(passes);
                };
                // known pending trials (prefetched, or a marked sweep's own
                // round trip): decide now; otherwise (a dense sweep over more
                // than 16 words) load rows and planes at once and decide after
                const bool known = pre || marked_only;
                if (known) {
                    pending();
                    if (passes == 0) continue;
                }
                const uint32_t src = pre ? fc.src : src_of(dcur);
                const uint2 info = pre ? fc.info : info_of(dcur);
                const uint32_t offl = info.x;
                // complemented threshold planes: 64 bytes from the lane's
                // first plane (the table is padded so this stays inside it);
                // planes beyond the node's S are those of a zero bit.
                // (Non-temporal loads here measured 5% slower per call.)
                auto load_planes = [&](uint32_t p, uint64_t (&k)[8]) {
#pragma unroll
                    for (uint32_t q = 0; q < 8; ++q) k[q] = ~0ull;
                    const uint32_t j = 4 * p + (lane >> 4);
                    const uint32_t f0 = (uint32_t)__shfl((int)info.y, (int)j);
                    const uint32_t S = (uint32_t)__shfl((int)info.y, (int)(j + 1)) - f0;
                    if (known && pq[p] == 0) return;
                    const u32x4a8* kp = reinterpret_cast<const u32x4a8*>(
                        P.kplanes + (uint64_t)f0 * kRowWords * G + (grp * kRowWords + xc) * S);
#pragma unroll
                    for (uint32_t q = 0; q < 4; ++q) {
                        const u32x4a8 t = kp[q];
                        k[2 * q] = (uint64_t)t.x | ((uint64_t)t.y << 32);
                        k[2 * q + 1] = (uint64_t)t.z | ((uint64_t)t.w << 32);
                    }
#pragma unroll
                    for (uint32_t b = 0; b < 8; ++b) k[b] = b < S ? k[b] : ~0ull;
                };
                uint64_t k0[8];
                load_planes(0, k0);
                // stage the source rows of this word group: R[i][x] = state of
                // in-arc i's source at word wg + x.  Plain loads: a mask read
                // stale within a sweep only delays a join to the next sweep,
                // and a sweep without joins saw the state it started from
                {
                    const uint64_t* rp = P.Anm + (uint64_t)src * W + wg;
                    __builtin_amdgcn_wave_barrier();
                    if ((W & 1) == 0 && gw == kRowWords) {
                        uint64_t row[kRowWords];
                        const uint4* rp4 = reinterpret_cast<const uint4*>(rp);
#pragma unroll
                        for (uint32_t y = 0; y < kRowWords / 2; ++y) {
                            const uint4 q = rp4[y];
                            row[2 * y] = (uint64_t)q.x | ((uint64_t)q.y << 32);
                            row[2 * y + 1] = (uint64_t)q.z | ((uint64_t)q.w << 32);
                        }
#pragma unroll
                        for (uint32_t y = 0; y < kRowWords; ++y) R[lane * kRowPitch + y] = lane < total ? row[y] : 0ull;
                    } else {
                        // odd word count or a short last group: 8-byte loads,
                        // all issued before the first is stored
                        uint64_t row[kRowWords];
#pragma unroll
                        for (uint32_t y = 0; y < kRowWords; ++y) row[y] = rp[y < gw ? y : 0u];
#pragma unroll
                        for (uint32_t y = 0; y < kRowWords; ++y) R[lane * kRowPitch + y] = lane < total && y < gw ? row[y] : 0ull;
                    }
                    __builtin_amdgcn_wave_barrier();
                }
                if (!known) {
                    pending();
                    if (passes == 0) continue;
                }
#pragma unroll
                for (uint32_t p = 0; p < 2; ++p) {
                    if (!((passes >> p) & 1u)) continue;
                    const uint32_t j = 4 * p + (lane >> 4);
                    const uint64_t pend = pq[p];
                    const uint64_t v = (uint64_t)vf + j;
                    uint64_t k[8];
                    if (p == 0) {
#pragma unroll
                        for (uint32_t q = 0; q < 8; ++q) k[q] = k0[q];
                    } else {
                        load_planes(1, k);
                    }
                    // node j's in-arc rows: lo .. lo + d - 1
                    const uint32_t oj = (uint32_t)__shfl((int)offl, (int)j);
                    const uint32_t oj1 = (uint32_t)__shfl((int)offl, (int)(j + 1));
                    const uint32_t lo = oj - (uint32_t)arc0;
                    const uint32_t dj = oj1 - oj;
                    const uint32_t d = pend ? dj : 0u;
                    // rows to add: the longest in-arc row among nodes with a
                    // pending trial in any word (lanes 16i .. 16i + 15 share
                    // node 4p + i)
                    const uint64_t bp = __ballot(pend != 0);
                    uint32_t maxd = 0;
#pragma unroll
                    for (uint32_t i = 0; i < 4; ++i) {
                        const uint32_t di = (uint32_t)__builtin_amdgcn_readlane((int)dj, (int)(16 * i));
                        if ((bp >> (16 * i)) & 0xFFFFull) maxd = di > maxd ? di : maxd;
                    }
                    uint64_t c[7] = {0, 0, 0, 0, 0, 0, 0};
                    for (uint32_t r = 0; r < maxd; r += 4) {
                        // rows lo + r .. lo + r + 3; a lane whose row has
                        // ended reads rows it masks (at most row 67)
                        const uint32_t base = lo + r < 64u ? lo + r : 64u;
                        const uint64_t* rr = R + base * kRowPitch + x;
                        uint64_t in[4];
#pragma unroll
                        for (uint32_t u = 0; u < 4; ++u) in[u] = rr[u * kRowPitch];
#pragma unroll
                        for (uint32_t u = 0; u < 4; ++u) in[u] = r + u < d ? in[u] : 0ull;
                        add4(c, in[0], in[1], in[2], in[3]);
                    }
                    const uint64_t dec = count_ge(c, k) & pend;
                    const uint64_t db = __ballot(dec != 0);
                    if (db == 0) continue;
                    if (dec) atomic_or64(&P.Anm[v * W + wg + x], dec);
                    changed += (uint32_t)__popcll(db);
                    if (marks_now) {
                        // node by node: one pass over its out-arcs stamps
                        // every word it changed in
#pragma unroll
                        for (uint32_t i = 0; i < 4; ++i) {
                            const uint32_t mw = (uint32_t)(db >> (16 * i)) & 0xFFFFu;
                            if (mw == 0) continue;
                            const uint64_t vm = (uint64_t)vf + 4 * p + i;
                            for (int64_t e = P.off[vm] + lane; e < P.off[vm + 1]; e += 64) {
                                const uint64_t t = P.idx[e];
                                uint32_t m = mw;
                                while (m) {
                                    const uint32_t xw = (uint32_t)__builtin_ctz(m);
                                    m &= m - 1;
                                    P.aux[t * W + wg + xw] = sw + 2;
                                }
                                P.nmark[t] = sw + 2;
                            }
                        }
                    }
                }
                __builtin_amdgcn_wave_barrier();
            }
        };
        if (marked_only) {
            // a marked sweep: a wavefront scans 64 of its batches at once
            // (lane = batch; the batches of a dense sweep's wavefront, so the
            // work stays balanced) for a node stamped for this sweep and
            // evaluates only those batches
            for (uint64_t k0 = 0; gwave + k0 * nwaves < P.nbatch; k0 += 64) {
                const uint64_t b = gwave + (k0 + lane) * nwaves;
                u32x4 d = {0, 0, 0, 0};
                if (b < P.nbatch) d = P.bdesc[b];
                const uint32_t bnn = d.y & 0xFFu, btot = d.y >> 8;
                bool hit = false;
                if (btot >= 1 && btot <= 64)
                    for (uint32_t j = 0; j < bnn; ++j) hit = hit || P.nmark[(uint64_t)d.x + j] >= min_mark;
                uint64_t m = __ballot(hit);
                auto desc_at = [&](int bit) -> u32x4 {
                    u32x4 dc;
                    dc.x = (uint32_t)__builtin_amdgcn_readlane((int)d.x, bit);
                    dc.y = (uint32_t)__builtin_amdgcn_readlane((int)d.y, bit);
                    dc.z = (uint32_t)__builtin_amdgcn_readlane((int)d.z, bit);
                    dc.w = (uint32_t)__builtin_amdgcn_readlane((int)d.w, bit);
                    return dc;
                };
                // the next hit's first loads are issued before this one runs
                First fA = {};
                u32x4 dA = {0, 0, 0, 0};
                if (m) {
                    dA = desc_at((int)__builtin_ctzll(m));
                    m &= m - 1;
                    if (pre) first_of(dA, fA);
                }
                while (true) {
                    const u32x4 dc = dA;
                    const First fc = fA;
                    const bool last = m == 0;
                    if (!last) {
                        dA = desc_at((int)__builtin_ctzll(m));
                        m &= m - 1;
                        if (pre) first_of(dA, fA);
                    }
                    process(dc, fc);
                    if (last) break;
                }
            }
        } else {
            u32x4 dA = {0, 0, 0, 0}, dB = {0, 0, 0, 0};
            First fA = {};
            if (gwave < P.nbatch) {
                dA = P.bdesc[gwave];
                if (pre) first_of(dA, fA);
            }
            if (gwave + nwaves < P.nbatch) dB = P.bdesc[gwave + nwaves];
            for (uint64_t bi = gwave; bi < P.nbatch; bi += nwaves) {
                const u32x4 dcur = dA;
                const First fc = fA;
                dA = dB;
                if (bi + 2 * nwaves < P.nbatch) dB = P.bdesc[bi + 2 * nwaves];
                if (pre && bi + nwaves < P.nbatch) first_of(dA, fA);
                process(dcur, fc);
            }
        }
    } else if (kMode == 3) {
        for (uint64_t i = gwave; i < P.nbig; i += nwaves) {
            const uint32_t bi = uniform32(P.bigb[i]);
            batch_generic(uniform32(P.bfirst[bi]), uniform32(P.bfirst[bi + 1]) - uniform32(P.bfirst[bi]));
        }
    } else {
        for (uint64_t bi = gwave; bi < P.nbatch; bi += nwaves)
            batch_generic(uniform32(P.bfirst[bi]), uniform32(P.bfirst[bi + 1]) - uniform32(P.bfirst[bi]));
    }
    if (changed && lane == 0) atomicAdd(&P.qcount[sw], changed);
}

// ====================================================== word-local shape
//
// One workgroup runs the whole cascade of one task with workgroup barriers
// between steps; workgroups take tasks from a counter and never wait for each
// other.  Three launch forms share the task bodies below:
//   single set  task = 64-trial word w, state rows indexed by w;
//   many sets   task = (set, word) on one graph (same rng_seed and trials),
//               state rows indexed by the workgroup's slot;
//   batch       task = (item, word) over several graphs, IC and LT mixed,
//               state rows indexed by the workgroup's slot.
// In the slot forms the nodes a task activates are listed, so that its
// counts can be taken and its state cleared sparsely before the next task.

constexpr int kTaskBlock = 512;  // word-local workgroup: 8 wavefronts per task
constexpr int kTaskWaves = kTaskBlock / 64;

// Workgroup-shared scratch of one task.
constexpr uint32_t kBigDeg = 512;  // out-arcs above which the whole workgroup walks a frontier node
constexpr uint32_t kBigMax = 64;   // such nodes handed over per step (more are walked by one wavefront)

struct TaskShared {
    uint32_t cnt[2];
    uint32_t farcs[2];  // IC: out-arcs of the frontier lists cnt[] count
    uint32_t full;      // IC: in-arcs of nodes whose trials of the task are all active
    uint32_t pull;      // IC: the current step pulls
    uint32_t next_item;
    uint32_t nbig;
    uint32_t nover;         // hand-overs refused because kBigMax nodes were already handed over
    uint32_t big[kBigMax];  // frontier-list positions of the nodes the workgroup walks together
    uint32_t cand;
    uint32_t act;
    uint32_t base;
    uint32_t task;
    unsigned long long total;
    uint32_t trial[64];
    uint32_t lvl[64];  // per-level counts of the task's 64 trials (level counting runs)
    ArcStage stage[kTaskWaves][64];
};

// Where one task keeps its state.
constexpr uint32_t kRemWords = 16;  // LT push form: remainder words per node and slot (tasks of at most 16 trials)

struct TaskCtx {
    uint32_t w;
    uint64_t tmask;        // the task's trials within word w (all 64 but in split batch tasks)
    uint32_t group;        // the 8-trial group holding all of the task's trials, or 8 when they span more
    uint64_t* Aw;          // active masks of the task's word
    const uint64_t* Bw;    // incremental sets form: the word's base masks (read only), else null
    uint64_t* Nw;          // IC: next-step masks (zero between steps)
    uint32_t* L[2];        // frontier node lists
    uint64_t* M[2];        // IC: frontier masks
    uint32_t* C;           // LT: candidates
    uint32_t* stamp;       // LT: last stamp that collected each node
    uint32_t stamp_base;   // LT: stamps of this task are stamp_base + step
    uint32_t* act;         // slot forms: activated nodes (else null)
    uint64_t* rem;         // batch slots, LT push form: threshold remainders, rem_stride per node (else null)
    uint32_t rem_stride;   // the task's trials when at most kRemWords (else 0)
    const uint32_t* seeds;
    uint32_t n_seeds;
};

// Level counting: every trial bit of `fresh` adds one to its trial's counter.
__device__ __forceinline__ void count_level_bits(TaskShared& sh, uint64_t fresh)
{
    while (fresh) {
        atomicAdd(&sh.lvl[__builtin_ctzll(fresh)], 1u);
        fresh &= fresh - 1;
    }
}

// Writes the counters of `level` for word w and clears them (threads < 64;
// the caller separates this from the counting with barriers).
__device__ __forceinline__ void flush_level(const SimParams& P, TaskShared& sh, uint32_t w, uint32_t level)
{
    if (threadIdx.x < 64) {
        const uint32_t t = 64 * w + threadIdx.x;
        if (level < P.max_levels && t < P.T) P.level_counts[(uint64_t)level * P.T + t] = sh.lvl[threadIdx.x];
        sh.lvl[threadIdx.x] = 0;
    }
}

// Narrow tasks (all trials in one 8-trial group): a lane takes a whole
// frontier node or candidate when it has at most kNarrowDeg arcs on the side
// walked, with every load of that walk issued before any is used; nodes with
// more arcs go through the wavefront-wide walk.
constexpr uint32_t kNarrowDeg = 16;

// Called by a whole wavefront: hand frontier-list position `it` (a node with
// more than kBigDeg out-arcs) to the whole workgroup, which walks it after
// this pass; false when kBigMax nodes were already handed over this step.
__device__ __forceinline__ bool hand_over(uint32_t it, uint32_t lane, TaskShared& sh)
{
    uint32_t pos = 0;
    if (lane == 0) pos = atomicAdd(&sh.nbig, 1u);
    pos = uniform32(__shfl(pos, 0));
    if (pos >= kBigMax) {
        if (lane == 0) atomicAdd(&sh.nover, 1u);  // counted for the run's status word 3
        return false;
    }
    if (lane == 0) sh.big[pos] = it;
    return true;
}

// One IC step of a task by pulling: the frontier masks are scattered into the
// dense row Nw (zero between steps); then every node v with a pending trial
// of the task walks its in-arcs (u, e) and takes arc e's coin (keyed by its
// out-CSR id, as a push draws it) for the pending trials in which u is in the
// frontier, until every pending trial has joined.  A node is owned by one
// lane, or by one wavefront when it has more than kPullLaneDeg in-arcs.  New nodes
// go to the next list with their masks; the caller clears Nw afterwards.
template <bool kChain = true>
__device__ __forceinline__ void ic_task_pull_step(const SimParams& P, const TaskCtx& c, TaskShared& sh, uint32_t cur, uint32_t cnt,
                                                  uint64_t vm, bool levels)
{
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t w = c.w;
    const uint32_t nxt = cur ^ 1u;
    const uint32_t* Lc = cur ? c.L[1] : c.L[0];
    const uint64_t* Mc = cur ? c.M[1] : c.M[0];
    for (uint32_t i = threadIdx.x; i < cnt; i += kTaskBlock) c.Nw[Lc[i]] = Mc[i];
    __syncthreads();
    const uint64_t* F = c.Nw;
    // node v (owned by the calling lane) gained trials `got`
    auto join = [&](uint32_t v, uint64_t a, uint64_t got, bool now_full) {
        c.Aw[v] = a | got;
        if (levels) count_level_bits(sh, got);
        if (c.act && a == 0) c.act[atomicAdd(&sh.act, 1u)] = v;
        if (now_full) atomicAdd(&sh.full, (uint32_t)ic_in_deg(P, v));
        const int64_t o0 = P.off[v], o1 = P.off[v + 1];
        if (o1 > o0) {
            const uint32_t pos = atomicAdd(&sh.cnt[nxt], 1u);
            (nxt ? c.L[1] : c.L[0])[pos] = v;
            (nxt ? c.M[1] : c.M[0])[pos] = got;
            atomicAdd(&sh.farcs[nxt], (uint32_t)(o1 - o0));
        }
    };
    const uint64_t n = (uint64_t)P.n;
    for (uint64_t base = threadIdx.x & ~63u; base < n; base += kTaskBlock) {
        const uint64_t v = base + lane;
        uint64_t a = 0, pend = 0;
        int64_t k0 = 0, k1 = 0;
        if (v < n) {
            a = c.Aw[v];
            pend = vm & ~(a | (c.Bw ? c.Bw[v] : 0ull));
            if (pend) {
                k0 = P.in_off[v];
                k1 = P.in_off[v + 1];
            }
        }
        const bool big = pend != 0 && (uint64_t)(k1 - k0) > kPullLaneDeg;
        if (pend && !big) {
            uint64_t rest = pend;
            const uint64_t got = ic_pull_lane<kChain>(P, F, k0, k1, w, rest);
            if (got) join((uint32_t)v, a, got, rest == 0);
        }
        // nodes with many in-arcs: the wavefront walks them 64 arcs at a time
        uint64_t bigs = __ballot(big);
        while (bigs) {
            const int j = __builtin_ctzll(bigs);
            bigs &= bigs - 1;
            uint64_t rest = uniform64(__shfl(pend, j));
            const uint64_t got = ic_pull_wave<kChain>(P, F, (int64_t)uniform64((uint64_t)__shfl(k0, j)),
                                              (int64_t)uniform64((uint64_t)__shfl(k1, j)), w, rest, lane);
            if (got && lane == (uint32_t)j) join((uint32_t)v, a, got, rest == 0);
        }
    }
}

// IC cascade of one task.  Per step every wavefront takes frontier entries
// and walks their out-arcs lane-strided; a node's first new bit of the step
// appends it to the next list (counter in LDS); after a barrier the next
// list picks up its masks from Nw and clears them.  Returns the step count.
template <bool kChain = true>
__device__ __forceinline__ uint32_t ic_task(const SimParams& P, const TaskCtx& c, TaskShared& sh, bool& guard)
{
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t w = c.w;
    const uint64_t vm = valid_mask(w, P.W, P.T) & c.tmask;
    const bool levels = P.level_counts != nullptr;
    const bool can_pull = P.ic_in != nullptr && P.ic_dir != 1;
    if (threadIdx.x == 0) {
        sh.cnt[0] = 0;
        sh.cnt[1] = 0;
        sh.act = 0;
        sh.farcs[0] = 0;
        sh.full = 0;
        sh.pull = 0;
    }
    if (levels && threadIdx.x < 64) sh.lvl[threadIdx.x] = 0;
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < c.n_seeds; i += kTaskBlock) {
        const uint32_t sd = c.seeds[i];
        const uint64_t nb = vm & ~(c.Bw ? c.Bw[sd] : 0ull);  // trials the seed newly activates
        if (nb == 0) continue;
        c.Aw[sd] = nb;
        if (levels) count_level_bits(sh, nb);
        if (c.act) c.act[atomicAdd(&sh.act, 1u)] = sd;
        if (can_pull) atomicAdd(&sh.full, (uint32_t)ic_in_deg(P, sd));
        const int64_t o0 = P.off[sd], o1 = P.off[sd + 1];
        if (o1 > o0) {
            const uint32_t pos = atomicAdd(&sh.cnt[0], 1u);
            c.L[0][pos] = sd;
            c.M[0][pos] = nb;
            atomicAdd(&sh.farcs[0], (uint32_t)(o1 - o0));
        }
    }
    __syncthreads();
    if (levels) {
        flush_level(P, sh, w, 0);
        __syncthreads();
    }
    uint32_t cur = 0, steps = 0;
    for (;;) {
        const uint32_t cnt = sh.cnt[cur];
        if (cnt == 0) break;
        if (steps + 1 >= P.cap) {
            guard = true;
            break;
        }
        ++steps;
        const uint32_t nxt = cur ^ 1u;
        __syncthreads();
        if (threadIdx.x == 0) {
            sh.cnt[nxt] = 0;
            sh.farcs[nxt] = 0;
            sh.next_item = 0;
            sh.nbig = 0;
            // direction of this step: Beamer's rule on the task's own
            // frontier (push -> pull when its out-arcs times alpha exceed the
            // in-arcs of nodes with a pending trial; pull -> push when it
            // holds fewer than n / beta nodes)
            bool pull = false;
            if (can_pull) {
                if (P.ic_dir == 2) {
                    pull = true;
                } else if (sh.pull) {
                    pull = (double)cnt * (double)P.ic_beta >= (double)P.n;
                } else {
                    const uint64_t in_m = (uint64_t)P.in_off[P.n];
                    const double todo = in_m > sh.full ? (double)(in_m - sh.full) : 0.0;
                    pull = (double)sh.farcs[cur] * (double)P.ic_alpha > todo;
                }
            }
            sh.pull = pull ? 1u : 0u;
        }
        __syncthreads();
        const bool pull = sh.pull != 0;
        // one out-arc e = (u, v) of a frontier node whose new trials are `mask`
        auto exam = [&](int64_t e, uint32_t v, uint32_t th, uint64_t mask) {
            if (th == 0) return;
            // without a base row the target's state is not read first: the
            // coins of trials already active at v only OR known bits in, and
            // the atomic's old value tells the new ones apart, so a failed
            // coin (the common case) costs no access to v at all
            const uint64_t bw = c.Bw ? c.Bw[v] : 0ull;
            const uint64_t todo = c.Bw ? mask & ~(c.Aw[v] | bw) : mask;
            if (todo == 0) return;
            const uint64_t live = ic_live<kChain>(todo, th, (uint64_t)e, w, P.seed);
            if (live == 0) return;
            const uint64_t old = atomic_or64(&c.Aw[v], live);
            const uint64_t fresh = live & ~old;
            if (levels) count_level_bits(sh, fresh);
            if (c.act && old == 0) c.act[atomicAdd(&sh.act, 1u)] = v;
            if (fresh == 0) return;
            if (can_pull && ((old | live | bw) & vm) == vm) atomicAdd(&sh.full, (uint32_t)ic_in_deg(P, v));
            const int64_t o0 = P.off[v], o1 = P.off[v + 1];
            if (o1 == o0) return;
            if (atomic_or64(&c.Nw[v], fresh) == 0) {
                const uint32_t pos = atomicAdd(&sh.cnt[nxt], 1u);
                (nxt ? c.L[1] : c.L[0])[pos] = v;
                atomicAdd(&sh.farcs[nxt], (uint32_t)(o1 - o0));
            }
        };
        if (pull) {
            ic_task_pull_step<kChain>(P, c, sh, cur, cnt, vm, levels);
        } else {
            // up to 64 frontier nodes per wavefront (a wavefront's share of a
            // small frontier), their out-arcs spread over the lanes (a prefix
            // sum of the degrees and, per arc, a binary search for its node),
            // so low-degree frontiers fill the wavefront; nodes with more than
            // kBigDeg out-arcs are handed to the workgroup
            const uint32_t chunk = cnt >= 64u * kTaskWaves ? 64u : (cnt + kTaskWaves - 1) / kTaskWaves;
            for (;;) {
                uint32_t it = 0;
                if (lane == 0) it = atomicAdd(&sh.next_item, chunk);
                it = __shfl(it, 0);
                if (it >= cnt) break;
                const bool have = lane < chunk && it + lane < cnt;
                const uint32_t u = have ? (cur ? c.L[1] : c.L[0])[it + lane] : 0u;
                const uint64_t mask = have ? (cur ? c.M[1] : c.M[0])[it + lane] : 0ull;
                const int64_t e0 = have ? P.off[u] : 0;
                uint32_t deg = have ? (uint32_t)(P.off[u + 1] - e0) : 0u;
                uint64_t big = __ballot(deg > kBigDeg);
                while (big) {
                    const int j = __builtin_ctzll(big);
                    big &= big - 1;
                    if (hand_over(it + (uint32_t)j, lane, sh) && lane == (uint32_t)j) deg = 0;
                }
                uint32_t incl = deg;
#pragma unroll
                for (int o = 1; o < 64; o <<= 1) {
                    const uint32_t y = __shfl_up(incl, o);
                    incl += lane >= (uint32_t)o ? y : 0u;
                }
                const uint32_t total = uniform32(__shfl(incl, 63));
                for (uint32_t base = 0; base < total; base += 64) {
                    const uint32_t q = base + lane;
                    uint32_t j = 0;
#pragma unroll
                    for (uint32_t stp = 32; stp > 0; stp >>= 1) {
                        const uint32_t im = (uint32_t)__shfl((int)incl, (int)(j + stp - 1));
                        j += im <= q ? stp : 0u;
                    }
                    const uint32_t jc = j < 64u ? j : 63u;
                    const uint32_t inc_j = (uint32_t)__shfl((int)incl, (int)jc);
                    const uint32_t deg_j = (uint32_t)__shfl((int)deg, (int)jc);
                    const int64_t e0_j = (int64_t)shfl64((uint64_t)e0, jc);
                    const uint64_t m_j = shfl64(mask, jc);
                    if (q >= total) continue;
                    const int64_t e = e0_j + (int64_t)(q - (inc_j - deg_j));
                    exam(e, P.idx[e], P.thr[e], m_j);
                }
            }
        }
        // the handed-over nodes, every wavefront on each
        __syncthreads();
        if (!pull) {
            const uint32_t nb = sh.nbig < kBigMax ? sh.nbig : kBigMax;
            for (uint32_t b = 0; b < nb; ++b) {
                const uint32_t it = sh.big[b];
                const uint32_t u = (cur ? c.L[1] : c.L[0])[it];
                const uint64_t mask = (cur ? c.M[1] : c.M[0])[it];
                const int64_t e1 = P.off[u + 1];
                for (int64_t e = P.off[u] + threadIdx.x; e < e1; e += kTaskBlock) exam(e, P.idx[e], P.thr[e], mask);
            }
        }
        __syncthreads();
        if (levels) flush_level(P, sh, w, steps);
        if (pull) {
            // the next list carries its masks already; clear the dense
            // frontier masks the step pulled from
            for (uint32_t i = threadIdx.x; i < cnt; i += kTaskBlock) c.Nw[(cur ? c.L[1] : c.L[0])[i]] = 0;
        } else {
            const uint32_t nc = sh.cnt[nxt];
            for (uint32_t i = threadIdx.x; i < nc; i += kTaskBlock) {
                const uint32_t v = (nxt ? c.L[1] : c.L[0])[i];
                (nxt ? c.M[1] : c.M[0])[i] = load_relaxed(&c.Nw[v]);
                c.Nw[v] = 0;
            }
        }
        __syncthreads();
        cur = nxt;
    }
    __syncthreads();
    return steps;
}


// byte j of the result = bit j of a (a < 256)
__device__ __forceinline__ uint64_t spread8(uint32_t a)
{
    uint64_t s = 0;
#pragma unroll
    for (uint32_t j = 0; j < 8; ++j) s |= (uint64_t)((a >> j) & 1u) << (8 * j);
    return s;
}

// LT decision for candidate v of a narrow task (trials 8g .. 8g + 7 of word
// w), pending trials `pend`, in-arc pieces k0 .. k0 + dg - 1 (dg <=
// kNarrowDeg), evaluated by one lane: the active in-weight of each pending
// trial against its threshold hash.  Returns the trials in which v joins.
__device__ __forceinline__ uint64_t lt_eval_lane(const SimParams& P, const uint64_t* Aw, const uint64_t* Bw, uint32_t w, uint32_t g,
                                                 uint64_t v, uint64_t pend, int64_t k0, uint32_t dg)
{
    const uint32_t sh = 8 * g;
    const uint32_t p8 = (uint32_t)(pend >> sh) & 0xFFu;
    uint64_t acc[8];
    if (P.lt_uniform) {
        // equal in-weights: count active sources per trial (bytes of `packed`)
        uint32_t src[kNarrowDeg];
#pragma unroll
        for (uint32_t i = 0; i < kNarrowDeg; ++i) src[i] = i < dg ? P.in_src32[k0 + i] : 0u;
        uint64_t packed = 0;
#pragma unroll
        for (uint32_t i = 0; i < kNarrowDeg; ++i)
            if (i < dg) {
                const uint64_t a = load_relaxed(&Aw[src[i]]) | (Bw ? Bw[src[i]] : 0ull);
                packed += spread8((uint32_t)(a >> sh) & p8);
            }
        const uint64_t wv = P.node_w[v];
#pragma unroll
        for (uint32_t j = 0; j < 8; ++j) acc[j] = ((packed >> (8 * j)) & 0xFFull) * wv;
    } else {
        uint64_t arc[kNarrowDeg];
#pragma unroll
        for (uint32_t i = 0; i < kNarrowDeg; ++i) arc[i] = i < dg ? P.in_arc[k0 + i] : 0ull;
#pragma unroll
        for (uint32_t j = 0; j < 8; ++j) acc[j] = 0;
#pragma unroll
        for (uint32_t i = 0; i < kNarrowDeg; ++i)
            if (i < dg) {
                const uint32_t s32 = (uint32_t)arc[i];
                const uint64_t a = load_relaxed(&Aw[s32]) | (Bw ? Bw[s32] : 0ull);
                const uint32_t a8 = (uint32_t)(a >> sh) & p8;
                const uint64_t wt = arc[i] >> 32;
#pragma unroll
                for (uint32_t j = 0; j < 8; ++j) acc[j] += ((a8 >> j) & 1u) ? wt : 0ull;
            }
    }
    const Block4 b = philox_block(v, (uint64_t)w * 8 + g, P.seed, kDomainLtNode);
    uint32_t d8 = 0;
#pragma unroll
    for (uint32_t j = 0; j < 8; ++j) d8 |= (((p8 >> j) & 1u) && acc[j] > (uint64_t)block_lane(b, j)) ? 1u << j : 0u;
    return (uint64_t)d8 << sh;
}

// LT cascade of one task of at most 16 trials in push form (the batch's
// tasks of 8 or 16 trials, without level counts).  Section 2's rule, v joins when the weight of its
// active in-neighbours exceeds its threshold h, is kept as a remainder
// r = h - (weight of the in-neighbours active so far) per (node, trial):
// a node that joins subtracts its out-arcs' weights from their targets'
// remainders in the next step, and a target joins in a trial when a
// subtraction takes its remainder below zero.  Each remainder is one 64-bit
// word, task tag (31 bits) | joined (1 bit) | remainder (32 bits), updated by
// compare-and-swap; a word that carries another task's tag holds nothing yet
// and starts from h = H(seed, LT, t, v), drawn then, so the words need no
// clearing between tasks.  Where the pull form reads every in-arc of every
// candidate once per step, this form touches one word per out-arc and newly
// joined trial.  Joins in a step become visible within it, but the fixpoint
// (the final state) is the same.  The wavefront spreads the out-arcs of up to 64
// frontier nodes (a wavefront's share of a small frontier) over its lanes (a
// prefix sum of their degrees and a binary search for each arc's node), so
// hubs and small nodes mix.  A node keeps
// one remainder word per trial of the task (c.rem_stride of them: the task's
// trials are consecutive bits of word w, from bit t0), at most kRemWords.

__device__ __forceinline__ uint32_t lt_task_push(const SimParams& P, const TaskCtx& c, TaskShared& sh, bool& guard)
{
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t w = c.w;
    const uint32_t t0 = (uint32_t)__builtin_ctzll(c.tmask);
    const uint64_t vm = valid_mask(w, P.W, P.T) & c.tmask;
    const uint64_t tag = (uint64_t)((c.stamp_base + 1u) & 0x7FFFFFFFu) << 33;
    constexpr uint64_t kJoined = 1ull << 32;
    uint64_t* Nn = c.Nw;  // trials that joined and are not pushed yet (zero between tasks)
    if (threadIdx.x == 0) {
        sh.cnt[0] = 0;
        sh.cnt[1] = 0;
        sh.act = 0;
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < c.n_seeds; i += kTaskBlock) {
        const uint32_t sd = c.seeds[i];
        const uint64_t nb = vm & ~(c.Bw ? c.Bw[sd] : 0ull);
        if (nb == 0) continue;
        c.Aw[sd] = nb;
        Nn[sd] = nb;
        // a seed's trials count as joined: its remainders never cross
        for (uint64_t bm = nb; bm; bm &= bm - 1) c.rem[(uint64_t)sd * c.rem_stride + (__builtin_ctzll(bm) - t0)] = tag | kJoined;
        c.L[0][atomicAdd(&sh.cnt[0], 1u)] = sd;
        if (c.act) c.act[atomicAdd(&sh.act, 1u)] = sd;
    }
    __syncthreads();
    uint32_t cur = 0, steps = 0;
    for (;;) {
        const uint32_t cnt = sh.cnt[cur];
        if (cnt == 0) break;
        const uint32_t* Lc = cur ? c.L[1] : c.L[0];
        if (steps + 1 >= P.cap) {
            guard = true;
            for (uint32_t i = threadIdx.x; i < cnt; i += kTaskBlock) Nn[Lc[i]] = 0;
            break;
        }
        ++steps;
        const uint32_t nxt = cur ^ 1u;
        uint32_t* Ln = nxt ? c.L[1] : c.L[0];
        __syncthreads();
        if (threadIdx.x == 0) {
            sh.cnt[nxt] = 0;
            sh.next_item = 0;
        }
        __syncthreads();
        const uint32_t chunk = cnt >= 64u * kTaskWaves ? 64u : (cnt + kTaskWaves - 1) / kTaskWaves;
        for (;;) {
            uint32_t it = 0;
            if (lane == 0) it = atomicAdd(&sh.next_item, chunk);
            it = __shfl(it, 0);
            if (it >= cnt) break;
            const bool have = lane < chunk && it + lane < cnt;
            const uint32_t u = have ? Lc[it + lane] : 0u;
            const uint64_t m = have ? atomicExch((unsigned long long*)&Nn[u], 0ull) & vm : 0ull;
            const int64_t e0 = m ? P.off[u] : 0;
            const uint32_t deg = m ? (uint32_t)(P.off[u + 1] - e0) : 0u;
            uint32_t incl = deg;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const uint32_t y = __shfl_up(incl, o);
                incl += lane >= (uint32_t)o ? y : 0u;
            }
            const uint32_t total = uniform32(__shfl(incl, 63));
            for (uint32_t base = 0; base < total; base += 64) {
                const uint32_t q = base + lane;
                // the arc's node: the number of lanes whose inclusive degree
                // sum is at most q
                uint32_t j = 0;
#pragma unroll
                for (uint32_t stp = 32; stp > 0; stp >>= 1) {
                    const uint32_t im = (uint32_t)__shfl((int)incl, (int)(j + stp - 1));
                    j += im <= q ? stp : 0u;
                }
                const uint32_t jc = j < 64u ? j : 63u;
                const uint32_t inc_j = (uint32_t)__shfl((int)incl, (int)jc);
                const uint32_t deg_j = (uint32_t)__shfl((int)deg, (int)jc);
                const int64_t e0_j = (int64_t)shfl64((uint64_t)e0, jc);
                const uint64_t m_j = shfl64(m, jc);
                if (q >= total) continue;
                const int64_t e = e0_j + (int64_t)(q - (inc_j - deg_j));
                const uint32_t v = P.idx[e];
                const uint64_t wt = P.lt_wout[e];
                if (wt == 0) continue;
                // trials where v is active already carry the joined bit (seeds
                // from the start, the others from their crossing)
                uint64_t todo = m_j;
                uint64_t* r = c.rem + (uint64_t)v * c.rem_stride;
                uint64_t dec = 0;
                uint32_t drawn = 8;  // the 8-trial group whose block blk holds (8: none)
                Block4 blk{0, 0, 0, 0};
                while (todo) {
                    const uint32_t b = (uint32_t)__builtin_ctzll(todo);
                    todo &= todo - 1;
                    const uint32_t k = b - t0;
                    uint64_t old = load_relaxed(&r[k]);
                    for (;;) {
                        uint64_t rem;
                        if ((old >> 33) != (tag >> 33)) {
                            if (drawn != (b >> 3)) {
                                drawn = b >> 3;
                                blk = philox_block(v, (uint64_t)w * 8 + drawn, P.seed, kDomainLtNode);
                            }
                            rem = block_lane(blk, b & 7u);
                        } else {
                            if (old & kJoined) break;  // this trial joined already
                            rem = (uint32_t)old;
                        }
                        const bool cross = wt > rem;
                        const uint64_t nw = tag | (cross ? kJoined : rem - wt);
                        const uint64_t prev = atomicCAS((unsigned long long*)&r[k], (unsigned long long)old, (unsigned long long)nw);
                        if (prev == old) {
                            if (cross) dec |= 1ull << b;
                            break;
                        }
                        old = prev;
                    }
                }
                if (dec) {
                    // each (node, trial) crosses once, so dec holds new trials only
                    const uint64_t oa = atomic_or64(&c.Aw[v], dec);
                    const uint64_t on = atomic_or64(&Nn[v], dec);
                    if (on == 0) Ln[atomicAdd(&sh.cnt[nxt], 1u)] = v;
                    if (c.act && oa == 0) c.act[atomicAdd(&sh.act, 1u)] = v;
                }
            }
        }
        __syncthreads();
        cur = nxt;
    }
    return steps;
}

// LT cascade of one task.  The frontier list holds the nodes that joined in
// the previous step (any trial); their out-neighbours with an inactive trial
// are collected once each into a candidate list (stamp_base + step marks the
// collection), then wavefronts evaluate candidates eight at a time; nodes
// that joined form the next frontier.  Returns the step count.
template <bool kPush = false>
__device__ __forceinline__ uint32_t lt_task(const SimParams& P, const TaskCtx& c, TaskShared& sh, bool& guard)
{
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t w = c.w;
    const uint64_t vm = valid_mask(w, P.W, P.T) & c.tmask;
    const bool narrow = c.group < 8;
    // with level counts the steps are synchronous: every candidate of a step
    // sees the state the step started from, and the joins (held in Nw) land
    // at the step's end, so step l activates exactly the nodes of level l
    const bool levels = P.level_counts != nullptr;
    if constexpr (kPush) {
        if (!levels && c.rem && c.rem_stride && !c.Bw && P.lt_wout) return lt_task_push(P, c, sh, guard);
    }
    if (threadIdx.x == 0) {
        sh.cnt[0] = 0;
        sh.cnt[1] = 0;
        sh.act = 0;
    }
    if (levels && threadIdx.x < 64) sh.lvl[threadIdx.x] = 0;
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < c.n_seeds; i += kTaskBlock) {
        const uint32_t sd = c.seeds[i];
        const uint64_t nb = vm & ~(c.Bw ? c.Bw[sd] : 0ull);  // trials the seed newly activates
        if (nb == 0) continue;
        c.Aw[sd] = nb;
        if (levels) count_level_bits(sh, nb);
        c.L[0][atomicAdd(&sh.cnt[0], 1u)] = sd;
        if (c.act) c.act[atomicAdd(&sh.act, 1u)] = sd;
    }
    __syncthreads();
    if (levels) {
        flush_level(P, sh, w, 0);
        __syncthreads();
    }
    uint32_t cur = 0, steps = 0;
    for (;;) {
        const uint32_t cnt = sh.cnt[cur];
        if (cnt == 0) break;
        if (steps + 1 >= P.cap) {
            guard = true;
            break;
        }
        ++steps;
        const uint32_t mark = c.stamp_base + steps;
        const uint32_t nxt = cur ^ 1u;
        __syncthreads();
        if (threadIdx.x == 0) {
            sh.cnt[nxt] = 0;
            sh.cand = 0;
            sh.next_item = 0;
            sh.nbig = 0;
        }
        __syncthreads();
        // push side: out-neighbours of the frontier with an inactive trial
        auto collect = [&](uint32_t v) {
            if ((vm & ~(c.Aw[v] | (c.Bw ? c.Bw[v] : 0ull))) == 0) return;
            if (atomicMax(&c.stamp[v], mark) < mark) c.C[atomicAdd(&sh.cand, 1u)] = v;
        };
        if (narrow) {
            // a lane per frontier node of at most kNarrowDeg out-arcs
            for (;;) {
                uint32_t it = 0;
                if (lane == 0) it = atomicAdd(&sh.next_item, 64u);
                it = __shfl(it, 0);
                if (it >= cnt) break;
                const bool have = it + lane < cnt;
                const uint32_t u = have ? (cur ? c.L[1] : c.L[0])[it + lane] : 0u;
                const int64_t e0 = have ? P.off[u] : 0;
                const uint32_t deg = have ? (uint32_t)(P.off[u + 1] - e0) : 0u;
                if (deg <= kNarrowDeg) {
                    uint32_t vv[kNarrowDeg];
#pragma unroll
                    for (uint32_t i = 0; i < kNarrowDeg; ++i) vv[i] = i < deg ? P.idx[e0 + i] : 0u;
#pragma unroll
                    for (uint32_t i = 0; i < kNarrowDeg; ++i)
                        if (i < deg) collect(vv[i]);
                }
                uint64_t big = __ballot(deg > kNarrowDeg);
                while (big) {
                    const int j = __builtin_ctzll(big);
                    big &= big - 1;
                    if (uniform32(__shfl(deg, j)) > kBigDeg && hand_over(it + (uint32_t)j, lane, sh)) continue;
                    const uint32_t ub = uniform32(__shfl(u, j));
                    const int64_t e1 = P.off[ub + 1];
                    for (int64_t e = P.off[ub] + lane; e < e1; e += 64) collect(P.idx[e]);
                }
            }
        } else {
            for (;;) {
                uint32_t it = 0;
                if (lane == 0) it = atomicAdd(&sh.next_item, 1u);
                it = __shfl(it, 0);
                if (it >= cnt) break;
                const uint32_t u = (cur ? c.L[1] : c.L[0])[it];
                const int64_t e0 = P.off[u], e1 = P.off[u + 1];
                if ((uint64_t)(e1 - e0) > kBigDeg && hand_over(it, lane, sh)) continue;
                for (int64_t e = e0 + lane; e < e1; e += 64) collect(P.idx[e]);
            }
        }
        // the handed-over nodes, every wavefront on each
        __syncthreads();
        {
            const uint32_t nb = sh.nbig < kBigMax ? sh.nbig : kBigMax;
            for (uint32_t b = 0; b < nb; ++b) {
                const uint32_t u = (cur ? c.L[1] : c.L[0])[sh.big[b]];
                const int64_t e1 = P.off[u + 1];
                for (int64_t e = P.off[u] + threadIdx.x; e < e1; e += kTaskBlock) collect(P.idx[e]);
            }
        }
        __syncthreads();
        if (threadIdx.x == 0) sh.next_item = 0;
        __syncthreads();
        // pull side: evaluate candidates eight at a time (narrow tasks: a lane
        // per candidate of at most kNarrowDeg in-arc pieces, the others eight
        // at a time)
        const uint32_t ncand = sh.cand;
        auto eval8 = [&](uint64_t mine) {
            uint64_t vs[8], joined[8];
            bool first[8];
            lt_eval8(P, c.Aw, c.Bw, w, c.tmask, mine, lane, vs, joined, first, sh.stage[threadIdx.x >> 6],
                     levels ? c.Nw : nullptr);
#pragma unroll
            for (int j = 0; j < 8; ++j)
                if (joined[j] && lane == 0) {
                    (nxt ? c.L[1] : c.L[0])[atomicAdd(&sh.cnt[nxt], 1u)] = (uint32_t)vs[j];
                    if (c.act && first[j]) c.act[atomicAdd(&sh.act, 1u)] = (uint32_t)vs[j];
                }
        };
        if (narrow) {
            for (;;) {
                uint32_t it = 0;
                if (lane == 0) it = atomicAdd(&sh.next_item, 64u);
                it = __shfl(it, 0);
                if (it >= ncand) break;
                const bool have = it + lane < ncand;
                const uint32_t v = have ? c.C[it + lane] : 0u;
                const uint64_t av = have ? load_relaxed(&c.Aw[v]) : 0ull;
                const uint64_t pend = have ? vm & ~(av | (c.Bw ? c.Bw[v] : 0ull)) : 0ull;
                const int64_t k0 = pend ? P.in_off[v] : 0;
                const uint32_t dg = pend ? (uint32_t)(P.in_off[v + 1] - k0) : 0u;
                const bool small = pend != 0 && dg <= kNarrowDeg;
                const uint64_t dec = small ? lt_eval_lane(P, c.Aw, c.Bw, w, c.group, v, pend, k0, dg) : 0ull;
                if (dec) {
                    if (levels) c.Nw[v] = dec;
                    else atomic_or64(&c.Aw[v], dec);
                    (nxt ? c.L[1] : c.L[0])[atomicAdd(&sh.cnt[nxt], 1u)] = v;
                    if (c.act && av == 0) c.act[atomicAdd(&sh.act, 1u)] = v;
                }
                uint64_t wide = __ballot(pend != 0 && !small);
                while (wide) {
                    uint64_t mine = ~0ull;
#pragma unroll
                    for (uint32_t q = 0; q < 8; ++q) {
                        if (!wide) break;
                        const int j = __builtin_ctzll(wide);
                        wide &= wide - 1;
                        const uint32_t vj = uniform32(__shfl(v, j));
                        if (lane == q) mine = vj;
                    }
                    eval8(mine);
                }
            }
        } else {
            for (;;) {
                uint32_t it = 0;
                if (lane == 0) it = atomicAdd(&sh.next_item, 8u);
                it = __shfl(it, 0);
                if (it >= ncand) break;
                eval8((lane < 8 && it + lane < ncand) ? (uint64_t)c.C[it + lane] : ~0ull);
            }
        }
        __syncthreads();
        if (levels) {
            // the step's joins land together; each joined node is listed once
            const uint32_t nj = sh.cnt[nxt];
            for (uint32_t i = threadIdx.x; i < nj; i += kTaskBlock) {
                const uint32_t v = (nxt ? c.L[1] : c.L[0])[i];
                const uint64_t d = c.Nw[v];
                c.Aw[v] |= d;
                c.Nw[v] = 0;
                count_level_bits(sh, d);
            }
            __syncthreads();
            flush_level(P, sh, w, steps);
            __syncthreads();
        }
        cur = nxt;
    }
    __syncthreads();
    return steps;
}

// Slot forms, after a task: fold the listed nodes' masks into the outputs and
// clear them.  total += sum of popcounts; node_counts[v] += popcount (when
// given); trial_counts[64w + b] += number of listed nodes with bit b (when
// given).
__device__ __forceinline__ void finish_slot_task(const TaskCtx& c, uint32_t n_act, TaskShared& sh, uint64_t* total, uint32_t* node_counts,
                                 uint32_t* trial_counts, uint32_t T)
{
    const uint32_t lane = threadIdx.x & 63u;
    if (threadIdx.x < 64) sh.trial[threadIdx.x] = 0;
    if (threadIdx.x == 0) sh.total = 0;
    __syncthreads();
    unsigned long long mine = 0;
    uint32_t tcount = 0;  // this lane's trial (bit) count over the wavefront's nodes
    for (uint32_t base = (threadIdx.x & ~63u); base < n_act; base += kTaskBlock) {
        const uint32_t i = base + lane;
        const uint32_t v = i < n_act ? c.act[i] : 0u;
        const uint64_t x = i < n_act ? c.Aw[v] : 0ull;
        const uint32_t pc = (uint32_t)__popcll(x);
        mine += pc;
        if (i < n_act) {
            if (node_counts) atomicAdd(&node_counts[v], pc);
            c.Aw[v] = 0;
        }
        if (trial_counts) {
            // only the task's trials can be set
            for (uint64_t bm = c.tmask; bm; bm &= bm - 1) {
                const uint32_t b = (uint32_t)__builtin_ctzll(bm);
                const uint64_t bal = __ballot((x >> b) & 1ull);
                tcount += (lane == b) ? (uint32_t)__popcll(bal) : 0u;
            }
        }
    }
    for (int o = 32; o > 0; o >>= 1) mine += __shfl_down(mine, o);
    if (lane == 0 && mine) atomicAdd(&sh.total, mine);
    if (trial_counts && tcount) atomicAdd(&sh.trial[lane], tcount);
    __syncthreads();
    if (threadIdx.x == 0 && sh.total) atomicAdd((unsigned long long*)total, sh.total);
    if (trial_counts && threadIdx.x < 64) {
        const uint64_t t = (uint64_t)c.w * 64 + threadIdx.x;
        if (sh.trial[threadIdx.x] && t < T) atomicAdd(&trial_counts[t], sh.trial[threadIdx.x]);
    }
    __syncthreads();
}

// Single-set and many-sets forms.
template <bool kSets, bool kLT>
__global__ __launch_bounds__(kTaskBlock, 2) void word_kernel(SimParams P, uint64_t list_cap)
{
    __shared__ TaskShared sh;
    const uint64_t n = (uint64_t)P.n;
    const uint32_t n_tasks = kSets ? P.n_sets * P.W : P.W;
    uint32_t max_steps = 0;
    bool guard = false;
    if (threadIdx.x == 0) sh.nover = 0;
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) sh.task = atomicAdd(P.task_counter, 1u);
        __syncthreads();
        const uint32_t t = sh.task;
        if (t >= n_tasks) break;
        TaskCtx c;
        c.rem = nullptr;
        c.rem_stride = 0;
        c.tmask = ~0ull;
        c.group = 8;
        uint32_t set = 0;
        uint64_t slot;
        if (kSets) {
            set = t / P.W;
            c.w = t % P.W;
            slot = blockIdx.x;
            const uint32_t b = P.set_off[set];
            c.seeds = P.set_nodes + b;
            c.n_seeds = P.set_off[set + 1] - b;
            c.act = P.act + slot * n;
        } else {
            c.w = t;
            slot = t;
            c.seeds = P.seeds;
            c.n_seeds = P.n_seeds;
            c.act = nullptr;
        }
        c.Aw = P.A + slot * n;
        c.Bw = (kSets && P.base) ? P.base + (uint64_t)c.w * n : nullptr;
        c.L[0] = (uint32_t*)P.Q[0] + slot * list_cap;
        c.L[1] = (uint32_t*)P.Q[1] + slot * list_cap;
        if (!kLT) {
            c.Nw = P.N[0] + slot * n;
            c.M[0] = (uint64_t*)P.Q[2] + slot * list_cap * 2;
            c.M[1] = c.M[0] + list_cap;
            c.C = nullptr;
            c.stamp = nullptr;
            c.stamp_base = 0;
        } else {
            c.Nw = (!kSets && P.level_counts) ? P.N[0] + slot * n : nullptr;
            c.M[0] = c.M[1] = nullptr;
            c.C = (uint32_t*)P.Q[2] + slot * list_cap;
            c.stamp = (kSets ? P.sstamp : P.aux) + slot * n;
            if (threadIdx.x == 0) sh.base = kSets ? P.slot_steps[slot] : 0u;
            __syncthreads();
            c.stamp_base = sh.base;
        }
        const uint32_t steps = kLT ? lt_task(P, c, sh, guard) : ic_task(P, c, sh, guard);
        if (kLT) {
            if (kSets) {
                if (threadIdx.x == 0) P.slot_steps[slot] = c.stamp_base + steps + 1;
            } else {
                for (uint64_t v = threadIdx.x; v < n; v += kTaskBlock) c.stamp[v] = 0;
            }
        }
        if (kSets) finish_slot_task(c, sh.act, sh, &P.totals[set], P.set_node_counts ? P.set_node_counts + (uint64_t)set * n : nullptr,
                                    nullptr, P.T);
        max_steps = steps > max_steps ? steps : max_steps;
    }
    if (threadIdx.x == 0) {
        atomicMax(&P.status[0], max_steps);
        if (sh.nover) atomicAdd(&P.status[3], sh.nover);
        if (guard) P.status[1] = 1;
    }
}

// One item of a batch: its graph and run parameters (P.seeds, P.n_seeds,
// P.T, P.W, P.seed) and its outputs.
struct BatchItem {
    SimParams P;
    int model;
    uint32_t* trial_counts;  // [T]
    uint32_t* node_counts;   // [n] or null
    uint64_t* total;         // [1]
};

// Batch form: tasks[t] = item << 32 | s << 24 | part << 16 | word, in the
// order the schedule chose: the task runs trials [part * 64 / 2^s,
// (part + 1) * 64 / 2^s) of the word (s = 0: the whole word).  Slot state
// rows are sized for the largest item.
__device__ __forceinline__ uint64_t split_mask(uint32_t s, uint32_t part)
{
    const uint32_t width = 64u >> s;
    return s == 0 ? ~0ull : ((1ull << width) - 1ull) << (width * part);
}

// Slot state of the batch and single-run slot forms: rows of max_n entries
// per workgroup slot.
struct SlotBufs {
    uint64_t max_n;
    uint64_t* sA;
    uint64_t* sN;
    uint32_t* sQ0;
    uint32_t* sQ1;
    uint64_t* sQ2;
    uint32_t* sact;
    uint32_t* sstamp;
    uint32_t* slot_steps;
    uint64_t* srem;  // [slot][max_n][kRemWords] LT threshold remainders (the batch form), else null
};

// IC slot runs on graphs of at most kLdsNodes nodes keep each task's active
// and next-step masks in LDS (2 x 32 KB per workgroup slot, two slots per
// compute unit): every target check and join of a step is then an LDS
// access instead of a round trip to L2.
constexpr uint32_t kLdsNodes = 4096;

// The persistent loop of the slot forms: workgroups take task indices from
// the counter; task_of(t, item, w, s, part) names the task's item, word and
// trial part.  kLds: the masks live in LDS (max_n <= kLdsNodes, IC items).
// kModel: 0 or 1 when every item is IC or LT (only that task body is built),
// -1 when the items mix both.
template <bool kChain, bool kPush, bool kLds, int kModel, typename TaskOf>
__device__ __forceinline__ void slot_tasks(TaskOf task_of, uint32_t n_tasks, uint32_t* task_counter, const SlotBufs& S,
                                           uint32_t* status, uint64_t* times = nullptr)
{
    __shared__ TaskShared sh;
    const uint64_t slot = blockIdx.x;
    const uint64_t max_n = S.max_n;
    uint32_t max_steps = 0;
    bool guard = false;
    if (threadIdx.x == 0) sh.nover = 0;
    uint64_t* lds_masks = nullptr;
    if constexpr (kLds) {
        // tasks leave the masks clear; LDS starts undefined, so clear once
        // (the loop's first barrier orders this before any task)
        __shared__ uint64_t masks[2 * kLdsNodes];
        for (uint32_t i = threadIdx.x; i < 2 * kLdsNodes; i += kTaskBlock) masks[i] = 0;
        lds_masks = masks;
    }
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) sh.task = atomicAdd(task_counter, 1u);
        __syncthreads();
        const uint32_t t = sh.task;
        if (t >= n_tasks) break;
        const BatchItem* itp;
        uint32_t w, sp, part;
        task_of(t, itp, w, sp, part);
        if (times && threadIdx.x == 0) {
            times[3 * (uint64_t)t] = wall_clock64();
            times[3 * (uint64_t)t + 2] = slot;
        }
        const BatchItem& it = *itp;
        const SimParams& P = it.P;
        TaskCtx c;
        c.w = w;
        c.tmask = split_mask(sp, part);
        c.group = sp >= 3 ? (part << (6 - sp)) >> 3 : 8u;
        c.seeds = P.seeds;
        c.n_seeds = P.n_seeds;
        c.act = S.sact + slot * max_n;
        c.Aw = kLds ? lds_masks : S.sA + slot * max_n;
        c.Bw = nullptr;
        c.L[0] = S.sQ0 + slot * max_n;
        c.L[1] = S.sQ1 + slot * max_n;
        c.Nw = kLds ? lds_masks + kLdsNodes : S.sN + slot * max_n;
        c.M[0] = S.sQ2 + slot * max_n * 2;
        c.M[1] = c.M[0] + max_n;
        c.C = (uint32_t*)(S.sQ2 + slot * max_n * 2);
        c.stamp = S.sstamp + slot * max_n;
        c.rem = S.srem ? S.srem + slot * max_n * kRemWords : nullptr;
        c.rem_stride = (64u >> sp) <= kRemWords ? 64u >> sp : 0u;
        if (threadIdx.x == 0) sh.base = S.slot_steps[slot];
        __syncthreads();
        c.stamp_base = sh.base;
        const bool lt = kModel < 0 ? it.model != 0 : kModel == 1;
        uint32_t steps;
        if constexpr (kModel == 0) steps = ic_task<kChain>(P, c, sh, guard);
        else if constexpr (kModel == 1) steps = lt_task<kPush>(P, c, sh, guard);
        else steps = lt ? lt_task<kPush>(P, c, sh, guard) : ic_task<kChain>(P, c, sh, guard);
        if (threadIdx.x == 0 && lt) S.slot_steps[slot] = c.stamp_base + steps + 1;
        finish_slot_task(c, sh.act, sh, it.total, it.node_counts, it.trial_counts, P.T);
        if (times && threadIdx.x == 0) times[3 * (uint64_t)t + 1] = wall_clock64();
        max_steps = steps > max_steps ? steps : max_steps;
    }
    if (threadIdx.x == 0) {
        atomicMax(&status[0], max_steps);
        if (sh.nover) atomicAdd(&status[3], sh.nover);
        if (guard) status[1] = 1;
    }
}

// times (or null): per task start and end of the device's constant-rate wall
// clock and the slot that ran it, [n_tasks][3].
__global__ __launch_bounds__(kTaskBlock, 4) void batch_kernel(const BatchItem* __restrict__ items, const uint64_t* __restrict__ tasks,
                                                       uint32_t n_tasks, uint32_t* task_counter, SlotBufs S, uint32_t* status,
                                                       uint64_t* times)
{
    slot_tasks<false, true, false, -1>(
        [&](uint32_t t, const BatchItem*& itp, uint32_t& w, uint32_t& sp, uint32_t& part) {
            const uint64_t code = tasks[t];
            itp = &items[code >> 32];
            w = (uint32_t)code & 0xFFFFu;
            sp = ((uint32_t)code >> 24) & 7u;
            part = ((uint32_t)code >> 16) & 63u;
        },
        n_tasks, task_counter, S, status, times);
}

// Single-run slot form: one item whose words run as 2^sp tasks each (task t =
// word t >> sp, part t & (2^sp - 1)); counts and the total accumulate into
// the item's outputs as in the batch form.  kModel: the item's model (0 IC,
// 1 LT); kLds: an IC item of at most kLdsNodes nodes, its masks in LDS.
template <int kModel, bool kLds>
__global__ __launch_bounds__(kTaskBlock, 4) void slot_run_kernel(const BatchItem* __restrict__ item, uint32_t sp, uint32_t n_tasks,
                                                          uint32_t* task_counter, SlotBufs S, uint32_t* status)
{
    static_assert(!kLds || kModel == 0, "LDS masks are for IC items");
    slot_tasks<true, false, kLds, kModel>(
        [&](uint32_t t, const BatchItem*& itp, uint32_t& w, uint32_t& spo, uint32_t& part) {
            itp = item;
            w = t >> sp;
            spo = sp;
            part = t & ((1u << sp) - 1u);
        },
        n_tasks, task_counter, S, status);
}

// ============================================================ reductions

// trial_counts[64w + b] += number of nodes with bit b of A[w*n + v] set.
// Grid: (blocks over nodes, W).  Lane b counts trial 64w + b.
// LT grid shape, last step: from the node-major state, in one pass over it,
// the per-node counts (and their total), the per-trial counts and, when asked
// for, the word-major copy A[w*n + v].  A wavefront takes 64 nodes at a time
// (lane = node) and one group of up to 16 words: a 64x64 bit transpose of each
// word turns "node v active in trial t" into lane t's 64-bit row over the
// nodes, whose popcount adds to trial t's count.  Per-trial sums meet in LDS
// before one atomic add per (block, trial).
__global__ __launch_bounds__(kBlock) void ltg_finish_kernel(const uint64_t* __restrict__ Anm, uint64_t* __restrict__ A, int64_t n,
                                                          uint32_t W, uint32_t T, uint32_t* __restrict__ trial_counts,
                                                          uint32_t* __restrict__ node_counts, unsigned long long* __restrict__ total,
                                                          int accumulate)
{
    __shared__ uint32_t part[kWaves][kRowWords][64];
    __shared__ unsigned long long tpart[kWaves];
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wave = threadIdx.x >> 6;
    const uint64_t gwave = ((uint64_t)blockIdx.x * kBlock + threadIdx.x) >> 6;
    const uint64_t nwaves = ((uint64_t)gridDim.x * kBlock) >> 6;
    const uint64_t ntiles = ((uint64_t)n + 63) / 64;
    unsigned long long sum = 0;
    for (uint32_t wg = 0; wg < W; wg += kRowWords) {
        const uint32_t gw = W - wg < kRowWords ? W - wg : kRowWords;
        uint32_t acc[kRowWords];
#pragma unroll
        for (uint32_t x = 0; x < kRowWords; ++x) acc[x] = 0;
        for (uint64_t tile = gwave; tile < ntiles; tile += nwaves) {
            const uint64_t v = tile * 64 + lane;
            const bool ok = v < (uint64_t)n;
            uint64_t wd[kRowWords];
            if ((W & 1) == 0 && gw == kRowWords) {
                const uint4* p4 = reinterpret_cast<const uint4*>(Anm + (ok ? v : 0) * W + wg);
#pragma unroll
                for (uint32_t y = 0; y < kRowWords / 2; ++y) {
                    const uint4 q = p4[y];
                    wd[2 * y] = ok ? (uint64_t)q.x | ((uint64_t)q.y << 32) : 0ull;
                    wd[2 * y + 1] = ok ? (uint64_t)q.z | ((uint64_t)q.w << 32) : 0ull;
                }
            } else {
#pragma unroll
                for (uint32_t x = 0; x < kRowWords; ++x) wd[x] = ok && x < gw ? Anm[v * W + wg + x] : 0ull;
            }
            uint32_t c = 0;
#pragma unroll
            for (uint32_t x = 0; x < kRowWords; ++x) {
                if (x >= gw) break;
                c += (uint32_t)__popcll(wd[x]);
                if (A && ok && 64u * (wg + x) < T) A[(uint64_t)(wg + x) * (uint64_t)n + v] = wd[x];
                acc[x] += (uint32_t)__popcll(wave_transpose64(wd[x], lane));
            }
            if (ok && node_counts) node_counts[v] = (wg == 0 && !accumulate ? 0u : node_counts[v]) + c;
            sum += c;
        }
#pragma unroll
        for (uint32_t x = 0; x < kRowWords; ++x) part[wave][x][lane] = acc[x];
        __syncthreads();
        for (uint32_t i = threadIdx.x; i < kRowWords * 64; i += kBlock) {
            const uint32_t x = i >> 6, t = i & 63u;
            uint32_t s2 = 0;
#pragma unroll
            for (int q = 0; q < kWaves; ++q) s2 += part[q][x][t];
            const uint64_t trial = (uint64_t)(wg + x) * 64 + t;
            if (s2 && x < gw && trial < T) atomicAdd(&trial_counts[trial], s2);
        }
        __syncthreads();
    }
    for (int o = 32; o > 0; o >>= 1) sum += __shfl_down(sum, o);
    if (lane == 0) tpart[wave] = sum;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long s2 = 0;
        for (int q = 0; q < kWaves; ++q) s2 += tpart[q];
        if (s2) atomicAdd(total, s2);
    }
}

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

// End of a grid-shape run, on the device so the host need not wait for it:
// status[0] = steps taken (the first step counter that is zero among steps
// 0 .. next - 1, else next; LT adds the final sweep that changed nothing),
// status[1] = 1 when the run was cut off at the step guard with work left.
__global__ void grid_status_kernel(const uint32_t* __restrict__ qcount, uint32_t next, uint32_t cap, uint32_t lt,
                                   uint32_t* __restrict__ status)
{
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    uint32_t steps = 0;
    while (steps < next && qcount[steps] != 0) ++steps;
    status[0] = steps + lt;
    const uint32_t last = (next + 1 < cap ? next + 1 : cap) - 1;
    if (next >= cap && qcount[last] != 0) status[1] = 1;
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
