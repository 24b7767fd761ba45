// HIP kernels of the IC / LT Monte Carlo simulator for gfx950 (wave64).
//
// Trial-bit-parallel state: for trial word w (trials 64w .. 64w+63) every node
// v owns one uint64 A[w*n + v] whose bit b says "v active in trial 64w + b".
// A wavefront works on one word at a time with lane b standing for trial
// 64w + b, so a per-node mask is at once a lane mask.
//
// IC (paper Section 2; Section 3 "Algorithms": only out-neighbours of the
// nodes activated in the previous step are examined): level-synchronous push.
// The frontier of a level is a queue of (node u, word w, arc chunk) items plus
// the mask N[w*n+u] of trials in which u joined at the previous level.  For an
// out-arc e = (u, v) the trials still to decide are mask & ~A[v]; coins are
// drawn only for the 8-trial groups that contain such a trial.  New bits are
// OR-ed into A with atomics, whose return value tells which bits are new, and
// the first writer of N[v] for the next level enqueues v.
//
// LT (Section 2): a node joins when the weight of its active in-neighbours
// exceeds its threshold.  The rule is monotone, so the final set of every trial
// is the least fixpoint above S, reached by any order of node updates.  The
// kernel therefore sweeps in place ("pull"): for every node with an inactive
// trial, sum the in-weights of active in-neighbours per trial (lane = trial)
// and compare with the threshold hash; sweeps repeat until one changes nothing.
//
// Both run inside one cooperative persistent launch; levels and sweeps are
// separated by grid-wide barriers, so the host never waits between steps.
#pragma once

#include <hip/hip_cooperative_groups.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "philox.hpp"

namespace imsim {

namespace cg = cooperative_groups;

constexpr int kBlock = 256;
constexpr uint32_t kChunk = 1024;   // out-arcs per IC work item
constexpr uint32_t kMaxWords = 4096;  // queue items carry the word in 12 bits

struct SimParams {
    int64_t n;
    uint32_t T;
    uint32_t W;
    uint64_t seed;
    int model;
    uint32_t cap;  // step guard (length of qcount)
    // out-CSR (IC)
    const int64_t* __restrict__ off;
    const uint32_t* __restrict__ idx;
    const uint32_t* __restrict__ thr;
    // in-CSR (LT): source node and 32-bit weight piece per in-arc
    const int64_t* __restrict__ in_off;
    const uint32_t* __restrict__ in_src;
    const uint32_t* __restrict__ in_w;
    // state
    uint64_t* A;
    uint64_t* N0;
    uint64_t* N1;
    uint64_t* N2;
    uint64_t* Q0;
    uint64_t* Q1;
    uint64_t* Q2;
    uint32_t* qcount;  // IC: items of level l; LT: nonzero if sweep l changed A
    const uint32_t* seeds;
    uint32_t n_seeds;
    uint32_t* status;  // [0] steps, [1] guard fired
};

__device__ __forceinline__ uint64_t valid_mask(uint32_t w, uint32_t W, uint32_t T)
{
    const uint32_t tail = T & 63u;
    return (w + 1 < W || tail == 0) ? ~0ull : ((1ull << tail) - 1ull);
}

__device__ __forceinline__ uint64_t pack_item(uint32_t v, uint32_t w, uint32_t chunk)
{
    return (uint64_t)v | ((uint64_t)w << 32) | ((uint64_t)chunk << 44);
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

__device__ __forceinline__ uint32_t n_chunks(uint64_t deg)
{
    return (uint32_t)((deg + kChunk - 1) / kChunk);
}

// ---------------------------------------------------------------- IC push

// Enqueue node v of word w for the next level (all its arc chunks).
__device__ __forceinline__ void ic_enqueue(const SimParams& P, uint64_t* Q, uint32_t* count, uint32_t v, uint32_t w)
{
    const uint64_t deg = (uint64_t)(P.off[v + 1] - P.off[v]);
    const uint32_t nc = n_chunks(deg);
    const uint32_t pos = atomicAdd(count, nc);
    for (uint32_t c = 0; c < nc; ++c) Q[pos + c] = pack_item(v, w, c);
}

// Decide the arcs of one queue item; lane-strided over its chunk of arcs.
__device__ void ic_expand_item(const SimParams& P, uint64_t item, const uint64_t* Ncur, uint64_t* Nnxt,
                               uint64_t* Qnxt, uint32_t* qnext, uint32_t lane)
{
    const uint32_t u = (uint32_t)item;
    const uint32_t w = (uint32_t)(item >> 32) & 0xFFFu;
    const uint32_t chunk = (uint32_t)(item >> 44);
    const uint64_t mask = load_relaxed(&Ncur[(uint64_t)w * P.n + u]);
    const int64_t row_end = P.off[u + 1];
    const int64_t e0 = P.off[u] + (int64_t)chunk * kChunk;
    const int64_t e1 = e0 + (int64_t)kChunk < row_end ? e0 + (int64_t)kChunk : row_end;
    uint64_t* Aw = P.A + (uint64_t)w * P.n;
    for (int64_t e = e0 + lane; e < e1; e += 64) {
        const uint32_t v = P.idx[e];
        const uint32_t th = P.thr[e];
        if (th == 0) continue;
        const uint64_t todo = mask & ~Aw[v];
        if (todo == 0) continue;
        uint64_t live;
        if (th == 0xFFFFFFFFu) {
            live = todo;
        } else {
            live = 0;
            uint64_t rest = todo;
            while (rest) {
                const uint32_t g = (uint32_t)__builtin_ctzll(rest) >> 3;
                rest &= ~(0xFFull << (8 * g));
                const Block4 b = philox_block((uint64_t)e, (uint64_t)w * 8 + g, P.seed, kDomainIcArc);
                uint32_t bits = 0;
#pragma unroll
                for (uint32_t j = 0; j < 8; ++j) bits |= (block_lane(b, j) < th ? 1u : 0u) << j;
                live |= (uint64_t)bits << (8 * g);
            }
            live &= todo;
        }
        if (live == 0) continue;
        const uint64_t old = atomic_or64(&Aw[v], live);
        const uint64_t fresh = live & ~old;
        if (fresh == 0) continue;
        if (P.off[v + 1] == P.off[v]) continue;  // no out-arcs: nothing to expand
        const uint64_t oldn = atomic_or64(&Nnxt[(uint64_t)w * P.n + v], fresh);
        if (oldn == 0) ic_enqueue(P, Qnxt, qnext, v, w);
    }
}

// ---------------------------------------------------------------- LT pull

// Evaluate nodes 8b .. 8b+7 of word w; returns true if any bit of A changed.
__device__ bool lt_eval_batch(const SimParams& P, uint32_t w, uint64_t b, uint32_t lane)
{
    const uint64_t vm = valid_mask(w, P.W, P.T);
    uint64_t* Aw = P.A + (uint64_t)w * P.n;
    const uint64_t v0 = b * 8;
    uint64_t pend[8];
    uint64_t any = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const uint64_t v = v0 + j;
        pend[j] = v < (uint64_t)P.n ? (vm & ~load_relaxed(&Aw[v])) : 0ull;
        any |= pend[j];
    }
    if (any == 0) return false;

    // per-trial active in-weight, exact in 64 bits
    uint64_t acc[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        acc[j] = 0;
        if (pend[j] == 0) continue;
        const uint64_t v = v0 + j;
        const int64_t k1 = P.in_off[v + 1];
        for (int64_t k = P.in_off[v]; k < k1; k += 4) {
            uint32_t us[4], ws[4];
            uint64_t as[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const bool ok = k + q < k1;
                us[q] = ok ? P.in_src[k + q] : 0u;
                ws[q] = ok ? P.in_w[k + q] : 0u;
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) as[q] = load_relaxed(&Aw[us[q]]);
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[j] += ((as[q] >> lane) & 1ull) ? (uint64_t)ws[q] : 0ull;
        }
    }

    // threshold hashes: lane 8j+g computes the block of node v0+j, trials
    // 64w+8g .. 64w+8g+7, when that group still has an inactive trial
    const uint32_t jj = lane >> 3, gg = lane & 7;
    uint64_t my_pend = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j) my_pend = (jj == (uint32_t)j) ? pend[j] : my_pend;
    Block4 blk{0, 0, 0, 0};
    if ((my_pend >> (8 * gg)) & 0xFFull) blk = philox_block(v0 + jj, (uint64_t)w * 8 + gg, P.seed, kDomainLtNode);

    bool changed = false;
    const uint32_t src_off = lane >> 3;
    const uint32_t sel = (lane & 7) >> 1;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        if (pend[j] == 0) continue;
        const int src = 8 * j + (int)src_off;
        const uint64_t x0 = __shfl(blk.w0, src);
        const uint64_t x1 = __shfl(blk.w1, src);
        const uint64_t x2 = __shfl(blk.w2, src);
        const uint64_t x3 = __shfl(blk.w3, src);
        const uint64_t word = sel == 0 ? x0 : sel == 1 ? x1 : sel == 2 ? x2 : x3;
        const uint32_t h = (lane & 1) ? (uint32_t)(word >> 32) : (uint32_t)word;
        const bool join = ((pend[j] >> lane) & 1ull) && acc[j] > (uint64_t)h;
        const uint64_t act = __ballot(join);
        if (act) {
            if (lane == 0) atomic_or64(&Aw[v0 + j], act);
            changed = true;
        }
    }
    return changed;
}

// ------------------------------------------------------- persistent kernel

__global__ __launch_bounds__(kBlock) void sim_persistent(SimParams P)
{
    cg::grid_group grid = cg::this_grid();
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t gtid = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    const uint64_t nthreads = (uint64_t)gridDim.x * kBlock;
    const uint64_t gwave = gtid >> 6;
    const uint64_t nwaves = nthreads >> 6;
    const uint64_t n = (uint64_t)P.n;

    // seeds: active in every trial; IC seeds with out-arcs form level 0
    const uint64_t pairs = (uint64_t)P.n_seeds * P.W;
    for (uint64_t i = gtid; i < pairs; i += nthreads) {
        const uint32_t s = P.seeds[i / P.W];
        const uint32_t w = (uint32_t)(i % P.W);
        const uint64_t vm = valid_mask(w, P.W, P.T);
        P.A[(uint64_t)w * n + s] = vm;
        if (P.model == 0 && P.off[s + 1] > P.off[s]) {
            P.N0[(uint64_t)w * n + s] = vm;
            ic_enqueue(P, P.Q0, &P.qcount[0], s, w);
        }
    }
    grid.sync();

    uint32_t steps = 0;
    bool guard = false;
    if (P.model == 0) {
        uint64_t* Nb[3] = {P.N0, P.N1, P.N2};
        uint64_t* Qb[3] = {P.Q0, P.Q1, P.Q2};
        for (uint32_t lev = 0;; ++lev) {
            // level lev-1's frontier masks are no longer needed: clear them so
            // the buffer is zero when it is reused as next-level masks
            if (lev >= 1) {
                const uint32_t oc = load_relaxed32(&P.qcount[lev - 1]);
                const uint64_t* Qo = Qb[(lev + 2) % 3];
                uint64_t* No = Nb[(lev + 2) % 3];
                for (uint64_t i = gtid; i < oc; i += nthreads) {
                    const uint64_t it = Qo[i];
                    if ((it >> 44) == 0) No[((it >> 32) & 0xFFFu) * n + (uint32_t)it] = 0;
                }
            }
            const uint32_t cnt = load_relaxed32(&P.qcount[lev]);
            if (cnt == 0) {
                steps = lev;
                break;
            }
            if (lev + 1 >= P.cap) {
                steps = lev;
                guard = true;
                break;
            }
            const uint64_t* Qc = Qb[lev % 3];
            const uint64_t* Nc = Nb[lev % 3];
            uint64_t* Nn = Nb[(lev + 1) % 3];
            uint64_t* Qn = Qb[(lev + 1) % 3];
            for (uint64_t it = gwave; it < cnt; it += nwaves)
                ic_expand_item(P, Qc[it], Nc, Nn, Qn, &P.qcount[lev + 1], lane);
            grid.sync();
        }
    } else {
        const uint64_t nb = (n + 7) / 8;
        const uint64_t items = nb * P.W;
        for (uint32_t sw = 0;; ++sw) {
            if (sw >= P.cap) {
                steps = sw;
                guard = true;
                break;
            }
            bool changed = false;
            for (uint64_t it = gwave; it < items; it += nwaves) {
                const uint32_t w = (uint32_t)(it / nb);
                const uint64_t b = it % nb;
                changed |= lt_eval_batch(P, w, b, lane);
            }
            if (changed && lane == 0) atomicAdd(&P.qcount[sw], 1u);
            grid.sync();
            if (load_relaxed32(&P.qcount[sw]) == 0) {
                steps = sw + 1;
                break;
            }
        }
    }
    if (gtid == 0) {
        P.status[0] = steps;
        P.status[1] = guard ? 1u : 0u;
    }
}

// ------------------------------------------------------------- reductions

// trial_counts[64w + b] += number of nodes with bit b of A[w*n + v] set.
// Grid: (blocks over nodes, W).  Lane b counts trial 64w + b.
__global__ __launch_bounds__(kBlock) void reduce_trial_counts(const uint64_t* __restrict__ A, int64_t n, uint32_t T,
                                                              uint32_t* __restrict__ trial_counts)
{
    __shared__ uint32_t part[kBlock / 64][64];
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
        for (int q = 0; q < kBlock / 64; ++q) s += part[q][lane];
        const uint64_t t = (uint64_t)w * 64 + lane;
        if (s && t < T) atomicAdd(&trial_counts[t], s);
    }
}

// node_counts[v] = sum_w popcount(A[w*n + v]); total += sum_v node_counts[v].
__global__ __launch_bounds__(kBlock) void reduce_node_counts(const uint64_t* __restrict__ A, int64_t n, uint32_t W,
                                                             uint32_t* __restrict__ node_counts,
                                                             unsigned long long* __restrict__ total)
{
    __shared__ unsigned long long part[kBlock / 64];
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
        for (int q = 0; q < kBlock / 64; ++q) s += part[q];
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
