// HIP kernels of the learned spread estimator (a message-passing network over
// the diffusion graph) for gfx950.
//
// Tensors of a batch of B seed sets on one graph are node-major: row r = v*B + b
// holds the features of node v for set b, so an aggregation over the arcs into
// v reads, per arc, one contiguous run of B*D values of the source node.
// Activations and gradients are stored in bf16 (raw uint16 bits); every sum is
// accumulated in fp32.  Dense layers run on the bf16 matrix cores
// (v_mfma_f32_16x16x32_bf16); the data-row axis is the MFMA column axis so a
// lane's four outputs are four consecutive channels of one row (8-byte stores).
// Reductions over rows write per-workgroup partials that a second kernel sums
// in a fixed order, so every result is deterministic.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace imsim_mpnn {

constexpr int kHidden = 64;    // channels of every hidden layer
constexpr int kIn = 16;        // padded width of the input features (4 used)
constexpr int kThreads = 256;  // threads of every workgroup here
constexpr int kWStage = 128;   // rows_per of the weight-gradient kernel is a multiple of this (4 waves x 32 rows)

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

// bf16 <-> fp32.  Rounding is to nearest, ties to even; NaN stays NaN.
__device__ __forceinline__ float bf2f(uint32_t h) { return __uint_as_float(h << 16); }

__device__ __forceinline__ uint32_t f2bf(float f)
{
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (u >> 16) | 0x40u;
    u += 0x7fffu + ((u >> 16) & 1u);
    return u >> 16;
}

__device__ __forceinline__ uint32_t pack2(float lo, float hi) { return f2bf(lo) | (f2bf(hi) << 16); }

// eight bf16 held as four 32-bit words -> eight floats
__device__ __forceinline__ void unpack8(const u32x4& r, float* f)
{
    #pragma unroll
    for (int i = 0; i < 4; ++i) {
        f[2 * i] = __uint_as_float(r[i] << 16);
        f[2 * i + 1] = __uint_as_float(r[i] & 0xffff0000u);
    }
}

__device__ __forceinline__ floatx4 mfma(const u32x4& a, const u32x4& b, floatx4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c, 0, 0,
                                                   0);
}

// A wavefront's 16 x 64 bf16 output tile goes through LDS so that its rows,
// which lie contiguously in memory, are stored 16 bytes per lane: the MFMA
// result gives each lane 8 bytes of one row only.  kTilePitch: LDS words per
// staged row (64 bf16 + 4 words, keeping 16-byte alignment).
constexpr int kTilePitch = 36;

// Lane (l16, g) puts the four values of channels c .. c+3 of row l16.
__device__ __forceinline__ void tile_put(uint32_t* tile, int l16, int c, float y0, float y1, float y2, float y3)
{
    *(u32x2*)(tile + l16 * kTilePitch + c / 2) = u32x2{pack2(y0, y1), pack2(y2, y3)};
}

// Stores the staged tile as rows row0 .. row0 + 15 of Y ([R][64]); only this
// wavefront touched `tile`, and LDS operations of one wavefront complete in
// order, so no barrier is needed.
__device__ __forceinline__ void tile_store(const uint32_t* tile, uint16_t* __restrict__ Y, int64_t row0, int64_t R, int lane)
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    #pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int c = 64 * j + lane;  // 16-byte piece c of the tile: row c / 8, piece c % 8
        const int r = c >> 3, pc = c & 7;
        const u32x4 v = *(const u32x4*)(tile + r * kTilePitch + 4 * pc);
        if (row0 + r < R) *(u32x4*)(Y + (row0 + r) * kHidden + 8 * pc) = v;
    }
    __builtin_amdgcn_wave_barrier();
}

// ---------------------------------------------------------------------------
// Input features.  Row r = v*B + b gets [s, f1(v), f2(v), f3(v), 0 ...] with
// s = 0; a second kernel sets s = 1 for the members of each set.

__global__ void features_kernel(int64_t rows, uint32_t B, const float* __restrict__ node_feat, uint16_t* __restrict__ X)
{
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < rows; r += (int64_t)gridDim.x * blockDim.x) {
        const int64_t v = r / B;
        u32x4 lo, hi = {0u, 0u, 0u, 0u};
        lo[0] = pack2(0.0f, node_feat[v * 3 + 0]);
        lo[1] = pack2(node_feat[v * 3 + 1], node_feat[v * 3 + 2]);
        lo[2] = 0u;
        lo[3] = 0u;
        u32x4* dst = (u32x4*)(X + r * kIn);
        dst[0] = lo;
        dst[1] = hi;
    }
}

__global__ void seed_scatter_kernel(uint32_t n_sets, uint32_t B, const uint32_t* __restrict__ set_off,
                                    const uint32_t* __restrict__ set_nodes, uint16_t* __restrict__ X)
{
    const uint32_t total = set_off[n_sets];
    for (uint32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < total; k += gridDim.x * blockDim.x) {
        // set b owns positions [set_off[b], set_off[b+1]): binary search
        uint32_t lo = 0, hi = n_sets;
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) / 2;
            if (set_off[mid] <= k) lo = mid; else hi = mid;
        }
        const uint64_t r = (uint64_t)set_nodes[k] * B + lo;
        X[r * kIn] = 0x3f80;  // 1.0
    }
}

// ---------------------------------------------------------------------------
// Sparse aggregation.  Y[v] = sum over arcs e of the CSR row of v of
// w[e] * X[nbr[e]], where a node row holds C = B*D bf16 values.  Forward: CSR
// = arcs into v, Y = M.  Backward: CSR = arcs out of v, and the epilogue adds
// `add` and zeroes where `relu_of` <= 0 (the ReLU of the layer below),
// producing that layer's pre-activation gradient.
//
// Work items are row segments of at most kSegArcs arcs, so a hub's row is
// spread over many workgroups: a node with a short row is one item that
// writes its output row; a long row's segments write fp32 partial rows to
// slots that a second kernel sums in slot order.  A lane owns eight
// consecutive values (16 bytes); items with C/8 < 256 chunks share a
// workgroup.

constexpr uint32_t kSegArcs = 256;
constexpr uint32_t kDirect = 0xFFFFFFFFu;

struct SpmmItem {
    uint32_t node;  // output row
    uint32_t slot;  // kDirect, or the partial row this segment writes
    uint32_t e0;    // first arc
    uint32_t len;   // arcs (<= kSegArcs for segments of split rows)
};

template <bool kBackward>
__device__ __forceinline__ void spmm_store(float* acc, uint64_t o, uint16_t* __restrict__ Y, const uint16_t* __restrict__ add,
                                           const uint16_t* __restrict__ relu_of)
{
    if constexpr (kBackward) {
        float d[8], h[8];
        unpack8(*(const u32x4*)(add + o), d);
        unpack8(*(const u32x4*)(relu_of + o), h);
        #pragma unroll
        for (int i = 0; i < 8; ++i) acc[i] = h[i] > 0.0f ? acc[i] + d[i] : 0.0f;
    }
    u32x4 out;
    #pragma unroll
    for (int i = 0; i < 4; ++i) out[i] = pack2(acc[2 * i], acc[2 * i + 1]);
    *(u32x4*)(Y + o) = out;
}

template <bool kBackward>
__global__ void __launch_bounds__(kThreads) spmm_kernel(uint32_t n_items, uint32_t C, const SpmmItem* __restrict__ items,
                                                        const uint32_t* __restrict__ nbr, const float* __restrict__ w,
                                                        const uint16_t* __restrict__ X, uint16_t* __restrict__ Y,
                                                        const uint16_t* __restrict__ add,
                                                        const uint16_t* __restrict__ relu_of, float* __restrict__ partial)
{
    const uint32_t nc = C / 8;
    const uint32_t per_block = nc >= kThreads ? 1u : kThreads / nc;
    const uint32_t local = nc >= kThreads ? 0u : threadIdx.x / nc;
    const uint64_t it = (uint64_t)blockIdx.x * per_block + local;
    if (local >= per_block || it >= n_items) return;
    const SpmmItem I = items[it];
    const uint64_t e0 = I.e0, e1 = e0 + I.len;
    const uint32_t step = nc >= kThreads ? kThreads : nc;
    for (uint32_t j = nc >= kThreads ? threadIdx.x : threadIdx.x % nc; j < nc; j += step) {
        float acc[8];
        #pragma unroll
        for (int i = 0; i < 8; ++i) acc[i] = 0.0f;
        uint64_t e = e0;
        for (; e + 8 <= e1; e += 8) {
            u32x4 r[8];
            float a[8];
            #pragma unroll
            for (int q = 0; q < 8; ++q) {
                const uint32_t u = nbr[e + q];
                a[q] = w[e + q];
                r[q] = *(const u32x4*)(X + (uint64_t)u * C + (uint64_t)j * 8);
            }
            #pragma unroll
            for (int q = 0; q < 8; ++q) {
                float f[8];
                unpack8(r[q], f);
                #pragma unroll
                for (int i = 0; i < 8; ++i) acc[i] = fmaf(a[q], f[i], acc[i]);
            }
        }
        for (; e < e1; ++e) {
            const uint32_t u = nbr[e];
            const float a = w[e];
            const u32x4 r = *(const u32x4*)(X + (uint64_t)u * C + (uint64_t)j * 8);
            float f[8];
            unpack8(r, f);
            #pragma unroll
            for (int i = 0; i < 8; ++i) acc[i] = fmaf(a, f[i], acc[i]);
        }
        if (I.slot != kDirect) {
            floatx4* dst = (floatx4*)(partial + (uint64_t)I.slot * C + (uint64_t)j * 8);
            dst[0] = floatx4{acc[0], acc[1], acc[2], acc[3]};
            dst[1] = floatx4{acc[4], acc[5], acc[6], acc[7]};
            continue;
        }
        spmm_store<kBackward>(acc, (uint64_t)I.node * C + (uint64_t)j * 8, Y, add, relu_of);
    }
}

// Rows split into segments: fin[3k .. 3k+2] = (node, first slot, slots);
// one workgroup per row sums its partial rows in slot order.
template <bool kBackward>
__global__ void __launch_bounds__(kThreads) spmm_finish_kernel(uint32_t C, const uint32_t* __restrict__ fin,
                                                               const float* __restrict__ partial, uint16_t* __restrict__ Y,
                                                               const uint16_t* __restrict__ add,
                                                               const uint16_t* __restrict__ relu_of)
{
    const uint32_t node = fin[3 * blockIdx.x], slot0 = fin[3 * blockIdx.x + 1], slots = fin[3 * blockIdx.x + 2];
    for (uint32_t j = threadIdx.x; j < C / 8; j += kThreads) {
        float acc[8];
        #pragma unroll
        for (int i = 0; i < 8; ++i) acc[i] = 0.0f;
        for (uint32_t k = 0; k < slots; ++k) {
            const floatx4* src = (const floatx4*)(partial + (uint64_t)(slot0 + k) * C + (uint64_t)j * 8);
            const floatx4 p0 = src[0], p1 = src[1];
            #pragma unroll
            for (int i = 0; i < 4; ++i) {
                acc[i] += p0[i];
                acc[4 + i] += p1[i];
            }
        }
        spmm_store<kBackward>(acc, (uint64_t)node * C + (uint64_t)j * 8, Y, add, relu_of);
    }
}

// ---------------------------------------------------------------------------
// Dense layer, forward.  Y = ReLU([Xs | Xn] W + b) for rows [0, R):
// Xs, Xn are [R][D] bf16, W is [2D][64] fp32 (rounded to bf16 here), b [64],
// Y [R][64] bf16.  MFMA: A = W^T tile (channel x k), B = X^T tile (k x row).

template <int D>
__global__ void __launch_bounds__(kThreads) dense_fwd_kernel(int64_t R, const uint16_t* __restrict__ Xs,
                                                             const uint16_t* __restrict__ Xn,
                                                             const float* __restrict__ W, const float* __restrict__ bias,
                                                             uint16_t* __restrict__ Y)
{
    constexpr int K = 2 * D;
    constexpr int KS = K / 32;      // MFMA k-steps
    constexpr int P = K + 8;        // LDS pitch (bf16) of W^T rows
    __shared__ uint16_t Wt[kHidden * P];
    __shared__ __attribute__((aligned(16))) uint32_t Ytile[kThreads / 64][16 * kTilePitch];
    uint32_t* tile = Ytile[threadIdx.x >> 6];
    for (int i = threadIdx.x; i < K * kHidden; i += kThreads) {
        const int k = i / kHidden, c = i % kHidden;
        Wt[c * P + k] = (uint16_t)f2bf(W[i]);
    }
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int l16 = lane & 15, g = lane >> 4;
    u32x4 A[4][KS];
    #pragma unroll
    for (int ct = 0; ct < 4; ++ct)
        #pragma unroll
        for (int ks = 0; ks < KS; ++ks) A[ct][ks] = *(const u32x4*)(Wt + (16 * ct + l16) * P + 32 * ks + 8 * g);
    float bv[4][4];
    #pragma unroll
    for (int ct = 0; ct < 4; ++ct)
        #pragma unroll
        for (int q = 0; q < 4; ++q) bv[ct][q] = bias[16 * ct + 4 * g + q];

    const int64_t tiles = (R + 15) / 16;
    const int64_t wave = (int64_t)blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6);
    const int64_t waves = (int64_t)gridDim.x * (kThreads / 64);
    // the next tile's rows are loaded before the current tile is computed
    auto load = [&](int64_t t, u32x4 (&Bf)[KS]) {
        const int64_t row = t * 16 + l16;
        const bool ok = row < R;
        #pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            const int kc = 32 * ks + 8 * g;
            const uint16_t* src = kc < D ? Xs + row * D + kc : Xn + row * D + (kc - D);
            Bf[ks] = ok ? *(const u32x4*)src : u32x4{0u, 0u, 0u, 0u};
        }
    };
    u32x4 Bn[KS];
    load(wave, Bn);
    for (int64_t t = wave; t < tiles; t += waves) {
        const int64_t row = t * 16 + l16;
        const bool ok = row < R;
        u32x4 Bf[KS];
        #pragma unroll
        for (int ks = 0; ks < KS; ++ks) Bf[ks] = Bn[ks];
        load(t + waves, Bn);
        floatx4 acc[4];
        #pragma unroll
        for (int ct = 0; ct < 4; ++ct) {
            acc[ct] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
            #pragma unroll
            for (int ks = 0; ks < KS; ++ks) acc[ct] = mfma(A[ct][ks], Bf[ks], acc[ct]);
        }
        (void)ok;
        #pragma unroll
        for (int ct = 0; ct < 4; ++ct) {
            float y[4];
            #pragma unroll
            for (int q = 0; q < 4; ++q) y[q] = fmaxf(acc[ct][q] + bv[ct][q], 0.0f);
            tile_put(tile, l16, 16 * ct + 4 * g, y[0], y[1], y[2], y[3]);
        }
        tile_store(tile, Y, t * 16, R, lane);
    }
}

// ---------------------------------------------------------------------------
// Dense layer, input gradient.  [dXs | dXn] = dZ W^T: dZ [R][64] bf16,
// W [2D][64] fp32; outputs [R][D] bf16 each.  MFMA: A = W tile (k x channel),
// B = dZ^T tile (channel x row).

template <int D>
__global__ void __launch_bounds__(kThreads) dense_bwd_data_kernel(int64_t R, const uint16_t* __restrict__ dZ,
                                                                  const float* __restrict__ W,
                                                                  uint16_t* __restrict__ dXs, uint16_t* __restrict__ dXn)
{
    constexpr int K = 2 * D;
    constexpr int KT = K / 16;       // 16-wide tiles of the output columns
    constexpr int P = kHidden + 8;   // LDS pitch of W rows
    __shared__ uint16_t Wb[K * P];
    static_assert(D == kHidden, "the staged output tiles hold rows of 64 values");
    __shared__ __attribute__((aligned(16))) uint32_t Otile[kThreads / 64][2][16 * kTilePitch];
    uint32_t* otile = Otile[threadIdx.x >> 6][0];
    for (int i = threadIdx.x; i < K * kHidden; i += kThreads) Wb[(i / kHidden) * P + i % kHidden] = (uint16_t)f2bf(W[i]);
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int l16 = lane & 15, g = lane >> 4;
    u32x4 A[KT][2];
    #pragma unroll
    for (int kt = 0; kt < KT; ++kt)
        #pragma unroll
        for (int ks = 0; ks < 2; ++ks) A[kt][ks] = *(const u32x4*)(Wb + (16 * kt + l16) * P + 32 * ks + 8 * g);

    const int64_t tiles = (R + 15) / 16;
    const int64_t wave = (int64_t)blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6);
    const int64_t waves = (int64_t)gridDim.x * (kThreads / 64);
    // the next tile's rows are loaded before the current tile is computed
    auto load = [&](int64_t t, u32x4 (&Bf)[2]) {
        const int64_t row = t * 16 + l16;
        const bool ok = row < R;
        #pragma unroll
        for (int ks = 0; ks < 2; ++ks)
            Bf[ks] = ok ? *(const u32x4*)(dZ + row * kHidden + 32 * ks + 8 * g) : u32x4{0u, 0u, 0u, 0u};
    };
    u32x4 Bn[2];
    load(wave, Bn);
    for (int64_t t = wave; t < tiles; t += waves) {
        const int64_t row = t * 16 + l16;
        const bool ok = row < R;
        u32x4 Bf[2] = {Bn[0], Bn[1]};
        load(t + waves, Bn);
        (void)ok;
        #pragma unroll
        for (int kt = 0; kt < KT; ++kt) {
            floatx4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
            acc = mfma(A[kt][0], Bf[0], acc);
            acc = mfma(A[kt][1], Bf[1], acc);
            const int k = 16 * kt + 4 * g;
            tile_put(otile + (k < D ? 0 : 16 * kTilePitch), l16, k < D ? k : k - D, acc[0], acc[1], acc[2], acc[3]);
        }
        tile_store(otile, dXs, t * 16, R, lane);
        tile_store(otile + 16 * kTilePitch, dXn, t * 16, R, lane);
    }
}

// ---------------------------------------------------------------------------
// 8x8 transpose of 16-bit values across each aligned group of 8 lanes: on
// entry lane 8q + j holds row j of its group's matrix (element i in half
// (i & 1) of word i >> 1), on exit it holds column j.  Three rounds swap the
// off-diagonal blocks of side 4, 2, 1 between lanes j and j ^ s; each lane
// sends the half of its row that its partner needs.

__device__ __forceinline__ u32x4 transpose8_b16(u32x4 v, uint32_t lane)
{
    {
        const bool up = (lane & 4u) != 0;
        const uint32_t r0 = (uint32_t)__shfl_xor((int)(up ? v[0] : v[2]), 4);
        const uint32_t r1 = (uint32_t)__shfl_xor((int)(up ? v[1] : v[3]), 4);
        if (up) {
            v[0] = r0;
            v[1] = r1;
        } else {
            v[2] = r0;
            v[3] = r1;
        }
    }
    {
        const bool up = (lane & 2u) != 0;
        const uint32_t r0 = (uint32_t)__shfl_xor((int)(up ? v[0] : v[1]), 2);
        const uint32_t r1 = (uint32_t)__shfl_xor((int)(up ? v[2] : v[3]), 2);
        if (up) {
            v[0] = r0;
            v[2] = r1;
        } else {
            v[1] = r0;
            v[3] = r1;
        }
    }
    {
        const bool up = (lane & 1u) != 0;
        // the lower lane sends its odd elements (high halves), the upper lane
        // its even ones (low halves), two per word
        const uint32_t p0 = up ? __builtin_amdgcn_perm(v[1], v[0], 0x05040100u) : __builtin_amdgcn_perm(v[1], v[0], 0x07060302u);
        const uint32_t p1 = up ? __builtin_amdgcn_perm(v[3], v[2], 0x05040100u) : __builtin_amdgcn_perm(v[3], v[2], 0x07060302u);
        const uint32_t q0 = (uint32_t)__shfl_xor((int)p0, 1);
        const uint32_t q1 = (uint32_t)__shfl_xor((int)p1, 1);
        if (up) {
            v[0] = __builtin_amdgcn_perm(v[0], q0, 0x07060100u);
            v[1] = __builtin_amdgcn_perm(v[1], q0, 0x07060302u);
            v[2] = __builtin_amdgcn_perm(v[2], q1, 0x07060100u);
            v[3] = __builtin_amdgcn_perm(v[3], q1, 0x07060302u);
        } else {
            v[0] = __builtin_amdgcn_perm(q0, v[0], 0x05040100u);
            v[1] = __builtin_amdgcn_perm(q0, v[1], 0x07060100u);
            v[2] = __builtin_amdgcn_perm(q1, v[2], 0x05040100u);
            v[3] = __builtin_amdgcn_perm(q1, v[3], 0x07060100u);
        }
    }
    return v;
}

// ---------------------------------------------------------------------------
// Dense layer, weight and bias gradients.  dW = [Xs | Xn]^T dZ ([2D][64]) and
// db = column sums of dZ, over rows [0, R).  Workgroup `blk` takes rows
// [blk*rows_per, (blk+1)*rows_per) (rows_per a multiple of 128); its four
// wavefronts take 32-row blocks in turn.  MFMA reduces over the row axis:
// dW^T tile (channel x column) += dZ^T (channel x 32 rows) X (32 rows x
// column).  A lane loads 16 bytes of one row (lane L: row 8 (L >> 4) +
// (L & 7) of the block, channels 8 ((L >> 3) & 1) .. + 7 of a 16-wide tile)
// and an 8x8 transpose across its group of 8 lanes turns that into the
// operand layout (eight consecutive rows of channel L & 15), so no staging in
// LDS is needed.  The wavefronts' tiles are added in LDS in wavefront order,
// then written as the workgroup's partial: part[blk * stride] holds dW
// ([2D][64]) followed by db ([64]).

template <int D>
__global__ void __launch_bounds__(kThreads) dense_bwd_weight_kernel(int64_t R, int64_t rows_per,
                                                                    const uint16_t* __restrict__ Xs,
                                                                    const uint16_t* __restrict__ Xn,
                                                                    const uint16_t* __restrict__ dZ,
                                                                    float* __restrict__ part, int64_t stride)
{
    constexpr int K = 2 * D;
    constexpr int KT = K / 16;      // 16-wide column tiles of [Xs | Xn]
    constexpr int CT = kHidden / 16;  // 16-wide channel tiles of dZ
    constexpr int kWaves = kThreads / 64;
    __shared__ floatx4 red[CT * KT][64];
    __shared__ float redb[CT][16];
    const int tid = threadIdx.x;
    const uint32_t lane = tid & 63;
    const int wv = tid >> 6;
    const int l16 = lane & 15, g = lane >> 4;
    const int64_t r_begin = (int64_t)blockIdx.x * rows_per;
    const int64_t r_end = r_begin + rows_per < R ? r_begin + rows_per : R;
    const int rl = 8 * (int)(lane >> 4) + (int)(lane & 7);  // the row of a block this lane loads
    const int half = (int)((lane >> 3) & 1u);               // which 8 columns of a 16-wide tile

    floatx4 acc[CT][KT];
    #pragma unroll
    for (int ct = 0; ct < CT; ++ct)
        #pragma unroll
        for (int kt = 0; kt < KT; ++kt) acc[ct][kt] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
    float db[CT];
    #pragma unroll
    for (int ct = 0; ct < CT; ++ct) db[ct] = 0.0f;

    for (int64_t r0 = r_begin + 32 * wv; r0 < r_end; r0 += 32 * kWaves) {
        const int64_t r = r0 + rl;
        const bool ok = r < r_end;
        u32x4 a[CT], b[KT];
        #pragma unroll
        for (int ct = 0; ct < CT; ++ct)
            a[ct] = ok ? *(const u32x4*)(dZ + r * kHidden + 16 * ct + 8 * half) : u32x4{0u, 0u, 0u, 0u};
        #pragma unroll
        for (int kt = 0; kt < KT; ++kt) {
            const int c = 16 * kt + 8 * half;
            const uint16_t* src = c < D ? Xs + r * D + c : Xn + r * D + (c - D);
            b[kt] = ok ? *(const u32x4*)src : u32x4{0u, 0u, 0u, 0u};
        }
        #pragma unroll
        for (int ct = 0; ct < CT; ++ct) {
            a[ct] = transpose8_b16(a[ct], lane);
            float f[8];
            unpack8(a[ct], f);
            #pragma unroll
            for (int i = 0; i < 8; ++i) db[ct] += f[i];
        }
        #pragma unroll
        for (int kt = 0; kt < KT; ++kt) b[kt] = transpose8_b16(b[kt], lane);
        #pragma unroll
        for (int ct = 0; ct < CT; ++ct)
            #pragma unroll
            for (int kt = 0; kt < KT; ++kt) acc[ct][kt] = mfma(a[ct], b[kt], acc[ct][kt]);
    }
    // bias: lanes l16, l16 + 16, + 32, + 48 hold rows of the same channel
    #pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
        db[ct] += __shfl_xor(db[ct], 16);
        db[ct] += __shfl_xor(db[ct], 32);
    }
    // add the wavefronts' tiles in wavefront order
    for (int w = 0; w < kWaves; ++w) {
        if (wv == w) {
            #pragma unroll
            for (int ct = 0; ct < CT; ++ct) {
                #pragma unroll
                for (int kt = 0; kt < KT; ++kt) {
                    floatx4& dst = red[ct * KT + kt][lane];
                    dst = w == 0 ? acc[ct][kt] : dst + acc[ct][kt];
                }
                if (lane < 16) redb[ct][lane] = w == 0 ? db[ct] : redb[ct][lane] + db[ct];
            }
        }
        __syncthreads();
    }
    float* pw = part + (int64_t)blockIdx.x * stride;
    for (int t = wv; t < CT * KT; t += kWaves) {
        const int ct = t / KT, kt = t % KT;
        const int k = 16 * kt + l16;
        *(floatx4*)(pw + k * kHidden + 16 * ct + 4 * g) = red[t][lane];
    }
    if (tid < kHidden) pw[K * kHidden + tid] = redb[tid >> 4][tid & 15];
}

// out[i] = sum over blk of part[blk * stride + i], i < count, in a fixed
// order: a workgroup takes 32 outputs; its slice s (of 8) sums blocks s, s+8,
// s+16, ... and the slices are added in order.
__global__ void __launch_bounds__(kThreads) sum_partials_kernel(int64_t count, int64_t blocks, int64_t stride,
                                                                const float* __restrict__ part, float* __restrict__ out)
{
    __shared__ float red[kThreads / 32][32];
    const uint32_t c = threadIdx.x & 31u, sl = threadIdx.x >> 5;
    const int64_t i = (int64_t)blockIdx.x * 32 + c;
    float s = 0.0f;
    if (i < count)
        for (int64_t b = sl; b < blocks; b += kThreads / 32) s += part[b * stride + i];
    red[sl][c] = s;
    __syncthreads();
    if (sl == 0 && i < count) {
        float t = red[0][c];
        for (uint32_t k = 1; k < kThreads / 32; ++k) t += red[k][c];
        out[i] = t;
    }
}

// ---------------------------------------------------------------------------
// Readout.  z = H3[r] . w_o + b_o (w_o rounded to bf16), yhat = 1 for a seed
// (input feature s = 1), else sigmoid(z).  Eight lanes per row.

__global__ void __launch_bounds__(kThreads) readout_fwd_kernel(int64_t R, const uint16_t* __restrict__ H,
                                                               const uint16_t* __restrict__ X0,
                                                               const float* __restrict__ w_o, float* __restrict__ Yhat)
{
    const int sub = threadIdx.x & 7;
    float wv[8];
    #pragma unroll
    for (int i = 0; i < 8; ++i) wv[i] = bf2f(f2bf(w_o[8 * sub + i]));
    const float b_o = w_o[kHidden];
    const int64_t groups = (int64_t)gridDim.x * (kThreads / 8);
    for (int64_t r = blockIdx.x * (int64_t)(kThreads / 8) + (threadIdx.x >> 3); r < R; r += groups) {
        float h[8];
        unpack8(*(const u32x4*)(H + r * kHidden + 8 * sub), h);
        float z = 0.0f;
        #pragma unroll
        for (int i = 0; i < 8; ++i) z = fmaf(h[i], wv[i], z);
        z += __shfl_xor(z, 1);
        z += __shfl_xor(z, 2);
        z += __shfl_xor(z, 4);
        if (sub == 0) {
            const bool seed = X0[r * kIn] != 0;
            Yhat[r] = seed ? 1.0f : 1.0f / (1.0f + expf(-(z + b_o)));
        }
    }
}

// part[blk][b] = sum over nodes v of workgroup blk's range of Yhat[v*B + b]
// (B <= 256).  Threads (b = tid % Bp, j = tid / Bp), Bp = pow2 >= B.
__global__ void __launch_bounds__(kThreads) column_partials_kernel(int64_t n, uint32_t B, uint32_t Bp, int64_t nodes_per,
                                                                   const float* __restrict__ Y, float* __restrict__ part)
{
    __shared__ float red[kThreads];
    const uint32_t b = threadIdx.x % Bp, j = threadIdx.x / Bp, J = kThreads / Bp;
    const int64_t v0 = (int64_t)blockIdx.x * nodes_per;
    const int64_t v1 = v0 + nodes_per < n ? v0 + nodes_per : n;
    float s = 0.0f;
    if (b < B)
        for (int64_t v = v0 + j; v < v1; v += J) s += Y[v * B + b];
    red[threadIdx.x] = s;
    __syncthreads();
    for (uint32_t h = J / 2; h > 0; h /= 2) {
        if (j < h) red[threadIdx.x] += red[threadIdx.x + h * Bp];
        __syncthreads();
    }
    if (j == 0 && b < B) part[(int64_t)blockIdx.x * B + b] = red[threadIdx.x];
}

// g[b] = d loss / d pred[b] and loss = mean over b of ((pred - target)/n)^2
__global__ void loss_kernel(uint32_t B, double n, const float* __restrict__ pred, const float* __restrict__ target,
                            float* __restrict__ g, float* __restrict__ loss)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    float L = 0.0f;
    const float inv_n = (float)(1.0 / n);
    for (uint32_t b = 0; b < B; ++b) {
        const float d = (pred[b] - target[b]) * inv_n;
        L += d * d;
        g[b] = 2.0f * d * inv_n / (float)B;
    }
    if (loss) loss[0] = L / (float)B;
}

// Readout backward.  dz = g[b] * yhat (1 - yhat) (zero for seeds, whose yhat
// is 1), dZ3 = [H3 > 0] * dz * w_o, and per-workgroup partials of
// dw_o = sum dz * H3 and db_o = sum dz over the workgroup's row range.
__global__ void __launch_bounds__(kThreads) readout_bwd_kernel(int64_t R, uint32_t B, int64_t rows_per,
                                                               const uint16_t* __restrict__ H,
                                                               const float* __restrict__ Yhat,
                                                               const float* __restrict__ g, const float* __restrict__ w_o,
                                                               uint16_t* __restrict__ dZ, float* __restrict__ part)
{
    __shared__ float red[kThreads / 8][kHidden + 1];
    const int sub = threadIdx.x & 7, grp = threadIdx.x >> 3;
    float wv[8], acc[8], accb = 0.0f;
    #pragma unroll
    for (int i = 0; i < 8; ++i) {
        wv[i] = bf2f(f2bf(w_o[8 * sub + i]));
        acc[i] = 0.0f;
    }
    const int64_t r0 = (int64_t)blockIdx.x * rows_per;
    const int64_t r1 = r0 + rows_per < R ? r0 + rows_per : R;
    for (int64_t r = r0 + grp; r < r1; r += kThreads / 8) {
        const float y = Yhat[r];
        const float dz = g[r % B] * y * (1.0f - y);
        float h[8];
        unpack8(*(const u32x4*)(H + r * kHidden + 8 * sub), h);
        u32x4 o;
        float d[8];
        #pragma unroll
        for (int i = 0; i < 8; ++i) {
            d[i] = h[i] > 0.0f ? dz * wv[i] : 0.0f;
            acc[i] = fmaf(dz, h[i], acc[i]);
        }
        #pragma unroll
        for (int i = 0; i < 4; ++i) o[i] = pack2(d[2 * i], d[2 * i + 1]);
        *(u32x4*)(dZ + r * kHidden + 8 * sub) = o;
        accb += dz;
    }
    #pragma unroll
    for (int i = 0; i < 8; ++i) red[grp][8 * sub + i] = acc[i];
    if (sub == 0) red[grp][kHidden] = accb;
    __syncthreads();
    if (threadIdx.x <= kHidden) {
        float s = 0.0f;
        for (int j = 0; j < kThreads / 8; ++j) s += red[j][threadIdx.x];
        part[(int64_t)blockIdx.x * (kHidden + 1) + threadIdx.x] = s;
    }
}

// ---------------------------------------------------------------------------
// Adam (Kingma and Ba), bias-corrected, on fp32 master parameters.
__global__ void adam_kernel(int64_t count, float* __restrict__ p, const float* __restrict__ grad, float* __restrict__ m,
                            float* __restrict__ v, float lr, float beta1, float beta2, float eps, float corr1, float corr2)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x) {
        const float gi = grad[i];
        const float mi = beta1 * m[i] + (1.0f - beta1) * gi;
        const float vi = beta2 * v[i] + (1.0f - beta2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        p[i] -= lr * (mi / corr1) / (sqrtf(vi / corr2) + eps);
    }
}

}  // namespace imsim_mpnn
