// Host runtime and C ABI of the learned spread estimator (include/imsim_mpnn.h).
//
// A plan owns the device in-CSR (forward aggregation), out-CSR (its
// transpose, for the backward pass), the static node features and one
// workspace of activations and gradients sized for n * max_batch rows.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "imsim_mpnn.h"
#include "mpnn_kernels.hpp"

namespace imsim {
int record_error(int code, const char* msg);
}

namespace {

using namespace imsim_mpnn;

int fail(int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    return imsim::record_error(code, buf);
}

#define MP_HIP(call)                                                                           \
    do {                                                                                       \
        hipError_t e_ = (call);                                                                \
        if (e_ != hipSuccess) return fail(IMS_E_HIP, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)

template <typename T>
int alloc(T** p, uint64_t count)
{
    *p = nullptr;
    if (count == 0) count = 1;
    hipError_t e = hipMalloc((void**)p, count * sizeof(T));
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return fail(e == hipErrorOutOfMemory ? IMS_E_OOM : IMS_E_HIP, "hipMalloc(%llu bytes): %s",
                    (unsigned long long)(count * sizeof(T)), hipGetErrorString(e));
    }
    return IMS_OK;
}

unsigned grid_for(int64_t work, int64_t per_block, int64_t cap)
{
    int64_t b = (work + per_block - 1) / per_block;
    b = std::max<int64_t>(1, std::min<int64_t>(b, cap));
    return (unsigned)b;
}

}  // namespace

struct ims_mpnn {
    int device = 0;
    int cus = 256;
    int64_t n = 0, m = 0;
    uint32_t max_batch = 0;
    uint32_t last_B = 0;
    bool have_forward = false;
    int64_t* in_off = nullptr;
    uint32_t* in_src = nullptr;
    float* in_w = nullptr;
    int64_t* out_off = nullptr;
    uint32_t* out_dst = nullptr;
    float* out_w = nullptr;
    float* feat = nullptr;          // [n][3]
    // aggregation work items of the in-CSR (0, forward) and out-CSR (1, backward)
    SpmmItem* items[2] = {nullptr, nullptr};
    uint32_t n_items[2] = {0, 0};
    uint32_t* fin[2] = {nullptr, nullptr};
    uint32_t n_fin[2] = {0, 0};
    float* seg_partial = nullptr;   // [slots][max_batch * 64]
    uint16_t* t[IMS_MPNN_T_COUNT] = {};
    float* part = nullptr;          // per-workgroup partial sums
    int64_t part_floats = 0;
    float* pred = nullptr;          // [max_batch]
    float* g = nullptr;             // [max_batch] d loss / d pred
    uint32_t* sets = nullptr;       // set offsets + nodes
    uint64_t sets_cap = 0;
};

namespace {

int tensor_width(int id) { return id == IMS_MPNN_T_X0 || id == IMS_MPNN_T_M0 ? kIn : (id == IMS_MPNN_T_YHAT ? 2 : kHidden); }

void destroy(ims_mpnn* p)
{
    if (!p) return;
    for (void* q : {(void*)p->in_off, (void*)p->in_src, (void*)p->in_w, (void*)p->out_off, (void*)p->out_dst,
                    (void*)p->out_w, (void*)p->feat, (void*)p->part, (void*)p->pred, (void*)p->g, (void*)p->sets})
        if (q) (void)hipFree(q);
    for (uint16_t* q : p->t)
        if (q) (void)hipFree(q);
    for (int k = 0; k < 2; ++k) {
        if (p->items[k]) (void)hipFree(p->items[k]);
        if (p->fin[k]) (void)hipFree(p->fin[k]);
    }
    if (p->seg_partial) (void)hipFree(p->seg_partial);
    delete p;
}

// Work items of one CSR: rows longer than kSegArcs become segments with
// partial slots (listed first, they are the long-running items), the rest
// one direct item each.
void build_items(int64_t n, const int64_t* off, std::vector<SpmmItem>& items, std::vector<uint32_t>& fin, uint32_t& slots)
{
    items.clear();
    fin.clear();
    slots = 0;
    for (int64_t v = 0; v < n; ++v) {
        const int64_t deg = off[v + 1] - off[v];
        if (deg <= (int64_t)kSegArcs) continue;
        fin.push_back((uint32_t)v);
        fin.push_back(slots);
        uint32_t k = 0;
        for (int64_t e = off[v]; e < off[v + 1]; e += kSegArcs, ++k)
            items.push_back(SpmmItem{(uint32_t)v, slots + k, (uint32_t)e, (uint32_t)std::min<int64_t>(kSegArcs, off[v + 1] - e)});
        fin.push_back(k);
        slots += k;
    }
    for (int64_t v = 0; v < n; ++v) {
        const int64_t deg = off[v + 1] - off[v];
        if (deg <= (int64_t)kSegArcs) items.push_back(SpmmItem{(uint32_t)v, kDirect, (uint32_t)off[v], (uint32_t)deg});
    }
}

// workgroups of the weight-gradient kernel and its rows per workgroup
void weight_grid(int64_t R, int64_t& blocks, int64_t& rows_per)
{
    blocks = std::min<int64_t>(1024, std::max<int64_t>(1, (R + kWStage - 1) / kWStage));
    rows_per = (R + blocks - 1) / blocks;
    rows_per = (rows_per + kWStage - 1) / kWStage * kWStage;
    blocks = (R + rows_per - 1) / rows_per;
}

constexpr int64_t kReadoutBlocks = 1024;
constexpr int64_t kColumnBlocks = 1024;

template <int D>
int dense_forward(ims_mpnn* p, int64_t R, const uint16_t* Xs, const uint16_t* Xn, const float* W, const float* b,
                  uint16_t* Y, hipStream_t s)
{
    const unsigned grid = grid_for((R + 15) / 16, kThreads / 64, (int64_t)p->cus * 8);
    hipLaunchKernelGGL(dense_fwd_kernel<D>, dim3(grid), dim3(kThreads), 0, s, R, Xs, Xn, W, b, Y);
    MP_HIP(hipGetLastError());
    return IMS_OK;
}

int spmm(ims_mpnn* p, bool backward, uint32_t C, const uint16_t* X, uint16_t* Y, const uint16_t* add,
         const uint16_t* relu_of, hipStream_t s)
{
    const int k = backward ? 1 : 0;
    const uint32_t nc = C / 8;
    const int64_t per_block = nc >= (uint32_t)kThreads ? 1 : kThreads / nc;
    const unsigned grid = grid_for(p->n_items[k], per_block, INT32_MAX);
    if (backward)
        hipLaunchKernelGGL(spmm_kernel<true>, dim3(grid), dim3(kThreads), 0, s, p->n_items[1], C, (const SpmmItem*)p->items[1],
                           (const uint32_t*)p->out_dst, (const float*)p->out_w, X, Y, add, relu_of, p->seg_partial);
    else
        hipLaunchKernelGGL(spmm_kernel<false>, dim3(grid), dim3(kThreads), 0, s, p->n_items[0], C, (const SpmmItem*)p->items[0],
                           (const uint32_t*)p->in_src, (const float*)p->in_w, X, Y, nullptr, nullptr, p->seg_partial);
    MP_HIP(hipGetLastError());
    if (p->n_fin[k]) {
        if (backward)
            hipLaunchKernelGGL(spmm_finish_kernel<true>, dim3(p->n_fin[1]), dim3(kThreads), 0, s, C, (const uint32_t*)p->fin[1],
                               (const float*)p->seg_partial, Y, add, relu_of);
        else
            hipLaunchKernelGGL(spmm_finish_kernel<false>, dim3(p->n_fin[0]), dim3(kThreads), 0, s, C, (const uint32_t*)p->fin[0],
                               (const float*)p->seg_partial, Y, nullptr, nullptr);
        MP_HIP(hipGetLastError());
    }
    return IMS_OK;
}

template <int D>
int dense_weight_grad(ims_mpnn* p, int64_t R, const uint16_t* Xs, const uint16_t* Xn, const uint16_t* dZ, float* grads,
                      hipStream_t s)
{
    int64_t blocks, rows_per;
    weight_grid(R, blocks, rows_per);
    const int64_t stride = 2 * D * kHidden + kHidden;
    if (blocks * stride > p->part_floats) return fail(IMS_E_INVALID_ARG, "internal: partial buffer too small");
    hipLaunchKernelGGL(dense_bwd_weight_kernel<D>, dim3((unsigned)blocks), dim3(kThreads), 0, s, R, rows_per, Xs, Xn, dZ,
                       p->part, stride);
    MP_HIP(hipGetLastError());
    hipLaunchKernelGGL(sum_partials_kernel, dim3(grid_for(stride, 32, INT32_MAX)), dim3(kThreads), 0, s, stride,
                       blocks, stride, (const float*)p->part, grads);
    MP_HIP(hipGetLastError());
    return IMS_OK;
}

uint64_t splitmix64(uint64_t& x)
{
    uint64_t z = (x += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

}  // namespace

extern "C" {

int ims_mpnn_create(int64_t n, int64_t m, const int64_t* offsets, const uint32_t* indices, const float* arc_weight,
                    uint32_t max_batch, ims_mpnn** out)
{
    if (!out) return fail(IMS_E_INVALID_ARG, "ims_mpnn_create: out is NULL");
    *out = nullptr;
    if (n < 1 || m < 0 || !offsets || (m > 0 && (!indices || !arc_weight)))
        return fail(IMS_E_INVALID_ARG, "ims_mpnn_create: bad n, m or NULL arrays");
    if (n >= (int64_t)1 << 32 || m >= (int64_t)1 << 32) return fail(IMS_E_UNSUPPORTED, "ims_mpnn_create: n or m >= 2^32");
    if (max_batch < 1 || max_batch > IMS_MPNN_MAX_BATCH)
        return fail(IMS_E_INVALID_ARG, "ims_mpnn_create: max_batch must be 1..%d", IMS_MPNN_MAX_BATCH);
    int rc = ims_validate_csr(n, m, offsets, indices);
    if (rc) return rc;
    for (int64_t e = 0; e < m; ++e)
        if (!std::isfinite(arc_weight[e])) return fail(IMS_E_INVALID_ARG, "ims_mpnn_create: arc weight %lld not finite", (long long)e);

    // in-CSR: arcs into v in increasing out-CSR position
    std::vector<int64_t> in_off(n + 1, 0);
    for (int64_t e = 0; e < m; ++e) in_off[indices[e] + 1]++;
    for (int64_t v = 0; v < n; ++v) in_off[v + 1] += in_off[v];
    std::vector<uint32_t> in_src(std::max<int64_t>(m, 1));
    std::vector<float> in_w(std::max<int64_t>(m, 1));
    {
        std::vector<int64_t> pos(in_off.begin(), in_off.end() - 1);
        for (int64_t u = 0; u < n; ++u)
            for (int64_t e = offsets[u]; e < offsets[u + 1]; ++e) {
                const int64_t q = pos[indices[e]]++;
                in_src[q] = (uint32_t)u;
                in_w[q] = arc_weight[e];
            }
    }
    std::vector<float> feat(3 * n);
    for (int64_t v = 0; v < n; ++v) {
        double sum = 0.0;
        for (int64_t e = offsets[v]; e < offsets[v + 1]; ++e) sum += arc_weight[e];
        feat[3 * v + 0] = (float)std::log1p((double)(offsets[v + 1] - offsets[v]));
        feat[3 * v + 1] = (float)std::log1p((double)(in_off[v + 1] - in_off[v]));
        feat[3 * v + 2] = (float)std::log1p(sum);
    }

    std::vector<SpmmItem> items[2];
    std::vector<uint32_t> fin[2];
    uint32_t slots[2];
    build_items(n, in_off.data(), items[0], fin[0], slots[0]);
    build_items(n, offsets, items[1], fin[1], slots[1]);

    ims_mpnn* p = new (std::nothrow) ims_mpnn;
    if (!p) return fail(IMS_E_OOM, "ims_mpnn_create: host allocation");
    p->n = n;
    p->m = m;
    p->max_batch = max_batch;
    if (hipGetDevice(&p->device) != hipSuccess) {
        destroy(p);
        return fail(IMS_E_HIP, "ims_mpnn_create: no current device");
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, p->device) == hipSuccess && prop.multiProcessorCount > 0) p->cus = prop.multiProcessorCount;
    const uint64_t rows = (uint64_t)n * max_batch;
    int64_t wblocks, wrows;
    weight_grid((int64_t)rows, wblocks, wrows);
    p->part_floats = std::max<int64_t>({wblocks * (2 * kHidden * kHidden + kHidden), kReadoutBlocks * (kHidden + 1),
                                        kColumnBlocks * (int64_t)max_batch});
    rc = IMS_OK;
    rc = rc ? rc : alloc(&p->in_off, n + 1);
    rc = rc ? rc : alloc(&p->in_src, m);
    rc = rc ? rc : alloc(&p->in_w, m);
    rc = rc ? rc : alloc(&p->out_off, n + 1);
    rc = rc ? rc : alloc(&p->out_dst, m);
    rc = rc ? rc : alloc(&p->out_w, m);
    rc = rc ? rc : alloc(&p->feat, 3 * n);
    rc = rc ? rc : alloc(&p->part, p->part_floats);
    rc = rc ? rc : alloc(&p->pred, max_batch);
    rc = rc ? rc : alloc(&p->g, max_batch);
    for (int id = 0; id < IMS_MPNN_T_COUNT && !rc; ++id) rc = alloc(&p->t[id], rows * tensor_width(id));
    for (int k = 0; k < 2 && !rc; ++k) {
        p->n_items[k] = (uint32_t)items[k].size();
        p->n_fin[k] = (uint32_t)(fin[k].size() / 3);
        rc = alloc(&p->items[k], items[k].size());
        rc = rc ? rc : alloc(&p->fin[k], fin[k].size());
    }
    rc = rc ? rc : alloc(&p->seg_partial, (uint64_t)std::max(slots[0], slots[1]) * max_batch * kHidden);
    if (rc) {
        destroy(p);
        return rc;
    }
    hipError_t e = hipSuccess;
    e = e != hipSuccess ? e : hipMemcpy(p->in_off, in_off.data(), (n + 1) * 8, hipMemcpyHostToDevice);
    e = e != hipSuccess ? e : hipMemcpy(p->out_off, offsets, (n + 1) * 8, hipMemcpyHostToDevice);
    e = e != hipSuccess ? e : hipMemcpy(p->feat, feat.data(), 3 * n * 4, hipMemcpyHostToDevice);
    if (m > 0) {
        e = e != hipSuccess ? e : hipMemcpy(p->in_src, in_src.data(), m * 4, hipMemcpyHostToDevice);
        e = e != hipSuccess ? e : hipMemcpy(p->in_w, in_w.data(), m * 4, hipMemcpyHostToDevice);
        e = e != hipSuccess ? e : hipMemcpy(p->out_dst, indices, m * 4, hipMemcpyHostToDevice);
        e = e != hipSuccess ? e : hipMemcpy(p->out_w, arc_weight, m * 4, hipMemcpyHostToDevice);
    }
    for (int k = 0; k < 2; ++k) {
        if (!items[k].empty())
            e = e != hipSuccess ? e : hipMemcpy(p->items[k], items[k].data(), items[k].size() * sizeof(SpmmItem), hipMemcpyHostToDevice);
        if (!fin[k].empty())
            e = e != hipSuccess ? e : hipMemcpy(p->fin[k], fin[k].data(), fin[k].size() * 4, hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) {
        destroy(p);
        return fail(IMS_E_HIP, "ims_mpnn_create: copy to device: %s", hipGetErrorString(e));
    }
    *out = p;
    return IMS_OK;
}

int ims_mpnn_destroy(ims_mpnn* p)
{
    if (p) (void)hipDeviceSynchronize();
    destroy(p);
    return IMS_OK;
}

int ims_mpnn_init_params(uint64_t seed, float* params)
{
    if (!params) return fail(IMS_E_INVALID_ARG, "ims_mpnn_init_params: params is NULL");
    uint64_t x = seed;
    auto uniform = [&](double a) { return (float)(((splitmix64(x) >> 11) * 0x1.0p-53 * 2.0 - 1.0) * a); };
    std::memset(params, 0, sizeof(float) * IMS_MPNN_NPARAMS);
    const double a0 = std::sqrt(6.0 / (8 + kHidden)), a1 = std::sqrt(6.0 / (2 * kHidden + kHidden)),
                 ao = std::sqrt(6.0 / (kHidden + 1));
    for (int i = 0; i < 2 * kIn * kHidden; ++i) params[IMS_MPNN_OFF_W0 + i] = uniform(a0);
    for (int i = 0; i < 2 * kHidden * kHidden; ++i) params[IMS_MPNN_OFF_W1 + i] = uniform(a1);
    for (int i = 0; i < 2 * kHidden * kHidden; ++i) params[IMS_MPNN_OFF_W2 + i] = uniform(a1);
    for (int i = 0; i < kHidden; ++i) params[IMS_MPNN_OFF_WO + i] = uniform(ao);
    return IMS_OK;
}

int ims_mpnn_forward(ims_mpnn* p, const float* params, const uint32_t* set_offsets, const uint32_t* set_nodes,
                     uint32_t n_sets, float* pred, void* stream)
{
    if (!p || !params || !set_offsets || !pred) return fail(IMS_E_INVALID_ARG, "ims_mpnn_forward: NULL argument");
    if (n_sets < 1 || n_sets > p->max_batch)
        return fail(IMS_E_INVALID_ARG, "ims_mpnn_forward: n_sets = %u outside 1..%u", n_sets, p->max_batch);
    if (set_offsets[0] != 0) return fail(IMS_E_INVALID_ARG, "ims_mpnn_forward: set_offsets[0] must be 0");
    for (uint32_t i = 0; i < n_sets; ++i)
        if (set_offsets[i + 1] < set_offsets[i]) return fail(IMS_E_INVALID_ARG, "ims_mpnn_forward: set_offsets decrease at %u", i);
    const uint32_t total = set_offsets[n_sets];
    if (total > 0 && !set_nodes) return fail(IMS_E_INVALID_ARG, "ims_mpnn_forward: set_nodes is NULL");
    for (uint32_t k = 0; k < total; ++k)
        if ((int64_t)set_nodes[k] >= p->n) return fail(IMS_E_SEED_RANGE, "ims_mpnn_forward: node %u >= n", set_nodes[k]);
    hipStream_t s = (hipStream_t)stream;
    const uint32_t B = n_sets;
    const int64_t R = p->n * (int64_t)B;
    int rc;

    const uint64_t need = (uint64_t)n_sets + 1 + total;
    if (need > p->sets_cap) {
        MP_HIP(hipStreamSynchronize(s));
        if (p->sets) (void)hipFree(p->sets);
        p->sets = nullptr;
        p->sets_cap = 0;
        if ((rc = alloc(&p->sets, need * 2))) return rc;
        p->sets_cap = need * 2;
    }
    MP_HIP(hipMemcpyAsync(p->sets, set_offsets, (n_sets + 1) * 4ull, hipMemcpyHostToDevice, s));
    if (total) MP_HIP(hipMemcpyAsync(p->sets + n_sets + 1, set_nodes, total * 4ull, hipMemcpyHostToDevice, s));

    uint16_t** t = p->t;
    hipLaunchKernelGGL(features_kernel, dim3(grid_for(R, kThreads, (int64_t)p->cus * 16)), dim3(kThreads), 0, s, R, B,
                       (const float*)p->feat, t[IMS_MPNN_T_X0]);
    MP_HIP(hipGetLastError());
    if (total) {
        hipLaunchKernelGGL(seed_scatter_kernel, dim3(grid_for(total, kThreads, 4096)), dim3(kThreads), 0, s, n_sets, B,
                           (const uint32_t*)p->sets, (const uint32_t*)(p->sets + n_sets + 1), t[IMS_MPNN_T_X0]);
        MP_HIP(hipGetLastError());
    }
    // layer 0 (input width 16), layers 1 and 2 (width 64)
    if ((rc = spmm(p, false, B * kIn, t[IMS_MPNN_T_X0], t[IMS_MPNN_T_M0], nullptr, nullptr, s))) return rc;
    if ((rc = dense_forward<kIn>(p, R, t[IMS_MPNN_T_X0], t[IMS_MPNN_T_M0], params + IMS_MPNN_OFF_W0, params + IMS_MPNN_OFF_B0,
                                 t[IMS_MPNN_T_H1], s)))
        return rc;
    if ((rc = spmm(p, false, B * kHidden, t[IMS_MPNN_T_H1], t[IMS_MPNN_T_M1], nullptr, nullptr, s))) return rc;
    if ((rc = dense_forward<kHidden>(p, R, t[IMS_MPNN_T_H1], t[IMS_MPNN_T_M1], params + IMS_MPNN_OFF_W1,
                                     params + IMS_MPNN_OFF_B1, t[IMS_MPNN_T_H2], s)))
        return rc;
    if ((rc = spmm(p, false, B * kHidden, t[IMS_MPNN_T_H2], t[IMS_MPNN_T_M2], nullptr, nullptr, s))) return rc;
    if ((rc = dense_forward<kHidden>(p, R, t[IMS_MPNN_T_H2], t[IMS_MPNN_T_M2], params + IMS_MPNN_OFF_W2,
                                     params + IMS_MPNN_OFF_B2, t[IMS_MPNN_T_H3], s)))
        return rc;
    // readout and the per-set sums
    float* yhat = (float*)t[IMS_MPNN_T_YHAT];
    hipLaunchKernelGGL(readout_fwd_kernel, dim3(grid_for(R, kThreads / 8, (int64_t)p->cus * 16)), dim3(kThreads), 0, s, R,
                       (const uint16_t*)t[IMS_MPNN_T_H3], (const uint16_t*)t[IMS_MPNN_T_X0], params + IMS_MPNN_OFF_WO, yhat);
    MP_HIP(hipGetLastError());
    uint32_t Bp = 1;
    while (Bp < B) Bp *= 2;
    const int64_t cblocks = std::min<int64_t>(kColumnBlocks, p->n);
    const int64_t nodes_per = (p->n + cblocks - 1) / cblocks;
    const int64_t cb = (p->n + nodes_per - 1) / nodes_per;
    hipLaunchKernelGGL(column_partials_kernel, dim3((unsigned)cb), dim3(kThreads), 0, s, p->n, B, Bp, nodes_per,
                       (const float*)yhat, p->part);
    MP_HIP(hipGetLastError());
    hipLaunchKernelGGL(sum_partials_kernel, dim3(grid_for(B, 32, INT32_MAX)), dim3(kThreads), 0, s, (int64_t)B, cb, (int64_t)B, (const float*)p->part,
                       p->pred);
    MP_HIP(hipGetLastError());
    MP_HIP(hipMemcpyAsync(pred, p->pred, B * 4ull, hipMemcpyDeviceToDevice, s));
    p->last_B = B;
    p->have_forward = true;
    return IMS_OK;
}

int ims_mpnn_backward(ims_mpnn* p, const float* params, const float* target, float* grads, float* loss, void* stream)
{
    if (!p || !params || !target || !grads) return fail(IMS_E_INVALID_ARG, "ims_mpnn_backward: NULL argument");
    if (!p->have_forward) return fail(IMS_E_INVALID_ARG, "ims_mpnn_backward: no forward on this plan");
    hipStream_t s = (hipStream_t)stream;
    const uint32_t B = p->last_B;
    const int64_t R = p->n * (int64_t)B;
    uint16_t** t = p->t;
    int rc;
    hipLaunchKernelGGL(loss_kernel, dim3(1), dim3(64), 0, s, B, (double)p->n, (const float*)p->pred, target, p->g, loss);
    MP_HIP(hipGetLastError());
    // readout: dZ3 and the head's gradient
    {
        const int64_t blocks = std::min<int64_t>(kReadoutBlocks, (R + kThreads / 8 - 1) / (kThreads / 8));
        const int64_t rows_per = (R + blocks - 1) / blocks;
        const int64_t nb = (R + rows_per - 1) / rows_per;
        hipLaunchKernelGGL(readout_bwd_kernel, dim3((unsigned)nb), dim3(kThreads), 0, s, R, B, rows_per,
                           (const uint16_t*)t[IMS_MPNN_T_H3], (const float*)t[IMS_MPNN_T_YHAT], (const float*)p->g,
                           params + IMS_MPNN_OFF_WO, t[IMS_MPNN_T_DZ3], p->part);
        MP_HIP(hipGetLastError());
        hipLaunchKernelGGL(sum_partials_kernel, dim3(grid_for(kHidden + 1, 32, INT32_MAX)), dim3(kThreads), 0, s, (int64_t)(kHidden + 1), nb,
                           (int64_t)(kHidden + 1), (const float*)p->part, grads + IMS_MPNN_OFF_WO);
        MP_HIP(hipGetLastError());
    }
    const unsigned dgrid = grid_for((R + 15) / 16, kThreads / 64, (int64_t)p->cus * 8);
    // layer 2
    if ((rc = dense_weight_grad<kHidden>(p, R, t[IMS_MPNN_T_H2], t[IMS_MPNN_T_M2], t[IMS_MPNN_T_DZ3], grads + IMS_MPNN_OFF_W2, s)))
        return rc;
    hipLaunchKernelGGL(dense_bwd_data_kernel<kHidden>, dim3(dgrid), dim3(kThreads), 0, s, R,
                       (const uint16_t*)t[IMS_MPNN_T_DZ3], params + IMS_MPNN_OFF_W2, t[IMS_MPNN_T_DH2], t[IMS_MPNN_T_DM2]);
    MP_HIP(hipGetLastError());
    if ((rc = spmm(p, true, B * kHidden, t[IMS_MPNN_T_DM2], t[IMS_MPNN_T_DZ2], t[IMS_MPNN_T_DH2], t[IMS_MPNN_T_H2], s)))
        return rc;
    // layer 1
    if ((rc = dense_weight_grad<kHidden>(p, R, t[IMS_MPNN_T_H1], t[IMS_MPNN_T_M1], t[IMS_MPNN_T_DZ2], grads + IMS_MPNN_OFF_W1, s)))
        return rc;
    hipLaunchKernelGGL(dense_bwd_data_kernel<kHidden>, dim3(dgrid), dim3(kThreads), 0, s, R,
                       (const uint16_t*)t[IMS_MPNN_T_DZ2], params + IMS_MPNN_OFF_W1, t[IMS_MPNN_T_DH1], t[IMS_MPNN_T_DM1]);
    MP_HIP(hipGetLastError());
    if ((rc = spmm(p, true, B * kHidden, t[IMS_MPNN_T_DM1], t[IMS_MPNN_T_DZ1], t[IMS_MPNN_T_DH1], t[IMS_MPNN_T_H1], s)))
        return rc;
    // layer 0: weights only
    if ((rc = dense_weight_grad<kIn>(p, R, t[IMS_MPNN_T_X0], t[IMS_MPNN_T_M0], t[IMS_MPNN_T_DZ1], grads + IMS_MPNN_OFF_W0, s)))
        return rc;
    return IMS_OK;
}

int ims_mpnn_adam_step(float* params, const float* grads, float* m, float* v, int64_t count, float lr, float beta1,
                       float beta2, float eps, uint32_t step, void* stream)
{
    if (!params || !grads || !m || !v || count < 0) return fail(IMS_E_INVALID_ARG, "ims_mpnn_adam_step: bad argument");
    if (step < 1) return fail(IMS_E_INVALID_ARG, "ims_mpnn_adam_step: step counts from 1");
    if (count == 0) return IMS_OK;
    const float c1 = (float)(1.0 - std::pow((double)beta1, (double)step));
    const float c2 = (float)(1.0 - std::pow((double)beta2, (double)step));
    hipLaunchKernelGGL(adam_kernel, dim3(grid_for(count, kThreads, 1024)), dim3(kThreads), 0, (hipStream_t)stream, count,
                       params, grads, m, v, lr, beta1, beta2, eps, c1, c2);
    MP_HIP(hipGetLastError());
    return IMS_OK;
}

int ims_mpnn_fetch(ims_mpnn* p, int tensor, void* host_out, int64_t bytes, int64_t* written, void* stream)
{
    if (!p || !host_out || bytes < 0) return fail(IMS_E_INVALID_ARG, "ims_mpnn_fetch: bad argument");
    if (tensor < 0 || tensor >= IMS_MPNN_T_COUNT) return fail(IMS_E_INVALID_ARG, "ims_mpnn_fetch: unknown tensor %d", tensor);
    if (!p->have_forward) return fail(IMS_E_INVALID_ARG, "ims_mpnn_fetch: no forward on this plan");
    const int64_t avail = p->n * (int64_t)p->last_B * tensor_width(tensor) * 2;
    const int64_t nb = std::min(avail, bytes);
    MP_HIP(hipStreamSynchronize((hipStream_t)stream));
    MP_HIP(hipMemcpy(host_out, p->t[tensor], nb, hipMemcpyDeviceToHost));
    if (written) *written = nb;
    return IMS_OK;
}

}  // extern "C"
