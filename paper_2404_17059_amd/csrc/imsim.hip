// Host runtime and C ABI of the imsim library (declared in include/imsim.h).
//
// A graph handle holds the device copy of the out-CSR (with IC thresholds), the
// in-CSR built here for the LT pull sweep, and a workspace that grows with the
// trial count.  ims_simulate enqueues: clear state -> one cooperative
// persistent launch (seed init + all levels / sweeps) -> two reductions.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "imsim.h"
#include "sim_kernels.hpp"

namespace {

thread_local std::string g_last_error;

int fail(int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

#define IMS_HIP(call)                                                                          \
    do {                                                                                       \
        hipError_t e_ = (call);                                                                \
        if (e_ != hipSuccess) return fail(IMS_E_HIP, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)

template <typename T>
int dev_alloc(T** p, uint64_t count)
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

template <typename T>
void dev_free(T*& p)
{
    if (p) (void)hipFree(p);
    p = nullptr;
}

template <typename Tv>
int fill_async(Tv* p, uint64_t count, Tv value, hipStream_t s)
{
    if (count == 0) return IMS_OK;
    uint64_t blocks = (count + imsim::kBlock - 1) / imsim::kBlock;
    blocks = std::min<uint64_t>(blocks, 65536);
    hipLaunchKernelGGL(imsim::fill_kernel<Tv>, dim3((unsigned)blocks), dim3(imsim::kBlock), 0, s, p, count, value);
    IMS_HIP(hipGetLastError());
    return IMS_OK;
}

}  // namespace

struct ims_graph {
    int device = 0;
    int64_t n = 0, m = 0;
    int model = 0;
    uint64_t total_chunks = 0;  // sum over nodes of ceil(outdeg / kChunk)
    int64_t* d_off = nullptr;
    uint32_t* d_idx = nullptr;
    uint32_t* d_thr = nullptr;
    int64_t* d_in_off = nullptr;
    uint32_t* d_in_src = nullptr;
    uint32_t* d_in_w = nullptr;
    // workspace
    uint32_t ws_W = 0;
    uint64_t* d_A = nullptr;
    uint64_t* d_N[3] = {nullptr, nullptr, nullptr};
    uint64_t* d_Q[3] = {nullptr, nullptr, nullptr};
    uint32_t* d_qcount = nullptr;
    uint32_t cap = 0;
    uint32_t* d_seeds = nullptr;
    uint32_t seeds_cap = 0;
    uint32_t* d_status = nullptr;
    bool n_dirty = true;
    int coop_blocks = 0;
    int coop_per_cu = 0;

    void free_workspace()
    {
        dev_free(d_A);
        for (auto& p : d_N) dev_free(p);
        for (auto& p : d_Q) dev_free(p);
        ws_W = 0;
    }
    ~ims_graph()
    {
        free_workspace();
        dev_free(d_off);
        dev_free(d_idx);
        dev_free(d_thr);
        dev_free(d_in_off);
        dev_free(d_in_src);
        dev_free(d_in_w);
        dev_free(d_qcount);
        dev_free(d_seeds);
        dev_free(d_status);
    }
};

namespace {

int ensure_workspace(ims_graph* g, uint32_t W, hipStream_t s)
{
    if (g->ws_W >= W) return IMS_OK;
    g->free_workspace();
    const uint64_t cells = (uint64_t)W * (uint64_t)g->n;
    int rc = dev_alloc(&g->d_A, cells);
    if (rc) return rc;
    if (g->model == IMS_MODEL_IC) {
        const uint64_t qcap = (uint64_t)W * std::max<uint64_t>(g->total_chunks, 1);
        for (int i = 0; i < 3; ++i) {
            if ((rc = dev_alloc(&g->d_N[i], cells))) return rc;
            if ((rc = dev_alloc(&g->d_Q[i], qcap))) return rc;
        }
    }
    g->ws_W = W;
    g->n_dirty = true;
    (void)s;
    return IMS_OK;
}

int coop_grid(ims_graph* g)
{
    if (g->coop_blocks > 0) return IMS_OK;
    int per_cu = 0;
    IMS_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, imsim::sim_persistent, imsim::kBlock, 0));
    hipDeviceProp_t prop;
    IMS_HIP(hipGetDeviceProperties(&prop, g->device));
    if (per_cu < 1) return fail(IMS_E_HIP, "sim_persistent cannot be resident (occupancy 0)");
    if (!prop.cooperativeLaunch) return fail(IMS_E_UNSUPPORTED, "device lacks cooperative launch");
    g->coop_per_cu = per_cu;
    g->coop_blocks = per_cu * prop.multiProcessorCount;
    return IMS_OK;
}

}  // namespace

extern "C" {

const char* ims_last_error(void) { return g_last_error.c_str(); }

const char* ims_version(void) { return "imsim 0.1 gfx950"; }

int ims_encode_p(const double* p, int64_t m, uint32_t* thr)
{
    if (m < 0 || (m > 0 && (!p || !thr))) return fail(IMS_E_INVALID_ARG, "ims_encode_p: bad arguments");
    for (int64_t e = 0; e < m; ++e) {
        const double x = p[e];
        if (!(x >= 0.0 && x <= 1.0)) return fail(IMS_E_INVALID_ARG, "ims_encode_p: p[%lld] = %g outside [0, 1]", (long long)e, x);
        const double f = std::floor(std::ldexp(x, 32));
        thr[e] = f >= 4294967295.0 ? 0xFFFFFFFFu : (uint32_t)f;
    }
    return IMS_OK;
}

int ims_encode_w(const double* w, int64_t m, uint64_t* w64)
{
    if (m < 0 || (m > 0 && (!w || !w64))) return fail(IMS_E_INVALID_ARG, "ims_encode_w: bad arguments");
    for (int64_t e = 0; e < m; ++e) {
        const double x = w[e];
        if (!(x >= 0.0 && x <= 1.0)) return fail(IMS_E_INVALID_ARG, "ims_encode_w: w[%lld] = %g outside [0, 1]", (long long)e, x);
        w64[e] = (uint64_t)std::floor(std::ldexp(x, 32));
    }
    return IMS_OK;
}

int ims_validate_csr(int64_t n, int64_t m, const int64_t* offsets, const uint32_t* indices)
{
    if (n < 0 || m < 0 || !offsets || (m > 0 && !indices)) return fail(IMS_E_INVALID_ARG, "ims_validate_csr: bad arguments");
    if (n >= (int64_t)0xFFFFFFFFll) return fail(IMS_E_INVALID_GRAPH, "n = %lld must be below 2^32 - 1", (long long)n);
    if (m >= (int64_t)0xFFFFFFFFll) return fail(IMS_E_INVALID_GRAPH, "m = %lld must be below 2^32 - 1", (long long)m);
    if (offsets[0] != 0) return fail(IMS_E_INVALID_GRAPH, "offsets[0] = %lld, expected 0", (long long)offsets[0]);
    for (int64_t u = 0; u < n; ++u)
        if (offsets[u + 1] < offsets[u]) return fail(IMS_E_INVALID_GRAPH, "offsets decrease at node %lld", (long long)u);
    if (offsets[n] != m) return fail(IMS_E_INVALID_GRAPH, "offsets[n] = %lld, expected m = %lld", (long long)offsets[n], (long long)m);
    for (int64_t e = 0; e < m; ++e)
        if ((int64_t)indices[e] >= n) return fail(IMS_E_INVALID_GRAPH, "indices[%lld] = %u >= n", (long long)e, indices[e]);
    return IMS_OK;
}

int ims_graph_create(int64_t n, int64_t m, const int64_t* offsets, const uint32_t* indices, int model, const void* param,
                     ims_graph** out)
{
    if (!out) return fail(IMS_E_INVALID_ARG, "ims_graph_create: out is NULL");
    *out = nullptr;
    if (model != IMS_MODEL_IC && model != IMS_MODEL_LT) return fail(IMS_E_INVALID_ARG, "unknown model %d", model);
    if (m > 0 && !param) return fail(IMS_E_INVALID_ARG, "ims_graph_create: param is NULL");
    int rc = ims_validate_csr(n, m, offsets, indices);
    if (rc) return rc;
    uint64_t max_deg = 0, chunks = 0;
    for (int64_t u = 0; u < n; ++u) {
        const uint64_t d = (uint64_t)(offsets[u + 1] - offsets[u]);
        max_deg = std::max(max_deg, d);
        chunks += (d + imsim::kChunk - 1) / imsim::kChunk;
    }
    if (max_deg >= (1ull << 30)) return fail(IMS_E_UNSUPPORTED, "out-degree %llu above 2^30", (unsigned long long)max_deg);

    // LT: check the in-weight bound and build the in-CSR; a weight of exactly
    // 2^32 is stored as two pieces of 2^31 so every piece fits 32 bits, and
    // zero weights are dropped (they never add to a sum).
    std::vector<int64_t> in_off;
    std::vector<uint32_t> in_src, in_w;
    if (model == IMS_MODEL_LT) {
        const uint64_t* w64 = (const uint64_t*)param;
        std::vector<uint64_t> wsum((size_t)std::max<int64_t>(n, 1), 0);
        std::vector<int64_t> cnt((size_t)n + 1, 0);
        for (int64_t e = 0; e < m; ++e) {
            const uint64_t w = w64[e];
            if (w > (1ull << 32)) return fail(IMS_E_WEIGHT_SUM, "LT weight of arc %lld above 2^32", (long long)e);
            const uint32_t v = indices[e];
            wsum[v] += w;
            if (wsum[v] > (1ull << 32)) return fail(IMS_E_WEIGHT_SUM, "LT in-weights of node %u sum above 2^32", v);
            cnt[v + 1] += w == 0 ? 0 : (w == (1ull << 32) ? 2 : 1);
        }
        in_off.assign((size_t)n + 1, 0);
        for (int64_t v = 0; v < n; ++v) in_off[v + 1] = in_off[v] + cnt[v + 1];
        const int64_t mi = in_off[n];
        in_src.resize((size_t)std::max<int64_t>(mi, 1));
        in_w.resize((size_t)std::max<int64_t>(mi, 1));
        std::vector<int64_t> pos(in_off.begin(), in_off.end() - 1);
        for (int64_t u = 0; u < n; ++u)
            for (int64_t e = offsets[u]; e < offsets[u + 1]; ++e) {
                const uint64_t w = w64[e];
                if (w == 0) continue;
                const uint32_t v = indices[e];
                if (w == (1ull << 32)) {
                    in_src[pos[v]] = (uint32_t)u;
                    in_w[pos[v]++] = 1u << 31;
                    in_src[pos[v]] = (uint32_t)u;
                    in_w[pos[v]++] = 1u << 31;
                } else {
                    in_src[pos[v]] = (uint32_t)u;
                    in_w[pos[v]++] = (uint32_t)w;
                }
            }
    }

    ims_graph* g = new (std::nothrow) ims_graph();
    if (!g) return fail(IMS_E_OOM, "host allocation failed");
    (void)hipGetDevice(&g->device);
    g->n = n;
    g->m = m;
    g->model = model;
    g->total_chunks = chunks;
    auto bail = [&](int code) {
        delete g;
        return code;
    };
    if ((rc = dev_alloc(&g->d_off, (uint64_t)n + 1))) return bail(rc);
    if ((rc = dev_alloc(&g->d_idx, (uint64_t)m))) return bail(rc);
    if (hipMemcpy(g->d_off, offsets, sizeof(int64_t) * (n + 1), hipMemcpyHostToDevice) != hipSuccess ||
        (m > 0 && hipMemcpy(g->d_idx, indices, sizeof(uint32_t) * m, hipMemcpyHostToDevice) != hipSuccess))
        return bail(fail(IMS_E_HIP, "graph upload failed"));
    if (model == IMS_MODEL_IC) {
        if ((rc = dev_alloc(&g->d_thr, (uint64_t)m))) return bail(rc);
        if (m > 0 && hipMemcpy(g->d_thr, param, sizeof(uint32_t) * m, hipMemcpyHostToDevice) != hipSuccess)
            return bail(fail(IMS_E_HIP, "threshold upload failed"));
    } else {
        const int64_t mi = in_off[n];
        if ((rc = dev_alloc(&g->d_in_off, (uint64_t)n + 1))) return bail(rc);
        if ((rc = dev_alloc(&g->d_in_src, (uint64_t)mi))) return bail(rc);
        if ((rc = dev_alloc(&g->d_in_w, (uint64_t)mi))) return bail(rc);
        if (hipMemcpy(g->d_in_off, in_off.data(), sizeof(int64_t) * (n + 1), hipMemcpyHostToDevice) != hipSuccess ||
            (mi > 0 && hipMemcpy(g->d_in_src, in_src.data(), sizeof(uint32_t) * mi, hipMemcpyHostToDevice) != hipSuccess) ||
            (mi > 0 && hipMemcpy(g->d_in_w, in_w.data(), sizeof(uint32_t) * mi, hipMemcpyHostToDevice) != hipSuccess))
            return bail(fail(IMS_E_HIP, "in-CSR upload failed"));
    }
    g->cap = (uint32_t)std::min<int64_t>(n + 8, 0xFFFFFFF0ll);
    if ((rc = dev_alloc(&g->d_qcount, g->cap))) return bail(rc);
    if ((rc = dev_alloc(&g->d_status, 2))) return bail(rc);
    *out = g;
    return IMS_OK;
}

int ims_graph_destroy(ims_graph* g)
{
    if (g) {
        (void)hipDeviceSynchronize();
        delete g;
    }
    return IMS_OK;
}

int ims_graph_info(const ims_graph* g, int64_t* n, int64_t* m, int* model)
{
    if (!g) return fail(IMS_E_INVALID_ARG, "ims_graph_info: NULL handle");
    if (n) *n = g->n;
    if (m) *m = g->m;
    if (model) *model = g->model;
    return IMS_OK;
}

int ims_simulate(ims_graph* g, const uint32_t* seeds, uint32_t n_seeds, uint32_t n_trials, uint64_t rng_seed,
                 const ims_opts* opts, uint32_t* trial_counts, uint32_t* node_counts, uint64_t* total,
                 uint64_t* active_bits, void* stream)
{
    if (!g) return fail(IMS_E_INVALID_ARG, "ims_simulate: NULL graph");
    if (n_trials == 0) return fail(IMS_E_INVALID_ARG, "ims_simulate: n_trials must be >= 1");
    if (n_trials > imsim::kMaxWords * 64u) return fail(IMS_E_UNSUPPORTED, "ims_simulate: n_trials above %u", imsim::kMaxWords * 64u);
    if (!trial_counts || !total) return fail(IMS_E_INVALID_ARG, "ims_simulate: trial_counts and total are required");
    if (n_seeds > 0 && !seeds) return fail(IMS_E_INVALID_ARG, "ims_simulate: seeds is NULL");
    hipStream_t s = (hipStream_t)stream;

    // seeds: range check and set semantics on the host
    std::vector<uint32_t> sv(seeds, seeds + n_seeds);
    for (uint32_t x : sv)
        if ((int64_t)x >= g->n) return fail(IMS_E_SEED_RANGE, "seed %u >= n = %lld", x, (long long)g->n);
    std::sort(sv.begin(), sv.end());
    sv.erase(std::unique(sv.begin(), sv.end()), sv.end());

    const uint32_t W = (n_trials + 63) / 64;
    int rc = ensure_workspace(g, W, s);
    if (rc) return rc;
    if ((rc = coop_grid(g))) return rc;
    if (g->seeds_cap < sv.size()) {
        dev_free(g->d_seeds);
        if ((rc = dev_alloc(&g->d_seeds, sv.size()))) return rc;
        g->seeds_cap = (uint32_t)sv.size();
    }
    if (!sv.empty()) IMS_HIP(hipMemcpyAsync(g->d_seeds, sv.data(), sv.size() * sizeof(uint32_t), hipMemcpyHostToDevice, s));

    const uint64_t cells = (uint64_t)W * (uint64_t)g->n;
    uint64_t* A = active_bits ? active_bits : g->d_A;
    if ((rc = fill_async<uint64_t>(A, cells, 0ull, s))) return rc;
    if (g->model == IMS_MODEL_IC && g->n_dirty) {
        for (int i = 0; i < 3; ++i)
            if ((rc = fill_async<uint64_t>(g->d_N[i], cells, 0ull, s))) return rc;
        g->n_dirty = false;
    }
    if ((rc = fill_async<uint32_t>(g->d_qcount, g->cap, 0u, s))) return rc;
    if ((rc = fill_async<uint32_t>(trial_counts, n_trials, 0u, s))) return rc;
    if ((rc = fill_async<unsigned long long>((unsigned long long*)total, 1, 0ull, s))) return rc;

    imsim::SimParams P;
    P.n = g->n;
    P.T = n_trials;
    P.W = W;
    P.seed = rng_seed;
    P.model = g->model;
    P.cap = g->cap;
    P.off = g->d_off;
    P.idx = g->d_idx;
    P.thr = g->d_thr;
    P.in_off = g->d_in_off;
    P.in_src = g->d_in_src;
    P.in_w = g->d_in_w;
    P.A = A;
    P.N0 = g->d_N[0];
    P.N1 = g->d_N[1];
    P.N2 = g->d_N[2];
    P.Q0 = g->d_Q[0];
    P.Q1 = g->d_Q[1];
    P.Q2 = g->d_Q[2];
    P.qcount = g->d_qcount;
    P.seeds = g->d_seeds;
    P.n_seeds = (uint32_t)sv.size();
    P.status = g->d_status;

    int blocks = g->coop_blocks;
    if (opts && opts->blocks_per_cu > 0) {
        const int cus = g->coop_blocks / g->coop_per_cu;
        blocks = std::min(opts->blocks_per_cu, g->coop_per_cu) * cus;
    }
    void* args[] = {&P};
    IMS_HIP(hipLaunchCooperativeKernel((const void*)imsim::sim_persistent, dim3(blocks), dim3(imsim::kBlock), args, 0, s));

    if (g->n > 0) {
        const uint64_t nblk = std::min<uint64_t>(((uint64_t)g->n + imsim::kBlock - 1) / imsim::kBlock, 1024);
        hipLaunchKernelGGL(imsim::reduce_trial_counts, dim3((unsigned)nblk, W), dim3(imsim::kBlock), 0, s, A, g->n, n_trials,
                           trial_counts);
        IMS_HIP(hipGetLastError());
        hipLaunchKernelGGL(imsim::reduce_node_counts, dim3((unsigned)std::min<uint64_t>(nblk * 4, 4096)), dim3(imsim::kBlock), 0, s, A,
                           g->n, W, node_counts, (unsigned long long*)total);
        IMS_HIP(hipGetLastError());
    }
    return IMS_OK;
}

int ims_graph_last_status(ims_graph* g, void* stream, uint32_t out[2])
{
    if (!g || !out) return fail(IMS_E_INVALID_ARG, "ims_graph_last_status: bad arguments");
    IMS_HIP(hipMemcpyAsync(out, g->d_status, 2 * sizeof(uint32_t), hipMemcpyDeviceToHost, (hipStream_t)stream));
    IMS_HIP(hipStreamSynchronize((hipStream_t)stream));
    if (out[1]) g->n_dirty = true;
    return IMS_OK;
}

int ims_debug_hash(uint64_t rng_seed, uint64_t domain, const uint64_t* trials, const uint64_t* ids, uint32_t* out, int64_t count,
                   void* stream)
{
    if (count < 0 || (count > 0 && (!trials || !ids || !out))) return fail(IMS_E_INVALID_ARG, "ims_debug_hash: bad arguments");
    if (count == 0) return IMS_OK;
    const uint64_t blocks = ((uint64_t)count + imsim::kBlock - 1) / imsim::kBlock;
    hipLaunchKernelGGL(imsim::debug_hash_kernel, dim3((unsigned)blocks), dim3(imsim::kBlock), 0, (hipStream_t)stream, rng_seed, domain,
                       trials, ids, out, count);
    IMS_HIP(hipGetLastError());
    return IMS_OK;
}

}  // extern "C"
