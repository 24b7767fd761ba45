// Host runtime and C ABI of the imsim library (declared in include/imsim.h).
//
// A graph handle holds the device copy of the out-CSR (with IC thresholds), the
// in-CSR built here for the LT pull sweep, and a workspace that grows with the
// trial count.  ims_simulate enqueues: clear state -> either one word-local
// launch (each workgroup runs whole 64-trial words) or seed init plus one launch
// per level / sweep in batches -> two reductions.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "imsim.h"
#include "plan.hpp"
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

namespace imsim {
// lets the other translation units of the library set the calling thread's
// ims_last_error() message
int record_error(int code, const char* msg)
{
    g_last_error = msg;
    return code;
}
}  // namespace imsim

struct ims_graph {
    int device = 0;
    int64_t n = 0, m = 0;
    int model = 0;
    uint64_t total_chunks = 0;  // sum over nodes of ceil(outdeg / kChunk)
    int cus = 0;
    std::vector<int64_t> h_off;  // host copy of the out-offsets (launch planning)
    int64_t* d_off = nullptr;
    uint32_t* d_idx = nullptr;
    uint32_t* d_thr = nullptr;
    int64_t* d_in_off = nullptr;     // in-CSR offsets (LT: weight pieces; IC: arcs of nonzero threshold)
    uint64_t* d_in_arc = nullptr;  // (source | weight piece << 32) per in-arc
    uint64_t* d_ic_in = nullptr;     // IC: (source | out-CSR arc id << 32) per in-arc
    uint32_t* d_ic_in_thr = nullptr; // IC: threshold per in-arc
    int64_t ic_in_m = 0;             // IC: in-arcs (arcs whose threshold is not 0)
    double ic_pbar = 0.0;            // IC: mean firing probability of those arcs
    uint64_t* d_lvl = nullptr;       // IC grid shape: per level frontier out-arcs [cap], full-pair in-arcs [cap]
    uint32_t* d_lvl_dir = nullptr;   // IC grid shape: direction of each level [cap]
    uint32_t* d_in_src32 = nullptr;  // source per in-arc (uniform-weight form)
    uint64_t* d_lt_wout = nullptr;   // LT weight per out-arc (push form of the batch's 8-trial tasks)
    uint32_t* d_node_w = nullptr;    // common weight piece per node (uniform-weight form)
    bool lt_uniform = false;
    uint32_t* d_kinfo = nullptr;     // per node: low half of its in-CSR offset, first plane in the count table
    uint64_t kplanes_total = 0;      // count-table planes per word summed over the nodes
    uint32_t* d_bfirst = nullptr;    // LT grid shape: first node of each batch
    uint32_t* d_bdesc = nullptr;     // LT grid shape: 4 words per batch (see SimParams::bdesc)
    uint32_t* d_bigb = nullptr;      // LT grid shape: batches with more than 64 in-arc pieces
    uint32_t nbig = 0;
    uint32_t nbatch = 0;
    // workspace: byte buffers that only grow
    struct Buf {
        void* p = nullptr;
        uint64_t bytes = 0;
    };
    Buf A, N[3], Q[3], aux, thp, Anm, nmark;
    // sets mode (ims_simulate_sets): per-slot state
    Buf sA, sN, sQ[3], sact, sstamp, ssteps, sets_dev;
    imsim::BatchItem* d_item = nullptr;  // the single-run slot form's item
    // Per-call host data (seed lists, set lists, the slot item) reaches the
    // device from pinned staging memory owned by the handle: such a copy
    // reads its source after the call has returned, so a stage is refilled
    // only once the previous copy out of it has completed (its event).
    struct Stage {
        void* h = nullptr;
        size_t bytes = 0;
        hipEvent_t done = nullptr;
    };
    Stage st_seeds, st_pre, st_setoff, st_setnodes, st_item;
    bool sets_zero_dirty = true;  // sA / sN / sstamp / ssteps must start zeroed
    bool zero_dirty = true;  // N / aux must be zero between runs
    uint32_t* d_qcount = nullptr;
    uint32_t cap = 0;
    uint32_t* d_seeds = nullptr;
    uint64_t* d_seed_pre = nullptr;  // prefix of seed out-degrees
    uint32_t seeds_cap = 0;
    uint32_t* d_status = nullptr;     // [0] steps, [1] guard, [2] task counter
    uint32_t* h_flag = nullptr;       // pinned readback of one step counter ([0]) and of the
                                      // last grid run's status words ([2], [3])
    hipEvent_t status_read = nullptr; // that status readback has landed
    bool status_pending = false;      // a grid run's status readback is still to be taken in
    uint32_t last_steps = 0;          // hint for the next grid-shape run
    uint32_t last_shape = 0;
    // kernel timing ring (ims_graph_profile)
    static constexpr int kProf = 256;
    hipEvent_t prof_ev[2 * kProf] = {};
    uint32_t prof_count = 0;

    static void release(Buf& b)
    {
        if (b.p) (void)hipFree(b.p);
        b.p = nullptr;
        b.bytes = 0;
    }
    ~ims_graph()
    {
        for (auto& e : prof_ev)
            if (e) (void)hipEventDestroy(e);
        release(A);
        for (auto& b : N) release(b);
        for (auto& b : Q) release(b);
        release(aux);
        release(nmark);
        release(thp);
        release(Anm);
        for (Buf* b : {&sA, &sN, &sQ[0], &sQ[1], &sQ[2], &sact, &sstamp, &ssteps, &sets_dev}) release(*b);
        dev_free(d_item);
        dev_free(d_off);
        dev_free(d_idx);
        dev_free(d_thr);
        dev_free(d_in_off);
        dev_free(d_in_arc);
        dev_free(d_ic_in);
        dev_free(d_ic_in_thr);
        dev_free(d_lvl);
        dev_free(d_lvl_dir);
        dev_free(d_in_src32);
        dev_free(d_lt_wout);
        dev_free(d_node_w);
        dev_free(d_bfirst);
        dev_free(d_bdesc);
        dev_free(d_kinfo);
        dev_free(d_bigb);
        dev_free(d_qcount);
        dev_free(d_seeds);
        dev_free(d_seed_pre);
        dev_free(d_status);
        if (status_read) (void)hipEventSynchronize(status_read);
        if (h_flag) (void)hipHostFree(h_flag);
        if (status_read) (void)hipEventDestroy(status_read);
        for (Stage* st : {&st_seeds, &st_pre, &st_setoff, &st_setnodes, &st_item}) {
            if (st->done) (void)hipEventSynchronize(st->done);
            if (st->h) (void)hipHostFree(st->h);
            if (st->done) (void)hipEventDestroy(st->done);
        }
    }
};

namespace {

// Device bytes the LT threshold table may take (W * n * 256).
constexpr uint64_t kThresholdTableBudget = 32ull << 30;
// device memory the single-run slot form may hold (48 B per slot and node)
constexpr uint64_t kSlotStateBudget = 32ull << 30;

// Grow a workspace buffer to at least `bytes`; a fresh buffer may hold garbage.
int ensure_buf(ims_graph* g, ims_graph::Buf& b, uint64_t bytes, bool zero_invariant)
{
    if (b.bytes >= bytes && b.p) return IMS_OK;
    ims_graph::release(b);
    uint8_t* p = nullptr;
    int rc = dev_alloc(&p, std::max<uint64_t>(bytes, 8));
    if (rc) return rc;
    b.p = p;
    b.bytes = std::max<uint64_t>(bytes, 8);
    if (zero_invariant) g->zero_dirty = true;
    return IMS_OK;
}

// Copy `bytes` of host data to device `dst` on stream s through stage `st`
// (see ims_graph::Stage).
int stage_upload(ims_graph::Stage& st, void* dst, const void* src, size_t bytes, hipStream_t s)
{
    if (bytes == 0) return IMS_OK;
    if (!st.done) IMS_HIP(hipEventCreateWithFlags(&st.done, hipEventDisableTiming));
    else IMS_HIP(hipEventSynchronize(st.done));
    if (st.bytes < bytes) {
        if (st.h) (void)hipHostFree(st.h);
        st.h = nullptr;
        st.bytes = 0;
        IMS_HIP(hipHostMalloc(&st.h, bytes, hipHostMallocDefault));
        st.bytes = bytes;
    }
    std::memcpy(st.h, src, bytes);
    IMS_HIP(hipMemcpyAsync(dst, st.h, bytes, hipMemcpyHostToDevice, s));
    IMS_HIP(hipEventRecord(st.done, s));
    return IMS_OK;
}

// The last grid-shape run's status, read back without blocking that run:
// its step count sizes the next run's step batches, and a cut-off run leaves
// frontier masks behind that the next run must clear.
int take_grid_status(ims_graph* g)
{
    if (!g->status_pending) return IMS_OK;
    IMS_HIP(hipEventSynchronize(g->status_read));
    g->status_pending = false;
    g->last_steps = g->h_flag[2];
    if (g->h_flag[3]) g->zero_dirty = true;
    return IMS_OK;
}

int device_cus(ims_graph* g)
{
    if (g->cus > 0) return IMS_OK;
    hipDeviceProp_t prop;
    IMS_HIP(hipGetDeviceProperties(&prop, g->device));
    g->cus = prop.multiProcessorCount;
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

    // LT: check the in-weight bound and build the in-CSR (plan.hpp)
    imsim_plan::LtInCsr lt_in;
    if (model == IMS_MODEL_LT) {
        int64_t bad_arc = -1, bad_node = -1;
        const int r = imsim_plan::build_lt_in_csr(n, m, offsets, indices, (const uint64_t*)param, lt_in, bad_arc, bad_node);
        if (r == 1) return fail(IMS_E_WEIGHT_SUM, "LT weight of arc %lld above 2^32", (long long)bad_arc);
        if (r == 2) return fail(IMS_E_WEIGHT_SUM, "LT in-weights of node %lld sum above 2^32", (long long)bad_node);
    }

    ims_graph* g = new (std::nothrow) ims_graph();
    if (!g) return fail(IMS_E_OOM, "host allocation failed");
    (void)hipGetDevice(&g->device);
    g->n = n;
    g->m = m;
    g->model = model;
    g->total_chunks = chunks;
    g->h_off.assign(offsets, offsets + n + 1);
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
        // pull side: per node its in-arcs with their out-CSR ids (plan.hpp)
        imsim_plan::IcInCsr ic_in;
        imsim_plan::build_ic_in_csr(n, m, offsets, indices, (const uint32_t*)param, ic_in);
        const std::vector<int64_t>& ioff = ic_in.off;
        const std::vector<uint64_t>& isa = ic_in.sa;
        const std::vector<uint32_t>& ithr = ic_in.thr;
        const int64_t mi = ioff[n];
        g->ic_in_m = mi;
        double psum = 0.0;
        for (int64_t k = 0; k < mi; ++k) psum += ithr[k] == 0xFFFFFFFFu ? 1.0 : std::ldexp((double)ithr[k], -32);
        g->ic_pbar = mi > 0 ? psum / (double)mi : 0.0;
        if ((rc = dev_alloc(&g->d_in_off, (uint64_t)n + 1)) || (rc = dev_alloc(&g->d_ic_in, (uint64_t)mi)) ||
            (rc = dev_alloc(&g->d_ic_in_thr, (uint64_t)mi)))
            return bail(rc);
        if (hipMemcpy(g->d_in_off, ioff.data(), sizeof(int64_t) * (n + 1), hipMemcpyHostToDevice) != hipSuccess ||
            (mi > 0 && (hipMemcpy(g->d_ic_in, isa.data(), sizeof(uint64_t) * mi, hipMemcpyHostToDevice) != hipSuccess ||
                        hipMemcpy(g->d_ic_in_thr, ithr.data(), sizeof(uint32_t) * mi, hipMemcpyHostToDevice) != hipSuccess)))
            return bail(fail(IMS_E_HIP, "IC in-CSR upload failed"));
    } else {
        const std::vector<int64_t>& in_off = lt_in.off;
        const std::vector<uint64_t>& in_arc = lt_in.arc;
        const int64_t mi = in_off[n];
        if ((rc = dev_alloc(&g->d_in_off, (uint64_t)n + 1))) return bail(rc);
        if ((rc = dev_alloc(&g->d_in_arc, (uint64_t)mi))) return bail(rc);
        if ((rc = dev_alloc(&g->d_lt_wout, (uint64_t)m))) return bail(rc);
        if (m > 0 && hipMemcpy(g->d_lt_wout, param, sizeof(uint64_t) * m, hipMemcpyHostToDevice) != hipSuccess)
            return bail(fail(IMS_E_HIP, "LT weight upload failed"));
        // equal in-weights form (every node's pieces equal) with its
        // count-threshold planes
        std::vector<uint32_t> node_w, src32;
        const bool uniform = imsim_plan::lt_uniform_form(n, lt_in, node_w, src32);
        g->lt_uniform = uniform;
        if (uniform) {
            std::vector<uint32_t> kinfo;
            g->kplanes_total = imsim_plan::lt_count_planes(n, in_off, kinfo);
            if ((rc = dev_alloc(&g->d_kinfo, kinfo.size()))) return bail(rc);
            if (hipMemcpy(g->d_kinfo, kinfo.data(), sizeof(uint32_t) * kinfo.size(), hipMemcpyHostToDevice) != hipSuccess)
                return bail(fail(IMS_E_HIP, "in-CSR upload failed"));
            if ((rc = dev_alloc(&g->d_in_src32, (uint64_t)mi))) return bail(rc);
            if ((rc = dev_alloc(&g->d_node_w, (uint64_t)n))) return bail(rc);
            if ((mi > 0 && hipMemcpy(g->d_in_src32, src32.data(), sizeof(uint32_t) * mi, hipMemcpyHostToDevice) != hipSuccess) ||
                (n > 0 && hipMemcpy(g->d_node_w, node_w.data(), sizeof(uint32_t) * n, hipMemcpyHostToDevice) != hipSuccess))
                return bail(fail(IMS_E_HIP, "in-CSR upload failed"));
        }
        if (hipMemcpy(g->d_in_off, in_off.data(), sizeof(int64_t) * (n + 1), hipMemcpyHostToDevice) != hipSuccess ||
            (mi > 0 && hipMemcpy(g->d_in_arc, in_arc.data(), sizeof(uint64_t) * mi, hipMemcpyHostToDevice) != hipSuccess))
            return bail(fail(IMS_E_HIP, "in-CSR upload failed"));
        // node batches of the grid-shape sweep
        imsim_plan::LtBatches lb;
        imsim_plan::lt_batches(n, in_off, lb);
        const std::vector<uint32_t>& bfirst = lb.bfirst;
        const std::vector<uint32_t>& bdesc = lb.bdesc;
        std::vector<uint32_t> bigb = lb.bigb;
        g->nbatch = lb.nbatch;
        if ((rc = dev_alloc(&g->d_bfirst, bfirst.size()))) return bail(rc);
        if ((rc = dev_alloc(&g->d_bdesc, bdesc.size()))) return bail(rc);
        g->nbig = (uint32_t)bigb.size();
        bigb.push_back(0);
        if ((rc = dev_alloc(&g->d_bigb, bigb.size()))) return bail(rc);
        if (hipMemcpy(g->d_bigb, bigb.data(), sizeof(uint32_t) * bigb.size(), hipMemcpyHostToDevice) != hipSuccess)
            return bail(fail(IMS_E_HIP, "batch upload failed"));
        if (hipMemcpy(g->d_bfirst, bfirst.data(), sizeof(uint32_t) * bfirst.size(), hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(g->d_bdesc, bdesc.data(), sizeof(uint32_t) * bdesc.size(), hipMemcpyHostToDevice) != hipSuccess)
            return bail(fail(IMS_E_HIP, "batch upload failed"));
    }
    g->cap = (uint32_t)std::min<int64_t>(n + 8, 0xFFFFFFF0ll);
    if ((rc = dev_alloc(&g->d_qcount, g->cap))) return bail(rc);
    if (model == IMS_MODEL_IC && ((rc = dev_alloc(&g->d_lvl, 2ull * g->cap)) || (rc = dev_alloc(&g->d_lvl_dir, g->cap))))
        return bail(rc);
    if ((rc = dev_alloc(&g->d_status, 4))) return bail(rc);
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

}  // extern "C"

namespace {

// Workgroups of `kernel` (kBlock threads) resident on the whole device at
// once: a grid of exactly this size runs in one round, with no second round
// of workgroups trailing behind.
template <typename K>
uint32_t resident_blocks(K kernel, uint32_t cus)
{
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, imsim::kBlock, 0) != hipSuccess || per_cu < 1) {
        (void)hipGetLastError();
        per_cu = 1;
    }
    return (uint32_t)per_cu * cus;
}

// IC pull side and direction rule of a run (P.W set): Beamer's switch points
// (alpha 14, beta 24, those of his direction-optimising BFS) unless given,
// with alpha scaled by the graph's mean arc probability: a pulled node stops
// early once its pending trials have joined, which an IC arc brings about
// only with its probability (p = 1 gives Beamer's BFS rule; measured on the
// paper's stand-in graphs, the scaled rule keeps low-probability cascades on
// hub graphs on the push side, where pulling was up to 2.8x slower, and still
// pulls the high-probability ones, 2-4.7x faster than push alone).
// Word-local runs default to alpha 2: their tasks of 4 to 16 trials push
// cheaply, and a pulled step scans the in-arcs of every pending node of the
// task (on the nine stand-ins and the 200k-node sets, alpha 2 is never slower
// than 14, and pulls uniform-p Watts-Strogatz 1.5x and ER 1.1x less often
// wrongly: 3.1 -> 2.1 ms and 0.35 -> 0.32 ms per 1,000 trials).
constexpr double kIcAlphaGrid = 14.0, kIcAlphaWordLocal = 2.0;
int set_ic_direction(imsim::SimParams& P, const ims_graph* g, double alpha, double beta, int dir, double alpha_default = kIcAlphaGrid)
{
    if (dir < 0 || dir > 2) return fail(IMS_E_INVALID_ARG, "IC direction %d not in 0..2", dir);
    if (!(alpha >= 0.0) || !(beta >= 0.0)) return fail(IMS_E_INVALID_ARG, "IC switch points must be >= 0 (0 = default)");
    P.ic_in = g->d_ic_in;
    P.ic_in_thr = g->d_ic_in_thr;
    P.lvl_farcs = (unsigned long long*)g->d_lvl;
    P.lvl_full = g->d_lvl ? (unsigned long long*)g->d_lvl + g->cap : nullptr;
    P.lvl_dir = g->d_lvl_dir;
    P.in_total = (uint64_t)P.W * (uint64_t)g->ic_in_m;
    P.ic_alpha = (float)((alpha > 0.0 ? alpha : alpha_default) * g->ic_pbar);
    // grid push: read the target first from a mean arc probability of 0.2 on
    // (measured on the stand-ins: uniform-p ER and BA-Facebook 6-8% faster
    // with the read, the low-probability cascades 2-11% faster without)
    P.ic_preload = g->ic_pbar >= 0.2 ? 1 : 0;
    P.ic_beta = beta > 0.0 ? (float)beta : 24.0f;
    P.ic_dir = dir;
    // word-local runs below a mean arc probability of 0.25 push only unless
    // the caller sets the direction or alpha: there a pulled step never paid
    // on the stand-ins, and the rule's bookkeeping (the in-arcs of every node
    // whose trials have all joined) cost 1-9% per run
    if (alpha_default == kIcAlphaWordLocal && dir == 0 && alpha == 0.0 && g->ic_pbar < 0.25) P.ic_dir = 1;
    return IMS_OK;
}

// One simulation; with level_counts the word-local shape also counts the
// nodes first activated at every level of every trial.
int simulate_impl(ims_graph* g, const uint32_t* seeds, uint32_t n_seeds, uint32_t n_trials, uint64_t rng_seed,
                  const ims_opts* opts, uint32_t* trial_counts, uint32_t* node_counts, uint64_t* total, uint64_t* active_bits,
                  void* stream, uint32_t* level_counts, uint32_t max_levels, uint32_t w0 = 0, bool accumulate = false)
{
    if (!g) return fail(IMS_E_INVALID_ARG, "ims_simulate: NULL graph");
    if (n_trials == 0) return fail(IMS_E_INVALID_ARG, "ims_simulate: n_trials must be >= 1");
    if (n_trials > imsim::kMaxWords * 64u) return fail(IMS_E_UNSUPPORTED, "ims_simulate: n_trials above %u", imsim::kMaxWords * 64u);
    if (!trial_counts || !total) return fail(IMS_E_INVALID_ARG, "ims_simulate: trial_counts and total are required");
    if (n_seeds > 0 && !seeds) return fail(IMS_E_INVALID_ARG, "ims_simulate: seeds is NULL");
    hipStream_t s = (hipStream_t)stream;
    int rc = device_cus(g);
    if (rc) return rc;
    if ((rc = take_grid_status(g))) return rc;

    // seeds: range check and set semantics on the host
    std::vector<uint32_t> sv(seeds, seeds + n_seeds);
    for (uint32_t x : sv)
        if ((int64_t)x >= g->n) return fail(IMS_E_SEED_RANGE, "seed %u >= n = %lld", x, (long long)g->n);
    std::sort(sv.begin(), sv.end());
    sv.erase(std::unique(sv.begin(), sv.end()), sv.end());

    uint32_t W = (n_trials + 63) / 64;
    const uint64_t n = (uint64_t)g->n;
    uint64_t cells = (uint64_t)W * n;
    // execution shape: word-local when there are enough words to occupy the
    // device (a word per workgroup, a quarter of the compute units or more);
    // grid-wide steps otherwise, whatever the graph size (measured faster at
    // 16 words on graphs of 1,000 to 1,000,000 nodes)
    int shape = opts ? opts->shape : 0;
    // automatic shape: IC takes the word-local shape once there are at least a
    // quarter as many words as compute units, and with fewer words when the
    // cascades stay small: the expected offspring of a node, p * m / n (p the
    // arcs' mean probability), at most 1.05 and the seeds' expected direct
    // reach, p times their out-degrees, at most 10,000 nodes, or a graph of
    // at most 5,000 nodes with offspring at most 2.5 (measured at 1,000
    // trials: word-local 1.1-3.5x faster on the ER / WS / BA stand-ins with
    // TV and WC weights, ER 2k with UR weights, ER 1k at p = 0.1 and a
    // 200k-node Chung-Lu graph with WC weights; the grid shape 1.2-4x faster
    // for offspring from 1.3 on larger graphs, from 5 on small ones, and for
    // 100 hub seeds on a 1M-node graph even at 0.3).  LT always takes the
    // grid shape (measured 1.2-16x faster than word-local on graphs of 1,000
    // to 1M nodes at 1,000 and 10,000 trials, except a 5,000-node BA graph at
    // 10,000 trials, 2.5x slower)
    if (shape == 0) {
        if (g->model == IMS_MODEL_LT) {
            shape = 2;
        } else if (W >= (uint32_t)g->cus / 4) {
            shape = 1;
        } else {
            double reach = 0.0;
            for (uint32_t x : sv) reach += (double)(g->h_off[x + 1] - g->h_off[x]);
            reach *= g->ic_pbar;
            const double offspring = n > 0 ? g->ic_pbar * (double)g->ic_in_m / (double)n : 0.0;
            shape = (offspring <= 1.05 && reach <= 10000.0) || (n <= 5000 && offspring <= 2.5) ? 1 : 2;
        }
    }
    if (level_counts) shape = 1;  // levels are the word-local (synchronous) steps
    if (shape != 1 && shape != 2) return fail(IMS_E_INVALID_ARG, "ims_simulate: unknown shape %d", shape);
    // LT grid shape over more than 16 words: runs of 16 words one after the
    // other (trials are independent; each run hashes its trials by their
    // global index), so every run takes the sweep's 16-word form; per-node
    // counts and the total accumulate over the runs
    if (shape == 2 && g->model == IMS_MODEL_LT && W > imsim::kRowWords && w0 == 0 && !accumulate) {
        ims_opts o = opts ? *opts : ims_opts{};
        o.shape = 2;
        for (uint32_t c0 = 0; c0 < W; c0 += imsim::kRowWords) {
            const uint32_t tc = std::min<uint32_t>(imsim::kRowWords * 64u, n_trials - 64u * c0);
            rc = simulate_impl(g, seeds, n_seeds, tc, rng_seed, &o, trial_counts + 64ull * c0, node_counts, total,
                               active_bits ? active_bits + (uint64_t)c0 * (uint64_t)g->n : nullptr, stream, nullptr, 0, c0,
                               c0 > 0);
            if (rc) return rc;
        }
        return IMS_OK;
    }
    // LT grid shape with 9 to 15 words: node-major rows padded to 16 words
    // (the words past n_trials hold no trial), so that a node's row is one
    // 128-byte line rather than straddling two; 6 and 7 words likewise to 8
    // (measured 3-4% faster; 5 words padded measured 1% slower)
    if (shape == 2 && g->model == IMS_MODEL_LT && W > 8 && W < imsim::kRowWords) {
        W = imsim::kRowWords;
        cells = (uint64_t)W * n;
    } else if (shape == 2 && g->model == IMS_MODEL_LT && (W == 6 || W == 7)) {
        W = 8;
        cells = (uint64_t)W * n;
    }

    // word-local runs that return only counts take the slot form: each word
    // runs as 4, 8 or 16 tasks (16, 8 or 4 trials each: the fewest that give
    // at least half as many tasks as there are slots) on workgroup slots whose
    // state is cleared sparsely, and the tasks add their own counts (no fill
    // of the full state, no reduction passes over it).  Measured at 1,000
    // trials (16 words) on the ER / WS / BA stand-ins: 4-trial tasks 1.2-2.8x
    // faster than 16-trial ones, 2-trial tasks faster only on the BA graphs;
    // at 10,000 trials 16-trial tasks fastest.
    // (graphs whose slot state would exceed kSlotStateBudget keep one
    // workgroup per word over the W x n state)
    const int slot_per_cu = opts && opts->blocks_per_cu > 0 ? opts->blocks_per_cu : 2;
    uint32_t slot_sp = 2;
    while (slot_sp < 4 && ((uint64_t)W << slot_sp) * 2 < (uint64_t)g->cus * slot_per_cu) ++slot_sp;
    const uint64_t slot_tasks = (uint64_t)W << slot_sp;
    const uint64_t slots = std::max<uint64_t>(1, std::min<uint64_t>(slot_tasks, (uint64_t)g->cus * slot_per_cu));
    const bool slot_run = shape == 1 && !active_bits && !level_counts && slots * n * 48 <= kSlotStateBudget;
    if (slot_run) {
        const uint64_t sc = slots * n;
        const uint64_t before = g->sA.bytes + g->sN.bytes + g->sstamp.bytes + g->ssteps.bytes;
        if ((rc = ensure_buf(g, g->sA, sc * 8, false)) || (rc = ensure_buf(g, g->sact, sc * 4, false)) ||
            (rc = ensure_buf(g, g->sQ[0], sc * 4, false)) || (rc = ensure_buf(g, g->sQ[1], sc * 4, false)) ||
            (rc = ensure_buf(g, g->sN, sc * 8, false)) || (rc = ensure_buf(g, g->sQ[2], sc * 16, false)) ||
            (rc = ensure_buf(g, g->sstamp, sc * 4, false)) || (rc = ensure_buf(g, g->ssteps, slots * 4, false)))
            return rc;
        if (g->sA.bytes + g->sN.bytes + g->sstamp.bytes + g->ssteps.bytes != before) {
            // fresh slot state starts clear (tasks leave it clear)
            for (ims_graph::Buf* b : {&g->sA, &g->sN, &g->sstamp, &g->ssteps})
                if ((rc = fill_async<uint8_t>((uint8_t*)b->p, b->bytes, 0, s))) return rc;
            g->sets_zero_dirty = false;
        }
        if (!g->d_item && (rc = dev_alloc(&g->d_item, 1))) return rc;
    }
    if (!active_bits && !slot_run && (rc = ensure_buf(g, g->A, cells * 8, false))) return rc;
    if (shape == 1 && !slot_run) {
        if (g->model == IMS_MODEL_IC) {
            if ((rc = ensure_buf(g, g->N[0], cells * 8, true))) return rc;
            if ((rc = ensure_buf(g, g->Q[0], cells * 4, false))) return rc;
            if ((rc = ensure_buf(g, g->Q[1], cells * 4, false))) return rc;
            if ((rc = ensure_buf(g, g->Q[2], cells * 16, false))) return rc;
        } else {
            if ((rc = ensure_buf(g, g->aux, cells * 4, true))) return rc;
            for (int i = 0; i < 3; ++i)
                if ((rc = ensure_buf(g, g->Q[i], cells * 4, false))) return rc;
            // synchronous steps (level counts) hold each step's joins here
            if (level_counts && (rc = ensure_buf(g, g->N[0], cells * 8, true))) return rc;
        }
    } else if (shape == 2 && g->model == IMS_MODEL_IC) {
        const uint64_t qcap = (uint64_t)W * std::max<uint64_t>(g->total_chunks, 1);
        for (int i = 0; i < 3; ++i) {
            if ((rc = ensure_buf(g, g->N[i], cells * 8, true))) return rc;
            if ((rc = ensure_buf(g, g->Q[i], qcap * 8, false))) return rc;
        }
    } else if (shape == 2) {
        if ((rc = ensure_buf(g, g->aux, cells * 4, true))) return rc;
        if ((rc = ensure_buf(g, g->Anm, cells * 8, false))) return rc;
        if ((rc = ensure_buf(g, g->nmark, (uint64_t)g->n * 4, false))) return rc;
    }
    // LT grid shape: threshold prefix table when it fits the budget
    const int test_flags = opts ? opts->test_flags : 0;
    // LT grid shape threshold form: count thresholds (equal in-weights, 8 B
    // per plane and node-word, words padded to whole groups), full hashes
    // (256 B), or hashes drawn in the kernel
    int lt_mode = 0;
    const uint64_t kmin_bytes = g->kplanes_total * ((W + imsim::kRowWords - 1) / imsim::kRowWords) * imsim::kRowWords * 8ull;
    if (shape == 2 && g->model == IMS_MODEL_LT && !(test_flags & 1)) {
        if (g->lt_uniform && !(test_flags & 4) && kmin_bytes <= kThresholdTableBudget && g->kplanes_total < (1ull << 32) &&
            !(test_flags & 8))
            lt_mode = 2;
        else if (cells * 256 <= kThresholdTableBudget) lt_mode = 1;
    }
    const bool use_table = lt_mode != 0;
    // (the count-threshold table has 64 bytes of padding: the sweep reads 64
    // bytes from each (node, word)'s first plane)
    if (use_table && (rc = ensure_buf(g, g->thp, lt_mode == 2 ? kmin_bytes + 64 : cells * 256, false))) return rc;
    if (g->seeds_cap < sv.size() || !g->d_seeds) {
        dev_free(g->d_seeds);
        dev_free(g->d_seed_pre);
        if ((rc = dev_alloc(&g->d_seeds, sv.size()))) return rc;
        if ((rc = dev_alloc(&g->d_seed_pre, sv.size() + 1))) return rc;
        g->seeds_cap = (uint32_t)sv.size();
    }
    std::vector<uint64_t> seed_pre(sv.size() + 1, 0);
    for (size_t i = 0; i < sv.size(); ++i) seed_pre[i + 1] = seed_pre[i] + (uint64_t)(g->h_off[sv[i] + 1] - g->h_off[sv[i]]);
    if (!g->h_flag) IMS_HIP(hipHostMalloc((void**)&g->h_flag, 4 * sizeof(uint32_t), hipHostMallocDefault));
    if ((rc = stage_upload(g->st_seeds, g->d_seeds, sv.data(), sv.size() * sizeof(uint32_t), s))) return rc;
    if ((rc = stage_upload(g->st_pre, g->d_seed_pre, seed_pre.data(), seed_pre.size() * sizeof(uint64_t), s))) return rc;

    uint64_t* A = active_bits ? active_bits : (uint64_t*)g->A.p;
    // the LT grid shape keeps its state node-major and writes A (when asked
    // for) from it at the end
    const bool ltg = shape == 2 && g->model == IMS_MODEL_LT;
    if (!ltg && !slot_run && (rc = fill_async<uint64_t>(A, cells, 0ull, s))) return rc;
    // LT word-local steps stamp candidates 1, 2, ... in aux, which earlier
    // runs (of either shape) leave holding their own stamps and sweep marks
    if (shape == 1 && !slot_run && g->model == IMS_MODEL_LT && (rc = fill_async<uint32_t>((uint32_t*)g->aux.p, cells, 0u, s)))
        return rc;
    if (g->zero_dirty) {
        for (auto& b : g->N)
            if (b.p && (rc = fill_async<uint8_t>((uint8_t*)b.p, b.bytes, 0, s))) return rc;
        if (g->aux.p && (rc = fill_async<uint8_t>((uint8_t*)g->aux.p, g->aux.bytes, 0, s))) return rc;
        g->zero_dirty = false;
    }
    // (a later 16-word run keeps an earlier run's guard flag)
    if (!accumulate && (rc = fill_async<uint32_t>(g->d_status, 4, 0u, s))) return rc;
    if ((rc = fill_async<uint32_t>(trial_counts, n_trials, 0u, s))) return rc;
    if (!accumulate && (rc = fill_async<unsigned long long>((unsigned long long*)total, 1, 0ull, s))) return rc;

    imsim::SimParams P;
    P.n = g->n;
    P.T = n_trials;
    P.W = W;
    P.seed = rng_seed;
    P.off = g->d_off;
    P.idx = g->d_idx;
    P.thr = g->d_thr;
    P.in_off = g->d_in_off;
    P.in_arc = g->d_in_arc;
    P.in_src32 = g->d_in_src32;
    P.node_w = g->d_node_w;
    P.lt_uniform = g->lt_uniform && !(test_flags & 4) ? 1 : 0;
    P.thp = nullptr;
    P.th32 = nullptr;
    P.kplanes = nullptr;
    P.kinfo = g->d_kinfo;
    P.thp_shift = (test_flags & 2) ? 31u : 16u;
    P.A = A;
    P.Anm = (uint64_t*)g->Anm.p;
    P.bfirst = g->d_bfirst;
    P.bdesc = reinterpret_cast<const imsim::u32x4*>(g->d_bdesc);
    P.bigb = g->d_bigb;
    P.nbig = g->nbig;
    P.nbatch = g->nbatch;
    for (int i = 0; i < 3; ++i) {
        P.N[i] = (uint64_t*)g->N[i].p;
        P.Q[i] = (uint64_t*)g->Q[i].p;
    }
    P.qcount = g->d_qcount;
    P.aux = (uint32_t*)g->aux.p;
    P.nmark = (uint32_t*)g->nmark.p;
    P.base = nullptr;
    P.level_counts = level_counts;
    P.w0 = w0;
    P.max_levels = max_levels;
    P.seeds = g->d_seeds;
    P.n_seeds = (uint32_t)sv.size();
    P.seed_arcs = seed_pre.back();
    P.task_counter = g->d_status + 2;
    P.set_off = nullptr;
    P.set_nodes = nullptr;
    P.n_sets = 0;
    P.totals = nullptr;
    P.set_node_counts = nullptr;
    P.act = nullptr;
    P.sstamp = nullptr;
    P.slot_steps = nullptr;
    P.status = g->d_status;
    P.cap = g->cap;
    if ((rc = set_ic_direction(P, g, opts ? opts->ic_alpha : 0.0, opts ? opts->ic_beta : 0.0, opts ? opts->ic_direction : 0,
                               shape == 1 ? kIcAlphaWordLocal : kIcAlphaGrid)))
        return rc;

    const bool prof = opts && opts->profile && g->prof_count < ims_graph::kProf;
    const uint32_t slot = g->prof_count;
    if (prof) {
        for (int k = 0; k < 2; ++k)
            if (!g->prof_ev[2 * slot + k]) IMS_HIP(hipEventCreate(&g->prof_ev[2 * slot + k]));
        IMS_HIP(hipEventRecord(g->prof_ev[2 * slot], s));
    }
    if (slot_run) {
        if (node_counts && (rc = fill_async<uint32_t>(node_counts, n, 0u, s))) return rc;
        imsim::BatchItem it;
        std::memset(&it, 0, sizeof it);
        it.P = P;
        it.model = g->model;
        it.trial_counts = trial_counts;
        it.node_counts = node_counts;
        it.total = total;
        if ((rc = stage_upload(g->st_item, g->d_item, &it, sizeof it, s))) return rc;
        imsim::SlotBufs S{n,
                          (uint64_t*)g->sA.p,
                          (uint64_t*)g->sN.p,
                          (uint32_t*)g->sQ[0].p,
                          (uint32_t*)g->sQ[1].p,
                          (uint64_t*)g->sQ[2].p,
                          (uint32_t*)g->sact.p,
                          (uint32_t*)g->sstamp.p,
                          (uint32_t*)g->ssteps.p};
        // IC on at most kLdsNodes nodes: the tasks' masks in LDS
        if (g->model == IMS_MODEL_IC && n <= imsim::kLdsNodes)
            hipLaunchKernelGGL((imsim::slot_run_kernel<0, true>), dim3((uint32_t)slots), dim3(imsim::kTaskBlock), 0, s,
                               (const imsim::BatchItem*)g->d_item, slot_sp, (uint32_t)slot_tasks, g->d_status + 2, S, g->d_status);
        else if (g->model == IMS_MODEL_IC)
            hipLaunchKernelGGL((imsim::slot_run_kernel<0, false>), dim3((uint32_t)slots), dim3(imsim::kTaskBlock), 0, s,
                               (const imsim::BatchItem*)g->d_item, slot_sp, (uint32_t)slot_tasks, g->d_status + 2, S, g->d_status);
        else
            hipLaunchKernelGGL((imsim::slot_run_kernel<1, false>), dim3((uint32_t)slots), dim3(imsim::kTaskBlock), 0, s,
                               (const imsim::BatchItem*)g->d_item, slot_sp, (uint32_t)slot_tasks, g->d_status + 2, S, g->d_status);
        IMS_HIP(hipGetLastError());
    } else if (shape == 1) {
        const int per_cu = opts && opts->blocks_per_cu > 0 ? opts->blocks_per_cu : 2;
        const uint32_t blocks = std::min<uint32_t>(W, (uint32_t)(g->cus * per_cu));
        if (g->model == IMS_MODEL_IC)
            hipLaunchKernelGGL((imsim::word_kernel<false, false>), dim3(blocks), dim3(imsim::kTaskBlock), 0, s, P, n);
        else
            hipLaunchKernelGGL((imsim::word_kernel<false, true>), dim3(blocks), dim3(imsim::kTaskBlock), 0, s, P, n);
        IMS_HIP(hipGetLastError());
    } else {
        // IC: 4 workgroups per compute unit by default (measured on the
        // benchmark graphs: up to 20% faster than 8, never slower than 1-3)
        const int per_cu = opts && opts->blocks_per_cu > 0 ? opts->blocks_per_cu : 4;
        const uint32_t blocks = (uint32_t)(g->cus * per_cu);
        // LT: by default every kernel of the run gets exactly its resident
        // grid (measured on the 1M-node count form: 13.0 ms against 15.7 ms
        // at 8 workgroups per compute unit)
        const bool fixed = opts && opts->blocks_per_cu > 0;
        auto lt_blocks = [&](auto kernel) -> uint32_t { return fixed ? blocks : resident_blocks(kernel, (uint32_t)g->cus); };
        if ((rc = fill_async<uint32_t>(g->d_qcount, g->cap, 0u, s))) return rc;
        // direction switch: sweeps mark once a sweep changes fewer than tau
        // (node, word) pairs; cells / 64 measured best on the 1M-node LT
        // graph (3.8% faster than cells / 32, the same as cells / 128)
        const uint32_t tau = opts && opts->alpha > 0.0 ? (uint32_t)std::min<double>(opts->alpha * (double)cells, 4e9)
                                                       : (uint32_t)std::min<uint64_t>(cells / 64 + 1, 0xFFFFFFFFull);
        if (g->model == IMS_MODEL_IC) {
            // per-level direction counters: entries 0 and 1 start at zero,
            // each level clears the entry two ahead of it
            if ((rc = fill_async<uint64_t>(g->d_lvl, 2, 0ull, s))) return rc;
            if ((rc = fill_async<uint64_t>(g->d_lvl + g->cap, 2, 0ull, s))) return rc;
            hipLaunchKernelGGL(imsim::grid_seed_kernel, dim3(std::max<uint32_t>(1, std::min<uint32_t>(blocks, (P.n_seeds * W + 255) / 256))),
                               dim3(imsim::kBlock), 0, s, P, g->model);
            IMS_HIP(hipGetLastError());
        } else {
            // node-major state and sweep marks start cleared every run
            if ((rc = fill_async<uint64_t>(P.Anm, cells, 0ull, s))) return rc;
            if ((rc = fill_async<uint32_t>((uint32_t*)g->aux.p, cells, 0u, s))) return rc;
            if ((rc = fill_async<uint32_t>((uint32_t*)g->nmark.p, (uint64_t)g->n, 0u, s))) return rc;
            if (lt_mode == 1) {
                P.th32 = (const uint32_t*)g->thp.p;
                hipLaunchKernelGGL(imsim::ltg_table_kernel, dim3(lt_blocks(imsim::ltg_table_kernel)), dim3(imsim::kBlock), 0, s, P,
                                   (uint32_t*)g->thp.p);
                IMS_HIP(hipGetLastError());
            } else if (lt_mode == 2) {
                P.kplanes = (const uint64_t*)g->thp.p;
                // (16 workgroups per compute unit measured 1% faster per call
                // than the resident grid for this ALU-bound kernel)
                hipLaunchKernelGGL(imsim::ltg_kmin_kernel, dim3(fixed ? blocks : (uint32_t)g->cus * 16), dim3(imsim::kBlock), 0, s, P,
                                   (uint64_t*)g->thp.p);
                IMS_HIP(hipGetLastError());
            }
            const uint64_t work = std::max<uint64_t>(seed_pre.back(), (uint64_t)P.n_seeds * W);
            hipLaunchKernelGGL(imsim::ltg_seed_kernel,
                               dim3((uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(blocks, (work + imsim::kBlock - 1) / imsim::kBlock))),
                               dim3(imsim::kBlock), 0, s, P, (const uint64_t*)g->d_seed_pre, P.seed_arcs * W < tau ? 1 : 0);
            IMS_HIP(hipGetLastError());
        }
        uint32_t sweep_blocks = blocks, big_blocks = blocks;
        if (g->model == IMS_MODEL_LT) {
            sweep_blocks = lt_mode == 2   ? lt_blocks(imsim::ltg_sweep_kernel<2>)
                           : lt_mode == 1 ? lt_blocks(imsim::ltg_sweep_kernel<1>)
                                          : lt_blocks(imsim::ltg_sweep_kernel<0>);
            big_blocks = lt_blocks(imsim::ltg_sweep_kernel<3>);
        }
        // steps in batches; a step after the last productive one returns at
        // once, so only the end of each batch is read back
        uint32_t next = 0, batch = std::max<uint32_t>(8, g->last_steps + 2);
        bool done = false;
        while (!done) {
            const uint32_t end = std::min<uint32_t>(next + batch, g->cap);
            for (uint32_t st = next; st < end; ++st) {
                if (g->model == IMS_MODEL_IC)
                    hipLaunchKernelGGL(imsim::grid_ic_level_kernel, dim3(blocks), dim3(imsim::kBlock), 0, s, P, st);
                else
                {
                    if (lt_mode == 2) {
                        hipLaunchKernelGGL(imsim::ltg_sweep_kernel<2>, dim3(sweep_blocks), dim3(imsim::kBlock), 0, s, P, st, tau);
                        if (g->nbig)
                            hipLaunchKernelGGL(imsim::ltg_sweep_kernel<3>,
                                               dim3(std::min<uint32_t>(big_blocks, (g->nbig + imsim::kWaves - 1) / imsim::kWaves)),
                                               dim3(imsim::kBlock), 0, s, P, st, tau);
                    }
                    else if (lt_mode == 1)
                        hipLaunchKernelGGL(imsim::ltg_sweep_kernel<1>, dim3(sweep_blocks), dim3(imsim::kBlock), 0, s, P, st, tau);
                    else
                        hipLaunchKernelGGL(imsim::ltg_sweep_kernel<0>, dim3(sweep_blocks), dim3(imsim::kBlock), 0, s, P, st, tau);
                }
            }
            IMS_HIP(hipGetLastError());
            // IC: level `end` has no items; LT: sweep end-1 changed nothing
            const uint32_t probe = g->model == IMS_MODEL_IC ? std::min(end, g->cap - 1) : end - 1;
            IMS_HIP(hipMemcpyAsync(g->h_flag, g->d_qcount + probe, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
            IMS_HIP(hipStreamSynchronize(s));
            done = g->h_flag[0] == 0 || end >= g->cap;
            next = end;
        }
        // IC: level `next` is empty and was not launched; launching it clears
        // the frontier masks of level next - 1 (the last expanded level), which
        // must be zero when the next run starts
        if (g->model == IMS_MODEL_IC && next < g->cap) {
            hipLaunchKernelGGL(imsim::grid_ic_level_kernel, dim3(blocks), dim3(imsim::kBlock), 0, s, P, next);
            IMS_HIP(hipGetLastError());
        }
        if (g->model == IMS_MODEL_LT && cells > 0) {
            hipLaunchKernelGGL(imsim::ltg_finish_kernel, dim3((uint32_t)std::min<uint64_t>((uint64_t)g->cus * 4, ((uint64_t)g->n + 255) / 256)),
                               dim3(imsim::kBlock), 0, s, (const uint64_t*)P.Anm, active_bits, g->n, W, n_trials, trial_counts,
                               node_counts, (unsigned long long*)total, accumulate ? 1 : 0);
            IMS_HIP(hipGetLastError());
        }
        // steps taken and the guard go into the status words on the device;
        // the host takes them in at its next call on this handle
        hipLaunchKernelGGL(imsim::grid_status_kernel, dim3(1), dim3(64), 0, s, (const uint32_t*)g->d_qcount, next, g->cap,
                           g->model == IMS_MODEL_LT ? 1u : 0u, g->d_status);
        IMS_HIP(hipGetLastError());
        if (!g->status_read) IMS_HIP(hipEventCreateWithFlags(&g->status_read, hipEventDisableTiming));
        IMS_HIP(hipMemcpyAsync(g->h_flag + 2, g->d_status, 2 * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
        IMS_HIP(hipEventRecord(g->status_read, s));
        g->status_pending = true;
    }
    if (prof) {
        IMS_HIP(hipEventRecord(g->prof_ev[2 * slot + 1], s));
        g->prof_count = slot + 1;
    }
    g->last_shape = (uint32_t)shape;

    if (n > 0 && !(ltg && cells > 0) && !slot_run) {
        const uint64_t nblk = std::min<uint64_t>((n + imsim::kBlock - 1) / imsim::kBlock, 1024);
        hipLaunchKernelGGL(imsim::reduce_trial_counts, dim3((unsigned)nblk, W), dim3(imsim::kBlock), 0, s, A, g->n, n_trials,
                           trial_counts);
        IMS_HIP(hipGetLastError());
        hipLaunchKernelGGL(imsim::reduce_node_counts, dim3((unsigned)std::min<uint64_t>(nblk * 4, 4096)), dim3(imsim::kBlock), 0, s, A,
                           g->n, W, node_counts, (unsigned long long*)total);
        IMS_HIP(hipGetLastError());
    }
    return IMS_OK;
}

}  // namespace

extern "C" {

int ims_simulate(ims_graph* g, const uint32_t* seeds, uint32_t n_seeds, uint32_t n_trials, uint64_t rng_seed,
                 const ims_opts* opts, uint32_t* trial_counts, uint32_t* node_counts, uint64_t* total,
                 uint64_t* active_bits, void* stream)
{
    return simulate_impl(g, seeds, n_seeds, n_trials, rng_seed, opts, trial_counts, node_counts, total, active_bits, stream,
                         nullptr, 0);
}

int ims_simulate_levels(ims_graph* g, const uint32_t* seeds, uint32_t n_seeds, uint32_t n_trials, uint64_t rng_seed,
                        uint32_t max_levels, uint32_t* level_counts, uint32_t* trial_counts, uint64_t* total, void* stream)
{
    if (!g) return fail(IMS_E_INVALID_ARG, "ims_simulate_levels: NULL graph");
    if (!level_counts || max_levels == 0) return fail(IMS_E_INVALID_ARG, "ims_simulate_levels: level_counts and max_levels >= 1 required");
    if (n_trials > 0 && (uint64_t)max_levels * n_trials > 0xFFFFFFFFull)
        return fail(IMS_E_UNSUPPORTED, "ims_simulate_levels: max_levels * n_trials above 2^32");
    int rc = fill_async<uint32_t>(level_counts, (uint64_t)max_levels * n_trials, 0u, (hipStream_t)stream);
    if (rc) return rc;
    return simulate_impl(g, seeds, n_seeds, n_trials, rng_seed, nullptr, trial_counts, nullptr, total, nullptr, stream,
                         level_counts, max_levels);
}

}  // extern "C"

namespace {

// Many seed sets under one trial range (common random numbers); with `base`
// the sets start from that word-major state and count new activations only.
int simulate_sets_impl(ims_graph* g, const uint64_t* base, const uint32_t* set_offsets, const uint32_t* set_nodes, uint32_t n_sets,
                       uint32_t n_trials, uint64_t rng_seed, const ims_opts* opts, uint64_t* totals, uint32_t* node_counts,
                       void* stream)
{
    if (!g) return fail(IMS_E_INVALID_ARG, "ims_simulate_sets: NULL graph");
    if (n_trials == 0) return fail(IMS_E_INVALID_ARG, "ims_simulate_sets: n_trials must be >= 1");
    if (n_trials > imsim::kMaxWords * 64u) return fail(IMS_E_UNSUPPORTED, "ims_simulate_sets: n_trials above %u", imsim::kMaxWords * 64u);
    if (n_sets > 0 && (!set_offsets || !totals)) return fail(IMS_E_INVALID_ARG, "ims_simulate_sets: set_offsets and totals are required");
    if (n_sets == 0) return IMS_OK;
    if (set_offsets[0] != 0) return fail(IMS_E_INVALID_ARG, "ims_simulate_sets: set_offsets[0] must be 0");
    for (uint32_t i = 0; i < n_sets; ++i)
        if (set_offsets[i + 1] < set_offsets[i]) return fail(IMS_E_INVALID_ARG, "ims_simulate_sets: set_offsets decrease at %u", i);
    if (set_offsets[n_sets] > 0 && !set_nodes) return fail(IMS_E_INVALID_ARG, "ims_simulate_sets: set_nodes is NULL");
    const uint32_t W = (n_trials + 63) / 64;
    if ((uint64_t)n_sets * W >= 0xFFFFFFFFull) return fail(IMS_E_UNSUPPORTED, "ims_simulate_sets: too many (set, word) tasks");
    hipStream_t s = (hipStream_t)stream;
    int rc = device_cus(g);
    if (rc) return rc;
    // set semantics per set: sort, drop duplicates, check the range
    std::vector<uint32_t> off(1, 0), nodes;
    nodes.reserve(set_offsets[n_sets]);
    for (uint32_t i = 0; i < n_sets; ++i) {
        const size_t b = nodes.size();
        for (uint32_t k = set_offsets[i]; k < set_offsets[i + 1]; ++k) {
            if ((int64_t)set_nodes[k] >= g->n) return fail(IMS_E_SEED_RANGE, "set %u: node %u >= n = %lld", i, set_nodes[k], (long long)g->n);
            nodes.push_back(set_nodes[k]);
        }
        std::sort(nodes.begin() + b, nodes.end());
        nodes.erase(std::unique(nodes.begin() + b, nodes.end()), nodes.end());
        off.push_back((uint32_t)nodes.size());
    }
    const uint64_t n = (uint64_t)g->n;
    const uint64_t tasks = (uint64_t)n_sets * W;
    const int per_cu = opts && opts->blocks_per_cu > 0 ? opts->blocks_per_cu : 2;
    const uint64_t slots = std::min<uint64_t>(tasks, (uint64_t)g->cus * per_cu);
    const uint64_t cells = slots * n;
    const uint64_t before = g->sA.bytes + g->sN.bytes + g->sstamp.bytes + g->ssteps.bytes;
    if ((rc = ensure_buf(g, g->sA, cells * 8, false))) return rc;
    if ((rc = ensure_buf(g, g->sact, cells * 4, false))) return rc;
    if ((rc = ensure_buf(g, g->sQ[0], cells * 4, false))) return rc;
    if ((rc = ensure_buf(g, g->sQ[1], cells * 4, false))) return rc;
    if (g->model == IMS_MODEL_IC) {
        if ((rc = ensure_buf(g, g->sN, cells * 8, false))) return rc;
        if ((rc = ensure_buf(g, g->sQ[2], cells * 16, false))) return rc;
    } else {
        if ((rc = ensure_buf(g, g->sQ[2], cells * 4, false))) return rc;
        if ((rc = ensure_buf(g, g->sstamp, cells * 4, false))) return rc;
        if ((rc = ensure_buf(g, g->ssteps, slots * 4, false))) return rc;
    }
    if (g->sA.bytes + g->sN.bytes + g->sstamp.bytes + g->ssteps.bytes != before) g->sets_zero_dirty = true;
    const uint64_t set_bytes = (off.size() + nodes.size()) * sizeof(uint32_t);
    if ((rc = ensure_buf(g, g->sets_dev, set_bytes, false))) return rc;
    uint32_t* d_off = (uint32_t*)g->sets_dev.p;
    uint32_t* d_nodes = d_off + off.size();
    if ((rc = stage_upload(g->st_setoff, d_off, off.data(), off.size() * sizeof(uint32_t), s))) return rc;
    if ((rc = stage_upload(g->st_setnodes, d_nodes, nodes.data(), nodes.size() * sizeof(uint32_t), s))) return rc;

    // slot state starts clear: fresh buffers are cleared once, and every task
    // clears what it touched (the rows of the nodes it activated, its next-
    // step masks; stamps only grow)
    if (g->sets_zero_dirty) {
        for (ims_graph::Buf* b : {&g->sA, &g->sN, &g->sstamp, &g->ssteps})
            if (b->p && (rc = fill_async<uint8_t>((uint8_t*)b->p, b->bytes, 0, s))) return rc;
        g->sets_zero_dirty = false;
    }
    if (!g->h_flag) IMS_HIP(hipHostMalloc((void**)&g->h_flag, 4 * sizeof(uint32_t), hipHostMallocDefault));
    if ((rc = fill_async<uint32_t>(g->d_status, 4, 0u, s))) return rc;
    if ((rc = fill_async<unsigned long long>((unsigned long long*)totals, n_sets, 0ull, s))) return rc;
    if (node_counts && (rc = fill_async<uint32_t>(node_counts, (uint64_t)n_sets * n, 0u, s))) return rc;

    imsim::SimParams P;
    std::memset(&P, 0, sizeof P);
    P.n = g->n;
    P.T = n_trials;
    P.W = W;
    P.seed = rng_seed;
    P.off = g->d_off;
    P.idx = g->d_idx;
    P.thr = g->d_thr;
    P.in_off = g->d_in_off;
    P.in_arc = g->d_in_arc;
    P.in_src32 = g->d_in_src32;
    P.node_w = g->d_node_w;
    P.lt_uniform = g->lt_uniform ? 1 : 0;
    if ((rc = set_ic_direction(P, g, opts ? opts->ic_alpha : 0.0, opts ? opts->ic_beta : 0.0, opts ? opts->ic_direction : 0,
                               kIcAlphaWordLocal)))
        return rc;
    P.A = (uint64_t*)g->sA.p;
    P.N[0] = (uint64_t*)g->sN.p;
    for (int i = 0; i < 3; ++i) P.Q[i] = (uint64_t*)g->sQ[i].p;
    P.set_off = d_off;
    P.set_nodes = d_nodes;
    P.n_sets = n_sets;
    P.totals = totals;
    P.base = base;
    P.set_node_counts = node_counts;
    P.act = (uint32_t*)g->sact.p;
    P.sstamp = (uint32_t*)g->sstamp.p;
    P.slot_steps = (uint32_t*)g->ssteps.p;
    P.task_counter = g->d_status + 2;
    P.status = g->d_status;
    P.cap = g->cap;
    if (g->model == IMS_MODEL_IC)
        hipLaunchKernelGGL((imsim::word_kernel<true, false>), dim3((uint32_t)slots), dim3(imsim::kTaskBlock), 0, s, P, n);
    else
        hipLaunchKernelGGL((imsim::word_kernel<true, true>), dim3((uint32_t)slots), dim3(imsim::kTaskBlock), 0, s, P, n);
    IMS_HIP(hipGetLastError());
    return IMS_OK;
}

}  // namespace

extern "C" {

int ims_simulate_sets(ims_graph* g, const uint32_t* set_offsets, const uint32_t* set_nodes, uint32_t n_sets, uint32_t n_trials,
                      uint64_t rng_seed, const ims_opts* opts, uint64_t* totals, uint32_t* node_counts, void* stream)
{
    return simulate_sets_impl(g, nullptr, set_offsets, set_nodes, n_sets, n_trials, rng_seed, opts, totals, node_counts, stream);
}

int ims_simulate_sets_from(ims_graph* g, const uint64_t* base_bits, const uint32_t* set_offsets, const uint32_t* set_nodes,
                           uint32_t n_sets, uint32_t n_trials, uint64_t rng_seed, const ims_opts* opts, uint64_t* totals,
                           uint32_t* node_counts, void* stream)
{
    if (!base_bits) return fail(IMS_E_INVALID_ARG, "ims_simulate_sets_from: base_bits is NULL");
    return simulate_sets_impl(g, base_bits, set_offsets, set_nodes, n_sets, n_trials, rng_seed, opts, totals, node_counts, stream);
}

}  // extern "C"

struct ims_batch {
    std::vector<ims_batch_item> items;
    std::vector<imsim::BatchItem> host_items;
    std::vector<uint32_t*> dev_seeds;
    std::vector<double> cost;
    ims_tuning tuning{2, 0, 8, 0.0, 0.0};  // 8 trials per task: measured 3-5% faster than 16 on the 64-item batch
    int device = 0, cus = 0;
    uint64_t max_n = 1;
    uint32_t n_tasks = 0;
    imsim::BatchItem* d_items = nullptr;
    uint64_t* d_tasks = nullptr;
    uint32_t* d_ctl = nullptr;  // [0] task counter, [1..4] status words (steps, guard, -, refused hand-overs)
    uint64_t* d_times = nullptr;  // per task (start, end, slot) when task timing is on (ims_batch_task_timing)
    bool timing = false;
    ims_graph::Buf sA, sN, sQ0, sQ1, sQ2, sact, sstamp, ssteps, srem;
    bool any_lt = false;
    uint32_t slots = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t capture_stream = nullptr;  // the null stream cannot be captured

    void drop_graph()
    {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        exec = nullptr;
        graph = nullptr;
    }
    ~ims_batch()
    {
        drop_graph();
        if (capture_stream) (void)hipStreamDestroy(capture_stream);
        for (auto* p : dev_seeds) dev_free(p);
        dev_free(d_items);
        dev_free(d_tasks);
        dev_free(d_ctl);
        dev_free(d_times);
        for (ims_graph::Buf* b : {&sA, &sN, &sQ0, &sQ1, &sQ2, &sact, &sstamp, &ssteps, &srem}) ims_graph::release(*b);
    }
};

namespace {

// Grow a batch buffer; fresh buffers are zero-filled (slot rows, next-step
// masks and stamps must start clear; tasks leave them clear).
int batch_buf(ims_graph::Buf& b, uint64_t bytes)
{
    if (b.p && b.bytes >= bytes) return IMS_OK;
    ims_graph::release(b);
    uint8_t* p = nullptr;
    int rc = dev_alloc(&p, std::max<uint64_t>(bytes, 8));
    if (rc) return rc;
    b.p = p;
    b.bytes = std::max<uint64_t>(bytes, 8);
    IMS_HIP(hipMemset(p, 0, b.bytes));
    return IMS_OK;
}

// Task list and slot state for the current tuning.
int batch_plan(ims_batch* b)
{
    const uint32_t n_items = (uint32_t)b->items.size();
    std::vector<uint32_t> order(n_items);
    for (uint32_t i = 0; i < n_items; ++i) order[i] = i;
    if (b->tuning.order == 0)
        std::stable_sort(order.begin(), order.end(), [&](uint32_t x, uint32_t y) { return b->cost[x] > b->cost[y]; });
    // each word of an item as 2^s tasks of 64 / 2^s trials (s from the
    // tuning's split); parts wholly past the item's last trial are left out
    uint32_t s = 0;
    while (s < 6 && (2u << s) <= (uint32_t)std::max(b->tuning.split, 1)) ++s;
    const uint32_t width = 64u >> s;
    std::vector<uint64_t> tasks;
    for (uint32_t i : order) {
        const uint32_t T = b->host_items[i].P.T;
        for (uint32_t w = 0; w < b->host_items[i].P.W; ++w)
            for (uint32_t part = 0; part < (1u << s); ++part)
                if ((uint64_t)w * 64 + (uint64_t)part * width < T)
                    tasks.push_back(((uint64_t)i << 32) | ((uint64_t)s << 24) | ((uint64_t)part << 16) | w);
    }
    if (tasks.size() >= 0xFFFFFFFFull) return fail(IMS_E_UNSUPPORTED, "ims_batch: more than 2^32 - 2 tasks");
    int rc0;
    // the tuning's IC switch points go into every item
    for (uint32_t i = 0; i < n_items; ++i) {
        int rc = set_ic_direction(b->host_items[i].P, b->items[i].graph, b->tuning.ic_alpha, b->tuning.ic_beta, 0);
        if (rc) return rc;
    }
    if (n_items > 0)
        IMS_HIP(hipMemcpy(b->d_items, b->host_items.data(), n_items * sizeof(imsim::BatchItem), hipMemcpyHostToDevice));
    b->n_tasks = (uint32_t)tasks.size();
    dev_free(b->d_times);
    if (b->timing && (rc0 = dev_alloc(&b->d_times, 3ull * std::max<uint32_t>(b->n_tasks, 1)))) return rc0;
    dev_free(b->d_tasks);
    int rc = dev_alloc(&b->d_tasks, tasks.size());
    if (rc) return rc;
    if (!tasks.empty()) IMS_HIP(hipMemcpy(b->d_tasks, tasks.data(), tasks.size() * sizeof(uint64_t), hipMemcpyHostToDevice));
    const int per_cu = std::min(std::max(b->tuning.blocks_per_cu, 1), 16);
    b->slots = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(b->n_tasks, (uint64_t)b->cus * per_cu));
    const uint64_t cells = (uint64_t)b->slots * b->max_n;
    if ((rc = batch_buf(b->sA, cells * 8)) || (rc = batch_buf(b->sN, cells * 8)) || (rc = batch_buf(b->sQ0, cells * 4)) ||
        (rc = batch_buf(b->sQ1, cells * 4)) || (rc = batch_buf(b->sQ2, cells * 16)) || (rc = batch_buf(b->sact, cells * 4)) ||
        (rc = batch_buf(b->sstamp, cells * 4)) || (rc = batch_buf(b->ssteps, (uint64_t)b->slots * 4)))
        return rc;
    // LT items split into tasks of at most 16 trials run in push form: 16
    // threshold remainders per node and slot
    if (b->any_lt && b->tuning.split >= 4 && (rc = batch_buf(b->srem, cells * 8 * imsim::kRemWords))) return rc;
    b->drop_graph();
    return IMS_OK;
}

// Enqueue one batch run: clear outputs and the task counter (fill kernels, no
// memset nodes, so the sequence can be captured), then the persistent launch.
int batch_enqueue(ims_batch* b, hipStream_t s)
{
    int rc;
    for (const auto& it : b->items) {
        if ((rc = fill_async<uint32_t>(it.trial_counts, it.n_trials, 0u, s))) return rc;
        if (it.node_counts) {
            int64_t n = 0;
            ims_graph_info(it.graph, &n, nullptr, nullptr);
            if ((rc = fill_async<uint32_t>(it.node_counts, (uint64_t)n, 0u, s))) return rc;
        }
        if ((rc = fill_async<unsigned long long>((unsigned long long*)it.total, 1, 0ull, s))) return rc;
    }
    if ((rc = fill_async<uint32_t>(b->d_ctl, 8, 0u, s))) return rc;
    imsim::SlotBufs S{b->max_n,
                      (uint64_t*)b->sA.p,
                      (uint64_t*)b->sN.p,
                      (uint32_t*)b->sQ0.p,
                      (uint32_t*)b->sQ1.p,
                      (uint64_t*)b->sQ2.p,
                      (uint32_t*)b->sact.p,
                      (uint32_t*)b->sstamp.p,
                      (uint32_t*)b->ssteps.p,
                      b->tuning.split >= 4 ? (uint64_t*)b->srem.p : nullptr};
    hipLaunchKernelGGL(imsim::batch_kernel, dim3(b->slots), dim3(imsim::kTaskBlock), 0, s, (const imsim::BatchItem*)b->d_items,
                       (const uint64_t*)b->d_tasks, b->n_tasks, b->d_ctl, S, b->d_ctl + 1, b->timing ? b->d_times : nullptr);
    IMS_HIP(hipGetLastError());
    return IMS_OK;
}

}  // namespace

extern "C" {

int ims_batch_create(const ims_batch_item* items, uint32_t n_items, const ims_tuning* tuning, ims_batch** out)
{
    if (!out || (n_items > 0 && !items)) return fail(IMS_E_INVALID_ARG, "ims_batch_create: bad arguments");
    *out = nullptr;
    if (n_items >= (1u << 20)) return fail(IMS_E_UNSUPPORTED, "ims_batch_create: at most 2^20 - 1 items");
    auto* b = new (std::nothrow) ims_batch();
    if (!b) return fail(IMS_E_OOM, "host allocation failed");
    auto bail = [&](int code) {
        delete b;
        return code;
    };
    (void)hipGetDevice(&b->device);
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, b->device) != hipSuccess) return bail(fail(IMS_E_HIP, "hipGetDeviceProperties failed"));
    b->cus = prop.multiProcessorCount;
    if (tuning) b->tuning = *tuning;
    for (uint32_t i = 0; i < n_items; ++i) {
        const ims_batch_item& it = items[i];
        if (!it.graph || !it.trial_counts || !it.total || it.n_trials == 0 || (it.n_seeds > 0 && !it.seeds))
            return bail(fail(IMS_E_INVALID_ARG, "ims_batch_create: item %u incomplete", i));
        if (it.n_trials > imsim::kMaxWords * 64u) return bail(fail(IMS_E_UNSUPPORTED, "item %u: n_trials above %u", i, imsim::kMaxWords * 64u));
        ims_graph* g = it.graph;
        std::vector<uint32_t> sv(it.seeds, it.seeds + it.n_seeds);
        for (uint32_t x : sv)
            if ((int64_t)x >= g->n) return bail(fail(IMS_E_SEED_RANGE, "item %u: seed %u >= n", i, x));
        std::sort(sv.begin(), sv.end());
        sv.erase(std::unique(sv.begin(), sv.end()), sv.end());
        uint32_t* d = nullptr;
        int rc = dev_alloc(&d, sv.size());
        if (rc) return bail(rc);
        b->dev_seeds.push_back(d);
        if (!sv.empty() && hipMemcpy(d, sv.data(), sv.size() * 4, hipMemcpyHostToDevice) != hipSuccess)
            return bail(fail(IMS_E_HIP, "seed upload failed"));
        imsim::BatchItem bi;
        std::memset(&bi, 0, sizeof bi);
        imsim::SimParams& P = bi.P;
        P.n = g->n;
        P.T = it.n_trials;
        P.W = (it.n_trials + 63) / 64;
        P.seed = it.rng_seed;
        P.off = g->d_off;
        P.idx = g->d_idx;
        P.thr = g->d_thr;
        P.in_off = g->d_in_off;
        P.in_arc = g->d_in_arc;
        P.in_src32 = g->d_in_src32;
        P.node_w = g->d_node_w;
        P.lt_uniform = g->lt_uniform ? 1 : 0;
        P.lt_wout = g->d_lt_wout;
        if ((rc = set_ic_direction(P, g, b->tuning.ic_alpha, b->tuning.ic_beta, 0))) return bail(rc);
        P.seeds = d;
        P.n_seeds = (uint32_t)sv.size();
        P.cap = g->cap;
        bi.model = g->model;
        if (g->model == IMS_MODEL_LT) b->any_lt = true;
        bi.trial_counts = it.trial_counts;
        bi.node_counts = it.node_counts;
        bi.total = it.total;
        b->host_items.push_back(bi);
        b->items.push_back(it);
        b->cost.push_back((double)P.W * (double)(g->m + g->n));
        b->max_n = std::max<uint64_t>(b->max_n, (uint64_t)g->n);
    }
    int rc = dev_alloc(&b->d_items, std::max<size_t>(b->host_items.size(), 1));
    if (rc) return bail(rc);
    if (!b->host_items.empty() &&
        hipMemcpy(b->d_items, b->host_items.data(), b->host_items.size() * sizeof(imsim::BatchItem), hipMemcpyHostToDevice) != hipSuccess)
        return bail(fail(IMS_E_HIP, "item upload failed"));
    if ((rc = dev_alloc(&b->d_ctl, 8))) return bail(rc);
    if ((rc = batch_plan(b))) return bail(rc);
    *out = b;
    return IMS_OK;
}

int ims_batch_launch(ims_batch* b, void* stream)
{
    if (!b) return fail(IMS_E_INVALID_ARG, "ims_batch_launch: NULL batch");
    hipStream_t s = (hipStream_t)stream;
    if (!b->exec) {
        // record the launch sequence on a private stream (default priority);
        // the instantiated graph then runs on the caller's stream
        if (!b->capture_stream) IMS_HIP(hipStreamCreateWithFlags(&b->capture_stream, hipStreamNonBlocking));
        hipStream_t cs = b->capture_stream;
        IMS_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
        int rc = batch_enqueue(b, cs);
        hipGraph_t gph = nullptr;
        hipError_t e = hipStreamEndCapture(cs, &gph);
        if (rc) {
            if (gph) (void)hipGraphDestroy(gph);
            return rc;
        }
        if (e != hipSuccess) return fail(IMS_E_HIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
        b->graph = gph;
        IMS_HIP(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    }
    IMS_HIP(hipGraphLaunch(b->exec, s));
    return IMS_OK;
}

int ims_batch_autotune(ims_batch* b, int repeats, void* stream, ims_tuning* chosen)
{
    if (!b || repeats < 1) return fail(IMS_E_INVALID_ARG, "ims_batch_autotune: bad arguments");
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t e0, e1;
    IMS_HIP(hipEventCreate(&e0));
    IMS_HIP(hipEventCreate(&e1));
    double best_ms = 1e300;
    ims_tuning best = b->tuning;
    // every output of every item, read back after each candidate
    std::vector<uint8_t> ref, cur;
    auto read_outputs = [&](std::vector<uint8_t>& out) -> int {
        out.clear();
        for (const auto& it : b->items) {
            int64_t n = 0;
            ims_graph_info(it.graph, &n, nullptr, nullptr);
            const size_t at = out.size();
            const size_t tc = (size_t)it.n_trials * 4, nc = it.node_counts ? (size_t)n * 4 : 0;
            out.resize(at + 8 + tc + nc);
            IMS_HIP(hipMemcpy(out.data() + at, it.total, 8, hipMemcpyDeviceToHost));
            IMS_HIP(hipMemcpy(out.data() + at + 8, it.trial_counts, tc, hipMemcpyDeviceToHost));
            if (nc) IMS_HIP(hipMemcpy(out.data() + at + 8 + tc, it.node_counts, nc, hipMemcpyDeviceToHost));
        }
        return IMS_OK;
    };
    int rc = IMS_OK;
    auto trial = [&](const ims_tuning& c) -> int {
        b->tuning = c;
        int r;
        if ((r = batch_plan(b))) return r;
        if ((r = batch_enqueue(b, s))) return r;  // warm-up
        IMS_HIP(hipEventRecord(e0, s));
        for (int k = 0; k < repeats; ++k)
            if ((r = batch_enqueue(b, s))) return r;
        IMS_HIP(hipEventRecord(e1, s));
        IMS_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        IMS_HIP(hipEventElapsedTime(&ms, e0, e1));
        if ((r = read_outputs(ref.empty() ? ref : cur))) return r;
        if (!cur.empty() && cur != ref)
            return fail(IMS_E_HIP, "ims_batch_autotune: schedule {%d,%d,%d,%g,%g} changed the results", c.blocks_per_cu, c.order,
                        c.split, c.ic_alpha, c.ic_beta);
        if (ms / repeats < best_ms) {
            best_ms = ms / repeats;
            best = c;
        }
        return IMS_OK;
    };
    // stage 1: launch shape and task size at the default switch points
    const ims_tuning shapes[] = {{2, 0, 2, 0, 0}, {2, 0, 4, 0, 0}, {4, 0, 4, 0, 0}, {2, 1, 4, 0, 0},
                                 {2, 0, 8, 0, 0}, {4, 0, 8, 0, 0}, {2, 0, 16, 0, 0}};
    for (const ims_tuning& c : shapes)
        if ((rc = trial(c))) break;
    // stage 2: IC switch points for the best shape (1e-9: push only)
    if (!rc) {
        const ims_tuning base = best;
        const double alphas[] = {1e-9, 2.0, 50.0, 400.0};
        for (double a : alphas) {
            ims_tuning c = base;
            c.ic_alpha = a;
            if ((rc = trial(c))) break;
        }
        if (!rc) {
            ims_tuning c = best;
            c.ic_beta = 4.0;
            rc = trial(c);
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    b->tuning = best;
    if ((rc = batch_plan(b))) return rc;
    if (chosen) *chosen = best;
    return IMS_OK;
}

int ims_batch_task_timing(ims_batch* b, int enable)
{
    if (!b) return fail(IMS_E_INVALID_ARG, "ims_batch_task_timing: NULL batch");
    if ((enable != 0) == b->timing) return IMS_OK;
    b->timing = enable != 0;
    return batch_plan(b);  // (re)allocates the record and drops the captured graph
}

int ims_batch_task_times(ims_batch* b, uint32_t max_tasks, uint64_t* tasks, uint64_t* times, uint32_t* count, void* stream)
{
    if (!b || !count || (max_tasks > 0 && (!tasks || !times))) return fail(IMS_E_INVALID_ARG, "ims_batch_task_times: bad arguments");
    *count = 0;
    if (!b->timing || !b->d_times) return fail(IMS_E_INVALID_ARG, "ims_batch_task_times: task timing is off");
    const uint32_t k = std::min<uint32_t>(max_tasks, b->n_tasks);
    IMS_HIP(hipStreamSynchronize((hipStream_t)stream));
    if (k > 0) {
        IMS_HIP(hipMemcpy(tasks, b->d_tasks, k * sizeof(uint64_t), hipMemcpyDeviceToHost));
        IMS_HIP(hipMemcpy(times, b->d_times, 3ull * k * sizeof(uint64_t), hipMemcpyDeviceToHost));
    }
    *count = k;
    return IMS_OK;
}

int ims_batch_destroy(ims_batch* b)
{
    if (b) {
        (void)hipDeviceSynchronize();
        delete b;
    }
    return IMS_OK;
}

int ims_graph_last_status(ims_graph* g, void* stream, uint32_t out[2])
{
    if (!g || !out) return fail(IMS_E_INVALID_ARG, "ims_graph_last_status: bad arguments");
    IMS_HIP(hipMemcpyAsync(out, g->d_status, 2 * sizeof(uint32_t), hipMemcpyDeviceToHost, (hipStream_t)stream));
    IMS_HIP(hipStreamSynchronize((hipStream_t)stream));
    if (out[1]) g->zero_dirty = true;
    return IMS_OK;
}

int ims_graph_last_counters(ims_graph* g, void* stream, uint32_t out[4])
{
    if (!g || !out) return fail(IMS_E_INVALID_ARG, "ims_graph_last_counters: bad arguments");
    IMS_HIP(hipMemcpyAsync(out, g->d_status, 4 * sizeof(uint32_t), hipMemcpyDeviceToHost, (hipStream_t)stream));
    IMS_HIP(hipStreamSynchronize((hipStream_t)stream));
    if (out[1]) g->zero_dirty = true;
    return IMS_OK;
}

int ims_graph_level_directions(ims_graph* g, uint32_t max_levels, uint32_t* dirs, uint32_t* count, void* stream)
{
    if (!g || !count || (max_levels > 0 && !dirs)) return fail(IMS_E_INVALID_ARG, "ims_graph_level_directions: bad arguments");
    *count = 0;
    IMS_HIP(hipStreamSynchronize((hipStream_t)stream));
    int rc = take_grid_status(g);
    if (rc) return rc;
    if (g->model != IMS_MODEL_IC || g->last_shape != 2) return IMS_OK;
    const uint32_t k = std::min<uint32_t>(max_levels, std::min<uint32_t>(g->last_steps, g->cap));
    if (k > 0) {
        IMS_HIP(hipMemcpyAsync(dirs, g->d_lvl_dir, k * sizeof(uint32_t), hipMemcpyDeviceToHost, (hipStream_t)stream));
        IMS_HIP(hipStreamSynchronize((hipStream_t)stream));
    }
    *count = k;
    return IMS_OK;
}

int ims_graph_profile(ims_graph* g, int reset, double* total_ms, uint32_t* count)
{
    if (!g || !total_ms || !count) return fail(IMS_E_INVALID_ARG, "ims_graph_profile: bad arguments");
    double sum = 0.0;
    for (uint32_t i = 0; i < g->prof_count; ++i) {
        IMS_HIP(hipEventSynchronize(g->prof_ev[2 * i + 1]));
        float ms = 0.f;
        IMS_HIP(hipEventElapsedTime(&ms, g->prof_ev[2 * i], g->prof_ev[2 * i + 1]));
        sum += ms;
    }
    *total_ms = sum;
    *count = g->prof_count;
    if (reset) g->prof_count = 0;
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

// ============================================ allocation-free single run
//
// ims_simulate_noalloc runs the count-only word-local form of ims_simulate
// (slot_run_kernel: each 64-trial word as four 16-trial tasks on persistent
// workgroup slots) with every per-call device buffer carved out of one fixed
// device array, `scratch`, instead of the graph's growing workspace.  The
// graph handle (created beforehand) and the caller's outputs are the only
// other device memory it touches; it calls no allocator.

namespace {

constexpr uint64_t kNoAllocBytes = (uint64_t)IMS_NOALLOC_SCRATCH_BYTES;
constexpr uint32_t kSeedChunk = 512;  // seeds carried by one upload launch's arguments
constexpr int kMaxDevices = 64;

}  // namespace

// One copy per GPU, resident from the library's load on that GPU until the
// process ends.  Host code never names it except to ask for its address.
static __device__ __align__(256) uint8_t scratch[IMS_NOALLOC_SCRATCH_BYTES];

namespace {

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on device `dev` (current), looked up once per
// device; the array's host-side name is not a device address.
int scratch_address(int dev, uint8_t** out)
{
    if (dev < 0 || dev >= kMaxDevices) return fail(IMS_E_UNSUPPORTED, "ims_simulate_noalloc: device %d above %d", dev, kMaxDevices - 1);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return fail(IMS_E_HIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
        }
        g_scratch_ptr[dev] = p;
    }
    *out = (uint8_t*)g_scratch_ptr[dev];
    return IMS_OK;
}

struct SeedChunk {
    uint32_t first;
    uint32_t count;
    uint32_t v[kSeedChunk];
};

// Seeds reach the device through kernel arguments (copied at launch), so the
// caller's host array is read only during the call, whatever memory it is.
__global__ __launch_bounds__(kSeedChunk) void noalloc_put_seeds_kernel(SeedChunk c, uint32_t* __restrict__ raw)
{
    if (threadIdx.x < c.count) raw[c.first + threadIdx.x] = c.v[threadIdx.x];
}

__global__ __launch_bounds__(64) void noalloc_put_item_kernel(imsim::BatchItem it, imsim::BatchItem* __restrict__ dst)
{
    if (threadIdx.x == 0) *dst = it;
}

// Set semantics on the device: the first position of every seed id wins
// (mark[] starts at 0xFFFFFFFF) ...
__global__ __launch_bounds__(imsim::kBlock) void noalloc_seed_first_kernel(const uint32_t* __restrict__ raw, uint32_t count,
                                                                          uint32_t* __restrict__ mark)
{
    for (uint32_t i = blockIdx.x * imsim::kBlock + threadIdx.x; i < count; i += gridDim.x * imsim::kBlock) atomicMin(&mark[raw[i]], i);
}

// ... and only winners are listed; their count lands in the item's n_seeds
// (the list order does not matter: every trial's final set is fixed).
__global__ __launch_bounds__(imsim::kBlock) void noalloc_seed_list_kernel(const uint32_t* __restrict__ raw, uint32_t count,
                                                                         const uint32_t* __restrict__ mark, uint32_t* __restrict__ seeds,
                                                                         uint32_t* __restrict__ n_out)
{
    for (uint32_t i = blockIdx.x * imsim::kBlock + threadIdx.x; i < count; i += gridDim.x * imsim::kBlock) {
        const uint32_t v = raw[i];
        if (mark[v] == i) seeds[atomicAdd(n_out, 1u)] = v;
    }
}

uint64_t align256(uint64_t x) { return (x + 255) & ~255ull; }

// Byte layout of `scratch` for one call.
struct NoAllocLayout {
    uint64_t item, counter, raw, seeds, mark, steps, sA, sN, sstamp, zero_end, sQ0, sQ1, sQ2, sact, end;
};

NoAllocLayout noalloc_layout(uint64_t n, uint64_t n_seeds, uint64_t slots)
{
    NoAllocLayout L;
    L.item = 0;
    L.counter = align256(sizeof(imsim::BatchItem));
    L.raw = L.counter + 256;
    L.seeds = L.raw + align256(4 * n_seeds);
    L.mark = L.seeds + align256(4 * n_seeds);
    L.steps = L.mark + align256(4 * n);
    // slot step counters, active rows, next-step masks and stamps must start
    // at zero: they are laid out together and cleared as one range
    L.sA = L.steps + align256(4 * slots);
    L.sN = L.sA + align256(8 * slots * n);
    L.sstamp = L.sN + align256(8 * slots * n);
    L.zero_end = L.sstamp + align256(4 * slots * n);
    L.sQ0 = L.zero_end;
    L.sQ1 = L.sQ0 + align256(4 * slots * n);
    L.sQ2 = L.sQ1 + align256(4 * slots * n);
    L.sact = L.sQ2 + align256(16 * slots * n);
    L.end = L.sact + align256(4 * slots * n);
    return L;
}

}  // namespace

extern "C" {

int ims_simulate_noalloc(ims_graph* g, const uint32_t* seeds, uint32_t n_seeds, uint32_t n_trials, uint64_t rng_seed,
                         uint32_t* trial_counts, uint32_t* node_counts, uint64_t* total, void* stream)
{
    if (!g) return fail(IMS_E_INVALID_ARG, "ims_simulate_noalloc: NULL graph");
    if (n_trials == 0) return fail(IMS_E_INVALID_ARG, "ims_simulate_noalloc: n_trials must be >= 1");
    if (n_trials > imsim::kMaxWords * 64u)
        return fail(IMS_E_UNSUPPORTED, "ims_simulate_noalloc: n_trials above %u", imsim::kMaxWords * 64u);
    if (!trial_counts || !total) return fail(IMS_E_INVALID_ARG, "ims_simulate_noalloc: trial_counts and total are required");
    if (n_seeds > 0 && !seeds) return fail(IMS_E_INVALID_ARG, "ims_simulate_noalloc: seeds is NULL");
    for (uint32_t i = 0; i < n_seeds; ++i)
        if ((int64_t)seeds[i] >= g->n) return fail(IMS_E_SEED_RANGE, "seed %u >= n = %lld", seeds[i], (long long)g->n);
    int dev = -1;
    IMS_HIP(hipGetDevice(&dev));
    if (dev != g->device) return fail(IMS_E_INVALID_ARG, "ims_simulate_noalloc: current device %d, graph on device %d", dev, g->device);
    int rc = device_cus(g);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    const uint64_t n = (uint64_t)g->n;
    const uint32_t W = (n_trials + 63) / 64;
    const uint32_t sp = 2;  // four 16-trial tasks per word, as the counts-only form of ims_simulate
    const uint64_t tasks = (uint64_t)W << sp;
    // as many slots as fit, up to two workgroups per compute unit
    uint64_t slots = std::min<uint64_t>(tasks, (uint64_t)g->cus * 2);
    while (slots > 0 && noalloc_layout(n, n_seeds, slots).end > kNoAllocBytes) slots = slots > 8 ? slots - slots / 8 : slots - 1;
    if (slots == 0)
        return fail(IMS_E_UNSUPPORTED,
                    "ims_simulate_noalloc: %lld nodes and %u seeds need %llu bytes of scratch for one workgroup slot, above the "
                    "fixed %llu (about 48 bytes per node plus 8 per seed)",
                    (long long)g->n, n_seeds, (unsigned long long)noalloc_layout(n, n_seeds, 1).end,
                    (unsigned long long)kNoAllocBytes);
    const NoAllocLayout L = noalloc_layout(n, n_seeds, slots);
    uint8_t* base = nullptr;
    if ((rc = scratch_address(dev, &base))) return rc;

    // clear what must start at zero (fill kernels, no memset nodes)
    if ((rc = fill_async<uint64_t>((uint64_t*)(base + L.counter), 256 / 8, 0ull, s))) return rc;
    if ((rc = fill_async<uint32_t>((uint32_t*)(base + L.mark), n, 0xFFFFFFFFu, s))) return rc;
    if ((rc = fill_async<uint64_t>((uint64_t*)(base + L.steps), (L.zero_end - L.steps) / 8, 0ull, s))) return rc;
    if ((rc = fill_async<uint32_t>(g->d_status, 4, 0u, s))) return rc;
    if ((rc = fill_async<uint32_t>(trial_counts, n_trials, 0u, s))) return rc;
    if ((rc = fill_async<unsigned long long>((unsigned long long*)total, 1, 0ull, s))) return rc;
    if (node_counts && (rc = fill_async<uint32_t>(node_counts, n, 0u, s))) return rc;

    // the item: graph, run parameters and outputs; n_seeds is counted below
    imsim::BatchItem it;
    std::memset(&it, 0, sizeof it);
    imsim::SimParams& P = it.P;
    P.n = g->n;
    P.T = n_trials;
    P.W = W;
    P.seed = rng_seed;
    P.off = g->d_off;
    P.idx = g->d_idx;
    P.thr = g->d_thr;
    P.in_off = g->d_in_off;
    P.in_arc = g->d_in_arc;
    P.in_src32 = g->d_in_src32;
    P.node_w = g->d_node_w;
    P.lt_uniform = g->lt_uniform ? 1 : 0;
    if ((rc = set_ic_direction(P, g, 0.0, 0.0, 0, kIcAlphaWordLocal))) return rc;
    P.seeds = (const uint32_t*)(base + L.seeds);
    P.n_seeds = 0;
    P.cap = g->cap;
    it.model = g->model;
    it.trial_counts = trial_counts;
    it.node_counts = node_counts;
    it.total = total;
    imsim::BatchItem* d_item = (imsim::BatchItem*)(base + L.item);
    hipLaunchKernelGGL(noalloc_put_item_kernel, dim3(1), dim3(64), 0, s, it, d_item);
    IMS_HIP(hipGetLastError());

    uint32_t* raw = (uint32_t*)(base + L.raw);
    for (uint32_t first = 0; first < n_seeds; first += kSeedChunk) {
        SeedChunk c;
        c.first = first;
        c.count = std::min<uint32_t>(kSeedChunk, n_seeds - first);
        std::memcpy(c.v, seeds + first, c.count * sizeof(uint32_t));
        hipLaunchKernelGGL(noalloc_put_seeds_kernel, dim3(1), dim3(kSeedChunk), 0, s, c, raw);
        IMS_HIP(hipGetLastError());
    }
    if (n_seeds > 0) {
        const uint32_t blocks = std::min<uint32_t>((n_seeds + imsim::kBlock - 1) / imsim::kBlock, 1024);
        uint32_t* mark = (uint32_t*)(base + L.mark);
        hipLaunchKernelGGL(noalloc_seed_first_kernel, dim3(blocks), dim3(imsim::kBlock), 0, s, (const uint32_t*)raw, n_seeds, mark);
        hipLaunchKernelGGL(noalloc_seed_list_kernel, dim3(blocks), dim3(imsim::kBlock), 0, s, (const uint32_t*)raw, n_seeds,
                           (const uint32_t*)mark, (uint32_t*)(base + L.seeds), &d_item->P.n_seeds);
        IMS_HIP(hipGetLastError());
    }

    imsim::SlotBufs S{n,
                      (uint64_t*)(base + L.sA),
                      (uint64_t*)(base + L.sN),
                      (uint32_t*)(base + L.sQ0),
                      (uint32_t*)(base + L.sQ1),
                      (uint64_t*)(base + L.sQ2),
                      (uint32_t*)(base + L.sact),
                      (uint32_t*)(base + L.sstamp),
                      (uint32_t*)(base + L.steps)};
    if (g->model == IMS_MODEL_IC)
        hipLaunchKernelGGL((imsim::slot_run_kernel<0, false>), dim3((uint32_t)slots), dim3(imsim::kTaskBlock), 0, s,
                           (const imsim::BatchItem*)d_item, sp, (uint32_t)tasks, (uint32_t*)(base + L.counter), S, g->d_status);
    else
        hipLaunchKernelGGL((imsim::slot_run_kernel<1, false>), dim3((uint32_t)slots), dim3(imsim::kTaskBlock), 0, s,
                           (const imsim::BatchItem*)d_item, sp, (uint32_t)tasks, (uint32_t*)(base + L.counter), S, g->d_status);
    IMS_HIP(hipGetLastError());
    g->last_shape = 1;
    return IMS_OK;
}

}  // extern "C"
