// Host-side graph plans of the imsim library: plain C++ (no HIP), so that the
// library uploads what these build and a sanitizer build on the CPU can
// exercise the same index arithmetic.
//
// Every array describes the graph of Section 3, "Data Structures" (out-CSR:
// the out-neighbours of u are indices[offsets[u] .. offsets[u+1]), arc id =
// position) from the other side, or in the blocks the LT grid sweep walks.
#pragma once

#include <stdint.h>

#include <algorithm>
#include <vector>

namespace imsim_plan {

constexpr uint64_t kOne = 1ull << 32;  // weight 1 in 2^-32 units

// IC pull side: for every node v its in-arcs (u, v) with a nonzero threshold,
// in out-CSR order of the arcs, each as source | out-CSR arc id << 32 with its
// threshold.  A pulled arc draws the coin of its out-CSR id, which is the coin
// its push draws.
struct IcInCsr {
    std::vector<int64_t> off;   // [n + 1]
    std::vector<uint64_t> sa;   // [mi]: source | arc id << 32
    std::vector<uint32_t> thr;  // [mi]
};

inline void build_ic_in_csr(int64_t n, int64_t m, const int64_t* offsets, const uint32_t* indices, const uint32_t* thr, IcInCsr& out)
{
    (void)m;
    out.off.assign((size_t)n + 1, 0);
    for (int64_t u = 0; u < n; ++u)
        for (int64_t e = offsets[u]; e < offsets[u + 1]; ++e)
            if (thr[e] != 0) ++out.off[(size_t)indices[e] + 1];
    for (int64_t v = 0; v < n; ++v) out.off[v + 1] += out.off[v];
    const int64_t mi = out.off[n];
    out.sa.assign((size_t)mi, 0);
    out.thr.assign((size_t)mi, 0);
    std::vector<int64_t> pos(out.off.begin(), out.off.end() - 1);
    for (int64_t u = 0; u < n; ++u)
        for (int64_t e = offsets[u]; e < offsets[u + 1]; ++e) {
            if (thr[e] == 0) continue;
            const int64_t k = pos[indices[e]]++;
            out.sa[k] = (uint64_t)u | ((uint64_t)e << 32);
            out.thr[k] = thr[e];
        }
}

// LT in-CSR (Section 2: v joins when the weight of its active in-neighbours
// exceeds its threshold).  A weight of exactly 2^32 is stored as two pieces of
// 2^31 so that every piece fits 32 bits; zero weights are dropped (they never
// add to a sum).  Per piece: source | piece << 32.
struct LtInCsr {
    std::vector<int64_t> off;   // [n + 1]
    std::vector<uint64_t> arc;  // [mi]
};

// Returns 0, or the first node (as bad_node) / arc (as bad_arc) that breaks
// the bound "in-weights sum to at most 2^32" (-1 where it does not apply):
// 1 = an arc weight above 2^32, 2 = a node's sum above 2^32.
inline int build_lt_in_csr(int64_t n, int64_t m, const int64_t* offsets, const uint32_t* indices, const uint64_t* w64, LtInCsr& out,
                           int64_t& bad_arc, int64_t& bad_node)
{
    bad_arc = bad_node = -1;
    std::vector<uint64_t> wsum((size_t)std::max<int64_t>(n, 1), 0);
    std::vector<int64_t> cnt((size_t)n + 1, 0);
    for (int64_t e = 0; e < m; ++e) {
        const uint64_t w = w64[e];
        if (w > kOne) {
            bad_arc = e;
            return 1;
        }
        const uint32_t v = indices[e];
        wsum[v] += w;
        if (wsum[v] > kOne) {
            bad_node = v;
            return 2;
        }
        cnt[v + 1] += w == 0 ? 0 : (w == kOne ? 2 : 1);
    }
    out.off.assign((size_t)n + 1, 0);
    for (int64_t v = 0; v < n; ++v) out.off[v + 1] = out.off[v] + cnt[v + 1];
    const int64_t mi = out.off[n];
    out.arc.assign((size_t)mi, 0);
    std::vector<int64_t> pos(out.off.begin(), out.off.end() - 1);
    for (int64_t u = 0; u < n; ++u)
        for (int64_t e = offsets[u]; e < offsets[u + 1]; ++e) {
            const uint64_t w = w64[e];
            if (w == 0) continue;
            const uint32_t v = indices[e];
            if (w == kOne) {
                out.arc[pos[v]++] = (uint64_t)u | ((uint64_t)(1u << 31) << 32);
                out.arc[pos[v]++] = (uint64_t)u | ((uint64_t)(1u << 31) << 32);
            } else {
                out.arc[pos[v]++] = (uint64_t)u | (w << 32);
            }
        }
    return 0;
}

// Equal in-weights form: true when every node's pieces are all equal (as for
// w = 1/indeg); then node_w[v] is that piece and src32 the sources alone.
inline bool lt_uniform_form(int64_t n, const LtInCsr& in, std::vector<uint32_t>& node_w, std::vector<uint32_t>& src32)
{
    node_w.assign((size_t)std::max<int64_t>(n, 1), 0);
    for (int64_t v = 0; v < n; ++v)
        for (int64_t k = in.off[v]; k < in.off[v + 1]; ++k) {
            const uint32_t piece = (uint32_t)(in.arc[k] >> 32);
            if (k == in.off[v]) node_w[v] = piece;
            else if (piece != node_w[v]) return false;
        }
    src32.assign(in.arc.size(), 0);
    for (size_t k = 0; k < in.arc.size(); ++k) src32[k] = (uint32_t)in.arc[k];
    return true;
}

// Count-threshold planes of the equal-weights form: node v keeps S_v bit
// planes, the fewest with 2^S_v - 1 above every count it can reach (its in-arc
// pieces; 1 plane without in-arcs; 0 above 64 pieces, where the table is not
// used).  kinfo[2v] = low half of in_off[v], kinfo[2v + 1] = planes of nodes
// before v (F(v)); entries n hold the totals.  Returns the planes of all nodes.
inline uint64_t lt_count_planes(int64_t n, const std::vector<int64_t>& in_off, std::vector<uint32_t>& kinfo)
{
    kinfo.assign(2 * ((size_t)n + 1), 0);
    uint64_t total = 0;
    for (int64_t v = 0; v <= n; ++v) {
        kinfo[2 * v] = (uint32_t)in_off[v];
        kinfo[2 * v + 1] = (uint32_t)total;
        if (v == n) break;
        const int64_t d = in_off[v + 1] - in_off[v];
        uint32_t planes = 0;
        if (d <= 64) {
            planes = 1;
            while (((1ll << planes) - 1) <= d) ++planes;
        }
        total += planes;
    }
    return total;
}

// Node batches of the LT grid sweep: at most 8 consecutive nodes whose
// in-arc pieces fit one 64-piece chunk, or one node with more.  bfirst[b] is
// the first node of batch b (bfirst[nbatch] = n); bdesc holds 4 words per
// batch (first node; node count | min(pieces, 2^24 - 1) << 8; the in-CSR
// position of its first piece, low and high half) and 4 zero words at the
// end; bigb lists the batches of more than 64 pieces.
struct LtBatches {
    std::vector<uint32_t> bfirst, bdesc, bigb;
    uint32_t nbatch = 0;
};

inline void lt_batches(int64_t n, const std::vector<int64_t>& in_off, LtBatches& out)
{
    out.bfirst.assign(1, 0);
    uint32_t bcnt = 0;
    uint64_t barcs = 0;
    for (int64_t v = 0; v < n; ++v) {
        const uint64_t d = (uint64_t)(in_off[v + 1] - in_off[v]);
        if (bcnt > 0 && (bcnt == 8 || barcs + d > 64)) {
            out.bfirst.push_back((uint32_t)v);
            bcnt = 0;
            barcs = 0;
        }
        ++bcnt;
        barcs += d;
        if (d > 64) {
            out.bfirst.push_back((uint32_t)(v + 1));
            bcnt = 0;
            barcs = 0;
        }
    }
    if (bcnt > 0) out.bfirst.push_back((uint32_t)n);
    out.nbatch = (uint32_t)(out.bfirst.size() - 1);
    out.bdesc.assign((size_t)out.nbatch * 4 + 4, 0);
    out.bigb.clear();
    for (uint32_t b = 0; b < out.nbatch; ++b) {
        const int64_t a0 = in_off[out.bfirst[b]], pieces = in_off[out.bfirst[b + 1]] - a0;
        if (pieces > 64) out.bigb.push_back(b);
        out.bdesc[4 * b] = out.bfirst[b];
        out.bdesc[4 * b + 1] = (out.bfirst[b + 1] - out.bfirst[b]) | ((uint32_t)std::min<int64_t>(pieces, 0xFFFFFF) << 8);
        out.bdesc[4 * b + 2] = (uint32_t)a0;
        out.bdesc[4 * b + 3] = (uint32_t)((uint64_t)a0 >> 32);
    }
}

}  // namespace imsim_plan
