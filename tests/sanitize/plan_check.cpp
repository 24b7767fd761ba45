// Sanitizer check of the library's host-side graph plans (csrc/plan.hpp):
// built with -fsanitize=address,undefined by tests/test_sanitizers.py and run
// on random graphs (self-loops, repeated arcs, empty rows, hubs above 64
// in-arcs, zero and full weights); every plan is compared with a brute-force
// recomputation from the out-CSR.  Prints "plan_check ok" on success.
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "plan.hpp"

using namespace imsim_plan;

static uint64_t rng_state = 0x9E3779B97F4A7C15ull;
static uint64_t next_u64()
{
    rng_state ^= rng_state << 13;
    rng_state ^= rng_state >> 7;
    rng_state ^= rng_state << 17;
    return rng_state;
}

#define CHECK(c)                                                             \
    do {                                                                     \
        if (!(c)) {                                                          \
            std::fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
            std::exit(1);                                                    \
        }                                                                    \
    } while (0)

struct Graph {
    int64_t n = 0;
    std::vector<int64_t> off;
    std::vector<uint32_t> idx;
};

static Graph random_graph(int64_t n, int64_t m, bool hub)
{
    Graph g;
    g.n = n;
    std::vector<std::vector<uint32_t>> rows((size_t)n);
    for (int64_t k = 0; k < m; ++k) {
        const uint32_t u = (uint32_t)(next_u64() % (uint64_t)n);
        uint32_t v = (uint32_t)(next_u64() % (uint64_t)n);
        if (hub && (next_u64() & 3) == 0) v = 0;  // node 0 collects many in-arcs
        rows[u].push_back(v);
    }
    g.off.assign((size_t)n + 1, 0);
    for (int64_t u = 0; u < n; ++u) {
        g.off[u + 1] = g.off[u] + (int64_t)rows[u].size();
        for (uint32_t v : rows[u]) g.idx.push_back(v);
    }
    return g;
}

static void check_ic(const Graph& g)
{
    const int64_t m = (int64_t)g.idx.size();
    std::vector<uint32_t> thr((size_t)m);
    for (auto& t : thr) {
        const uint64_t r = next_u64() % 4;
        t = r == 0 ? 0u : (r == 1 ? 0xFFFFFFFFu : (uint32_t)next_u64());
    }
    IcInCsr in;
    build_ic_in_csr(g.n, m, g.off.data(), g.idx.data(), thr.data(), in);
    CHECK((int64_t)in.off.size() == g.n + 1 && in.off[0] == 0);
    // brute force: for each v, arcs (u, v) with thr != 0 in increasing arc id
    std::vector<std::vector<uint64_t>> want((size_t)g.n);
    for (int64_t u = 0; u < g.n; ++u)
        for (int64_t e = g.off[u]; e < g.off[u + 1]; ++e)
            if (thr[e]) want[g.idx[e]].push_back((uint64_t)u | ((uint64_t)e << 32));
    for (int64_t v = 0; v < g.n; ++v) {
        CHECK(in.off[v + 1] - in.off[v] == (int64_t)want[v].size());
        for (int64_t k = in.off[v]; k < in.off[v + 1]; ++k) {
            CHECK(in.sa[k] == want[v][k - in.off[v]]);
            CHECK(in.thr[k] == thr[in.sa[k] >> 32]);
        }
    }
}

static void check_lt(const Graph& g, int weights)
{
    const int64_t m = (int64_t)g.idx.size();
    std::vector<int64_t> indeg((size_t)g.n, 0);
    for (uint32_t v : g.idx) ++indeg[v];
    std::vector<uint64_t> w((size_t)m);
    for (int64_t e = 0; e < m; ++e) {
        const int64_t d = indeg[g.idx[e]];
        if (weights == 0) w[e] = kOne / (uint64_t)d;  // 1 / indeg: equal pieces
        else w[e] = (next_u64() % 5 == 0) ? 0 : (kOne / (uint64_t)d) - (next_u64() % 3);
    }
    LtInCsr in;
    int64_t bad_arc, bad_node;
    CHECK(build_lt_in_csr(g.n, m, g.off.data(), g.idx.data(), w.data(), in, bad_arc, bad_node) == 0);
    std::vector<std::vector<uint64_t>> want((size_t)g.n);
    for (int64_t u = 0; u < g.n; ++u)
        for (int64_t e = g.off[u]; e < g.off[u + 1]; ++e) {
            if (w[e] == 0) continue;
            if (w[e] == kOne) {
                want[g.idx[e]].push_back((uint64_t)u | (1ull << 63));
                want[g.idx[e]].push_back((uint64_t)u | (1ull << 63));
            } else {
                want[g.idx[e]].push_back((uint64_t)u | (w[e] << 32));
            }
        }
    for (int64_t v = 0; v < g.n; ++v) {
        CHECK(in.off[v + 1] - in.off[v] == (int64_t)want[v].size());
        for (int64_t k = in.off[v]; k < in.off[v + 1]; ++k) CHECK(in.arc[k] == want[v][k - in.off[v]]);
    }
    // equal pieces
    std::vector<uint32_t> node_w, src32;
    const bool uni = lt_uniform_form(g.n, in, node_w, src32);
    bool uni_bf = true;
    for (int64_t v = 0; v < g.n; ++v)
        for (size_t k = 1; k < want[v].size(); ++k)
            if ((want[v][k] >> 32) != (want[v][0] >> 32)) uni_bf = false;
    CHECK(uni == uni_bf);
    if (uni) {
        for (int64_t v = 0; v < g.n; ++v)
            if (!want[v].empty()) CHECK(node_w[v] == (uint32_t)(want[v][0] >> 32));
        for (size_t k = 0; k < in.arc.size(); ++k) CHECK(src32[k] == (uint32_t)in.arc[k]);
    }
    // count planes
    std::vector<uint32_t> kinfo;
    const uint64_t total = lt_count_planes(g.n, in.off, kinfo);
    uint64_t f = 0;
    for (int64_t v = 0; v < g.n; ++v) {
        CHECK(kinfo[2 * v] == (uint32_t)in.off[v] && kinfo[2 * v + 1] == (uint32_t)f);
        const int64_t d = in.off[v + 1] - in.off[v];
        uint32_t s = 0;
        if (d <= 64) {
            s = 1;
            while ((1ll << s) - 1 <= d) ++s;
            CHECK((1ll << s) - 1 > d && (s == 1 || (1ll << (s - 1)) - 1 <= d));
        }
        f += s;
    }
    CHECK(total == f && kinfo[2 * g.n + 1] == (uint32_t)f);
    // batches
    LtBatches b;
    lt_batches(g.n, in.off, b);
    CHECK(b.bfirst.front() == 0 && b.bfirst.back() == (uint32_t)g.n && b.nbatch + 1 == b.bfirst.size());
    size_t nbig = 0;
    for (uint32_t k = 0; k < b.nbatch; ++k) {
        const uint32_t v0 = b.bfirst[k], v1 = b.bfirst[k + 1];
        CHECK(v1 > v0);
        const int64_t pieces = in.off[v1] - in.off[v0];
        CHECK((v1 - v0 <= 8 && pieces <= 64) || (v1 - v0 == 1));
        CHECK(b.bdesc[4 * k] == v0 && (b.bdesc[4 * k + 1] & 0xFF) == v1 - v0);
        CHECK((int64_t)(b.bdesc[4 * k + 1] >> 8) == std::min<int64_t>(pieces, 0xFFFFFF));
        CHECK(((uint64_t)b.bdesc[4 * k + 3] << 32 | b.bdesc[4 * k + 2]) == (uint64_t)in.off[v0]);
        if (pieces > 64) {
            CHECK(nbig < b.bigb.size() && b.bigb[nbig] == k);
            ++nbig;
        }
        // a batch ends early only where the next node would not fit
        if (k + 1 < b.nbatch && v1 - v0 < 8 && pieces <= 64) CHECK(pieces + (in.off[v1 + 1] - in.off[v1]) > 64);
    }
    CHECK(nbig == b.bigb.size());
}

static void check_lt_errors()
{
    Graph g = random_graph(5, 0, false);
    g.off = {0, 2, 3, 3, 3, 3};
    g.idx = {2, 2, 2};
    LtInCsr in;
    int64_t a, v;
    std::vector<uint64_t> w = {kOne / 2, kOne / 2, 1};
    CHECK(build_lt_in_csr(g.n, 3, g.off.data(), g.idx.data(), w.data(), in, a, v) == 2 && v == 2);
    w = {kOne + 1, 0, 0};
    CHECK(build_lt_in_csr(g.n, 3, g.off.data(), g.idx.data(), w.data(), in, a, v) == 1 && a == 0);
    w = {kOne, 0, 0};
    CHECK(build_lt_in_csr(g.n, 3, g.off.data(), g.idx.data(), w.data(), in, a, v) == 0 && in.arc.size() == 2);
}

int main()
{
    for (int rep = 0; rep < 40; ++rep) {
        const int64_t n = 1 + (int64_t)(next_u64() % 300);
        const int64_t m = (int64_t)(next_u64() % 2500);
        const Graph g = random_graph(n, m, rep % 3 == 0);
        check_ic(g);
        check_lt(g, 0);
        check_lt(g, 1);
    }
    const Graph empty = random_graph(1, 0, false);
    check_ic(empty);
    check_lt(empty, 0);
    check_lt_errors();
    std::printf("plan_check ok\n");
    return 0;
}
