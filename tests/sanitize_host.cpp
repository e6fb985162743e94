// sanitize_host.cpp -- drives the host-only logic of libmech under
// AddressSanitizer and UndefinedBehaviorSanitizer (tests/test_sanitizers.py
// builds it with the library sources and runs it; no device is touched):
//   * the cut of cell trees into units (mech_cable_plan,
//     mech_cable_required_bytes) on random forests of random trees, chains
//     and stars, for unit bounds from 1 node to larger than any cell, and the
//     rejection of trees that are not in Hines order or not contiguous;
//   * buffer layouts of random type sets in both precisions
//     (mech_required_bytes);
//   * the node-index check of mech_alloc, reached after the earlier types
//     have been sorted on the host, which fails before any device call.
// Exit status 0 when every call returned what it should.
#include "mech.h"

#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

int main() {
    std::mt19937_64 rng(20190506);
    int bad = 0, cases = 0;
    auto check = [&](bool ok, const char *what, int trial) {
        if (!ok) {
            ++bad;
            std::printf("FAILED %s (trial %d)\n", what, trial);
        }
    };
    const int caps[] = {0, 1, 2, 7, 64, 1000, 5000};
    for (int trial = 0; trial < 210; ++trial) {
        const int n = 1 + (int)(rng() % 3000);
        std::vector<int32_t> parent(n);
        for (int i = 0; i < n;) {
            int size = 1 + (int)(rng() % (trial % 3 == 0 ? 2500 : 60));
            if (i + size > n) size = n - i;
            parent[i] = -1;
            const int shape = (int)(rng() % 3);   // random tree, chain, star
            for (int j = 1; j < size; ++j)
                parent[i + j] = i + (shape == 0 ? (int)(rng() % j) : shape == 1 ? j - 1 : 0);
            i += size;
        }
        const int cap = caps[trial % 7];
        size_t need = 0;
        check(mech_cable_required_bytes(n, parent.data(), cap, &need) == MECH_OK && need > 0, "required bytes", trial);
        int32_t sizes[14];
        if (mech_cable_plan(n, parent.data(), cap, sizes, nullptr, 0) != MECH_OK) {
            check(false, "plan sizes", trial);
            continue;
        }
        int64_t total = 0;
        for (int k = 0; k < 14; ++k) total += sizes[k];
        std::vector<int32_t> buf((size_t)total);
        check(mech_cable_plan(n, parent.data(), cap, sizes, buf.data(), total) == MECH_OK, "plan", trial);
        check(mech_cable_plan(n, parent.data(), cap, sizes, buf.data(), total - 1) == MECH_ERR_NOMEM, "short buffer",
              trial);
        // parent, then per position its node: every node has a position
        check(sizes[0] == n && sizes[1] >= n, "plan array sizes", trial);
        std::vector<int> seen(n, 0);
        const int32_t *pos_node = buf.data() + sizes[0], *pos_src = pos_node + sizes[1] + sizes[2];
        for (int32_t i = 0; i < sizes[1]; ++i)
            if (pos_node[i] >= 0 && pos_node[i] < n && pos_src[i] < 0) ++seen[pos_node[i]];
        bool once = true;
        for (int v : seen) once = once && v == 1;
        check(once, "one own position per node", trial);
        ++cases;
    }
    {
        int32_t sizes[14];
        const int32_t not_hines[] = {-1, 1}, split[] = {-1, -1, 0}, no_root[] = {0};
        check(mech_cable_plan(2, not_hines, 4, sizes, nullptr, 0) == MECH_ERR_INVAL, "parent >= n", -1);
        check(mech_cable_plan(3, split, 4, sizes, nullptr, 0) == MECH_ERR_INVAL, "cell not contiguous", -1);
        check(mech_cable_plan(1, no_root, 4, sizes, nullptr, 0) == MECH_ERR_INVAL, "node 0 not a root", -1);
        check(mech_cable_plan(0, nullptr, 4, sizes, nullptr, 0) == MECH_OK, "empty forest", -1);
        check(mech_cable_plan(2, not_hines, -1, sizes, nullptr, 0) == MECH_ERR_INVAL, "negative bound", -1);
    }
    // layouts of random type sets, and the node-index check of mech_alloc
    void *fake = std::aligned_alloc(256, 256);
    for (int trial = 0; trial < 200; ++trial) {
        const int64_t n_nodes = 1 + (int64_t)(rng() % 5000);
        const int n_types = 1 + (int)(rng() % 8);
        std::vector<std::vector<int32_t>> idx(n_types);
        std::vector<mech_type_desc> types(n_types);
        for (int s = 0; s < n_types; ++s) {
            const int64_t count = (int64_t)(rng() % (3 * n_nodes));
            idx[s].resize((size_t)count);
            for (auto &x : idx[s]) x = (int32_t)(rng() % n_nodes);
            types[s].kind = (int32_t)(rng() % 8);
            types[s].count = count;
            types[s].node_index = idx[s].data();
        }
        for (int prec = 0; prec <= 1; ++prec) {
            size_t bytes = 0;
            check(mech_required_bytes(n_nodes, types.data(), n_types, prec, &bytes) == MECH_OK && bytes % 256 == 0,
                  "required bytes", trial);
        }
        // one index out of range in the last type with instances
        int last = -1;
        for (int s = 0; s < n_types; ++s)
            if (types[s].count > 0) last = s;
        if (last < 0) continue;
        idx[last][idx[last].size() - 1] = (int32_t)n_nodes;
        mech_ctx *ctx = nullptr;
        check(mech_alloc(&ctx, n_nodes, types.data(), n_types, (int)(trial & 1), fake, 256, nullptr) ==
                      MECH_ERR_RANGE &&
                  ctx == nullptr,
              "node index out of range", trial);
        ++cases;
    }
    std::free(fake);
    std::printf("%d cases, %d failed\n", cases, bad);
    return bad == 0 ? 0 : 1;
}
