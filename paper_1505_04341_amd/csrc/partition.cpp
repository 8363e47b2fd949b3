// Graph partitioning for general sparse matrices.
//
// The method takes a partition of the unknowns into p subdomains as input
// (Sec. 2.1: a graph partitioner is applied to the adjacency graph of A).
// This is a plain, deterministic recursive bisection so that matrices without
// a geometric box split can be used:
//   * a set of vertices with q parts to form is split into the first t and
//     the remaining vertices of a breadth-first order of its induced
//     subgraph, t = round(|set| * floor(q/2) / q), and the two halves receive
//     floor(q/2) and q - floor(q/2) parts recursively;
//   * the breadth-first order starts from a pseudo-peripheral vertex (George
//     and Liu): from the lowest-numbered vertex of the set, move to the
//     lowest-numbered vertex of the deepest level as long as that gives more
//     levels (at most 8 moves); neighbours are visited in ascending order and
//     components not reached are appended, each from its lowest vertex;
//   * part ids follow the recursion: the first half gets the lower ids.
// Only the sparsity pattern is used; the diagonal is ignored.
#include <algorithm>
#include <cstdint>
#include <vector>

#include "host_setup.hpp"

namespace ddlr {

namespace {

struct Bisector {
    int64_t n;
    const int64_t* rp;
    const int32_t* ci;
    std::vector<int32_t> mark;  // subset stamp of each vertex
    std::vector<int32_t> seen;  // visit stamp
    std::vector<int32_t> lev;
    int32_t stamp = 0, vstamp = 0;

    // BFS over the subset marked `stamp` from `root`, appending to order;
    // returns the deepest level reached.
    int bfs(int32_t root, std::vector<int32_t>& order) {
        const size_t start = order.size();
        order.push_back(root);
        seen[root] = vstamp;
        lev[root] = 0;
        int depth = 0;
        for (size_t h = start; h < order.size(); ++h) {
            const int32_t u = order[h];
            for (int64_t t = rp[u]; t < rp[u + 1]; ++t) {
                const int32_t v = ci[t];
                if (v == u || mark[v] != stamp || seen[v] == vstamp) continue;
                seen[v] = vstamp;
                lev[v] = lev[u] + 1;
                depth = std::max(depth, lev[v]);
                order.push_back(v);
            }
        }
        return depth;
    }

    // lowest-numbered vertex of the deepest level of the last BFS
    int32_t deepest(const std::vector<int32_t>& order, int d) const {
        int32_t far = -1;
        for (int32_t v : order)
            if (lev[v] == d && (far < 0 || v < far)) far = v;
        return far;
    }

    // breadth-first order of the subset (sorted ascending) from a pseudo-peripheral vertex
    std::vector<int32_t> order_of(const std::vector<int32_t>& set) {
        std::vector<int32_t> order, trial;
        int32_t root = set.front();
        ++vstamp;
        int depth = bfs(root, order);
        for (int it = 0; it < 8; ++it) {
            const int32_t far = deepest(order, depth);
            trial.clear();
            ++vstamp;
            const int d = bfs(far, trial);
            if (d <= depth) break;
            root = far;
            depth = d;
            order.swap(trial);
        }
        // the order from root, then unreached components from their lowest vertex
        order.clear();
        ++vstamp;
        bfs(root, order);
        for (int32_t v : set)
            if (seen[v] != vstamp) bfs(v, order);
        return order;
    }

    void split(const std::vector<int32_t>& set, int32_t q, int32_t base, int32_t* part) {
        if (q == 1 || set.size() <= 1) {
            for (int32_t v : set) part[v] = base;
            return;
        }
        ++stamp;
        for (int32_t v : set) mark[v] = stamp;
        const std::vector<int32_t> order = order_of(set);
        const int32_t q1 = q / 2, q2 = q - q1;
        const int64_t t = ((int64_t)set.size() * q1 * 2 + q) / (2 * (int64_t)q);  // round(|set| q1 / q)
        std::vector<int32_t> a(order.begin(), order.begin() + t), b(order.begin() + t, order.end());
        std::sort(a.begin(), a.end());
        std::sort(b.begin(), b.end());
        split(a, q1, base, part);
        split(b, q2, base + q1, part);
    }
};

}  // namespace

void partition_graph(int64_t n, const int64_t* rp, const int32_t* ci, int32_t p, int32_t* part) {
    if (n < 1 || p < 1) throw SetupError{-1, "partition: n and p must be positive"};
    if (p > n) throw SetupError{-1, "partition: more parts than vertices"};
    Bisector B{n, rp, ci, std::vector<int32_t>(n, 0), std::vector<int32_t>(n, 0), std::vector<int32_t>(n, 0)};
    std::vector<int32_t> all(n);
    for (int64_t i = 0; i < n; ++i) all[i] = (int32_t)i;
    B.split(all, p, 0, part);
    std::vector<int64_t> cnt(p, 0);
    for (int64_t i = 0; i < n; ++i) ++cnt[part[i]];
    for (int32_t q = 0; q < p; ++q)
        if (cnt[q] == 0) throw SetupError{-1, "partition: a part came out empty (too few vertices for p parts)"};
}

}  // namespace ddlr
