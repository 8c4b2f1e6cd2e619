// Nested dissection by geometric bisection (domain-decomposition clustering
// of the hierarchical-matrix literature the paper builds on, Sec. 5.3).
//
// A vertex set larger than the leaf size is split at the median of its
// longest bounding-box axis; the vertices of the lower half that touch the
// upper half form the separator, so the two remaining domains are decoupled
// in the matrix graph and their Cholesky factors carry no coupling block.
// The elimination order is the post-order of the tree: both domains
// (recursively), then the separator.  Separator and leaf vertices are
// ordered by recursive coordinate bisection, so that halving an index range
// of a separator halves it geometrically; the hierarchical compression of
// the factor relies on that.
#include <algorithm>
#include <cmath>
#include <numeric>

#include "host.h"

namespace bido {
namespace {

struct Builder {
    const Csr& g;
    const double* xyz;
    int dim;
    int leaf;
    NdTree& t;
    std::vector<int64_t> stamp;
    std::vector<char> side;
    int64_t next = 0;
    int64_t cur_stamp = 0;

    Builder(const Csr& g_, const double* x, int d, int l, NdTree& t_)
        : g(g_), xyz(x), dim(d), leaf(l), t(t_), stamp(g_.n, -1), side(g_.n, 0) {}

    int longest_axis(const std::vector<int64_t>& v) const {
        double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
        for (int64_t i : v)
            for (int a = 0; a < dim; ++a) {
                double c = xyz[i * dim + a];
                lo[a] = std::min(lo[a], c);
                hi[a] = std::max(hi[a], c);
            }
        int best = 0;
        for (int a = 1; a < dim; ++a)
            if (hi[a] - lo[a] > hi[best] - lo[best]) best = a;
        return best;
    }

    // median split of v[lo, hi) on its longest axis (lower half first)
    void median_split(std::vector<int64_t>& v, size_t lo, size_t hi, size_t mid) {
        std::vector<int64_t> sub(v.begin() + lo, v.begin() + hi);
        int ax = longest_axis(sub);
        auto cmp = [&](int64_t a, int64_t b) {
            double ca = xyz[a * dim + ax], cb = xyz[b * dim + ax];
            return ca < cb || (ca == cb && a < b);
        };
        std::nth_element(v.begin() + lo, v.begin() + mid, v.begin() + hi, cmp);
    }

    // recursive coordinate bisection order, in place
    void kd_order(std::vector<int64_t>& v, size_t lo, size_t hi) {
        if (hi - lo <= 8) {
            std::sort(v.begin() + lo, v.begin() + hi);
            return;
        }
        size_t mid = lo + (hi - lo) / 2;
        median_split(v, lo, hi, mid);
        kd_order(v, lo, mid);
        kd_order(v, mid, hi);
    }

    void emit(std::vector<int64_t>& v) {
        kd_order(v, 0, v.size());
        for (int64_t i : v) t.perm.push_back(i);
        next += (int64_t)v.size();
    }

    int build(std::vector<int64_t>& v, int depth) {
        NdNode nd;
        nd.sub_begin = next;
        nd.depth = depth;
        if ((int64_t)v.size() <= leaf) {
            nd.begin = next;
            emit(v);
            nd.end = next;
            t.nodes.push_back(nd);
            return (int)t.nodes.size() - 1;
        }
        size_t mid = v.size() / 2;
        median_split(v, 0, v.size(), mid);
        const int64_t st = ++cur_stamp;
        for (size_t i = 0; i < v.size(); ++i) {
            stamp[v[i]] = st;
            side[v[i]] = i < mid ? 0 : 1;
        }
        std::vector<int64_t> sep, d1, d2;
        for (size_t i = 0; i < mid; ++i) {
            int64_t a = v[i];
            bool touches = false;
            for (int64_t p = g.ptr[a]; p < g.ptr[a + 1] && !touches; ++p) {
                int64_t b = g.col[p];
                touches = stamp[b] == st && side[b] == 1;
            }
            (touches ? sep : d1).push_back(a);
        }
        d2.assign(v.begin() + mid, v.end());
        if (sep.empty()) {  // the halves are not coupled: cut the last lower vertex
            sep.push_back(d1.back());
            d1.pop_back();
        }
        std::vector<int64_t>().swap(v);
        int c1 = d1.empty() ? -1 : build(d1, depth + 1);
        int c2 = d2.empty() ? -1 : build(d2, depth + 1);
        nd.begin = next;
        emit(sep);
        nd.end = next;
        nd.child[0] = c1 >= 0 ? c1 : c2;
        nd.child[1] = c1 >= 0 ? c2 : -1;
        t.nodes.push_back(nd);
        int me = (int)t.nodes.size() - 1;
        for (int c = 0; c < 2; ++c)
            if (nd.child[c] >= 0) t.nodes[nd.child[c]].parent = me;
        return me;
    }
};

}  // namespace

void nested_dissection(const Csr& g, const double* xyz, int dim, int leaf,
                       NdTree& t) {
    t = NdTree();
    t.perm.reserve(g.n);
    Builder b(g, xyz, dim, std::max(leaf, 1), t);
    std::vector<int64_t> all(g.n);
    std::iota(all.begin(), all.end(), 0);
    t.root = b.build(all, 0);
    t.iperm.assign(g.n, -1);
    for (int64_t i = 0; i < g.n; ++i) t.iperm[t.perm[i]] = i;
    // heights (post-order: children first)
    t.height = 0;
    for (auto& nd : t.nodes) {
        int h = 0;
        for (int c = 0; c < 2; ++c)
            if (nd.child[c] >= 0) h = std::max(h, t.nodes[nd.child[c]].height + 1);
        nd.height = h;
        t.height = std::max(t.height, h);
    }
}

Csr permute(const Csr& a, const std::vector<int64_t>& perm,
            const std::vector<int64_t>& iperm) {
    Csr b;
    b.n = a.n;
    b.ptr.assign(a.n + 1, 0);
    for (int64_t r = 0; r < a.n; ++r) b.ptr[r + 1] = b.ptr[r] + (a.ptr[perm[r] + 1] - a.ptr[perm[r]]);
    b.col.resize(b.ptr[a.n]);
    b.val.resize(b.ptr[a.n]);
#pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t r = 0; r < a.n; ++r) {
        int64_t o = perm[r], base = b.ptr[r];
        std::vector<std::pair<int32_t, double>> row;
        row.reserve(a.ptr[o + 1] - a.ptr[o]);
        for (int64_t p = a.ptr[o]; p < a.ptr[o + 1]; ++p)
            row.emplace_back((int32_t)iperm[a.col[p]], a.val[p]);
        std::sort(row.begin(), row.end(),
                  [](const std::pair<int32_t, double>& x, const std::pair<int32_t, double>& y) {
                      return x.first < y.first;
                  });
        for (size_t k = 0; k < row.size(); ++k) {
            b.col[base + k] = row[k].first;
            b.val[base + k] = row[k].second;
        }
    }
    return b;
}

}  // namespace bido

namespace bido {

// Reverse Cuthill-McKee order of a symmetric pattern (perm and iperm only:
// no elimination tree).  Per connected component: a pseudo-peripheral start
// (breadth-first searches from a vertex of least degree, moving to a vertex
// of least degree in the last level while the depth grows), then a
// breadth-first numbering that takes each vertex's unnumbered neighbours in
// increasing degree; the whole order is reversed at the end.  Neighbours of
// a vertex then lie within a narrow band of its own index (for a k x k x k
// grid about k^2 on either side), which the inner solves that need no
// factor use for compact column offsets and cache locality.
void rcm_order(const Csr& g, NdTree& t) {
    t = NdTree();
    const int64_t n = g.n;
    std::vector<int64_t> deg(n);
    for (int64_t i = 0; i < n; ++i) deg[i] = g.ptr[i + 1] - g.ptr[i];
    std::vector<int64_t> level(n, -1), order;
    order.reserve(n);
    std::vector<char> done(n, 0);
    std::vector<int64_t> queue, nb;
    // breadth-first levels from s among the unnumbered vertices; returns
    // the depth and leaves the last level's vertices in `last`
    auto bfs = [&](int64_t s, std::vector<int64_t>& last) {
        queue.assign(1, s);
        level[s] = 0;
        size_t h = 0;
        int64_t depth = 0;
        while (h < queue.size()) {
            const int64_t v = queue[h++];
            for (int64_t q = g.ptr[v]; q < g.ptr[v + 1]; ++q) {
                const int64_t u = g.col[q];
                if (done[u] || level[u] >= 0) continue;
                level[u] = level[v] + 1;
                depth = std::max(depth, level[u]);
                queue.push_back(u);
            }
        }
        last.clear();
        for (int64_t v : queue)
            if (level[v] == depth) last.push_back(v);
        for (int64_t v : queue) level[v] = -1;
        return depth;
    };
    std::vector<int64_t> last;
    for (int64_t seed = 0; seed < n; ++seed) {
        if (done[seed]) continue;
        // least-degree vertex of the component as the first start
        bfs(seed, last);
        int64_t s = seed;
        for (int64_t v : queue)
            if (deg[v] < deg[s]) s = v;
        int64_t depth = bfs(s, last);
        for (int it = 0; it < 8; ++it) {
            int64_t c = last[0];
            for (int64_t v : last)
                if (deg[v] < deg[c]) c = v;
            std::vector<int64_t> l2;
            const int64_t d2 = bfs(c, l2);
            if (d2 <= depth) break;
            s = c;
            depth = d2;
            last.swap(l2);
        }
        // Cuthill-McKee numbering of the component from s
        size_t h = order.size();
        order.push_back(s);
        done[s] = 1;
        while (h < order.size()) {
            const int64_t v = order[h++];
            nb.clear();
            for (int64_t q = g.ptr[v]; q < g.ptr[v + 1]; ++q) {
                const int64_t u = g.col[q];
                if (!done[u]) {
                    done[u] = 1;
                    nb.push_back(u);
                }
            }
            std::stable_sort(nb.begin(), nb.end(), [&](int64_t a, int64_t b) { return deg[a] < deg[b]; });
            order.insert(order.end(), nb.begin(), nb.end());
        }
    }
    t.perm.assign(order.rbegin(), order.rend());
    t.iperm.assign(n, -1);
    for (int64_t i = 0; i < n; ++i) t.iperm[t.perm[i]] = i;
}

}  // namespace bido
