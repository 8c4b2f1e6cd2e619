// Execution plan of the hierarchical-Cholesky sweeps and its CPU emulation.
#include "plan.h"

#include <omp.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <stdexcept>

namespace bido {
namespace {

int pow2_at_least(int n, int cap) {
    int g = 1;
    while (g < n && g < cap) g <<= 1;
    return g;
}

int64_t panel_row_off(int64_t r, int64_t nI) {
    return r < nI ? r * (r + 1) / 2 : nI * (nI + 1) / 2 + (r - nI) * nI;
}


// S_top^-1 column by column: the sweeps of the top fronts applied to unit
// vectors e_j (top numbering), in blocks of TB columns.  The forward sweep of
// column j only reaches the fronts whose top subtree holds j (post-order
// numbering makes that a contiguous range per front); the backward sweep
// reaches every top front.
void top_inverse(const Factor& f, const std::vector<int>& top, const std::vector<int32_t>& tmap,
                 int64_t ntop, std::vector<double>& inv, int n_threads) {
    constexpr int TB = 32;
    const int nt = (int)top.size();
    std::vector<const double*> P(nt);
    std::vector<int64_t> sb(nt), eb(nt);          // top-subtree range [sb, eb) per front
    std::vector<int> local(f.fronts.size(), -1);
    for (int q = 0; q < nt; ++q) {
        const Front& fr = f.fronts[top[q]];
        P[q] = fr.P.data();
        local[top[q]] = q;
        eb[q] = tmap[fr.off] + fr.nI;
        sb[q] = tmap[fr.off];
        for (int c = 0; c < 2; ++c) {
            const int ch = f.tree.nodes[top[q]].child[c];
            if (ch >= 0 && local[ch] >= 0) sb[q] = std::min(sb[q], sb[local[ch]]);
        }
    }
    inv.assign((size_t)ntop * ntop, 0.0);
    std::vector<char> gnd(f.n, 0);
    for (int64_t g : f.grounds) gnd[g] = 1;
    const int64_t nblk = (ntop + TB - 1) / TB;
#pragma omp parallel num_threads(n_threads > 0 ? n_threads : omp_get_max_threads())
    {
        std::vector<double> acc((size_t)ntop * TB), Y((size_t)ntop * TB), X((size_t)ntop * TB), W, O;
#pragma omp for schedule(dynamic)
        for (int64_t blk = 0; blk < nblk; ++blk) {
            const int64_t j0 = blk * TB, j1 = std::min<int64_t>(ntop, j0 + TB);
            const int m = (int)(j1 - j0);
            std::fill(acc.begin(), acc.end(), 0.0);
            std::fill(Y.begin(), Y.end(), 0.0);
            for (int q = 0; q < nt; ++q) {
                if (j1 <= sb[q] || j0 >= eb[q]) continue;   // no column of the block reaches it
                const Front& fr = f.fronts[top[q]];
                const int nI = fr.nI, nF = nI + fr.nB;
                W.assign((size_t)nI * TB, 0.0);
                for (int i = 0; i < nI; ++i) {
                    const int64_t g = fr.off + i, ti = tmap[g];
                    if (gnd[g]) continue;
                    for (int k = 0; k < m; ++k)
                        W[(size_t)i * TB + k] = (ti == j0 + k ? 1.0 : 0.0) - acc[(size_t)ti * TB + k];
                }
                O.assign((size_t)nF * TB, 0.0);
                for (int r = 0; r < nF; ++r) {
                    double* o = &O[(size_t)r * TB];
                    const double* pr = P[q] + (size_t)r * nI;
                    const int len = r < nI ? r + 1 : nI;
                    for (int c = 0; c < len; ++c) {
                        const double a = pr[c];
                        const double* w = &W[(size_t)c * TB];
                        for (int k = 0; k < TB; ++k) o[k] += a * w[k];
                    }
                }
                for (int i = 0; i < nI; ++i)
                    std::copy(&O[(size_t)i * TB], &O[(size_t)i * TB] + TB, &Y[(size_t)tmap[fr.off + i] * TB]);
                for (int r = 0; r < fr.nB; ++r) {
                    double* a = &acc[(size_t)tmap[fr.B[r]] * TB];
                    const double* o = &O[(size_t)(nI + r) * TB];
                    for (int k = 0; k < TB; ++k) a[k] += o[k];
                }
            }
            for (int q = nt - 1; q >= 0; --q) {
                const Front& fr = f.fronts[top[q]];
                const int nI = fr.nI, nF = nI + fr.nB;
                W.assign((size_t)nF * TB, 0.0);
                for (int i = 0; i < nI; ++i)
                    std::copy(&Y[(size_t)tmap[fr.off + i] * TB], &Y[(size_t)tmap[fr.off + i] * TB] + TB,
                              &W[(size_t)i * TB]);
                for (int r = 0; r < fr.nB; ++r) {
                    const double* xb = &X[(size_t)tmap[fr.B[r]] * TB];
                    for (int k = 0; k < TB; ++k) W[(size_t)(nI + r) * TB + k] = -xb[k];
                }
                O.assign((size_t)nI * TB, 0.0);
                for (int r = 0; r < nF; ++r) {
                    const double* pr = P[q] + (size_t)r * nI;
                    const double* z = &W[(size_t)r * TB];
                    const int len = r < nI ? r + 1 : nI;
                    for (int c = 0; c < len; ++c) {
                        const double a = pr[c];
                        double* o = &O[(size_t)c * TB];
                        for (int k = 0; k < TB; ++k) o[k] += a * z[k];
                    }
                }
                for (int i = 0; i < nI; ++i)
                    std::copy(&O[(size_t)i * TB], &O[(size_t)i * TB] + TB, &X[(size_t)tmap[fr.off + i] * TB]);
            }
            for (int64_t i = 0; i < ntop; ++i)
                for (int k = 0; k < m; ++k) inv[(size_t)i * ntop + j0 + k] = X[(size_t)i * TB + k];
        }
    }
}

}  // namespace

bool build_plan(const Factor& f, FactorPlan& p, std::string& err, int n_threads, const PlanOptions* opt) {
    const PlanOptions o = opt ? *opt : PlanOptions();
    const NdTree& t = f.tree;
    const int nn = (int)t.nodes.size();
    p = FactorPlan();
    p.n = f.n;
    p.ground = f.ground;
    p.height = t.height;
    p.nodes.resize(nn);
    // update workspace entry 0 stays 0.0 (read in place of a missing child's
    // update); the boundary index and extend-add arrays end with a spare entry
    int64_t poff = 0, boff = 0, uoff = 1, eoff = 0;
    for (int id = 0; id < nn; ++id) {
        const Front& fr = f.fronts[id];
        TriNode& d = p.nodes[id];
        d.off = fr.off;
        d.nI = fr.nI;
        d.nB = fr.nB;
        d.panel = poff;
        d.bidx = boff;
        d.upd = uoff;
        d.ea = eoff;
        d.child[0] = t.nodes[id].child[0];
        d.child[1] = t.nodes[id].child[1];
        poff += (int64_t)fr.nI * (fr.nI + 1) / 2 + (int64_t)fr.nB * fr.nI;
        boff += fr.nB;
        uoff += fr.nB;
        eoff += fr.nI + fr.nB;
        p.max_nI = std::max(p.max_nI, fr.nI);
    }
    if (p.max_nI > PLAN_LDS_MAXW) {
        err = "separator of " + std::to_string(p.max_nI) + " vertices exceeds the " +
              std::to_string(PLAN_LDS_MAXW) + "-entry LDS staging limit";
        return false;
    }
    p.upd_size = uoff;
    for (int id = 0; id < nn; ++id) {
        TriNode& d = p.nodes[id];
        d.u0 = d.child[0] >= 0 ? p.nodes[d.child[0]].upd : 0;
        d.u1 = d.child[1] >= 0 ? p.nodes[d.child[1]].upd : 0;
        d.gi = -1;
        for (int64_t g : f.grounds)
            if (g >= d.off && g < d.off + d.nI) d.gi = (int32_t)(g - d.off);
    }
    p.panel.assign((size_t)poff, 0.0);
    p.panel_cm.assign((size_t)poff, 0.0);
    p.bidx.assign((size_t)boff + 1, 0);
    p.ea.assign((size_t)eoff + 1, Ea{-1, -1});        // (plus a spare entry)
    for (int id = 0; id < nn; ++id) {
        const Front& fr = f.fronts[id];
        const TriNode& d = p.nodes[id];
        const int nI = fr.nI;
        const std::vector<double>* P = &fr.P;
        int64_t o = d.panel;
        for (int r = 0; r < nI + fr.nB; ++r) {
            const int len = r < nI ? r + 1 : nI;
            for (int c = 0; c < len; ++c) p.panel[o++] = (*P)[(size_t)r * nI + c];
        }
        o = d.panel;
        for (int c = 0; c < nI; ++c)
            for (int r = c; r < nI + fr.nB; ++r) p.panel_cm[o++] = (*P)[(size_t)r * nI + c];
        for (int r = 0; r < fr.nB; ++r) p.bidx[d.bidx + r] = fr.B[r];
        const NdNode& nd = t.nodes[id];
        for (int c = 0; c < 2; ++c) {
            const int ch = nd.child[c];
            if (ch < 0) continue;
            const Front& cf = f.fronts[ch];
            for (int j = 0; j < cf.nB; ++j) {
                const int64_t g = cf.B[j];
                int pos;
                if (g < nd.end) pos = (int)(g - nd.begin);
                else pos = nI + (int)(std::lower_bound(fr.B.begin(), fr.B.end(), g) - fr.B.begin());
                Ea& m = p.ea[d.ea + pos];
                if (c == 0) m.a = j; else m.b = j;
            }
        }
    }

    // ---- subtree cut: per tree, the largest height whose subtrees are numerous
    // enough (a merged forest keeps each tree's own cut)
    const int H = t.height;
    std::vector<std::vector<int>> by_h(H + 1);
    for (int id = 0; id < nn; ++id) by_h[t.nodes[id].height].push_back(id);
    std::vector<int> root_of(nn, -1), roots;
    for (int id = nn - 1; id >= 0; --id) {
        const int par = t.nodes[id].parent;
        root_of[id] = par < 0 ? id : root_of[par];
        if (par < 0) roots.push_back(id);
    }
    std::reverse(roots.begin(), roots.end());
    const bool forest = roots.size() > 1;
    // part of a merged forest that holds node id (-1: none recorded)
    auto part_of = [&](int id) {
        int k = -1;
        for (size_t q = 0; q < f.parts.size() && q < f.part_node0.size(); ++q)
            if (f.part_node0[q] <= id) k = (int)q;
        return k < (int)f.part_top_h.size() && k < (int)f.part_off.size() ? k : -1;
    };
    for (int id = 0; id < nn; ++id) p.nodes[id].tree = std::max(0, part_of(root_of[id]));
    std::vector<int> hc_of(nn, -1);
    // cap of every tree's cut
    const int sub_cap = o.sub_h;
    {
        std::vector<std::vector<int>> members(nn);
        for (int id = 0; id < nn; ++id) members[root_of[id]].push_back(id);
        int64_t all_v = 0;
        for (int id = 0; id < nn; ++id) all_v += f.fronts[id].nI;
        // a forest may share a subtree budget
        const int sub_total = o.sub_total > 0 ? o.sub_total : 0;
        for (int r : roots) {
            const int Hr = t.nodes[r].height;
            std::vector<int> mw(Hr + 1, 0), mf(Hr + 1, 0), nroots(Hr + 2, 0);
            for (int id : members[r]) {
                const int h = t.nodes[id].height;
                mw[h] = std::max(mw[h], f.fronts[id].nI);
                mf[h] = std::max(mf[h], f.fronts[id].nI + f.fronts[id].nB);
                // id is a subtree root for every cut in [its height, its parent's height)
                const int hp = t.nodes[id].parent < 0 ? Hr + 1 : t.nodes[t.nodes[id].parent].height;
                nroots[h] += 1;
                nroots[hp] -= 1;
            }
            for (int h = 1; h <= Hr; ++h) {
                mw[h] = std::max(mw[h], mw[h - 1]);
                mf[h] = std::max(mf[h], mf[h - 1]);
                nroots[h] += nroots[h - 1];
            }
            int cut = -1;
            int want0 = o.sub_want > 0 ? o.sub_want : 256;
            if (sub_total > 0 && all_v > 0) {
                int64_t tv = 0;
                for (int id : members[r]) tv += f.fronts[id].nI;
                want0 = (int)std::max<int64_t>(1, (int64_t)sub_total * tv / all_v);
            }
            for (int want : {want0, 64, 16, 1}) {
                for (int h = Hr; h >= 0 && cut < 0; --h)
                    if (mw[h] <= PLAN_SUB_MAXW && mf[h] <= PLAN_SUB_MAXF && nroots[h] >= want) cut = h;
                if (cut >= 0) break;
            }
            if (sub_cap >= 0) cut = std::min(cut, sub_cap);
            if (sub_total > 0) {
                // keep the tree's recorded top cut (and so its cached top)
                const int k = part_of(r);
                if (k >= 0 && f.part_top_h[k] >= 0) cut = std::min(cut, f.part_top_h[k] - 1);
            }
            for (int id : members[r]) hc_of[id] = cut;
        }
    }
    auto in_sub = [&](int id) { return t.nodes[id].height <= hc_of[id]; };
    int hc = -1;
    for (int id = 0; id < nn; ++id) hc = std::max(hc, hc_of[id]);
    p.hc = hc;
    if (hc >= 0) {
        for (int rt = 0; rt < nn; ++rt) {
            const NdNode& nr = t.nodes[rt];
            if (!in_sub(rt) || (nr.parent >= 0 && in_sub(nr.parent))) continue;
            std::vector<std::vector<int>> byh(hc + 1);
            std::vector<int> stack{rt};
            while (!stack.empty()) {
                const int id = stack.back();
                stack.pop_back();
                byh[t.nodes[id].height].push_back(id);
                for (int c = 0; c < 2; ++c)
                    if (t.nodes[id].child[c] >= 0) stack.push_back(t.nodes[id].child[c]);
            }
            for (int h = 0; h <= hc; ++h) {
                p.sub_hoff.push_back((int32_t)p.sub_nodes.size());
                for (int id : byh[h]) p.sub_nodes.push_back(id);
            }
            p.sub_hoff.push_back((int32_t)p.sub_nodes.size());
            ++p.n_sub;
        }
        for (int id : p.sub_nodes) p.sub_maxw = std::max(p.sub_maxw, f.fronts[id].nI);
    }
    p.sub_tn.clear();
    for (int id : p.sub_nodes) p.sub_tn.push_back(p.nodes[id]);

    // ---- top: cut height by a cost model -------------------------------------
    // A level of the sweeps costs about one forward and one backward launch
    // of dependent memory latency (or its panel bytes at level-phase
    // bandwidth when larger); the top costs two launches plus n_top^2 FP64
    // entries at streaming bandwidth.  A forest (the factor of several
    // independent blocks) gets one cut per tree and one hierarchical top per
    // tree, concatenated.  The plan option top_h forces a single tree's cut
    // (a value above the tree height switches the top off).
    // cost-model cut of the tree rooted at r (heights of its own nodes)
    auto model_cut = [&](int r, int& lowest) {
        constexpr double T_FWD = 10e-6, T_BWD = 25e-6, BW_LVL = 2.0e12, T_TOP = 10e-6, BW_TOP = 4.5e12;
        const int Hr = t.nodes[r].height;
        int best = Hr + 1;
        lowest = Hr + 1;
        double best_cost = 0.0, saved = 0.0;
        int64_t cum = 0;
        for (int h = Hr; h > hc_of[r]; --h) {
            double pb = 0.0;
            for (int id : by_h[h]) {
                if (root_of[id] != r) continue;
                cum += f.fronts[id].nI;
                pb += 8.0 * ((double)f.fronts[id].nI * (f.fronts[id].nI + 1) / 2 +
                             (double)f.fronts[id].nB * f.fronts[id].nI);
            }
            if (cum > PLAN_TOP_MAX) break;
            lowest = h;
            saved += std::max(T_FWD, pb / BW_LVL) + std::max(T_BWD, pb / BW_LVL);
            const double cost = T_TOP + 8.0 * (double)cum * (double)cum / BW_TOP - saved;
            if (cost < best_cost) { best_cost = cost; best = h; }
        }
        return best;
    };
    std::vector<int> cut_of(nn, H + 1);      // first top height of each node's tree
    if (!forest) {
        int lowest = H + 1;
        int best = roots.empty() ? H + 1 : model_cut(roots[0], lowest);
        if (roots.empty()) lowest = H + 1;
        // a forced cut is raised as far as the top-size bound requires
        if (o.top_h >= 0) best = std::max(lowest, std::min(H + 1, o.top_h));
        for (int id = 0; id < nn; ++id) cut_of[id] = best;
        p.top_h = best;
    } else {
        // a merged forest may carry each tree's cut (the one its own plan uses)
        std::vector<int> rc(nn, H + 1);
        for (int r : roots) {
            int lowest;
            rc[r] = model_cut(r, lowest);
            const int k = part_of(r);
            if (k >= 0 && f.part_top_h[k] >= 0)
                rc[r] = std::max(lowest, std::min(t.nodes[r].height + 1, f.part_top_h[k]));
        }
        for (int id = 0; id < nn; ++id) cut_of[id] = rc[root_of[id]];
        p.top_h = -1;
    }
    p.used.top_h = p.top_h;
    p.used.sub_h = sub_cap;
    std::vector<char> is_top(nn, 0);
    for (int id = 0; id < nn; ++id) is_top[id] = t.nodes[id].height >= cut_of[id];

    // top index of each vertex (-1 elsewhere); reset after each use
    std::vector<int32_t> tmap(f.n, -1);
    // gather lists of the bottom roots below the nodes `top` into T (top
    // indices from tmap)
    auto gather_lists = [&](const std::vector<int>& top, TopPart& T) -> bool {
        const int64_t nt = T.n_top;
        std::vector<char> intop(nn, 0);
        for (int id : top) intop[id] = 1;
        // bottom roots: the update vector of each one covers its boundary,
        // which lies in the top
        std::vector<std::vector<int64_t>> lists(nt);
        for (int id = 0; id < nn; ++id) {
            const NdNode& nd = t.nodes[id];
            if (intop[id] || nd.parent < 0 || !intop[nd.parent]) continue;
            const Front& fr = f.fronts[id];
            for (int r = 0; r < fr.nB; ++r) {
                const int32_t ti = tmap[fr.B[r]];
                if (ti < 0) { err = "boundary of a bottom root outside the top"; return false; }
                lists[ti].push_back(p.nodes[id].upd + r);
            }
        }
        T.gptr.assign(nt + 1, 0);
        T.gsrc.clear();
        for (int64_t k = 0; k < nt; ++k) {
            T.gptr[k + 1] = T.gptr[k] + (int32_t)lists[k].size();
            for (int64_t src : lists[k]) T.gsrc.push_back(src);
        }
        if (T.gsrc.empty()) T.gsrc.push_back(0);
        return true;
    };
    // a merged tree whose own plan holds a hierarchical top of the same cut:
    // take its vertices (shifted by the tree's offset, same order) and its
    // hierarchical form; only the gather lists are rebuilt
    auto reuse_top = [&](const std::vector<int>& top, const TopPart& src, int64_t off, TopPart& T) -> bool {
        int64_t cnt = 0;
        for (int id : top) cnt += f.fronts[id].nI;
        if (!src.hodlr || src.n_top != cnt) return false;
        bool ok = true;
        for (int64_t k = 0; k < src.n_top && ok; ++k) {
            const int64_t v = src.pos[k] + off;
            ok = v >= 0 && v < f.n && tmap[v] < 0;
            if (ok) tmap[v] = (int32_t)k;
        }
        for (int id : top)
            for (int i = 0; i < f.fronts[id].nI && ok; ++i) ok = tmap[f.fronts[id].off + i] >= 0;
        if (ok) {
            T = TopPart();
            T.eps = src.eps;
            T.n_top = src.n_top;
            T.pos.resize(src.n_top);
            for (int64_t k = 0; k < src.n_top; ++k) T.pos[k] = src.pos[k] + off;
            T.hodlr = true;
            T.hd = src.hd;
            T.cols = src.cols;
            ok = gather_lists(top, T);
        }
        for (int64_t k = 0; k < src.n_top; ++k) {
            const int64_t v = src.pos[k] + off;
            if (v >= 0 && v < f.n) tmap[v] = -1;
        }
        return ok;
    };

    // the top of the nodes `top` (post-order): vertices, gather lists of the
    // bottom roots, S_top^-1 (hierarchical when eps > 0 or `hier`)
    auto build_top = [&](const std::vector<int>& top, bool hier, TopPart& T) -> bool {
        auto t0 = std::chrono::steady_clock::now();
        T.eps = f.eps;
        int64_t nt = 0;
        for (int id : top)
            for (int i = 0; i < f.fronts[id].nI; ++i) {
                tmap[f.fronts[id].off + i] = (int32_t)nt++;
                T.pos.push_back(f.fronts[id].off + i);
            }
        T.n_top = nt;
        bool ok = nt <= PLAN_TOP_MAX;
        if (!ok) err = "dense top too large";
        if (ok) ok = gather_lists(top, T);
        if (ok) top_inverse(f, top, tmap, nt, T.inv, n_threads);
        for (int64_t v : T.pos) tmap[v] = -1;
        if (!ok) return false;
        if ((f.eps > 0.0 || hier) && f.dim > 0 && (int64_t)f.xyz.size() >= f.n * f.dim) {
            // hierarchical form: bisection order of the top vertices, then
            // low-rank off-diagonal blocks at relative accuracy eps
            std::vector<double> xt((size_t)nt * f.dim);
            for (int64_t k = 0; k < nt; ++k)
                for (int d = 0; d < f.dim; ++d) xt[k * f.dim + d] = f.xyz[T.pos[k] * f.dim + d];
            std::vector<int64_t> ord;
            hodlr_order(nt, xt.data(), f.dim, PLAN_HODLR_LEAF, ord);
            std::vector<double> Ap((size_t)nt * nt);
            for (int64_t a = 0; a < nt; ++a)
                for (int64_t b = 0; b < nt; ++b) Ap[(size_t)a * nt + b] = T.inv[(size_t)ord[a] * nt + ord[b]];
            std::vector<int64_t> pos(nt);
            std::vector<int32_t> gptr(nt + 1, 0);
            std::vector<int64_t> gsrc;
            for (int64_t a = 0; a < nt; ++a) {
                pos[a] = T.pos[ord[a]];
                for (int32_t q = T.gptr[ord[a]]; q < T.gptr[ord[a] + 1]; ++q) gsrc.push_back(T.gsrc[q]);
                gptr[a + 1] = (int32_t)gsrc.size();
            }
            if (gsrc.empty()) gsrc.push_back(0);
            T.pos.swap(pos);
            T.gptr.swap(gptr);
            T.gsrc.swap(gsrc);
            hodlr_build(Ap, nt, f.eps, PLAN_HODLR_LEAF, n_threads, T.hd);
            std::vector<double>().swap(T.inv);
            T.hodlr = true;
            for (size_t b = 0; b < T.hd.blocks.size(); ++b)
                for (int j = 0; j < 2 * T.hd.blocks[b].k; ++j) T.cols.push_back((int32_t)((b << 16) | j));
        }
        T.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        return true;
    };
    // append top part B to A (hierarchical forms; indices shifted)
    auto append_top = [](TopPart& A, const TopPart& B) {
        const int64_t to = A.n_top, go = (int64_t)A.gsrc.size();
        const int64_t vo = (int64_t)A.hd.val.size(), ao = (int64_t)A.hd.anc.size();
        const int32_t bo = (int32_t)A.hd.blocks.size(), tso = (int32_t)(A.n_top ? A.hd.t_size : 0);
        for (int64_t v : B.pos) A.pos.push_back(v);
        if (A.gptr.empty()) A.gptr.push_back(0);
        for (size_t k = 1; k < B.gptr.size(); ++k) A.gptr.push_back((int32_t)(B.gptr[k] + go));
        for (int64_t v : B.gsrc) A.gsrc.push_back(v);
        for (HodlrBlock hb : B.hd.blocks) {
            hb.a += (int32_t)to; hb.m += (int32_t)to; hb.e += (int32_t)to;
            hb.u += vo; hb.v += vo; hb.t += tso;
            A.hd.blocks.push_back(hb);
        }
        for (HodlrLeaf lf : B.hd.leaves) {
            lf.a += (int32_t)to; lf.e += (int32_t)to; lf.d += vo; lf.anc += (int32_t)ao;
            A.hd.leaves.push_back(lf);
        }
        for (int32_t c : B.hd.anc) A.hd.anc.push_back(c + 2 * bo);
        A.hd.val.insert(A.hd.val.end(), B.hd.val.begin(), B.hd.val.end());
        for (int32_t c : B.cols) A.cols.push_back(c + (bo << 16));
        A.hd.t_size = tso + B.hd.t_size;
        A.hd.max_rank = std::max(A.hd.max_rank, B.hd.max_rank);
        A.hd.n += B.hd.n;
        A.n_top += B.n_top;
        A.seconds += B.seconds;
        A.hodlr = true;
    };
    std::shared_ptr<const TopPart> tp;
    if (!forest) {
        const int top_h = p.top_h;
        if (top_h <= H) {
            auto hit = f.top_cache.find(top_h);
            if (hit != f.top_cache.end() && hit->second->eps == f.eps) tp = hit->second;
            if (!tp) {
                auto np = std::make_shared<TopPart>();
                std::vector<int> top;
                for (int id = 0; id < nn; ++id)
                    if (is_top[id]) top.push_back(id);     // post-order
                if (!build_top(top, false, *np)) return false;
                f.top_cache[top_h] = np;
                tp = np;
            }
        }
    } else {
        auto np = std::make_shared<TopPart>();
        np->eps = f.eps;
        np->gptr.push_back(0);
        for (int r : roots) {
            std::vector<int> top;
            for (int id = 0; id < nn; ++id)
                if (is_top[id] && root_of[id] == r) top.push_back(id);
            if (top.empty()) continue;
            TopPart T;
            const int k = part_of(r);
            bool reused = false;
            if (k >= 0) {
                auto hit = f.parts[k]->top_cache.find(cut_of[r]);
                if (hit != f.parts[k]->top_cache.end() && hit->second->eps == f.eps)
                    reused = reuse_top(top, *hit->second, f.part_off[k], T);
            }
            if (!reused && !build_top(top, true, T)) return false;
            if (!T.hodlr) { err = "a forest needs vertex coordinates for its tops"; return false; }
            append_top(*np, T);
        }
        if (np->n_top > 0) {
            if (np->gsrc.empty()) np->gsrc.push_back(0);
            tp = np;
        }
    }
    if (tp) {
        if (tp->hodlr && (tp->hd.blocks.size() >= (1u << 15) || tp->hd.max_rank >= (1 << 15))) {
            err = "hierarchical top too large";
            return false;
        }
        p.n_top = tp->n_top;
        p.top_pos = tp->pos;
        p.top_zero.assign(tp->n_top, 0);
        {
            std::vector<char> gnd(f.n, 0);
            for (int64_t g : f.grounds) gnd[g] = 1;
            for (int64_t k = 0; k < tp->n_top; ++k) p.top_zero[k] = gnd[tp->pos[k]] ? 1 : 0;
        }
        p.top_gptr = tp->gptr;
        p.top_gsrc = tp->gsrc;
        p.top_inv = tp->inv;
        p.top_hodlr = tp->hodlr;
        p.hodlr = tp->hd;
        p.hodlr_cols = tp->cols;
        p.top_seconds = tp->seconds;
    }

    // ---- level phases above the cut ------------------------------------------
    // Work-item limits: columns per forward item and rows per backward item.
    // Splitting a tile over several items exposes more workgroups but needs a
    // combine launch after the level, so the limits are tunable
    // (PlanOptions fwd_cols, bwd_rows) within the LDS staging bound.
    const int fwd_cols = o.fwd_cols > 0 ? std::max(32, std::min(PLAN_LDS_DOUBLES, o.fwd_cols)) : PLAN_FWD_COLS;
    const int bwd_maxr = o.bwd_rows > 0 ? std::max(64, std::min(PLAN_LDS_DOUBLES, o.bwd_rows)) : PLAN_BWD_MAXR;
    p.used.fwd_cols = fwd_cols;
    p.used.bwd_rows = bwd_maxr == PLAN_BWD_MAXR ? 0 : bwd_maxr;
    p.bwd_wide = o.bwd_wide >= 0 ? o.bwd_wide != 0 : true;
    p.used.bwd_wide = p.bwd_wide ? 1 : 0;
    // wide backward items wanted per level of tall tiles (0 keeps every tile whole)
    const int want_items = o.level_items >= 0 ? std::min(o.level_items, 1 << 20) : PLAN_BWD_LEVEL_ITEMS;
    p.used.level_items = o.level_items;
    p.used.sub_want = o.sub_want;
    p.used.bwd_group_max = o.bwd_group_max;
    std::vector<std::pair<size_t, size_t>> fspan, bspan, fcspan, bcspan;
    struct LdsSz { size_t f, b; };
    std::vector<LdsSz> lds;
    // level heights lvl0 .. Hl: the nodes neither in the subtree phase nor in the top
    int lvl0 = H + 1;
    for (int r : roots) lvl0 = std::min(lvl0, hc_of[r] + 1);
    if (roots.empty()) lvl0 = 0;
    p.lvl0 = lvl0;
    int Hl = lvl0 - 1;
    for (int id = 0; id < nn; ++id)
        if (!is_top[id] && !in_sub(id) && t.nodes[id].height > Hl) Hl = t.nodes[id].height;
    for (int h = lvl0; h <= Hl; ++h) {
        const size_t f0 = p.fwd_items.size(), fc0 = p.fwd_comb.size();
        size_t ldsf = 0;
        for (int id : by_h[h]) {
            if (is_top[id] || in_sub(id)) continue;
            const Front& fr = f.fronts[id];
            const int nI = fr.nI, nF = fr.nI + fr.nB;
            if (nI == 0) continue;
            for (int r0 = 0; r0 < nF; r0 += PLAN_FWD_ROWS) {
                const int nrows = std::min(PLAN_FWD_ROWS, nF - r0);
                // own rows only need the columns c <= r
                const int cmax = r0 < nI ? std::min(nI, r0 + nrows) : nI;
                const int nparts = (cmax + fwd_cols - 1) / fwd_cols;
                const int64_t part0 = p.scratch_size;
                for (int k = 0; k < nparts; ++k) {
                    TriItem it{};
                    it.node = id;
                    it.r0 = r0;
                    it.nrows = nrows;
                    it.cs = k * fwd_cols;
                    it.ce = std::min(cmax, it.cs + fwd_cols);
                    it.nparts = nparts;
                    it.tile = p.n_tiles;
                    it.part = part0 + (int64_t)k * PLAN_FWD_ROWS;
                    it.part0 = part0;
                    p.fwd_items.push_back(it);
                    if (k == 0 && nparts > 1) p.fwd_comb.push_back(it);
                    ldsf = std::max(ldsf, (size_t)(it.ce - it.cs) * sizeof(double));
                }
                if (nparts > 1) p.scratch_size += (int64_t)nparts * PLAN_FWD_ROWS;
                ++p.n_tiles;
            }
        }
        fspan.push_back({f0, p.fwd_items.size() - f0});
        fcspan.push_back({fc0, p.fwd_comb.size() - fc0});
        lds.push_back({ldsf, 0});
    }
    for (int h = lvl0; h <= Hl; ++h) {
        const size_t b0 = p.bwd_items.size(), bc0 = p.bwd_comb.size();
        size_t ldsb = 0;
        // wide items take a whole column tile (up to the LDS staging bound).
        // A level of few, tall tiles (3D separators: thousands of rows under
        // each 64-column tile) would then leave most of the device idle, so
        // without an explicit row limit its tiles are cut into row ranges
        // until the level has about BWD_LEVEL_ITEMS items (never below 256
        // rows; the thin tiles of 2D levels are left whole)
        int level_rb = PLAN_LDS_DOUBLES;
        if (p.bwd_wide && o.bwd_rows <= 0 && want_items > 0) {
            int64_t tiles = 0, rows = 0;
            for (int id : by_h[h]) {
                if (is_top[id] || in_sub(id)) continue;
                const Front& fr = f.fronts[id];
                const int W = pow2_at_least(std::min(std::max(fr.nI, 1), 64), 64);
                for (int c0 = 0; c0 < fr.nI; c0 += W) {
                    ++tiles;
                    rows += fr.nI + fr.nB - c0;
                }
            }
            if (tiles > 0 && tiles < want_items && rows / tiles > 1024) {
                int64_t rb = rows / want_items;
                int pw = 256;
                while (pw * 2 <= rb && pw * 2 <= PLAN_LDS_DOUBLES) pw *= 2;
                level_rb = pw;
            }
        }
        for (int id : by_h[h]) {
            if (is_top[id] || in_sub(id)) continue;
            const Front& fr = f.fronts[id];
            const int nI = fr.nI, nF = fr.nI + fr.nB;
            if (nI == 0) continue;
            const int W = pow2_at_least(std::min(nI, 64), 64);
            const int RB = p.bwd_wide ? (o.bwd_rows > 0 ? bwd_maxr : level_rb)
                           : bwd_maxr == PLAN_BWD_MAXR ? std::min(PLAN_BWD_MAXR, std::max(64, 8192 / W))
                                                       : bwd_maxr;
            for (int c0 = 0; c0 < nI; c0 += W) {
                const int nparts = (nF - c0 + RB - 1) / RB;
                const int64_t part0 = p.scratch_size;
                for (int k = 0; k < nparts; ++k) {
                    BwdItem b{};
                    b.node = id;
                    b.c0 = c0;
                    b.ncols = std::min(W, nI - c0);
                    b.W = W;
                    b.rs = c0 + k * RB;
                    b.re = std::min(nF, b.rs + RB);
                    b.nparts = nparts;
                    b.tile = p.n_tiles;
                    b.part = part0 + (int64_t)k * W;
                    b.part0 = part0;
                    p.bwd_items.push_back(b);
                    if (k == 0 && nparts > 1) p.bwd_comb.push_back(b);
                    ldsb = std::max(ldsb, (size_t)(b.re - b.rs) * sizeof(double));
                }
                if (nparts > 1) p.scratch_size += (int64_t)nparts * W;
                ++p.n_tiles;
            }
        }
        bspan.push_back({b0, p.bwd_items.size() - b0});
        bcspan.push_back({bc0, p.bwd_comb.size() - bc0});
        lds[h - lvl0].b = ldsb;
    }
    for (size_t k = 0; k < fspan.size(); ++k)
        p.spans.push_back({fspan[k].first, fspan[k].second, bspan[k].first, bspan[k].second,
                           lds[k].f, lds[k].b, fcspan[k].first, fcspan[k].second, bcspan[k].first,
                           bcspan[k].second});

    // ---- algorithmic bytes per height ------------------------------------------
    p.fwd_bytes64.assign(H + 1, 0.0);
    p.bwd_bytes64.assign(H + 1, 0.0);
    p.fwd_bytes32.assign(H + 1, 0.0);
    p.bwd_bytes32.assign(H + 1, 0.0);
    for (int h = 0; h <= H; ++h)
        for (int id : by_h[h]) {
            if (is_top[id]) continue;
            const Front& fr = f.fronts[id];
            const double pe = (double)fr.nI * (fr.nI + 1) / 2 + (double)fr.nB * fr.nI;
            double cb = 0.0;
            for (int c = 0; c < 2; ++c)
                if (t.nodes[id].child[c] >= 0) cb += f.fronts[t.nodes[id].child[c]].nB;
            // forward: panel + b_t + extend-add maps + children's updates + y_t + c_t
            const double fv = 8.0 * (fr.nI + (fr.nI + fr.nB) + cb + fr.nI + fr.nB);
            // backward: panel + y_t + boundary ids + x_B + x_t
            const double bv = 8.0 * (fr.nI + 2.0 * fr.nB + fr.nI);
            if (in_sub(id)) {
                p.sub_fwd_bytes64 += 8.0 * pe + fv;
                p.sub_bwd_bytes64 += 8.0 * pe + bv;
                p.sub_fwd_bytes32 += 4.0 * pe + fv;
                p.sub_bwd_bytes32 += 4.0 * pe + bv;
                continue;
            }
            p.fwd_bytes64[h] += 8.0 * pe + fv;
            p.bwd_bytes64[h] += 8.0 * pe + bv;
            p.fwd_bytes32[h] += 4.0 * pe + fv;
            p.bwd_bytes32[h] += 4.0 * pe + bv;
        }
    p.meta_bytes = (int64_t)(p.nodes.size() * sizeof(TriNode) + p.bidx.size() * 8 + p.ea.size() * 8 +
                             p.fwd_items.size() * sizeof(TriItem) + p.bwd_items.size() * sizeof(BwdItem));
    if (p.scratch_size > (int64_t)1 << 31) { err = "plan scratch too large"; return false; }
    return true;
}

// ---------------------------------------------------------------------------
// CPU emulation: the per-node work of each kernel, in launch order, with
// bounds-checked accesses.
// ---------------------------------------------------------------------------
namespace {

int64_t col_off(int64_t c, int64_t nI, int64_t nB) { return c * (nI + nB) - c * (c - 1) / 2; }

struct Emu {
    const FactorPlan& p;
    const double* b;
    std::vector<double> y, upd, x, scratch;
    explicit Emu(const FactorPlan& pl, const double* bb)
        : p(pl), b(bb), y(pl.n, std::nan("")), upd(std::max<int64_t>(pl.upd_size, 1), std::nan("")),
          x(pl.n, std::nan("")), scratch(std::max<int64_t>(pl.scratch_size, 1), std::nan("")) {}

    int64_t upd_of(int child) const { return child >= 0 ? p.nodes.at(child).upd : 0; }

    double gather_w(const TriNode& nd, int i) const {
        if (nd.u0 != upd_of(nd.child[0]) || nd.u1 != upd_of(nd.child[1]))
            throw std::runtime_error("children's update offsets");
        const int64_t u0 = nd.u0, u1 = nd.u1;
        double v = b[nd.off + i];
        const Ea m = p.ea.at(nd.ea + i);
        if (m.a >= 0) v -= upd.at(u0 + m.a);
        if (m.b >= 0) v -= upd.at(u1 + m.b);
        return i == nd.gi ? 0.0 : v;
    }

    // sum over columns [cs, ce) of P(r, c) w(c) from the column-major copy
    double row_part(const TriNode& nd, int r, int cs, int ce, const std::vector<double>& w) const {
        const int cend = r < nd.nI ? std::min(ce, r + 1) : ce;
        double s = 0.0;
        for (int c = cs; c < cend; ++c)
            s += p.panel_cm.at(nd.panel + col_off(c, nd.nI, nd.nB) + (r - c)) * w.at(c - cs);
        return s;
    }

    void store_row(const TriNode& nd, int r, double s) {
        if (r < nd.nI) {
            y.at(nd.off + r) = s;
        } else {
            const Ea m = p.ea.at(nd.ea + r);
            if (m.a >= 0) s += upd.at(nd.u0 + m.a);
            if (m.b >= 0) s += upd.at(nd.u1 + m.b);
            upd.at(nd.upd + (r - nd.nI)) = s;
        }
    }

    double z_of(const TriNode& nd, int r) const {
        return r < nd.nI ? y.at(nd.off + r) : -x.at(p.bidx.at(nd.bidx + (r - nd.nI)));
    }

    // sum over rows [rs, re) of P(r, c) z(r) from the row-major copy
    double col_part(const TriNode& nd, int c, int rs, int re, const std::vector<double>& z, int z0) const {
        const int nI = nd.nI;
        double s = 0.0;
        for (int r = std::max(rs, c); r < re; ++r)
            s += p.panel.at(nd.panel + panel_row_off(r, nI) + c) * z.at(r - z0);
        return s;
    }

    void fwd_sub() {
        for (int s = 0; s < p.n_sub; ++s) {
            const int32_t* hoff = &p.sub_hoff.at((size_t)s * (p.hc + 2));
            for (int h = 0; h <= p.hc; ++h)
                for (int k = hoff[h]; k < hoff[h + 1]; ++k) {
                    const TriNode& nd = p.sub_tn.at(k);
                    if (nd.nI > PLAN_SUB_MAXW || nd.nI + nd.nB > PLAN_SUB_MAXF)
                        throw std::runtime_error("subtree node too large");
                    std::vector<double> w(nd.nI);
                    for (int i = 0; i < nd.nI; ++i) w[i] = gather_w(nd, i);
                    std::vector<double> out(nd.nI + nd.nB);
                    for (int r = 0; r < nd.nI + nd.nB; ++r) out[r] = row_part(nd, r, 0, nd.nI, w);
                    for (int r = 0; r < nd.nI + nd.nB; ++r) store_row(nd, r, out[r]);
                }
        }
    }

    void bwd_sub() {
        for (int s = 0; s < p.n_sub; ++s) {
            const int32_t* hoff = &p.sub_hoff.at((size_t)s * (p.hc + 2));
            for (int h = p.hc; h >= 0; --h)
                for (int k = hoff[h]; k < hoff[h + 1]; ++k) {
                    const TriNode& nd = p.sub_tn.at(k);
                    const int nF = nd.nI + nd.nB;
                    std::vector<double> z(nF);
                    for (int r = 0; r < nF; ++r) z[r] = z_of(nd, r);
                    for (int c = 0; c < nd.nI; ++c) x.at(nd.off + c) = col_part(nd, c, 0, nF, z, 0);
                }
        }
    }

    void fwd_lvl(const FactorPlan::Span& sp) {
        for (size_t q = sp.f0; q < sp.f0 + sp.nf; ++q) {
            const TriItem it = p.fwd_items.at(q);
            const TriNode& nd = p.nodes.at(it.node);
            if ((size_t)(it.ce - it.cs) * 8 > sp.lds_f) throw std::runtime_error("forward LDS too small");
            if (it.nrows > PLAN_FWD_ROWS) throw std::runtime_error("forward row tile too large");
            std::vector<double> w(it.ce - it.cs);
            for (int i = it.cs; i < it.ce; ++i) w[i - it.cs] = gather_w(nd, i);
            std::vector<double> s(PLAN_FWD_ROWS, 0.0);
            for (int l = 0; l < it.nrows; ++l) s[l] = row_part(nd, it.r0 + l, it.cs, it.ce, w);
            if (it.nparts == 1) {
                for (int l = 0; l < it.nrows; ++l) store_row(nd, it.r0 + l, s[l]);
                continue;
            }
            for (int l = 0; l < PLAN_FWD_ROWS; ++l) scratch.at(it.part + l) = s[l];
        }
        // combine launch: one entry per split tile
        for (size_t q = sp.cf0; q < sp.cf0 + sp.ncf; ++q) {
            const TriItem it = p.fwd_comb.at(q);
            const TriNode& nd = p.nodes.at(it.node);
            for (int l = 0; l < it.nrows; ++l) {
                double t = 0.0;
                for (int k = 0; k < it.nparts; ++k) t += scratch.at(it.part0 + (int64_t)k * PLAN_FWD_ROWS + l);
                store_row(nd, it.r0 + l, t);
            }
        }
    }

    // dense top: w_top = b - updates of the bottom roots, x_top = S_top^-1 w_top
    void top() {
        const int64_t nt = p.n_top;
        if (nt == 0) return;
        std::vector<double> w(nt);
        for (int64_t k = 0; k < nt; ++k) {
            double v = b[p.top_pos.at(k)];
            for (int32_t q = p.top_gptr.at(k); q < p.top_gptr.at(k + 1); ++q) v -= upd.at(p.top_gsrc.at(q));
            w[k] = p.top_zero.at(k) ? 0.0 : v;
        }
        if (p.top_hodlr) {
            std::vector<double> y(nt);
            hodlr_apply(p.hodlr, w.data(), y.data());
            for (int64_t i = 0; i < nt; ++i) x.at(p.top_pos[i]) = y[i];
            return;
        }
        for (int64_t i = 0; i < nt; ++i) {
            double s = 0.0;
            for (int64_t j = 0; j < nt; ++j) s += p.top_inv.at((size_t)i * nt + j) * w[j];
            x.at(p.top_pos[i]) = s;
        }
    }

    void bwd_lvl(const FactorPlan::Span& sp) {
        for (size_t q = sp.b0; q < sp.b0 + sp.nb; ++q) {
            const BwdItem it = p.bwd_items.at(q);
            const TriNode& nd = p.nodes.at(it.node);
            if ((size_t)(it.re - it.rs) * 8 > sp.lds_b) throw std::runtime_error("backward LDS too small");
            std::vector<double> z(it.re - it.rs);
            for (int r = it.rs; r < it.re; ++r) z[r - it.rs] = z_of(nd, r);
            std::vector<double> s(it.W, 0.0);
            for (int col = 0; col < it.ncols; ++col) s[col] = col_part(nd, it.c0 + col, it.rs, it.re, z, it.rs);
            if (it.nparts == 1) {
                for (int col = 0; col < it.ncols; ++col) x.at(nd.off + it.c0 + col) = s[col];
                continue;
            }
            for (int col = 0; col < it.W; ++col) scratch.at(it.part + col) = s[col];
        }
        for (size_t q = sp.cb0; q < sp.cb0 + sp.ncb; ++q) {
            const BwdItem it = p.bwd_comb.at(q);
            const TriNode& nd = p.nodes.at(it.node);
            for (int col = 0; col < it.ncols; ++col) {
                double t = 0.0;
                for (int k = 0; k < it.nparts; ++k) t += scratch.at(it.part0 + (int64_t)k * it.W + col);
                x.at(nd.off + it.c0 + col) = t;
            }
        }
    }
};

}  // namespace

void emulate_plan(const FactorPlan& p, const double* b, double* x) {
    Emu e(p, b);
    e.fwd_sub();
    for (const auto& sp : p.spans) e.fwd_lvl(sp);
    e.top();
    for (size_t k = p.spans.size(); k-- > 0;) e.bwd_lvl(p.spans[k]);
    e.bwd_sub();
    for (int64_t i = 0; i < p.n; ++i) x[i] = e.x[i];
}

}  // namespace bido
