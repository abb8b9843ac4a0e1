// Host junction-tree compiler of the library.
//
// The paper converts a Bayesian network into a junction tree whose cliques
// and separators hold potential tables (Section 1), marks the layer of every
// clique and separator by a breadth-first traversal, and picks the root that
// gives the fewest layers (Section 2).  It does not say how the tree is
// built; this follows the textbook construction with these fixed choices,
// so that the result is a function of the network alone:
//   moral graph -> min-fill elimination, key (fill-in, clique weight, id)
//   -> maximal elimination cliques numbered in elimination order
//   -> maximum-weight spanning tree over all clique pairs by Kruskal, key
//      (-|separator|, product of separator cardinalities, i, j)
//   -> root: a centre of the tree (minimum eccentricity), lowest id on ties
//   -> layouts: root ascending; a separator's variables in the order they
//      take in the parent clique's layout; other cliques [parent separator,
//      in that order] ++ [remaining variables ascending]; last variable
//      fastest
//   -> CPT homes and posterior homes: smallest containing clique, lowest id.
#include <algorithm>
#include <cmath>
#include <numeric>
#include <queue>
#include <functional>
#include <tuple>

#include "fbn_internal.h"

namespace fbn {
namespace {

// Fixed-width bit set over the variables.
struct Bits {
    std::vector<uint64_t> w;
    explicit Bits(int n = 0) : w((size_t)(n + 63) / 64, 0) {}
    void set(int i) { w[(size_t)i >> 6] |= 1ull << (i & 63); }
    void reset(int i) { w[(size_t)i >> 6] &= ~(1ull << (i & 63)); }
    bool test(int i) const { return (w[(size_t)i >> 6] >> (i & 63)) & 1; }
    int count() const {
        int c = 0;
        for (uint64_t x : w) c += __builtin_popcountll(x);
        return c;
    }
    template <class F> void each(F f) const {
        for (size_t k = 0; k < w.size(); k++) {
            uint64_t x = w[k];
            while (x) {
                int b = __builtin_ctzll(x);
                f((int)(k * 64 + (size_t)b));
                x &= x - 1;
            }
        }
    }
    bool subset_of(const Bits& o) const {
        for (size_t k = 0; k < w.size(); k++)
            if (w[k] & ~o.w[k]) return false;
        return true;
    }
};

inline uint64_t mul_sat(uint64_t a, uint64_t b) {
    unsigned __int128 p = (unsigned __int128)a * b;
    return p > UINT64_MAX ? UINT64_MAX : (uint64_t)p;
}

}  // namespace

std::string compile_tree(const Net& net, uint64_t max_entries, Tree& t, int& code) {
    const int n = net.n;
    t = Tree();
    t.n = n;
    t.card = net.card;
    code = 0;

    // ---- moral graph
    std::vector<Bits> adj(n, Bits(n));
    for (int v = 0; v < n; v++) {
        const auto& ps = net.parents[v];
        for (size_t a = 0; a < ps.size(); a++) {
            adj[v].set(ps[a]);
            adj[ps[a]].set(v);
            for (size_t b = a + 1; b < ps.size(); b++) {
                adj[ps[a]].set(ps[b]);
                adj[ps[b]].set(ps[a]);
            }
        }
    }

    // ---- min-fill with cached keys; after eliminating v only N(v) and the
    // neighbours of N(v) can change key
    std::vector<long long> fill(n);
    std::vector<uint64_t> weight(n);
    std::vector<char> alive(n, 1);
    auto score = [&](int v) {
        const Bits& nb = adj[v];
        long long missing = 0;
        uint64_t w = (uint64_t)net.card[v];
        nb.each([&](int a) {
            w = mul_sat(w, (uint64_t)net.card[a]);
            // neighbours of v not adjacent to a (a itself included once)
            int c = 0;
            for (size_t k = 0; k < nb.w.size(); k++) c += __builtin_popcountll(nb.w[k] & ~adj[a].w[k]);
            missing += c - 1;
        });
        fill[v] = missing / 2;
        weight[v] = w;
    };
    for (int v = 0; v < n; v++) score(v);

    std::vector<Bits> ecl;   // elimination cliques
    std::vector<int> evar;   // eliminated variable of each
    ecl.reserve(n);
    for (int step = 0; step < n; step++) {
        int best = -1;
        for (int v = 0; v < n; v++) {
            if (!alive[v]) continue;
            if (best < 0 || std::make_tuple(fill[v], weight[v], v) < std::make_tuple(fill[best], weight[best], best))
                best = v;
        }
        const int v = best;
        if (max_entries && weight[v] > max_entries) {
            code = 6;
            return "a clique exceeds max_clique_entries";
        }
        Bits nb = adj[v];
        Bits cl = nb;
        cl.set(v);
        ecl.push_back(cl);
        evar.push_back(v);
        t.elim_order.push_back(v);
        // complete N(v), drop v
        nb.each([&](int a) {
            for (size_t k = 0; k < nb.w.size(); k++) adj[a].w[k] |= nb.w[k];
            adj[a].reset(a);
            adj[a].reset(v);
        });
        adj[v] = Bits(n);
        alive[v] = 0;
        Bits touched = nb;
        nb.each([&](int a) {
            for (size_t k = 0; k < nb.w.size(); k++) touched.w[k] |= adj[a].w[k];
        });
        touched.each([&](int u) {
            if (alive[u]) score(u);
        });
    }

    // ---- maximal cliques: an elimination clique can only be contained in
    // an earlier one (it holds its own eliminated variable, absent later)
    std::vector<Bits> cliques;
    for (int i = 0; i < n; i++) {
        bool dominated = false;
        for (int j = 0; j < i && !dominated; j++)
            if (ecl[j].test(evar[i]) && ecl[i].subset_of(ecl[j])) dominated = true;
        if (!dominated) cliques.push_back(ecl[i]);
    }
    const int nc = (int)cliques.size();
    t.nc = nc;
    std::vector<std::vector<int>> asc(nc);
    std::vector<uint64_t> csize(nc, 1);
    for (int c = 0; c < nc; c++) {
        cliques[c].each([&](int v) {
            asc[c].push_back(v);
            csize[c] = mul_sat(csize[c], (uint64_t)net.card[v]);
        });
        if ((max_entries && csize[c] > max_entries) || csize[c] > 0x7fffffffull) {
            code = 6;
            return "a clique exceeds max_clique_entries";
        }
    }

    // ---- Kruskal over every pair (an empty separator joins components)
    struct Cand {
        int w;
        uint64_t prod;
        int i, j;
    };
    std::vector<Cand> cand;
    cand.reserve((size_t)nc * (nc > 0 ? nc - 1 : 0) / 2);
    for (int i = 0; i < nc; i++)
        for (int j = i + 1; j < nc; j++) {
            int w = 0;
            uint64_t prod = 1;
            for (size_t k = 0; k < cliques[i].w.size(); k++) {
                uint64_t x = cliques[i].w[k] & cliques[j].w[k];
                w += __builtin_popcountll(x);
                while (x) {
                    int b = __builtin_ctzll(x);
                    prod = mul_sat(prod, (uint64_t)net.card[k * 64 + (size_t)b]);
                    x &= x - 1;
                }
            }
            cand.push_back({w, prod, i, j});
        }
    std::sort(cand.begin(), cand.end(), [](const Cand& a, const Cand& b) {
        return std::make_tuple(-a.w, a.prod, a.i, a.j) < std::make_tuple(-b.w, b.prod, b.i, b.j);
    });
    std::vector<int> uf(nc);
    std::iota(uf.begin(), uf.end(), 0);
    std::function<int(int)> find = [&](int x) { return uf[x] == x ? x : uf[x] = find(uf[x]); };
    std::vector<std::vector<int>> nbr(nc);
    int got = 0;
    for (const Cand& cd : cand) {
        if (got == nc - 1) break;
        int a = find(cd.i), b = find(cd.j);
        if (a == b) continue;
        uf[a] = b;
        nbr[cd.i].push_back(cd.j);
        nbr[cd.j].push_back(cd.i);
        got++;
    }

    // ---- root: the centre of a longest path (lowest id of two centres)
    auto bfs = [&](int s, std::vector<int>& dist, std::vector<int>& from) {
        dist.assign(nc, -1);
        from.assign(nc, -1);
        std::queue<int> q;
        dist[s] = 0;
        q.push(s);
        int last = s;
        while (!q.empty()) {
            int c = q.front();
            q.pop();
            if (dist[c] > dist[last] || (dist[c] == dist[last] && c < last)) last = c;
            for (int d : nbr[c])
                if (dist[d] < 0) {
                    dist[d] = dist[c] + 1;
                    from[d] = c;
                    q.push(d);
                }
        }
        return last;
    };
    std::vector<int> dist, from;
    int a = bfs(0, dist, from);
    int b = bfs(a, dist, from);
    std::vector<int> path;
    for (int c = b; c >= 0; c = from[c]) path.push_back(c);
    const int diam = (int)path.size() - 1;
    int root = path[(size_t)diam / 2];
    if (diam % 2 == 1) root = std::min(root, path[(size_t)diam / 2 + 1]);
    t.root = root;
    t.roots.assign(1, root);

    // ---- depth, parent, height, children
    t.parent.assign(nc, -1);
    t.depth.assign(nc, 0);
    t.height.assign(nc, 0);
    t.children.assign(nc, {});
    {
        std::vector<int> order;
        std::vector<char> seen(nc, 0);
        order.push_back(root);
        seen[root] = 1;
        for (size_t q = 0; q < order.size(); q++) {
            int c = order[q];
            for (int d : nbr[c])
                if (!seen[d]) {
                    seen[d] = 1;
                    t.parent[d] = c;
                    t.depth[d] = t.depth[c] + 1;
                    order.push_back(d);
                }
        }
        for (size_t q = order.size(); q-- > 0;) {
            int c = order[q];
            if (t.parent[c] >= 0) t.height[t.parent[c]] = std::max(t.height[t.parent[c]], t.height[c] + 1);
        }
        for (int c = 0; c < nc; c++)
            if (t.parent[c] >= 0) t.children[t.parent[c]].push_back(c);
    }

    // ---- edges by ascending child id; then layouts from the root down: the
    // root ascending, a separator in the order its variables take in the
    // parent's layout, a non-root clique [parent separator] ++ [rest ascending]
    t.pedge.assign(nc, -1);
    t.vars.assign(nc, {});
    t.size = csize;
    std::vector<std::vector<int>> rest(nc);
    for (int c = 0; c < nc; c++) {
        if (c == root) continue;
        const int p = t.parent[c];
        uint64_t ssz = 1;
        for (int v : asc[c]) {
            if (cliques[p].test(v)) ssz *= (uint64_t)net.card[v];
            else rest[c].push_back(v);
        }
        t.pedge[c] = t.ne++;
        t.e_parent.push_back(p);
        t.e_child.push_back(c);
        t.e_sep.push_back({});
        t.e_size.push_back(ssz);
    }
    std::vector<int> topdown(nc);
    std::iota(topdown.begin(), topdown.end(), 0);
    std::stable_sort(topdown.begin(), topdown.end(), [&](int a, int b) { return t.depth[a] < t.depth[b]; });
    for (int c : topdown) {
        if (c == root) {
            t.vars[c] = asc[c];
            continue;
        }
        const int p = t.parent[c];
        std::vector<int>& sep = t.e_sep[(size_t)t.pedge[c]];
        for (int v : t.vars[p])
            if (cliques[c].test(v)) sep.push_back(v);
        std::vector<int> lay = sep;
        lay.insert(lay.end(), rest[c].begin(), rest[c].end());
        t.vars[c] = lay;
    }

    // ---- homes
    t.cpt_home.assign(n, -1);
    t.var_home.assign(n, -1);
    for (int v = 0; v < n; v++) {
        for (int c = 0; c < nc; c++) {
            if (!cliques[c].test(v)) continue;
            if (t.var_home[v] < 0 || csize[c] < csize[t.var_home[v]]) t.var_home[v] = c;
            bool fam = true;
            for (int p : net.parents[v]) fam = fam && cliques[c].test(p);
            if (fam && (t.cpt_home[v] < 0 || csize[c] < csize[t.cpt_home[v]])) t.cpt_home[v] = c;
        }
    }

    // ---- prior potentials: product of the homed CPTs (ascending variable
    // id), walked with an odometer over the clique's layout
    t.prior.assign(nc, {});
    std::vector<std::vector<int>> homed(nc);
    for (int v = 0; v < n; v++) homed[t.cpt_home[v]].push_back(v);
    std::vector<int> pos(n, -1);
    for (int c = 0; c < nc; c++) {
        const auto& lay = t.vars[c];
        const int m = (int)lay.size();
        for (int k = 0; k < m; k++) pos[lay[k]] = k;
        // for each homed CPT: stride of each layout position in the CPT
        struct Fac {
            const double* p;
            std::vector<uint64_t> st;  // per layout position
        };
        std::vector<Fac> facs;
        for (int v : homed[c]) {
            Fac f;
            f.p = net.cpt[v].empty() ? nullptr : net.cpt[v].data();
            f.st.assign(m, 0);
            uint64_t s = 1;
            f.st[pos[v]] = s;
            s *= (uint64_t)net.card[v];
            for (size_t k = net.parents[v].size(); k-- > 0;) {
                f.st[pos[net.parents[v][k]]] = s;
                s *= (uint64_t)net.card[net.parents[v][k]];
            }
            facs.push_back(std::move(f));
        }
        std::vector<double>& out = t.prior[c];
        out.resize(csize[c]);
        std::vector<int> dg(m, 0);
        std::vector<uint64_t> idx(facs.size(), 0);
        for (uint64_t i = 0; i < csize[c]; i++) {
            double phi = 1.0;
            for (size_t f = 0; f < facs.size(); f++) phi *= facs[f].p ? facs[f].p[idx[f]] : 1.0;
            out[i] = phi;
            // advance the odometer (last position fastest)
            for (int k = m - 1; k >= 0; k--) {
                for (size_t f = 0; f < facs.size(); f++) idx[f] += facs[f].st[k];
                if (++dg[k] < net.card[lay[k]]) break;
                for (size_t f = 0; f < facs.size(); f++) idx[f] -= facs[f].st[k] * (uint64_t)net.card[lay[k]];
                dg[k] = 0;
            }
        }
        for (int k = 0; k < m; k++) pos[lay[k]] = -1;
    }
    return "";
}

Tree merge_forest(const std::vector<Tree>& parts) {
    Tree f;
    int v0 = 0, c0 = 0, e0 = 0;
    for (const Tree& t : parts) {
        f.card.insert(f.card.end(), t.card.begin(), t.card.end());
        for (int v : t.elim_order) f.elim_order.push_back(v + v0);
        for (int c = 0; c < t.nc; c++) {
            std::vector<int> lay = t.vars[(size_t)c];
            for (int& v : lay) v += v0;
            f.vars.push_back(std::move(lay));
            f.size.push_back(t.size[(size_t)c]);
            f.parent.push_back(t.parent[(size_t)c] < 0 ? -1 : t.parent[(size_t)c] + c0);
            f.pedge.push_back(t.pedge[(size_t)c] < 0 ? -1 : t.pedge[(size_t)c] + e0);
            f.height.push_back(t.height[(size_t)c]);
            f.depth.push_back(t.depth[(size_t)c]);
            std::vector<int> ch = t.children[(size_t)c];
            for (int& d : ch) d += c0;
            f.children.push_back(std::move(ch));
            f.prior.push_back(t.prior[(size_t)c]);
        }
        for (int r : t.roots) f.roots.push_back(r + c0);
        for (int e = 0; e < t.ne; e++) {
            f.e_parent.push_back(t.e_parent[(size_t)e] + c0);
            f.e_child.push_back(t.e_child[(size_t)e] + c0);
            std::vector<int> sv = t.e_sep[(size_t)e];
            for (int& v : sv) v += v0;
            f.e_sep.push_back(std::move(sv));
            f.e_size.push_back(t.e_size[(size_t)e]);
        }
        for (int v = 0; v < t.n; v++) {
            f.cpt_home.push_back(t.cpt_home[(size_t)v] + c0);
            f.var_home.push_back(t.var_home[(size_t)v] + c0);
        }
        v0 += t.n;
        c0 += t.nc;
        e0 += t.ne;
    }
    f.n = v0;
    f.nc = c0;
    f.ne = e0;
    f.root = f.roots.empty() ? 0 : f.roots[0];
    return f;
}

}  // namespace fbn
