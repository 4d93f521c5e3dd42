// Symbolic analysis: the cluster tree from recursive bisection of the grid
// box (Alg. 1 "Partition the graph of A"; the recursive-bisection case of the
// relation to LoRaSp in Sec. 2.2), the block pattern A_B of Eq. (quotient),
// the distance-2 colouring of Sec. 3.4 that lets clusters more than two apart
// run together (Sec. 2.3), and the structural fill of Sec. 2.3: eliminating a
// cluster couples every pair of its neighbours, so after a level the pattern
// is that of A_B^2, and the fill partners of a cluster are the clusters two
// steps away that an earlier cluster has already coupled to it.
#include "symbolic.h"

#include <algorithm>
#include <atomic>
#include <array>
#include <cstdint>
#include <cstring>
#include <thread>

#include "hs.h"

namespace hs {

int LevelSymbolic::block_id(int a, int b) const {
    const int* lo = pat.data() + pat_ptr[a];
    const int* hi = pat.data() + pat_ptr[a + 1];
    const int* it = std::lower_bound(lo, hi, b);
    if (it == hi || *it != b) return -1;
    return static_cast<int>(it - pat.data());
}

namespace {

struct Box {
    std::array<int, 3> lo, hi;
};

constexpr int DENSE_MAX = 1 << 14;  // levels up to this many clusters use word bitsets

// Greedy distance-2 colouring by ascending index; returns the colour count.
// Word-bitset form: the clusters within distance 2 of i are the union of
// N(j) + {j} over j in N(i); those below i are already coloured.
int colour_distance2_bits(int ncl, const ivec& ptr, const ivec& adj, ivec& color) {
    const int w = (ncl + 63) >> 6;
    std::vector<uint64_t> nb((size_t)ncl * w, 0), d(w);
    for (int j = 0; j < ncl; ++j) {
        uint64_t* r = nb.data() + (size_t)j * w;
        r[j >> 6] |= uint64_t(1) << (j & 63);
        for (int e = ptr[j]; e < ptr[j + 1]; ++e) r[adj[e] >> 6] |= uint64_t(1) << (adj[e] & 63);
    }
    color.assign(ncl, -1);
    std::vector<int> mark;
    int ncolors = 0;
    for (int i = 0; i < ncl; ++i) {
        std::fill(d.begin(), d.end(), 0);
        for (int e = ptr[i]; e < ptr[i + 1]; ++e) {
            const uint64_t* r = nb.data() + (size_t)adj[e] * w;
            for (int k = 0; k <= (i >> 6); ++k) d[k] |= r[k];
        }
        for (int k = 0; k <= (i >> 6); ++k) {
            uint64_t x = d[k];
            if (k == (i >> 6)) x &= (uint64_t(1) << (i & 63)) - 1;  // coloured: below i
            for (; x; x &= x - 1) {
                const int c = color[(k << 6) + __builtin_ctzll(x)];
                if ((int)mark.size() <= c) mark.resize(c + 1, -1);
                mark[c] = i;
            }
        }
        int c = 0;
        while (c < (int)mark.size() && mark[c] == i) ++c;
        color[i] = c;
        ncolors = std::max(ncolors, c + 1);
    }
    return ncolors;
}

int colour_distance2(int ncl, const ivec& ptr, const ivec& adj, ivec& color) {
    if (ncl <= DENSE_MAX) return colour_distance2_bits(ncl, ptr, adj, color);
    color.assign(ncl, -1);
    std::vector<int> mark;  // mark[c] == i  <=> colour c used near i
    int ncolors = 0;
    for (int i = 0; i < ncl; ++i) {
        for (int e = ptr[i]; e < ptr[i + 1]; ++e) {
            int j = adj[e];
            if (color[j] >= 0) {
                if ((int)mark.size() <= color[j]) mark.resize(color[j] + 1, -1);
                mark[color[j]] = i;
            }
            for (int f = ptr[j]; f < ptr[j + 1]; ++f) {
                int l = adj[f];
                if (l != i && color[l] >= 0) {
                    if ((int)mark.size() <= color[l]) mark.resize(color[l] + 1, -1);
                    mark[color[l]] = i;
                }
            }
        }
        int c = 0;
        while (c < (int)mark.size() && mark[c] == i) ++c;
        color[i] = c;
        ncolors = std::max(ncolors, c + 1);
    }
    return ncolors;
}

// Sorted-row set with membership test; for levels up to 2^14 clusters, rows
// of 64-bit words (row scans skip empty words and walk set bits).
class Pattern {
   public:
    explicit Pattern(int n) : w_((n + 63) >> 6), dense_(n <= DENSE_MAX) {
        if (dense_)
            bits_.assign((size_t)n * w_, 0);
        else
            rows_.assign(n, {});
    }
    void add(int a, int b) {
        if (dense_) {
            bits_[(size_t)a * w_ + (b >> 6)] |= uint64_t(1) << (b & 63);
            return;
        }
        auto& r = rows_[a];
        auto it = std::lower_bound(r.begin(), r.end(), b);
        if (it == r.end() || *it != b) r.insert(it, b);
    }
    bool dense() const { return dense_; }
    int words() const { return w_; }
    void or_row(int a, const uint64_t* mask) {  // dense only
        uint64_t* r = bits_.data() + (size_t)a * w_;
        for (int k = 0; k < w_; ++k) r[k] |= mask[k];
    }
    void row(int a, std::vector<int>& out) const {
        out.clear();
        if (dense_) {
            const uint64_t* p = bits_.data() + (size_t)a * w_;
            for (int k = 0; k < w_; ++k)
                for (uint64_t x = p[k]; x; x &= x - 1) out.push_back((k << 6) + __builtin_ctzll(x));
        } else {
            out = rows_[a];
        }
    }

   private:
    int w_;
    bool dense_;
    std::vector<uint64_t> bits_;
    std::vector<std::vector<int>> rows_;
};

void simulate_level(LevelSymbolic& L, ivec& next_ptr, ivec& next_adj) {
    const int ncl = L.ncl;
    L.ncolors = colour_distance2(ncl, L.adj_ptr, L.adj, L.color);
    L.order.resize(ncl);
    for (int i = 0; i < ncl; ++i) L.order[i] = i;
    std::stable_sort(L.order.begin(), L.order.end(), [&](int a, int b) { return L.color[a] < L.color[b]; });
    L.pos.assign(ncl, 0);
    for (int p = 0; p < ncl; ++p) L.pos[L.order[p]] = p;
    L.color_ptr.assign(L.ncolors + 1, 0);
    for (int i = 0; i < ncl; ++i) L.color_ptr[L.color[i] + 1]++;
    for (int c = 0; c < L.ncolors; ++c) L.color_ptr[c + 1] += L.color_ptr[c];

    Pattern P(ncl);
    for (int a = 0; a < ncl; ++a) {
        P.add(a, a);
        for (int e = L.adj_ptr[a]; e < L.adj_ptr[a + 1]; ++e) P.add(a, L.adj[e]);
    }
    std::vector<std::vector<int>> fill(ncl);
    std::vector<int> row;
    std::vector<char> isnbr(ncl, 0);
    std::vector<uint64_t> mask(P.words(), 0);
    for (int s : L.order) {
        for (int e = L.adj_ptr[s]; e < L.adj_ptr[s + 1]; ++e) isnbr[L.adj[e]] = 1;
        P.row(s, row);
        for (int t : row)
            if (t != s && !isnbr[t]) fill[s].push_back(L.pos[t]);  // by position, mapped back below
        for (int e = L.adj_ptr[s]; e < L.adj_ptr[s + 1]; ++e) isnbr[L.adj[e]] = 0;
        // eliminating s couples every pair of its neighbours
        if (P.dense()) {
            for (int e = L.adj_ptr[s]; e < L.adj_ptr[s + 1]; ++e) mask[L.adj[e] >> 6] |= uint64_t(1) << (L.adj[e] & 63);
            for (int e = L.adj_ptr[s]; e < L.adj_ptr[s + 1]; ++e) P.or_row(L.adj[e], mask.data());
            for (int e = L.adj_ptr[s]; e < L.adj_ptr[s + 1]; ++e) mask[L.adj[e] >> 6] = 0;
        } else {
            for (int e = L.adj_ptr[s]; e < L.adj_ptr[s + 1]; ++e)
                for (int f = L.adj_ptr[s]; f < L.adj_ptr[s + 1]; ++f) P.add(L.adj[e], L.adj[f]);
        }
    }
    // every fill list in processing order: its positions sorted (short
    // lists; the caller runs systems on several host threads), then the
    // clusters at those positions
    L.fill_ptr.resize(ncl + 1);
    L.fill_ptr[0] = 0;
    for (int s = 0; s < ncl; ++s) L.fill_ptr[s + 1] = L.fill_ptr[s] + (int)fill[s].size();
    L.fill.resize(L.fill_ptr[ncl]);
    for (int s = 0; s < ncl; ++s) {
        std::vector<int>& f = fill[s];
        for (size_t i = 1; i < f.size(); ++i) {  // insertion sort
            const int v = f[i];
            size_t j = i;
            for (; j > 0 && f[j - 1] > v; --j) f[j] = f[j - 1];
            f[j] = v;
        }
        int* out = L.fill.data() + L.fill_ptr[s];
        for (size_t i = 0; i < f.size(); ++i) out[i] = L.order[f[i]];
    }
    L.pat_ptr.assign(ncl + 1, 0);
    L.pat.clear();
    for (int a = 0; a < ncl; ++a) {
        P.row(a, row);
        L.pat.insert(L.pat.end(), row.begin(), row.end());
        L.pat_ptr[a + 1] = (int)L.pat.size();
    }
    // quotient of the final pattern over parent clusters: the row of parent
    // p holds the parents of the columns of its children's rows 2p and 2p+1,
    // other than p; each parent is taken once (marker) and the row sorted
    const int npar = (ncl + 1) / 2;
    next_ptr.assign(npar + 1, 0);
    next_adj.clear();
    std::vector<char> seen(npar, 0);
    std::vector<int> cur;
    for (int p = 0; p < npar; ++p) {
        cur.clear();
        for (int a = 2 * p; a < std::min(2 * p + 2, ncl); ++a)
            for (int e = L.pat_ptr[a]; e < L.pat_ptr[a + 1]; ++e) {
                const int pb = L.pat[e] / 2;
                if (pb != p && !seen[pb]) {
                    seen[pb] = 1;
                    cur.push_back(pb);
                }
            }
        std::sort(cur.begin(), cur.end());
        for (int q : cur) seen[q] = 0;
        next_adj.insert(next_adj.end(), cur.begin(), cur.end());
        next_ptr[p + 1] = (int)next_adj.size();
    }
}

}  // namespace

// The level-0 block graph and every level's symbolic analysis, once the
// leaves (S.leaf_ptr, leaf_dofs, cluster_of, local_of) are set.
static int finish_symbolic(int64_t n, const int64_t* row_ptr, const int32_t* col_idx, Symbolic& S) {
    (void)n;
    const int nleaf = (int)S.leaf_ptr.size() - 1;
    // level-0 block graph from the stored entries, symmetrised: the distinct
    // clusters that each cluster's rows reach (marker over its own rows), then
    // every such pair entered in both directions
    std::vector<std::vector<int>> adj(nleaf);
    {
        std::vector<char> seen(nleaf, 0);
        std::vector<int> out;
        for (int c = 0; c < nleaf; ++c) {
            out.clear();
            for (int w0 = S.leaf_ptr[c]; w0 < S.leaf_ptr[c + 1]; ++w0) {
                const int64_t i = S.leaf_dofs[w0];
                for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
                    const int cj = S.cluster_of[col_idx[e]];
                    if (cj != c && !seen[cj]) {
                        seen[cj] = 1;
                        out.push_back(cj);
                    }
                }
            }
            for (int d : out) {
                seen[d] = 0;
                adj[c].push_back(d);
                adj[d].push_back(c);
            }
        }
    }
    LevelSymbolic L0;
    L0.ncl = nleaf;
    L0.adj_ptr.assign(nleaf + 1, 0);
    for (int c = 0; c < nleaf; ++c) {
        auto& v = adj[c];
        std::sort(v.begin(), v.end());
        v.erase(std::unique(v.begin(), v.end()), v.end());
        L0.adj.insert(L0.adj.end(), v.begin(), v.end());
        L0.adj_ptr[c + 1] = (int)L0.adj.size();
    }
    S.levels.clear();
    S.levels.push_back(std::move(L0));
    for (int lvl = 0; lvl < S.nlevels; ++lvl) {
        ivec nptr, nadj;
        simulate_level(S.levels[lvl], nptr, nadj);
        if (lvl + 1 < S.nlevels) {
            LevelSymbolic N;
            N.ncl = (int)nptr.size() - 1;
            N.adj_ptr = std::move(nptr);
            N.adj = std::move(nadj);
            S.levels.push_back(std::move(N));
        }
    }
    return HS_OK;
}

// Leaves by complete recursive bisection of the graph of A + A^T (no grid):
// every set S of a tree level is put in level-structure order (breadth first
// from a pseudo-peripheral vertex, one connected component of the induced
// subgraph after the other, components by their lowest vertex; the root
// search starts at the component's lowest vertex and moves to the lowest
// vertex of the last breadth-first level while that increases the
// eccentricity, at most 8 times; neighbours in ascending order), and its
// first floor(|S| / 2) vertices form the left child.  Leaves list their
// unknowns in ascending order.
static void algebraic_leaves(int64_t n, const int64_t* row_ptr, const int32_t* col_idx, int depth,
                      std::vector<std::vector<int>>& nodes) {
    // symmetrised pattern without the diagonal, rows sorted
    std::vector<int> deg(n, 0);
    for (int64_t i = 0; i < n; ++i)
        for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
            const int j = col_idx[e];
            if (j != i) {
                ++deg[i];
                ++deg[j];
            }
        }
    std::vector<int64_t> ptr(n + 1, 0);
    for (int64_t i = 0; i < n; ++i) ptr[i + 1] = ptr[i] + deg[i];
    std::vector<int> nb(ptr[n]);
    {
        std::vector<int64_t> w(ptr.begin(), ptr.end() - 1);
        for (int64_t i = 0; i < n; ++i)
            for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
                const int j = col_idx[e];
                if (j != i) {
                    nb[w[i]++] = j;
                    nb[w[j]++] = (int)i;
                }
            }
        for (int64_t i = 0; i < n; ++i) {
            auto b = nb.begin() + ptr[i], en = nb.begin() + ptr[i + 1];
            std::sort(b, en);
            en = std::unique(b, en);
            // keep the row's length; duplicates (a_ij and a_ji both stored) are marked -1
            for (auto it = en; it != nb.begin() + ptr[i + 1]; ++it) *it = -1;
        }
    }
    std::vector<int> tag(n, -1), seen(n, 0);
    std::vector<char> done(n, 0);
    int stamp = 0, ntag = 0;
    std::vector<int> flat, lp, flat2, lp2, order;
    auto bfs = [&](int root, int cur, std::vector<int>& fl, std::vector<int>& lv) {
        ++stamp;
        fl.assign(1, root);
        seen[root] = stamp;
        lv.assign({0, 1});
        for (;;) {
            const int a = lv[lv.size() - 2], b = lv.back();
            for (int q = a; q < b; ++q) {
                const int u = fl[q];
                for (int64_t e = ptr[u]; e < ptr[u + 1]; ++e) {
                    const int v = nb[e];
                    if (v < 0) break;
                    if (tag[v] == cur && !done[v] && seen[v] != stamp) {
                        seen[v] = stamp;
                        fl.push_back(v);
                    }
                }
            }
            if ((int)fl.size() == b) return;
            lv.push_back((int)fl.size());
        }
    };
    nodes.assign(1, std::vector<int>(n));
    for (int64_t i = 0; i < n; ++i) nodes[0][i] = (int)i;
    for (int d = 0; d < depth; ++d) {
        std::vector<std::vector<int>> nxt;
        nxt.reserve(nodes.size() * 2);
        for (const std::vector<int>& S : nodes) {
            const int cur = ntag++;
            for (int v : S) {
                tag[v] = cur;
                done[v] = 0;
            }
            order.clear();
            size_t start = 0;
            for (;;) {
                while (start < S.size() && done[S[start]]) ++start;
                if (start == S.size()) break;
                int root = S[start];
                bfs(root, cur, flat, lp);
                for (int it = 0; it < 8; ++it) {
                    int cand = INT32_MAX;
                    for (int q = lp[lp.size() - 2]; q < lp.back(); ++q) cand = std::min(cand, flat[q]);
                    bfs(cand, cur, flat2, lp2);
                    if (lp2.size() <= lp.size()) break;
                    root = cand;
                    flat.swap(flat2);
                    lp.swap(lp2);
                }
                for (int v : flat) {
                    order.push_back(v);
                    done[v] = 1;
                }
            }
            const size_t h = order.size() / 2;
            std::vector<int> l(order.begin(), order.begin() + h), r(order.begin() + h, order.end());
            std::sort(l.begin(), l.end());
            std::sort(r.begin(), r.end());
            nxt.push_back(std::move(l));
            nxt.push_back(std::move(r));
        }
        nodes.swap(nxt);
    }
}

int build_symbolic(int64_t n, const int64_t* row_ptr, const int32_t* col_idx, int nx, int ny, int nz, int leaf,
                   Symbolic& S) {
    const bool algebraic = nx == 0 && ny == 0 && nz == 0;
    if (n <= 0 || leaf <= 0 || (!algebraic && (nx <= 0 || ny <= 0 || nz <= 0))) return HS_ERR_ARG;
    if (!algebraic && (int64_t)nx * ny * nz != n) return HS_ERR_GEOMETRY;
    S = Symbolic();
    S.n = n;
    int depth = 0;
    while ((int64_t)leaf << depth < n) ++depth;
    if (depth > 30) return HS_ERR_ARG;
    S.depth = depth;
    S.nlevels = depth + 1;

    if (algebraic) {
        std::vector<std::vector<int>> nodes;
        algebraic_leaves(n, row_ptr, col_idx, depth, nodes);
        const int nleaf = (int)nodes.size();
        S.leaf_ptr.assign(nleaf + 1, 0);
        S.leaf_dofs.resize(n);  // the leaves partition the unknowns: every entry below is written
        S.cluster_of.resize(n);
        S.local_of.resize(n);
        int64_t w = 0;
        for (int c = 0; c < nleaf; ++c) {
            int loc = 0;
            for (int id : nodes[c]) {
                S.leaf_dofs[w++] = id;
                S.cluster_of[id] = c;
                S.local_of[id] = loc++;
            }
            S.leaf_ptr[c + 1] = (int)w;
        }
        return finish_symbolic(n, row_ptr, col_idx, S);
    }

    std::vector<Box> boxes{Box{{0, 0, 0}, {nx, ny, nz}}};
    for (int d = 0; d < depth; ++d) {
        std::vector<Box> nxt;
        nxt.reserve(boxes.size() * 2);
        for (const Box& b : boxes) {
            int axis = 0;
            int best = b.hi[0] - b.lo[0];
            for (int a = 1; a < 3; ++a)
                if (b.hi[a] - b.lo[a] > best) {
                    best = b.hi[a] - b.lo[a];
                    axis = a;
                }
            int cut = b.lo[axis] + best / 2;
            Box l = b, r = b;
            l.hi[axis] = cut;
            r.lo[axis] = cut;
            nxt.push_back(l);
            nxt.push_back(r);
        }
        boxes.swap(nxt);
    }
    const int nleaf = (int)boxes.size();
    S.leaf_ptr.assign(nleaf + 1, 0);
    S.leaf_dofs.resize(n);  // the boxes tile the grid: every entry below is written
    S.cluster_of.resize(n);
    S.local_of.resize(n);
    int64_t w = 0;
    for (int c = 0; c < nleaf; ++c) {
        const Box& b = boxes[c];
        int loc = 0;
        // ids x + nx*(y + ny*z) ascending: z outermost, x innermost
        for (int z = b.lo[2]; z < b.hi[2]; ++z)
            for (int y = b.lo[1]; y < b.hi[1]; ++y)
                for (int x = b.lo[0]; x < b.hi[0]; ++x) {
                    int64_t id = x + (int64_t)nx * (y + (int64_t)ny * z);
                    S.leaf_dofs[w++] = id;
                    S.cluster_of[id] = c;
                    S.local_of[id] = loc++;
                }
        S.leaf_ptr[c + 1] = (int)w;
    }

    return finish_symbolic(n, row_ptr, col_idx, S);
}

int complete_level(const Symbolic& S) {
    for (int l = 0; l < S.nlevels; ++l) {
        const LevelSymbolic& L = S.levels[l];
        bool c = true;
        for (int s = 0; s < L.ncl && c; ++s)
            if (L.adj_ptr[s + 1] - L.adj_ptr[s] != L.ncl - 1 || L.order[s] != s) c = false;
        if (c) return l;
    }
    return S.nlevels - 1;
}

void combine_symbolic(std::vector<Symbolic>& parts, bool keep_empty_levels, Symbolic& out, Forest& F) {
    const int ns = (int)parts.size();
    F = Forest();
    F.nsys = ns;
    F.row_off.assign(ns + 1, 0);
    for (int i = 0; i < ns; ++i) F.row_off[i + 1] = F.row_off[i] + parts[i].n;
    std::vector<int> dense(ns), last(ns);
    for (int i = 0; i < ns; ++i) {
        dense[i] = complete_level(parts[i]);
        last[i] = keep_empty_levels ? parts[i].nlevels - 1 : dense[i];
    }
    F.sys.resize(ns);
    for (int i = 0; i < ns; ++i) F.sys[i] = i;
    std::stable_sort(F.sys.begin(), F.sys.end(), [&](int a, int b) { return last[a] > last[b]; });
    F.last.resize(ns);
    F.dense.resize(ns);
    for (int j = 0; j < ns; ++j) {
        F.last[j] = last[F.sys[j]];
        F.dense[j] = dense[F.sys[j]];
    }
    out = Symbolic();
    out.n = F.row_off[ns];
    out.nlevels = ns ? F.last[0] + 1 : 0;
    for (auto& P : parts) out.depth = std::max(out.depth, P.depth);
    F.cl_off.assign(out.nlevels, {});

    const int hw = (int)std::min(16u, std::max(1u, std::thread::hardware_concurrency()));
    // run fn(q) for q < count on up to hw host threads
    auto run = [&](int count, const auto& fn) {
        const int nth = std::min(count, hw);
        if (nth <= 1) {
            for (int q = 0; q < count; ++q) fn(q);
            return;
        }
        std::atomic<int> next(0);
        std::vector<std::thread> pool;
        for (int t = 0; t < nth; ++t)
            pool.emplace_back([&] {
                for (int q = next++; q < count; q = next++) fn(q);
            });
        for (auto& th : pool) th.join();
    };

    // leaves in placement order; unknown ids in the caller's system order.
    // Each system fills its own slices (leaf_ptr after its first leaf, its
    // rows of cluster_of and local_of), so the systems run on host threads.
    {
        std::vector<int> off(ns + 1, 0);
        std::vector<int64_t> dof0(ns + 1, 0);  // first leaf entry of every placement
        for (int j = 0; j < ns; ++j) {
            off[j + 1] = off[j] + parts[F.sys[j]].levels[0].ncl;
            dof0[j + 1] = dof0[j] + parts[F.sys[j]].n;
        }
        const int nleaf = off[ns];
        out.leaf_ptr.resize(nleaf + 1);
        out.leaf_ptr[0] = 0;
        out.cluster_of.resize(out.n);
        out.local_of.resize(out.n);
        run(ns, [&](int j) {
            Symbolic& P = parts[F.sys[j]];
            const int64_t r0 = F.row_off[F.sys[j]];
            const int c0 = off[j];
            for (int c = 0; c < P.levels[0].ncl; ++c) out.leaf_ptr[c0 + c + 1] = (int)(dof0[j] + P.leaf_ptr[c + 1]);
            for (int64_t i = 0; i < P.n; ++i) {
                out.cluster_of[r0 + i] = c0 + P.cluster_of[i];
                out.local_of[r0 + i] = P.local_of[i];
            }
            ivec().swap(P.cluster_of);
            ivec().swap(P.local_of);
            i64vec().swap(P.leaf_dofs);
        });
    }

    out.levels.resize(out.nlevels);
    // every level on its own, every system's clusters copied into their slice
    // of the combined arrays; (level, system) tasks on host threads
    std::vector<std::array<int, 2>> tasks;
    std::vector<int> alive_of(out.nlevels);
    struct Base {
        int64_t adj, fill, pat;
    };
    std::vector<std::vector<Base>> base(out.nlevels);
    std::vector<std::vector<int>> obase(out.nlevels);  // per (system, colour) start in order
    for (int l = 0; l < out.nlevels; ++l) {
        int alive = 0;
        while (alive < ns && F.last[alive] >= l) ++alive;
        alive_of[l] = alive;
        std::vector<int>& off = F.cl_off[l];
        off.assign(alive + 1, 0);
        int ncolors = 0;
        base[l].assign(alive + 1, Base{0, 0, 0});
        for (int j = 0; j < alive; ++j) {
            const LevelSymbolic& L = parts[F.sys[j]].levels[l];
            off[j + 1] = off[j] + L.ncl;
            ncolors = std::max(ncolors, L.ncolors);
            base[l][j + 1] = Base{base[l][j].adj + (int64_t)L.adj.size(), base[l][j].fill + (int64_t)L.fill.size(),
                                  base[l][j].pat + (int64_t)L.pat.size()};
        }
        LevelSymbolic& C = out.levels[l];
        C.ncl = off[alive];
        C.ncolors = ncolors;
        // every entry below is written by the (level, system) tasks, except
        // the leading zeros of the row pointers
        C.color.resize(C.ncl);
        C.adj_ptr.resize(C.ncl + 1);
        C.fill_ptr.resize(C.ncl + 1);
        C.pat_ptr.resize(C.ncl + 1);
        C.adj_ptr[0] = C.fill_ptr[0] = C.pat_ptr[0] = 0;
        C.adj.resize(base[l][alive].adj);
        C.fill.resize(base[l][alive].fill);
        C.pat.resize(base[l][alive].pat);
        // processing order: colour by colour, systems in placement order
        C.color_ptr.assign(ncolors + 1, 0);
        obase[l].assign((size_t)alive * ncolors, 0);
        int w = 0;
        for (int c = 0; c < ncolors; ++c) {
            for (int j = 0; j < alive; ++j) {
                const LevelSymbolic& L = parts[F.sys[j]].levels[l];
                obase[l][(size_t)j * ncolors + c] = w;
                if (c < L.ncolors) w += L.color_ptr[c + 1] - L.color_ptr[c];
            }
            C.color_ptr[c + 1] = w;
        }
        C.order.resize(C.ncl);
        C.pos.resize(C.ncl);
        for (int j = 0; j < alive; ++j) tasks.push_back({l, j});
    }
    auto task = [&](int q) {
        const int l = tasks[q][0], j = tasks[q][1];
        LevelSymbolic& C = out.levels[l];
        const LevelSymbolic& L = parts[F.sys[j]].levels[l];
        const int c0 = F.cl_off[l][j];
        const Base& b = base[l][j];
        for (int s = 0; s < L.ncl; ++s) {
            C.color[c0 + s] = L.color[s];
            C.adj_ptr[c0 + s + 1] = (int)(b.adj + L.adj_ptr[s + 1]);
            C.fill_ptr[c0 + s + 1] = (int)(b.fill + L.fill_ptr[s + 1]);
            C.pat_ptr[c0 + s + 1] = (int)(b.pat + L.pat_ptr[s + 1]);
        }
        for (size_t e = 0; e < L.adj.size(); ++e) C.adj[b.adj + e] = c0 + L.adj[e];
        for (size_t e = 0; e < L.fill.size(); ++e) C.fill[b.fill + e] = c0 + L.fill[e];
        for (size_t e = 0; e < L.pat.size(); ++e) C.pat[b.pat + e] = c0 + L.pat[e];
        for (int c = 0; c < L.ncolors; ++c) {
            int w = obase[l][(size_t)j * C.ncolors + c];
            for (int x = L.color_ptr[c]; x < L.color_ptr[c + 1]; ++x, ++w) {
                C.order[w] = c0 + L.order[x];
                C.pos[c0 + L.order[x]] = w;
            }
        }
    };
    run((int)tasks.size(), task);
    for (int l = 0; l < out.nlevels; ++l)
        for (int j = 0; j < alive_of[l]; ++j) parts[F.sys[j]].levels[l] = LevelSymbolic();
}

}  // namespace hs
