// Host-side preprocessing: tree validation, bond clamping and compilation of
// the SOP generator into a sparse tree operator (hierarchical SOP).
//
// Paper: pyTTN (arXiv 2503.15460), Sec. II A (tree ansatz, N_i = min(16, N_i)
// style bond limits) and Sec. II B 2 (hierarchical SOP: the per-node form
// (A) + (B) + (C), built with a bipartite-graph construction and a pre-order
// pass for the mean-field operators; identity operators become copies).
#include <algorithm>
#include <cmath>
#include <functional>
#include <map>
#include <set>

#include "ttn_internal.h"

namespace ttn {

void Tree::update_dims() {
    dims.assign(n, {});
    size.assign(n, 0);
    for (int z = 0; z < n; ++z) {
        if (local_dim[z] > 0) dims[z].push_back(local_dim[z]);
        else
            for (int c : kids[z]) dims[z].push_back(bond[c]);
        dims[z].push_back(z == root ? 1 : bond[z]);
        int64_t s = 1;
        for (int d : dims[z]) s *= d;
        size[z] = s;
    }
}

Tree build_tree(int n, const int32_t *parent, const int32_t *local_dim, const int32_t *bond_req,
                const int32_t *bond_max) {
    if (n < 2 || !parent || !local_dim || !bond_req) throw Error(TTN_E_TREE, "need at least 2 nodes");
    Tree t;
    t.n = n;
    t.parent.assign(parent, parent + n);
    t.local_dim.assign(local_dim, local_dim + n);
    t.kids.assign(n, {});
    for (int z = 0; z < n; ++z) {
        int p = t.parent[z];
        if (p == -1) {
            if (t.root >= 0) throw Error(TTN_E_TREE, "more than one root");
            t.root = z;
        } else if (p < 0 || p >= n || p == z) {
            throw Error(TTN_E_TREE, "parent id out of range at node " + std::to_string(z));
        } else {
            t.kids[p].push_back(z);
        }
    }
    if (t.root < 0) throw Error(TTN_E_TREE, "no root");
    for (int z = 0; z < n; ++z) {  // every node reaches the root
        int w = z, steps = 0;
        while (w != t.root) {
            w = t.parent[w];
            if (++steps > n) throw Error(TTN_E_TREE, "cycle in parent array");
        }
    }
    for (int z = 0; z < n; ++z) {
        bool leaf = t.kids[z].empty();
        if (leaf != (t.local_dim[z] > 0))
            throw Error(TTN_E_DIMS, "node " + std::to_string(z) + ": local_dim > 0 iff leaf");
        if (t.local_dim[z] < 0) throw Error(TTN_E_DIMS, "negative local_dim");
        if (z != t.root && bond_req[z] < 1) throw Error(TTN_E_DIMS, "bond_dim must be >= 1");
    }
    if (t.kids[t.root].empty()) throw Error(TTN_E_TREE, "root must have children");
    for (int z = 0; z < n; ++z)
        if ((int)t.kids[z].size() > MAX_CHILDREN)
            throw Error(TTN_E_TREE, "node " + std::to_string(z) + " has more than " + std::to_string(MAX_CHILDREN) +
                                        " children");
    // post-order
    std::function<void(int)> rec = [&](int z) {
        for (int c : t.kids[z]) rec(c);
        t.postorder.push_back(z);
    };
    rec(t.root);
    t.leaf_index.assign(n, -1);
    for (int z = 0; z < n; ++z)
        if (t.local_dim[z] > 0) {
            t.leaf_index[z] = (int)t.leaves.size();
            t.leaves.push_back(z);
        }
    // product of primitive dims inside every subtree (as double)
    std::vector<double> inside(n, 1.0);
    for (int z : t.postorder) {
        if (t.local_dim[z] > 0) inside[z] = t.local_dim[z];
        else {
            double p = 1.0;
            for (int c : t.kids[z]) p *= inside[c];
            inside[z] = p;
        }
    }
    const double total = inside[t.root];
    auto clamp = [&](const int32_t *req) {
        std::vector<int> b(n, 1);
        for (int c = 0; c < n; ++c) {
            if (c == t.root) continue;
            double v = std::min({(double)req[c], inside[c], total / inside[c]});
            b[c] = (int)v;
        }
        // lower each bond to the product of the other indices at both end nodes
        bool changed = true;
        while (changed) {
            changed = false;
            for (int z = 0; z < n; ++z) {
                std::vector<std::pair<int, int>> inc;  // (owner or -1, dim), snapshot
                if (t.local_dim[z] > 0) inc.push_back({-1, t.local_dim[z]});
                else
                    for (int c : t.kids[z]) inc.push_back({c, b[c]});
                if (z != t.root) inc.push_back({z, b[z]});
                for (size_t i = 0; i < inc.size(); ++i) {
                    if (inc[i].first < 0) continue;
                    double other = 1.0;
                    for (size_t j = 0; j < inc.size(); ++j)
                        if (j != i) other *= inc[j].second;
                    if ((double)inc[i].second > other) {
                        b[inc[i].first] = (int)other;
                        changed = true;
                    }
                }
            }
        }
        return b;
    };
    t.bond = clamp(bond_req);
    t.cap = t.bond;
    if (bond_max) {
        for (int z = 0; z < n; ++z)
            if (z != t.root && bond_max[z] < 1) throw Error(TTN_E_DIMS, "bond_max must be >= 1");
        std::vector<int> c = clamp(bond_max);
        for (int z = 0; z < n; ++z) t.cap[z] = std::max(t.bond[z], c[z]);
    }
    std::swap(t.bond, t.cap);  // shapes at capacity first
    t.update_dims();
    t.capdims = t.dims;
    t.capsize = t.size;
    std::swap(t.bond, t.cap);
    t.update_dims();
    return t;
}

SopInput read_sop(const Tree &t, int32_t n_ops, const int32_t *op_leaf, const int64_t *op_offset,
                  const double *op_data, int32_t n_terms, const double *coeff,
                  const int64_t *term_ptr, const int32_t *term_ops) {
    if (n_ops < 0 || n_terms < 0) throw Error(TTN_E_INVALID, "negative counts");
    if (n_ops > 0 && (!op_leaf || !op_offset || !op_data)) throw Error(TTN_E_INVALID, "null operator arrays");
    if (n_terms > 0 && (!coeff || !term_ptr || !term_ops)) throw Error(TTN_E_INVALID, "null term arrays");
    SopInput s;
    s.n_ops = n_ops;
    s.n_terms = n_terms;
    for (int o = 0; o < n_ops; ++o) {
        int l = op_leaf[o];
        if (l < 0 || l >= t.n || t.local_dim[l] <= 0)
            throw Error(TTN_E_INVALID, "operator " + std::to_string(o) + " is not on a leaf");
        int64_t d = t.local_dim[l];
        if (op_offset[o + 1] - op_offset[o] != d * d)
            throw Error(TTN_E_DIMS, "operator " + std::to_string(o) + " size != d*d");
        std::vector<cplx> m(d * d);
        for (int64_t i = 0; i < d * d; ++i) {
            m[i] = cplx(op_data[2 * (op_offset[o] + i)], op_data[2 * (op_offset[o] + i) + 1]);
            if (!std::isfinite(m[i].real()) || !std::isfinite(m[i].imag()))
                throw Error(TTN_E_INVALID, "non-finite operator element");
        }
        s.op_leaf.push_back(l);
        s.op_mat.push_back(std::move(m));
    }
    for (int r = 0; r < n_terms; ++r) {
        cplx c(coeff[2 * r], coeff[2 * r + 1]);
        if (!std::isfinite(c.real()) || !std::isfinite(c.imag()))
            throw Error(TTN_E_INVALID, "non-finite coefficient in term " + std::to_string(r));
        std::vector<int> ops;
        std::set<int> seen;
        for (int64_t q = term_ptr[r]; q < term_ptr[r + 1]; ++q) {
            int o = term_ops[q];
            if (o < 0 || o >= n_ops) throw Error(TTN_E_INVALID, "term operator id out of range");
            if (!seen.insert(s.op_leaf[o]).second)
                throw Error(TTN_E_INVALID, "term " + std::to_string(r) + " has two operators on one leaf");
            ops.push_back(o);
        }
        if (ops.empty()) throw Error(TTN_E_INVALID, "term " + std::to_string(r) + " has no operator");
        s.coeff.push_back(c);
        s.term_ops.push_back(ops);
    }
    return s;
}

// ||G - G^dag||_F against ||G||_F from the leaf operators and coefficients.
// Operators on one leaf that agree to `cluster` (relative Frobenius) are given
// one id, and so are adjoints; the two operator strings of G and G^dag are
// collected with their summed coefficients.  For two strings a, b the trace
// Tr(S_a^dag S_b) / prod d_l is the product over the leaves either string
// touches of Tr(X^dag Y) / d_l (X or Y the identity where a string has no
// operator), so ||.||_F^2 / prod d_l is a double sum over the strings that
// never forms a dense matrix.
double sop_hermiticity_defect(const SopInput &s, double cluster) {
    // per leaf: representative matrices of the distinct operators
    int nleaf = 1;
    for (int o = 0; o < s.n_ops; ++o) nleaf = std::max(nleaf, s.op_leaf[o] + 1);
    std::vector<std::vector<std::vector<cplx>>> reps(nleaf);
    auto fro = [](const std::vector<cplx> &m) {
        double a = 0.0;
        for (auto &x : m) a += std::norm(x);
        return std::sqrt(a);
    };
    auto id_of = [&](int leaf, const std::vector<cplx> &m) {
        auto &v = reps[leaf];
        const double nm = fro(m);
        for (size_t k = 0; k < v.size(); ++k) {
            double d2 = 0.0;
            for (size_t q = 0; q < m.size(); ++q) d2 += std::norm(m[q] - v[k][q]);
            if (std::sqrt(d2) <= cluster * std::max(nm, fro(v[k]))) return (int)k;
        }
        v.push_back(m);
        return (int)v.size() - 1;
    };
    std::vector<int> cid(s.n_ops), aid(s.n_ops);
    for (int o = 0; o < s.n_ops; ++o) {
        const auto &m = s.op_mat[o];
        const int d = (int)std::lround(std::sqrt((double)m.size()));
        std::vector<cplx> adj(m.size());
        for (int i = 0; i < d; ++i)
            for (int j = 0; j < d; ++j) adj[(size_t)i * d + j] = std::conj(m[(size_t)j * d + i]);
        cid[o] = id_of(s.op_leaf[o], m);
        aid[o] = id_of(s.op_leaf[o], adj);
    }
    // Gram tables per leaf: g[x][y] = Tr(X^dag Y)/d, plus tr[y] = Tr(Y)/d
    std::vector<std::vector<std::vector<cplx>>> gram(nleaf);
    std::vector<std::vector<cplx>> trn(nleaf);
    for (int leaf = 0; leaf < nleaf; ++leaf) {
        const auto &v = reps[leaf];
        if (v.empty()) continue;
        const int d = (int)std::lround(std::sqrt((double)v[0].size()));
        auto &g = gram[leaf];
        auto &tr = trn[leaf];
        g.assign(v.size(), std::vector<cplx>(v.size(), cplx(0)));
        tr.assign(v.size(), cplx(0));
        for (size_t x = 0; x < v.size(); ++x) {
            for (int i = 0; i < d; ++i) tr[x] += v[x][(size_t)i * d + i];
            tr[x] /= (double)d;
            for (size_t y = 0; y < v.size(); ++y) {
                cplx a(0);
                for (size_t q = 0; q < v[x].size(); ++q) a += std::conj(v[x][q]) * v[y][q];
                g[x][y] = a / (double)d;
            }
        }
    }
    using Str = std::vector<std::pair<int, int>>;  // (leaf, operator id), sorted by leaf
    std::map<Str, cplx> G, D;
    for (int r = 0; r < s.n_terms; ++r) {
        Str a, b;
        for (int o : s.term_ops[r]) {
            a.push_back({s.op_leaf[o], cid[o]});
            b.push_back({s.op_leaf[o], aid[o]});
        }
        std::sort(a.begin(), a.end());
        std::sort(b.begin(), b.end());
        G[a] += s.coeff[r];
        D[a] += s.coeff[r];
        D[b] -= std::conj(s.coeff[r]);
    }
    auto norm2 = [&](const std::map<Str, cplx> &T) {
        std::vector<std::pair<const Str *, cplx>> v;
        for (auto &kv : T)
            if (kv.second != cplx(0)) v.push_back({&kv.first, kv.second});
        double acc = 0.0;
        for (size_t i = 0; i < v.size(); ++i)
            for (size_t j = 0; j < v.size(); ++j) {
                const Str &a = *v[i].first, &b = *v[j].first;
                cplx f(1.0);
                size_t p = 0, q = 0;
                while (p < a.size() || q < b.size()) {
                    if (q == b.size() || (p < a.size() && a[p].first < b[q].first)) {
                        f *= std::conj(trn[a[p].first][a[p].second]);
                        ++p;
                    } else if (p == a.size() || b[q].first < a[p].first) {
                        f *= trn[b[q].first][b[q].second];
                        ++q;
                    } else {
                        f *= gram[a[p].first][a[p].second][b[q].second];
                        ++p;
                        ++q;
                    }
                }
                acc += (std::conj(v[i].second) * v[j].second * f).real();
            }
        return std::max(acc, 0.0);
    };
    const double g2 = norm2(G);
    if (g2 == 0.0) return 0.0;
    return std::sqrt(norm2(D) / g2);
}

bool sop_is_hermitian(const SopInput &s, double rtol) { return sop_hermiticity_defect(s, 1e-12) <= rtol; }

namespace {

using SlotVec = std::vector<std::pair<int, int>>;  // (node, value) sorted by node

struct CTerm {
    cplx coef;
    SlotVec slots;
};

// Minimum vertex cover of a bipartite graph (Konig's theorem).
// adj[l] lists right vertices; returns (left in cover, right in cover).
std::pair<std::vector<char>, std::vector<char>> min_vertex_cover(int nl, int nr,
                                                                const std::vector<std::vector<int>> &adj) {
    std::vector<int> matchR(nr, -1), matchL(nl, -1);
    for (int l = 0; l < nl; ++l) {
        std::vector<char> vis(nr, 0);
        std::function<bool(int)> aug = [&](int u) -> bool {
            for (int r : adj[u]) {
                if (vis[r]) continue;
                vis[r] = 1;
                if (matchR[r] < 0 || aug(matchR[r])) {
                    matchR[r] = u;
                    matchL[u] = r;
                    return true;
                }
            }
            return false;
        };
        aug(l);
    }
    // alternating reachability from unmatched left vertices
    std::vector<char> zl(nl, 0), zr(nr, 0);
    std::vector<int> stack;
    for (int l = 0; l < nl; ++l)
        if (matchL[l] < 0) {
            zl[l] = 1;
            stack.push_back(l);
        }
    while (!stack.empty()) {
        int u = stack.back();
        stack.pop_back();
        for (int r : adj[u]) {
            if (zr[r] || matchL[u] == r) continue;
            zr[r] = 1;
            int w = matchR[r];
            if (w >= 0 && !zl[w]) {
                zl[w] = 1;
                stack.push_back(w);
            }
        }
    }
    std::vector<char> cl(nl), cr(nr);
    for (int l = 0; l < nl; ++l) cl[l] = !zl[l];
    for (int r = 0; r < nr; ++r) cr[r] = zr[r];
    return {cl, cr};
}

}  // namespace

TreeOp compile_tree_operator(const Tree &t, const SopInput &s) {
    TreeOp op;
    op.entries.assign(t.n, {});
    op.n_ch.assign(t.n, 2);
    op.inside_used.assign(t.n, 0);
    op.outside_used.assign(t.n, 0);
    op.leafU.assign(t.leaves.size(), {});
    op.n_ch[t.root] = 1;

    std::vector<CTerm> terms;
    for (int r = 0; r < s.n_terms; ++r) {
        if (s.coeff[r] == cplx(0)) continue;
        CTerm ct;
        ct.coef = s.coeff[r];
        for (int o : s.term_ops[r]) ct.slots.push_back({s.op_leaf[o], o});
        std::sort(ct.slots.begin(), ct.slots.end());
        terms.push_back(ct);
    }

    for (int c : t.postorder) {
        if (c == t.root) continue;
        const bool leaf = t.local_dim[c] > 0;
        const std::vector<int> &kids = t.kids[c];
        std::vector<CTerm> untouched;
        std::map<std::pair<std::vector<int>, SlotVec>, cplx> edges;
        for (auto &ct : terms) {
            std::vector<int> in(leaf ? 1 : kids.size(), -1);
            SlotVec out;
            bool touch = false;
            for (auto &sv : ct.slots) {
                int k = -1;
                if (leaf) {
                    if (sv.first == c) k = 0;
                } else {
                    auto it = std::find(kids.begin(), kids.end(), sv.first);
                    if (it != kids.end()) k = (int)(it - kids.begin());
                }
                if (k >= 0) {
                    in[k] = sv.second;
                    touch = true;
                } else {
                    out.push_back(sv);
                }
            }
            if (!touch) {
                untouched.push_back(ct);
                continue;
            }
            edges[{in, out}] += ct.coef;
        }
        op.outside_used[c] = !untouched.empty();
        // inside terms (nothing outside the subtree) and crossing terms
        std::vector<std::pair<std::vector<int>, cplx>> inside;
        std::map<std::vector<int>, int> lidx;
        std::map<SlotVec, int> ridx;
        for (auto &e : edges) {
            if (e.second == cplx(0)) continue;
            if (e.first.second.empty()) inside.push_back({e.first.first, e.second});
            else {
                lidx.emplace(e.first.first, 0);
                ridx.emplace(e.first.second, 0);
            }
        }
        std::vector<std::vector<int>> lkeys;
        std::vector<SlotVec> rkeys;
        for (auto &kv : lidx) {
            kv.second = (int)lkeys.size();
            lkeys.push_back(kv.first);
        }
        for (auto &kv : ridx) {
            kv.second = (int)rkeys.size();
            rkeys.push_back(kv.first);
        }
        int nl = (int)lkeys.size(), nr = (int)rkeys.size();
        std::vector<std::vector<int>> adj(nl);
        std::vector<std::vector<std::pair<int, cplx>>> ladj(nl);  // (r, w)
        for (auto &e : edges) {
            if (e.second == cplx(0) || e.first.second.empty()) continue;
            int l = lidx[e.first.first], r = ridx[e.first.second];
            adj[l].push_back(r);
            ladj[l].push_back({r, e.second});
        }
        auto cover = min_vertex_cover(nl, nr, adj);
        // channel ids: 0 identity, 1 inside, then left cover, then right cover
        std::vector<int> lch(nl, -1), rch(nr, -1);
        int nch = 2;
        for (int l = 0; l < nl; ++l)
            if (cover.first[l]) lch[l] = nch++;
        for (int r = 0; r < nr; ++r)
            if (cover.second[r]) rch[r] = nch++;
        op.n_ch[c] = nch;
        op.inside_used[c] = !inside.empty();
        // channel combinations: channel -> list of (in key, weight)
        std::vector<std::vector<std::pair<std::vector<int>, cplx>>> combo(nch);
        combo[1] = inside;
        std::vector<CTerm> next = untouched;
        if (!inside.empty()) next.push_back({cplx(1.0), SlotVec{{c, 1}}});
        for (int l = 0; l < nl; ++l) {
            if (lch[l] >= 0) {
                combo[lch[l]].push_back({lkeys[l], cplx(1.0)});
                for (auto &rw : ladj[l]) {
                    CTerm nt{rw.second, rkeys[rw.first]};
                    nt.slots.push_back({c, lch[l]});
                    std::sort(nt.slots.begin(), nt.slots.end());
                    next.push_back(nt);
                }
            } else {
                for (auto &rw : ladj[l]) combo[rch[rw.first]].push_back({lkeys[l], rw.second});
            }
        }
        for (int r = 0; r < nr; ++r)
            if (rch[r] >= 0) {
                CTerm nt{cplx(1.0), rkeys[r]};
                nt.slots.push_back({c, rch[r]});
                std::sort(nt.slots.begin(), nt.slots.end());
                next.push_back(nt);
            }
        terms.swap(next);
        // node entries
        auto &ent = op.entries[c];
        if (leaf) {
            int li = t.leaf_index[c];
            int d = t.local_dim[c];
            op.leafU[li].assign(nch, {});
            for (int b = 1; b < nch; ++b) {
                if (combo[b].empty()) continue;
                std::vector<cplx> U((size_t)d * d, cplx(0));
                for (auto &kw : combo[b]) {
                    const auto &m = s.op_mat[kw.first[0]];
                    for (size_t i = 0; i < U.size(); ++i) U[i] += kw.second * m[i];
                }
                op.leafU[li][b] = U;
                ent.push_back({cplx(1.0), {b}, b});
            }
        } else {
            for (int b = 1; b < nch; ++b)
                for (auto &kw : combo[b]) ent.push_back({kw.second, kw.first, b});
        }
        if (op.outside_used[c]) ent.push_back({cplx(1.0), std::vector<int>(leaf ? 1 : kids.size(), -1), 0});
    }
    // root: every remaining term lives on the root's child bonds
    {
        const auto &kids = t.kids[t.root];
        std::map<std::vector<int>, cplx> acc;
        for (auto &ct : terms) {
            std::vector<int> in(kids.size(), -1);
            for (auto &sv : ct.slots) {
                auto it = std::find(kids.begin(), kids.end(), sv.first);
                if (it == kids.end()) throw Error(TTN_E_INVALID, "internal: unprocessed slot at root");
                in[it - kids.begin()] = sv.second;
            }
            acc[in] += ct.coef;
        }
        for (auto &kv : acc)
            if (kv.second != cplx(0)) op.entries[t.root].push_back({kv.second, kv.first, 0});
    }
    return op;
}

bool same_tree_operator_structure(const TreeOp &a, const TreeOp &b) {
    if (a.n_ch != b.n_ch || a.inside_used != b.inside_used || a.outside_used != b.outside_used) return false;
    if (a.entries.size() != b.entries.size() || a.leafU.size() != b.leafU.size()) return false;
    for (size_t z = 0; z < a.entries.size(); ++z) {
        const auto &ea = a.entries[z], &eb = b.entries[z];
        if (ea.size() != eb.size()) return false;
        for (size_t e = 0; e < ea.size(); ++e)
            if (ea[e].slot != eb[e].slot || ea[e].bp != eb[e].bp) return false;
    }
    for (size_t l = 0; l < a.leafU.size(); ++l) {
        if (a.leafU[l].size() != b.leafU[l].size()) return false;
        for (size_t ch = 0; ch < a.leafU[l].size(); ++ch)
            if (a.leafU[l][ch].empty() != b.leafU[l][ch].empty()) return false;
    }
    return true;
}

// Greedy: every (item, position) gives a candidate key (group, number of
// factors, position, slots, ids of the other factors); the largest candidate
// sets are taken first and every item joins at most one set.
std::vector<MergeSet> plan_entry_merge(const std::vector<MergeItem> &items) {
    const int ne = (int)items.size();
    std::map<std::vector<int64_t>, std::vector<int>> buckets;
    for (int e = 0; e < ne; ++e) {
        const MergeItem &E = items[e];
        for (int f = 0; f < E.nf; ++f) {
            std::vector<int64_t> key = {E.group, E.nf, f};
            for (int g = 0; g < E.nf; ++g) {
                key.push_back(E.slot[g]);
                if (g != f) key.push_back(E.id[g]);
            }
            buckets[key].push_back(e);
        }
    }
    std::vector<std::pair<int, const std::vector<int64_t> *>> order;
    for (auto &kv : buckets)
        if (kv.second.size() >= 2) order.push_back({(int)kv.second.size(), &kv.first});
    std::stable_sort(order.begin(), order.end(), [](const auto &a, const auto &b) { return a.first > b.first; });
    std::vector<char> used(ne, 0);
    std::vector<MergeSet> out;
    for (auto &o : order) {
        MergeSet m{(int)(*o.second)[2], {}};
        for (int e : buckets[*o.second])
            if (!used[e]) m.members.push_back(e);
        if (m.members.size() < 2) continue;
        for (int e : m.members) used[e] = 1;
        out.push_back(std::move(m));
    }
    return out;
}

}  // namespace ttn
