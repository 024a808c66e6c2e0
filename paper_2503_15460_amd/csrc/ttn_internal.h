// Internal host-side structures of the TTN library (not part of the C boundary).
#pragma once

#include <complex>
#include <cstdint>
#include <stdexcept>
#include <string>
#include <vector>

#include "ttn.h"

namespace ttn {

using cplx = std::complex<double>;

// Error carrying a ttn_status code; converted to a return value at the boundary.
struct Error : std::runtime_error {
    ttn_status code;
    Error(ttn_status c, const std::string &m) : std::runtime_error(m), code(c) {}
};

// Children per node: node tensors have at most 8 indices (children + parent).
constexpr int MAX_CHILDREN = 7;

// Tree geometry after validation and bond clamping.
struct Tree {
    int n = 0, root = -1;
    std::vector<int> parent, local_dim, bond;  // bond: effective, root = 1
    std::vector<std::vector<int>> kids;         // children in increasing id
    std::vector<int> postorder;                 // children before parents
    std::vector<int> leaves;                    // increasing id
    std::vector<int> leaf_index;                // node -> position in leaves (-1)
    // slot dims of node tensors: children bonds (or the physical index of a
    // leaf) followed by the parent bond (1 for the root)
    std::vector<std::vector<int>> dims;
    std::vector<int64_t> size;  // number of elements of each node tensor
    // capacity: the largest bond each bond may reach (subspace expansion), with
    // the node shapes and sizes at capacity; equal to the bonds without one
    std::vector<int> cap;
    std::vector<std::vector<int>> capdims;
    std::vector<int64_t> capsize;
    // recompute dims and size from bond
    void update_dims();
};

// bond_max (may be NULL): per node, the largest bond the subspace expansion
// may grow that bond to (clamped like the requests; never below the bond)
Tree build_tree(int n, const int32_t *parent, const int32_t *local_dim, const int32_t *bond_req,
                const int32_t *bond_max = nullptr);

// One nonzero of a node's sparse tree-operator tensor (one hSOP channel).
//   slot[k]: channel id on the bond of child k (>= 1), or -1 for the identity;
//            for a leaf slot[0] is the index of its primitive operator U (>= 1)
//            or -1 (identity)
//   bp     : channel id on the node's own bond (root: always 0)
struct OpEntry {
    cplx coef;
    std::vector<int> slot;
    int bp;
};

// Sparse tree operator (hierarchical SOP).  On every bond, channel 0 is the
// identity on the subtree side (its mean field collects every term not
// touching the subtree) and channel 1 collects the terms lying entirely inside
// the subtree (its mean field is the identity).  Channels >= 2 come from the
// minimum vertex cover of the bipartite graph of the crossing terms.
struct TreeOp {
    std::vector<std::vector<OpEntry>> entries;  // per node
    std::vector<int> n_ch;                      // channels on the bond above each node (root 1)
    std::vector<char> inside_used;              // channel 1 carries terms
    std::vector<char> outside_used;             // channel 0 carries terms (some term misses the subtree)
    // per leaf, per channel: d*d operator (channel 0 empty: identity)
    std::vector<std::vector<std::vector<cplx>>> leafU;
};

struct SopInput {
    int n_ops = 0, n_terms = 0;
    std::vector<int> op_leaf;
    std::vector<std::vector<cplx>> op_mat;  // dense d*d row-major
    std::vector<cplx> coeff;
    std::vector<std::vector<int>> term_ops;
};

SopInput read_sop(const Tree &t, int32_t n_ops, const int32_t *op_leaf, const int64_t *op_offset,
                  const double *op_data, int32_t n_terms, const double *coeff,
                  const int64_t *term_ptr, const int32_t *term_ops);

// ||G - G^dag||_F / ||G||_F from the leaf operators and coefficients (leaf
// operators that agree to `cluster` relative are identified first).
double sop_hermiticity_defect(const SopInput &s, double cluster);
// True if ||G - G^dag||_F <= rtol ||G||_F.
bool sop_is_hermitian(const SopInput &s, double rtol = 1e-7);

TreeOp compile_tree_operator(const Tree &t, const SopInput &s);
// True if two compiled operators differ at most in values: the same channels
// on every bond, the same entries (slots and parent channel) at every node and
// the same non-empty leaf channel operators.  Programs, environments and
// scratch built for one then fit the other.
bool same_tree_operator_structure(const TreeOp &a, const TreeOp &b);

// Node form of the operator (Sec. II B 2, terms (B) and (C)): products that
// share every factor but one are summed into one product whose remaining
// factor is the coefficient-weighted sum of theirs.  An item is one product:
// its group (products of different groups are never combined), and per
// factor position f the tensor slot and an identity of the factor (equal ids
// mean the same matrix).  The plan lists the sets to combine, each with the
// factor position f that is summed; items in no set stay as they are.
struct MergeItem {
    int group = 0, nf = 0;
    int slot[8] = {0};
    int64_t id[8] = {0};
};
struct MergeSet {
    int f;
    std::vector<int> members;
};
std::vector<MergeSet> plan_entry_merge(const std::vector<MergeItem> &items);

}  // namespace ttn
