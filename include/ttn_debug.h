/*
 * ttn_debug.h - host-only diagnostic entry points of the TTN library.
 * They allocate no device memory and run on machines without a GPU.
 */
#ifndef TTN_DEBUG_H
#define TTN_DEBUG_H

#include "ttn.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Compile the SOP generator of a tree (arguments as for ttn_create and
 * ttn_set_sop) into the library's sparse tree operator (hierarchical SOP,
 * Sec. II B 2 of the paper) and assemble it back into a dense matrix over the
 * leaves in depth-first order (children in increasing id).  `out` receives
 * dim*dim complex values (row-major) where dim = prod of leaf dims, which must
 * not exceed max_dim.  n_entries (may be NULL) receives the number of
 * tree-operator entries (hSOP channels summed over nodes).
 * Errors: TTN_E_TREE, TTN_E_DIMS, TTN_E_INVALID (including dim > max_dim). */
ttn_status ttn_debug_dense_tree_operator(int32_t n_nodes, const int32_t *parent, const int32_t *local_dim,
                                         int32_t n_ops, const int32_t *op_leaf, const int64_t *op_offset,
                                         const double *op_data, int32_t n_terms, const double *coeff,
                                         const int64_t *term_ptr, const int32_t *term_ops, int64_t max_dim,
                                         double *out, int64_t *n_entries);

/* ||G - G^dag||_F / ||G||_F of an SOP generator (arguments as for ttn_create
 * and ttn_set_sop), the quantity ttn_set_sop checks when hermitian = 1,
 * computed from traces of products of leaf operators; host only.
 * Errors: TTN_E_TREE, TTN_E_DIMS, TTN_E_INVALID. */
ttn_status ttn_debug_hermiticity_defect(int32_t n_nodes, const int32_t *parent, const int32_t *local_dim,
                                        int32_t n_ops, const int32_t *op_leaf, const int64_t *op_offset,
                                        const double *op_data, int32_t n_terms, const double *coeff,
                                        const int64_t *term_ptr, const int32_t *term_ops, double *defect);

/* Size of the compiled sparse tree operator per node (host only), each output
 * [n_nodes] and optional (NULL):
 *   n_channels    channels on the bond above each node (the root: 1)
 *   n_entries     operator entries of each node (hierarchical SOP)
 *   n_merged      products the node's effective generator applies after the
 *                 node-form compression (products equal in every factor but
 *                 one summed into one; Sec. II B 2, terms (B) and (C))
 *   n_sop_terms   SOP terms crossing the bond above each node (a plain SOP
 *                 keeps one SPO and one mean field per such term; root: 0)
 * Arguments as for ttn_create / ttn_set_sop.
 * Errors: TTN_E_TREE, TTN_E_DIMS, TTN_E_INVALID. */
ttn_status ttn_debug_tree_operator_stats(int32_t n_nodes, const int32_t *parent, const int32_t *local_dim,
                                         int32_t n_ops, const int32_t *op_leaf, const int64_t *op_offset,
                                         const double *op_data, int32_t n_terms, const double *coeff,
                                         const int64_t *term_ptr, const int32_t *term_ops, int32_t *n_channels,
                                         int32_t *n_entries, int32_t *n_merged, int32_t *n_sop_terms);

/* Number of step graphs a handle with use_graph = 1 has captured so far (a
 * replayed step captures nothing).  Errors: TTN_E_INVALID. */
ttn_status ttn_debug_graph_captures(ttn_t h, int64_t *captures);

/* Effective (clamped) bond dimensions for a tree, host only.
 * Errors: TTN_E_TREE, TTN_E_DIMS. */
ttn_status ttn_debug_clamp_bonds(int32_t n_nodes, const int32_t *parent, const int32_t *local_dim,
                                 const int32_t *bond_dim, int32_t *effective);

/* Householder QR of a dense complex matrix on the GPU with the library's own
 * kernels (LAPACK convention with the zero-snap of the sweep's gauge shifts).
 * m (x) in row-major (rows, cols), rows >= cols, cols <= 64; q_out receives
 * (rows, cols) and r_out (cols, cols), all complex interleaved host buffers.
 * variant 0: one work-group; 1: many work-groups (one launch per column);
 * 2: many work-groups in one cooperative launch (grid-wide barriers);
 * 3: the Cholesky route (Cholesky QR twice, reflector signs from an LU of the
 *    leading block), the variant-1 kernels taking over when the matrix is
 *    outside its range (rank-deficient, near the zero-snap, ill-conditioned);
 * 4: the Cholesky route alone: TTN_E_NOCONV when the matrix is outside its range.
 * Uses device 0 and the null stream; allocates and frees its own device memory.
 * Errors: TTN_E_INVALID (shape), TTN_E_NOCONV (variant 4), TTN_E_DEVICE. */
ttn_status ttn_debug_qr(int64_t rows, int32_t cols, const double *m, int32_t variant, double *q_out,
                        double *r_out);

#ifdef __cplusplus
}
#endif

#endif /* TTN_DEBUG_H */
