/*
 * ttn.h - C boundary of the MI355X (gfx950) one-site TDVP library for tree
 * tensor networks (multilayer MCTDH), after pyTTN (arXiv 2503.15460).
 *
 * The calls follow the paper's problem statement:
 *   ttn_create     - the tree tensor network ansatz (Sec. II A: a tree of
 *                    coefficient tensors, the number of single-particle
 *                    functions n on every bond, primitive dimensions at leaves);
 *   ttn_set_sop    - the sum-of-product generator H = sum_r c_r prod h_{a,r}
 *                    (Sec. II B 1, SOP equation);
 *   ttn_set_coefficients - new coefficients c_r for the same terms between
 *                    steps (time-dependent coefficients, Sec. II B);
 *   ttn_step       - the projector-splitting solution of the local equation of
 *                    motion dA/dt = -i sum_r c_r h_r A H_r (Sec. II C) over dt;
 *   ttn_ground_sweeps - ground-state optimisation by the same single-site
 *                    sweep with lowest-eigenvector node updates (Sec. II C,
 *                    DMRG on trees);
 *   ttn_observe    - autocorrelation a(t) (Sec. IV A), populations and spin
 *                    expectation values (Secs. IV, V A), and the HEOM reduced
 *                    density matrix by vacuum projection (SI, FP-HEOM section).
 *
 * Conventions common to every call
 *   - Every function returns a ttn_status: TTN_OK (0) or a negative error.
 *     After an error, ttn_last_error() returns a message; the state of the
 *     handle is unchanged, with two exceptions: TTN_E_DEVICE leaves the handle
 *     unusable (destroy it), and ttn_set_sop failing with TTN_E_OOM leaves the
 *     handle without an operator (set one again before stepping or observing).
 *     A sweep stopped by a failed kernel launch reports TTN_E_DEVICE.
 *   - All pointer arguments are HOST pointers owned by the caller.  The library
 *     copies what it needs during the call and never keeps a caller pointer.
 *   - Complex numbers are two consecutive doubles (re, im).
 *   - The library owns all device memory of a handle.  A handle is not thread
 *     safe and runs all its work on one HIP stream (ttn_options.hip_stream, for
 *     example a PyTorch stream, or the null stream).
 *   - Time evolution is d/dt psi = -i G psi (G = H/hbar for unitary models).
 *
 * Tensor layout (used by ttn_get_state / ttn_set_state)
 *   Node z holds A^z with the children's indices first, in increasing node id,
 *   and the index toward the parent last; leaves hold (d, n); the root's parent
 *   index has dimension 1.  Row-major, complex interleaved, nodes concatenated
 *   in node-id order.
 */
#ifndef TTN_H
#define TTN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t ttn_status;
#define TTN_OK 0
#define TTN_E_INVALID (-1) /* bad argument, or hermitian=1 with a non-Hermitian G */
#define TTN_E_TREE (-2)    /* parent array is not a single rooted tree */
#define TTN_E_DIMS (-3)    /* local/bond dimensions invalid or buffer size mismatch */
#define TTN_E_OOM (-4)     /* device allocation failed or workspace too small */
#define TTN_E_DEVICE (-5)  /* HIP runtime error; the handle is unusable */
#define TTN_E_NOCONV (-6)  /* local exponential did not converge */
#define TTN_E_STATE (-7)   /* call out of order (e.g. ttn_step before ttn_set_sop) */

/* Precision of the H_eff / environment contractions.  TTN_FP32: the operator
 * stages, group sums and environment contractions of the multi-kernel path run
 * in complex FP32 with FP32 accumulation (the FP64 state is rounded when read,
 * results are widened when written); node tensors, environments, QR gauge
 * shifts, Krylov orthogonalisation and the small projected exponential stay
 * FP64, and local problems of at most 1024 elements keep the fused FP64 solver.
 * From a full-rank state observables stay within about 1e-6 of FP64 over tens
 * of steps; from a product state the rank-deficient first gauge shifts amplify
 * rounding of any precision (FP64 included) to about 1e-3 in the first steps. */
#define TTN_FP64 0
#define TTN_FP32 1
/* TTN_BF16X3: as TTN_FP32, and the dense operator stages whose factors have
 * dimensions 24..64 run on the matrix cores with split precision: each FP32
 * operand is split into bf16 hi + lo and products are taken as hi*hi + hi*lo +
 * lo*hi with FP32 accumulation (about 1e-5 relative per contraction). */
#define TTN_BF16X3 2

/* observable kinds for ttn_observe */
#define TTN_OBS_EXPECT 0      /* <Psi| prod_i op_ids[i] |Psi>, ops on distinct leaves */
#define TTN_OBS_NORM 1        /* <Psi|Psi> */
#define TTN_OBS_ENERGY 2      /* <Psi|G|Psi> */
#define TTN_OBS_OVERLAP_T0 3  /* a(t) = <Psi(0)|Psi(t)>, Psi(0) = last state set */
#define TTN_OBS_BILINEAR 4    /* (b|Psi) = sum_x b_x Psi_x, b a product vector (no conj.) */

typedef struct ttn_ctx *ttn_t;
typedef struct ttn_batch_ctx *ttn_batch_t;

typedef struct {
    int32_t precision;      /* TTN_FP64, TTN_FP32 or TTN_BF16X3 */
    double krylov_tol;      /* local exponential error target, relative (0 -> 1e-13, FP32/BF16X3: 1e-10) */
    int32_t krylov_mmax;    /* max Krylov dimension per solve (0 -> 40) */
    int32_t hermitian;      /* 1: Lanczos (G must be Hermitian), 0: Arnoldi */
    void *hip_stream;       /* hipStream_t for all work of the handle, NULL = null stream */
    void *workspace;        /* optional DEVICE buffer (caller-owned, on `device`, >= 256-byte aligned)
                               that holds the sweep's scratch: contraction temporaries, Krylov
                               bases, QR work arrays, the step snapshot.  NULL: the library
                               allocates the scratch itself.  Must stay valid until
                               ttn_destroy; ttn_set_sop fails with TTN_E_OOM when
                               workspace_bytes is below what the operator needs
                               (ttn_workspace_size reports it, also after that failure). */
    size_t workspace_bytes; /* size of `workspace` in bytes */
    int32_t use_graph;      /* 1: each step is captured into a hipGraph once per (dt, Krylov dimension
                               hints) and replayed from then on (one graph launch per step instead
                               of hundreds of kernel launches); the gauge QRs then take the
                               non-cooperative kernels.  A NULL hip_stream is replaced by a stream
                               of the handle's own.  Not with spawn_tol > 0 (TTN_E_INVALID). */
    int32_t autotune;       /* 1: ttn_set_sop times every register tile of the tiled operator stages on
                               the handle's own programs and records the fastest in the process-wide
                               tile table (see ttn_tile_table_*); stages already in the table are not
                               timed again.  Results do not depend on the tile. */
    int32_t device;         /* HIP device ordinal */
    uint64_t seed;          /* seeds the start vectors of the subspace expansion's Krylov iteration */
    double spawn_tol;       /* subspace expansion (Sec. II D): 0 = fixed bonds; > 0: when the sweep
                               crosses a bond, new single-particle functions (going up) or single
                               hole functions (going down) are added with zero coefficients along
                               the dominant singular vectors sigma_s of the two-site residual
                               while |dt/2| sigma_s >= spawn_tol, up to bond_max */
    const int32_t *bond_max;/* [n_nodes] largest bond each bond may grow to (read by ttn_create,
                               clamped like bond_dim; NULL: no growth).  Device memory is
                               allocated for these bonds from the start. */
} ttn_options;

/* Fill *opt with the defaults (FP64, tol 0 = the precision's default, mmax 40,
 * Hermitian). */
void ttn_default_options(ttn_options *opt);

/* Create a tree tensor network.
 *   n_nodes   number of nodes (>= 2)
 *   parent    [n_nodes] parent id, exactly one -1 (the root); children of a node
 *             are ordered by increasing node id; a node has at most 7 children
 *             (node tensors have at most 8 indices)
 *   local_dim [n_nodes] primitive dimension d > 0 for leaves, 0 for interior nodes
 *   bond_dim  [n_nodes] requested number of SPFs on the bond to the parent
 *             (ignored for the root).  Requests the tree cannot support are
 *             clamped: n = min(request, prod dims below, prod dims above), then
 *             lowered until every matricisation has rows >= columns.  The
 *             effective values are returned by ttn_get_info; effective bonds
 *             above 64 are refused (TTN_E_DIMS).
 * Errors: TTN_E_TREE (not a tree, or a node with more than 7 children),
 *         TTN_E_DIMS (leaf/interior dims invalid), TTN_E_INVALID (options),
 *         TTN_E_DEVICE.  On success *out receives the handle. */
ttn_status ttn_create(int32_t n_nodes, const int32_t *parent, const int32_t *local_dim,
                      const int32_t *bond_dim, const ttn_options *opt, ttn_t *out);

/* Set the SOP generator G = sum_r coeff[r] prod_{o in term r} op_o.
 *   n_ops, op_leaf[n_ops]      leaf each operator acts on
 *   op_offset[n_ops+1]         offsets (in complex elements) into op_data
 *   op_data                    dense d x d row-major complex matrices
 *   n_terms, coeff[2*n_terms]  complex coefficients
 *   term_ptr[n_terms+1], term_ops[...]  operator ids of each term, at most one
 *                              per leaf, at least one per term
 * The generator is compiled into a hierarchical SOP (sparse tree operator)
 * whose bond operators are chosen by a minimum vertex cover of the bipartite
 * term graph of every bond (Sec. II B 2).  With hermitian=1, G is checked for
 * Hermiticity: ||G - G^dag||_F <= 1e-7 ||G||_F, evaluated from the leaf
 * operators and coefficients (traces of products of leaf operators, never the
 * dense matrix; operators on one leaf that agree to 1e-12 relative count as
 * one), and TTN_E_INVALID is returned if it fails.  Device environments are
 * rebuilt if a state is already set.  Argument errors (TTN_E_INVALID,
 * TTN_E_DIMS) leave the handle unchanged; after TTN_E_OOM or TTN_E_DEVICE it
 * has no operator.
 * Errors: TTN_E_INVALID, TTN_E_DIMS, TTN_E_OOM (device memory, or the
 * caller's workspace too small), TTN_E_DEVICE. */
ttn_status ttn_set_sop(ttn_t h, int32_t n_ops, const int32_t *op_leaf, const int64_t *op_offset,
                       const double *op_data, int32_t n_terms, const double *coeff,
                       const int64_t *term_ptr, const int32_t *term_ops);

/* Time-dependent coefficients (Sec. II B: the operator front-end allows
 * coefficients that depend on time; Sec. II E 2: the interaction-picture chain
 * form of the spin-boson model has time-dependent couplings g_k(t)).  Replaces the coefficients c_r of the
 * terms given to ttn_set_sop (same operators, same terms, same order) for the
 * following steps.  coeff (host): n_terms complex values, 2 doubles each.  A
 * step then propagates with the coefficients frozen: a caller integrating
 * H(t) sets c_r(t + dt/2) before every step of dt (the midpoint rule, second
 * order like the symmetric sweep).
 * The operator is compiled again on the host.  When its structure is the same
 * (the same channels on every bond and the same entries at every node, which
 * holds while no coefficient or sum of coefficients becomes or stops being
 * exactly zero), the leaf channel operators and the coefficient tables on the
 * device are overwritten in place, with no device allocation; otherwise the
 * operator is rebuilt as by ttn_set_sop.  Either way the state is kept and its
 * environments are rebuilt.  Step graphs (use_graph) stay valid when only
 * values changed and the band of every leaf channel operator is the same (the
 * graphs read the rewritten tables); otherwise they are recorded again at the
 * next step.
 * rebuilt (host, may be NULL) receives 1 if the operator was rebuilt, else 0.
 * Errors: TTN_E_STATE (no SOP yet), TTN_E_INVALID (n_terms differs from the
 * operator's, null coeff, a coefficient not finite, or hermitian = 1 and the
 * generator with these coefficients fails the Hermiticity check of
 * ttn_set_sop; the operator in place is then unchanged), TTN_E_OOM (rebuild
 * only; the handle then has no operator), TTN_E_DEVICE. */
ttn_status ttn_set_coefficients(ttn_t h, int32_t n_terms, const double *coeff, int32_t *rebuilt);

/* Product initial state (the Hartree product the paper starts its
 * propagations from, Secs. III and IV A, where the unoccupied single-particle
 * functions are included in the initial tensors).  leaf_vecs holds one complex
 * vector of length d per leaf, concatenated in increasing leaf id.  The
 * unoccupied functions are completed with unit vectors (leaf: modified
 * Gram-Schmidt of e_0, e_1, ... against the given vector, skipping residuals
 * below 1e-6; interior node: the first n columns of the identity; root:
 * e_(0..0)).
 * This state becomes Psi(0) for TTN_OBS_OVERLAP_T0.
 * Errors: TTN_E_STATE (no SOP yet), TTN_E_INVALID (zero vector), TTN_E_DEVICE. */
ttn_status ttn_set_product_state(ttn_t h, const double *leaf_vecs);

/* Advance n_steps steps of dt (dt may be negative).  One step is the symmetric
 * projector-splitting sweep S(dt/2) S*(dt/2) with the two root forward half
 * steps merged (2N-1 forward, 2(N-1) backward local exponentials, 4(N-1) QRs).
 * n_steps = 0 does nothing.
 * Errors: TTN_E_INVALID (n_steps < 0, dt not finite), TTN_E_STATE,
 * TTN_E_NOCONV (state restored to before the failed step), TTN_E_DEVICE. */
ttn_status ttn_step(ttn_t h, double dt, int32_t n_steps);

/* Ground-state optimisation (Sec. II C: the single-site machinery also serves
 * ground states, one-site alternating least squares, DMRG on trees): n_sweeps
 * sweeps over the nodes in the order of one ttn_step (S, the root, S*), every
 * node's tensor replaced by the eigenvector of the lowest eigenvalue of its
 * local effective generator (Lanczos on the state's current tensor, FP64
 * orthogonalisation; the fused solver restarts from the Ritz vector up to 8
 * times until the residual |beta y_m| falls below the Krylov tolerance, the
 * multi-kernel path takes one pass of the largest Krylov dimension) and the R
 * factor of every QR gauge move absorbed unchanged (no backward bond step).
 * The state stays normalised; Psi(0) and the propagation time are untouched.
 * energy (host, 1 double) receives <Psi|G|Psi> / <Psi|Psi> after the last
 * sweep; unconverged (host, may be NULL) the number of fused local solves
 * whose residual stayed above the tolerance.  Needs a Hermitian generator
 * (options.hermitian = 1) and no subspace expansion; precision as set by
 * options.precision (the H_eff contractions in FP32 in the mixed modes).
 * Errors: TTN_E_INVALID (n_sweeps < 1, null energy, non-Hermitian generator,
 * subspace expansion on, handle in a batch), TTN_E_STATE (no SOP or state),
 * TTN_E_DEVICE. */
ttn_status ttn_ground_sweeps(ttn_t h, int32_t n_sweeps, double *energy, int32_t *unconverged);

/* Observables; out receives complex values (2 doubles each), caller-owned.
 *   TTN_OBS_EXPECT     n op ids (distinct leaves) -> 1 value
 *   TTN_OBS_NORM       n = 0 -> 1 value
 *   TTN_OBS_ENERGY     n = 0 -> 1 value
 *   TTN_OBS_OVERLAP_T0 n = 0 -> 1 value
 *   TTN_OBS_BILINEAR   op_ids unused; vecs = one complex vector per leaf
 *                      (concatenated by leaf id), passed in `vecs` -> 1 value
 * Values are raw (not divided by the norm).
 * Errors: TTN_E_STATE, TTN_E_INVALID, TTN_E_DEVICE. */
ttn_status ttn_observe(ttn_t h, int32_t kind, int32_t n, const int32_t *op_ids,
                       const double *vecs, double *out);

/* Apply the effective generator of the root node to x (complex, size of the
 * root tensor) -> y, using the current environments.  Diagnostic entry point
 * for brute-force checks of the contraction kernels.
 * Errors: TTN_E_STATE, TTN_E_DEVICE. */
ttn_status ttn_apply_root_heff(ttn_t h, const double *x, double *y);

/* Info: effective bond dims [n_nodes]; counters[8] = {steps, forward solves,
 * backward solves, total Krylov matvecs, algorithmic H_eff flops (8 per complex
 * MAC), bytes of device memory in use, tree-operator entries, redo count}.
 * Either pointer may be NULL. */
ttn_status ttn_get_info(ttn_t h, int32_t *effective_bond_dim, int64_t *counters);

/* Local exponentials of the last completed step, in sweep order: for each
 * solve i < *n_solves (at most max_solves written) node[i] is the node of a
 * forward solve or the node below the bond of a backward solve, forward[i] is
 * 1 or 0, matvecs[i] the effective-generator applications it took.  Any
 * output may be NULL.  Errors: TTN_E_STATE (no step yet). */
ttn_status ttn_get_step_solves(ttn_t h, int32_t max_solves, int32_t *node, int32_t *forward, int32_t *matvecs,
                               int32_t *n_solves);

/* Bytes of device scratch the handle's current operator needs (the size a
 * caller-provided ttn_options.workspace must have); 0 before ttn_set_sop.  Also
 * valid after ttn_set_sop failed with TTN_E_OOM. */
ttn_status ttn_workspace_size(ttn_t h, size_t *bytes);

/* Size in bytes (complex128 elements * 16) of the state for get/set_state. */
ttn_status ttn_state_size(ttn_t h, size_t *bytes);

/* Copy all node tensors to/from a host buffer of exactly ttn_state_size bytes.
 * ttn_set_state expects every non-root node to be an isometry toward its
 * parent (the orthogonality centre at the root); it rebuilds the environments
 * and makes the state Psi(0).  Errors: TTN_E_DIMS, TTN_E_STATE, TTN_E_DEVICE. */
ttn_status ttn_get_state(ttn_t h, double *buf, size_t bytes);
ttn_status ttn_set_state(ttn_t h, const double *buf, size_t bytes);

/* Kernel launch profile.  ttn_profile_begin switches on timing of every
 * kernel launch of the library and clears earlier records: ordinary launches
 * carry a start and a stop event stamped from the dispatch itself, the
 * cooperative QR reads the device's constant-rate clock at its first
 * work-group start and last end (adds a little overhead per launch).
 * ttn_profile_end synchronises the device, switches the timing off and writes
 * one row per kernel name: launches, summed duration, and the algorithmic
 * flops (8 per complex MAC) and bytes of those launches as modelled by the
 * library.  n_rows receives the number of rows (at most max_rows written).
 * The profiler is process wide (all handles).  Errors: TTN_E_DEVICE. */
typedef struct {
    char name[48];
    int64_t calls;
    double total_ms;
    double flops;
    double bytes;
} ttn_kernel_stat;
ttn_status ttn_profile_begin(void);
ttn_status ttn_profile_end(ttn_kernel_stat *rows, int32_t max_rows, int32_t *n_rows);

/* Batches: many independent instances (trajectories, parameter sweeps, uneven
 * trees and bond dimensions) advanced together.  Each instance keeps its own
 * tensors, operator and Krylov hints; the batch gives the instances
 * n_streams HIP streams (round robin; <= 0 -> 8, at most one per instance,
 * default priority), enqueues one step of every instance before waiting for
 * any, so that their sweeps overlap on the device.  Results are those of
 * ttn_step on each instance alone.
 *   ttn_batch_create: insts[n] are created handles (same device, each in at
 *     most one batch, not repeated); while in the batch an instance runs on a
 *     batch stream, ttn_batch_destroy gives it back its own.  The handles stay
 *     owned by the caller; destroying one removes it from its batch.
 *     Errors: TTN_E_INVALID, TTN_E_DEVICE.
 *   ttn_batch_step: n_steps steps; dt[i] is instance i's step (insertion
 *     order).  Every instance needs an operator and a state.  On an error the
 *     instances have completed different numbers of steps; the failing
 *     instance is named by ttn_batch_last_error and keeps the state of
 *     ttn_step's error behaviour.  Errors: those of ttn_step.
 *   ttn_batch_last_error: message of the last failed batch call (NULL batch:
 *     last error of this thread), owned by the library.
 */
ttn_status ttn_batch_create(int32_t n, ttn_t const *insts, int32_t n_streams, ttn_batch_t *out);
ttn_status ttn_batch_step(ttn_batch_t b, const double *dt, int32_t n_steps);
/* Lockstep mode (on = 1; 0 returns to the streams): every instance runs on the
 * batch's first stream and a step proceeds in sweep layers: in layer j every
 * instance runs its sweep's operations (QRs with their environment updates,
 * absorptions, multi-kernel local exponentials) up to its j-th local
 * exponential that fits the fused one-work-group solver, and those
 * exponentials of all instances go out as ONE grouped launch (one work-group
 * per instance).  Results are those of ttn_step on each instance.
 * Not with subspace expansion.  After a device error every instance of the
 * batch is unusable.  Errors: TTN_E_INVALID, TTN_E_DEVICE. */
ttn_status ttn_batch_set_lockstep(ttn_batch_t b, int32_t on);
const char *ttn_batch_last_error(ttn_batch_t b);
void ttn_batch_destroy(ttn_batch_t b);

/* Per-handle message of the last error (NULL handle: last error of this
 * thread).  The string is owned by the library. */
const char *ttn_last_error(ttn_t h);

/* Release all resources of the handle. */
void ttn_destroy(ttn_t h);

/* The process-wide tile table of the operator stages (filled by autotune = 1,
 * consulted by every handle): save writes it as JSON (one entry per line:
 * ["shape key", rows per thread, row groups, microseconds]), load merges such a
 * file into it (entries with tiles this build lacks are skipped) and returns
 * the number read, clear empties it.  Host only.
 * Errors: TTN_E_INVALID (file cannot be opened). */
ttn_status ttn_tile_table_save(const char *path);
ttn_status ttn_tile_table_load(const char *path, int32_t *n_loaded);
ttn_status ttn_tile_table_size(int64_t *n_entries);
void ttn_tile_table_clear(void);

/* Release the library's process-wide device resources (the launch profiler's
 * clock slots and event pool).  Call after destroying every handle and before
 * the HIP runtime is torn down (e.g. from an exit hook); the library stays
 * usable and re-creates them on demand. */
void ttn_release_process_resources(void);

#ifdef __cplusplus
}
#endif

#endif /* TTN_H */
