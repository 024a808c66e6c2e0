// Device-side data structures and kernel launchers of the TTN library (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

namespace ttn {

constexpr int MAXD = 8;        // slots of a node tensor (children + parent)
constexpr int MAXF = 8;        // non-identity factors of one operator entry
constexpr int SMALL_MAX = 1024;   // local problems up to this size use the fused solver
constexpr int SMALL_MMAX = 24;    // Krylov dimension limit of the fused solver (LDS budget; sub-steps beyond)
constexpr int SMALL_THREADS = 1024;
constexpr int VEC_BLOCKS = 256;   // work-groups of the multi-kernel vector operations
constexpr int VEC_THREADS = 256;
// QR zero-snap: Householder sub-columns with norm <= QR_SNAP * |M|_F are treated
// as exactly zero, so that rounding noise in structurally empty columns of a
// product state cannot choose the completion of a rank-deficient factor.
constexpr double QR_SNAP = 1e-12;

// Geometry of a node tensor: slot s has L[s] = prod dims[<s], R[s] = prod dims[>s].
struct Geom {
    int D;
    int dims[MAXD];
    int64_t L[MAXD];
    int64_t R[MAXD];
    int64_t N;
};

// One operator entry: coef * (x)_f M_f applied on slots slot[f] (ascending).
// Factor f is banded: M[i][j] == 0 unless i - lo[f] <= j <= i + hi[f] (dense
// factors carry lo = hi = n - 1).  Leaf operators in a number basis (ladder,
// position, number operators and their sums) are detected as banded.
struct DevEntry {
    double2 coef;
    int nf;
    int group;
    int src;  // input slice the entry reads (ProgView::in_stride apart; 0 for ordinary programs)
    int slot[MAXF];
    int lo[MAXF];
    int hi[MAXF];
    const double2 *M[MAXF];
};

// Linear combination of factor matrices, dst = sum_q coef_q src_q (n2
// elements each): the factor of a merged operator entry (entries equal in all
// factors but one are summed into one entry before a program is applied).
struct CombJob {
    double2 *dst;
    int n2;     // elements of the matrix
    int first;  // sources srcs[first .. first + count)
    int count;
    int n;      // rows = columns (for the transposing modes)
    int mode;   // 0: sum coef src; 1: transpose; 2: conjugate; 3: conjugate transpose (coef applied as given)
};
struct CombSrc {
    double2 coef;
    const double2 *src;
};

// Grouped application of entries to a tensor (H_eff matvec, K_eff matvec,
// SPO / mean-field rebuilds).  Device tables are owned by the engine.
struct ProgView {
    Geom g;
    const DevEntry *ent;
    int n_ent;
    int max_nf;
    const int *gptr;          // [n_groups+1] entries of group g: gent[gptr[g]..gptr[g+1])
    const int *gent;
    int n_groups;
    double2 *const *gdst;     // contraction destination per group (env programs)
    int contract_slot;        // -1: none
    int f32;                  // 1: stages, group sums and contractions in complex FP32
    int bf16x3;               // 1 (with f32): dense stages with factors of 24..64 on BF16x3 MFMA
    unsigned short *mprep;    // bf16 hi/lo realified factors, n_ent * 2 * 128 * 128 (BF16x3 mode)
    int mfma32;               // 1 (FP32 mode): dense stages with factors of 24..64 on the FP32 matrix cores
    int mfma64;               // 1 (FP64 mode): dense stages with factors of 16..64 on the FP64 matrix cores
    double2 *tmp;             // 2 * n_ent * N (float2 elements in the FP32 mode)
    double2 *gsum;            // n_groups * N (float2 elements in the FP32 mode)
    int64_t in_stride;        // distance of the input slices read by entries with src > 0
    double2 *cpart;           // contraction partials
    double sflops[MAXF];      // algorithmic flops / bytes of each stage launch (host side)
    double sbytes[MAXF];
    int snmin[MAXF], snmax[MAXF];  // smallest / largest factor dimension of each stage
    int stile[MAXF];               // stage runs on the tiled kernel (dense factors, n <= 64)
};

// Pair-operator form of an H_eff program of a large node (FP32 mode): when
// every product acts on at most one child slot k and the parent slot P, the
// program is sum_k W_k applied on the index pair (k, P), where the dense pair
// operator W_k = sum_e c_e F_e (x) P_e ((n_k n_P)^2 elements) is rebuilt from
// the current factors before each use and applied as one complex GEMM on the
// matrix cores (rows: the other indices of the node tensor).
struct PairTerm {
    double2 coef;
    const double2 *F;  // n_k x n_k on slot k, or null (identity)
    const double2 *P;  // n_P x n_P on the parent slot, or null (identity)
};
struct PairPass {
    int nk, np;        // dims of slot k and of the parent slot
    int64_t L, Mid;    // products of the dims before k and between k and P
    float2 *W;         // W[q][kappa], q = (a, b) output pair, kappa = (a', b') input pair
    const PairTerm *terms;
    int n_terms;
    unsigned short *Wb;  // BF16x3 form: realified bf16 hi then lo parts, [2Q][2Q] each (null otherwise)
    int v4;              // FP32 form: stage four kappa at a time (16-byte loads and LDS stores; needs np % 4 == 0)
};
constexpr int PAIR_KC = 16;  // complex K per LDS chunk of the pair GEMM
void launch_pair_build(const PairPass &pp, hipStream_t st);
// out (FP64) = (accumulate ? out : 0) + W_k applied to in (complex FP32) on (k, P).
// ws (pair_gemm_ws_bytes(ws_slots) bytes, or null): the work is shared evenly
// by ws_slots work-groups (0: the device's resident capacity), tiles cut
// between two of them summed from ws by a second kernel in a fixed order;
// null: one work-group per tile.
void launch_pair_gemm(const PairPass &pp, const float2 *in, double2 *out, int accumulate, double flops, float *ws,
                      int ws_slots, hipStream_t st);
size_t pair_gemm_ws_bytes(int ws_slots, int bf16x3);  // workspace of the shared schedule on the current device
// rows and columns >= keep of the n x n matrix C set to zero
void launch_zero_tail(double2 *C, int n, int keep, hipStream_t st);
// y = x rounded to complex FP32 (n elements)
void launch_to_f32(const double2 *x, float2 *y, int64_t n, hipStream_t st);
// BF16x3 form: (Re, Im) of x as bf16 hi and lo pairs; the pair operator split
// into its realified bf16 hi / lo parts; the GEMM on v_mfma_f32_32x32x16_bf16
void launch_to_bf16x2(const double2 *x, unsigned *xh, unsigned *xl, int64_t n, hipStream_t st);
void launch_pair_split(const PairPass &pp, hipStream_t st);
// (ws, ws_slots: the shared schedule as for launch_pair_gemm, workspace of
// pair_gemm_ws_bytes(ws_slots, 1) bytes)
void launch_pair_gemm_bf(const PairPass &pp, const unsigned *xh, const unsigned *xl, double2 *out, int accumulate,
                         double flops, float *ws, int ws_slots, hipStream_t st);

// Statistics written by one Krylov solve.
struct SolveStat {
    int m;         // Krylov dimension used (last sub-step)
    int level;     // sub-stepping level (0: none)
    int fail;      // 1: not converged
    int matvecs;   // matrix-vector products
    double err;    // final error estimate (relative)
    double err_lo; // error estimate at a smaller dimension (big path)
    double eval;   // ground-state mode: the lowest Ritz value of the local generator
};

struct SmallSolveArgs {
    Geom g;
    const DevEntry *ent;
    int n_ent;
    double2 *x;        // in/out
    double2 *V;        // scratch (SMALL_MMAX + 2) * N
    double tau;        // computes exp(-i tau G) x
    double tol;
    int mmax;
    int hermitian;
    int m_hint;
    int batched;       // two-slot problem with the batched matvec
    int vlds;          // 1: the Krylov basis lives in LDS (when it fits), else in V
    int mlds;          // 1: the factor matrices are copied to LDS (batched matvec, when they fit)
    int mlds_elems;    // their total size in complex elements
    int nA;            // entries with a slot-1 factor (batched)
    SolveStat *stat;
    int ground;        // 1: x <- the lowest eigenvector of G instead of exp(-i tau G) x (Hermitian G)
};
constexpr int SMALL_MAXENT = 128;  // entries of the batched two-slot matvec
constexpr int SMALL_UB = 2048;     // slot-0 operator size limit of the batched two-slot matvec
constexpr int SMALL_US = 1024;     // LDS elements for the entry-group partial sums (batched matvec)
constexpr int64_t SMALL_SEQ_WORK = 8192;  // entries x elements limit of the fused solver's generic matvec
// static LDS of the fused solver: three int tables and the staged entry fields per entry, plus reduction scratch
constexpr size_t SMALL_STATIC_LDS = (size_t)SMALL_MAXENT * (3 * sizeof(int) + 48) + 1024;
size_t small_solve_lds_bytes(int64_t N, int mmax, int batched, int nA);
inline size_t small_solve_vlds_bytes(int64_t N, int mmax) { return 16 * (size_t)(mmax + 1) * N; }

// Scratch of the multi-kernel Krylov path.
struct BigKrylov {
    double2 *V;        // (mmax + 1) * N basis
    double2 *Hm;       // (mmax + 1) * mmax projected matrix, column-major by iteration
    double2 *h;        // mmax + 1 reduced dots
    double2 *y;        // mmax coefficients
    double *part;      // VEC_BLOCKS * (mmax + 2) * 2 partial sums
    double *scal;      // [0] beta0 [1] beta
    int *meff;         // breakdown dimension (0: none)
    unsigned *counter; // last-block reduction counter (starts at 0)
    double2 *G;        // (mmax + 1)^2 Gram matrix of the basis, column j = V^H v_j (one-pass orthogonalisation)
    int *refine;       // 1: the last update cancelled most of w, one more classical pass follows
};

// Scratch of the many-work-group Householder QR.
constexpr int QRM_BLOCKS_MAX = 256;
constexpr int64_t QR_MULTI_MIN = 16384;  // matrices with at least this many elements use the many-work-group QR
struct QRWork {
    double2 *tau, *scl, *diag;  // [64] per reflector
    int *snapped;               // [64]
    double2 *w;                 // [64*64] w[i*64+j] = v_i^H a_j
    double2 *rowi;              // [64] row i of the current column step
    double *part;               // [QRM_BLOCKS_MAX * (2 + 2*64)]
    double2 *S;                 // [QRM_BLOCKS_MAX * 64*63/2] partial reflector Gram
    double2 *K;                 // [64*64] T V_top^H
    double *thr;                // [1] snap threshold
    unsigned *counter;          // last-block ticket (starts at 0)
    double *cpart;              // [2][QRM_BLOCKS_MAX][QRC_REC] column partials of the cooperative QR
    unsigned *bar;              // [192] grid barrier of the cooperative QR (starts at 0); bar[128] != 0: failed
    unsigned long long bar_base;  // arrivals counted in bar[0..1] by the launches made so far (host side)
    // nullable: the Householder kernels return at once while *gate == 0 (the
    // Cholesky route of the same launch sequence produced the factors)
    const int *gate;
    // Cholesky route (launch_qr_chol)
    double2 *cq_part;     // [CQR_BLOCKS_MAX][64*64] per-work-group Gram partials
    double2 *cq_G;        // [64*64] reduced Gram matrix
    double2 *cq_R1;       // [64*64] first Cholesky factor
    double2 *cq_R1inv;    // [64*64] its inverse
    double2 *cq_M;        // [64*64] R2^{-1} S
    double2 *cq_Y;        // [cq_ycap] first-pass factor A R1^{-1}, row-major m x n
    int64_t cq_ycap;
    double *cq_scal;      // [4] |A|_F^2
    int *cq_state;        // [4] 0: the Cholesky route holds, 1: the Householder kernels run
    unsigned *cq_counter; // [4] last-block ticket (starts at 0)
};
constexpr int QRC_REC = 2 + 4 * 64;  // xn2, fro, g_j (complex), row i (complex)

// ---- launch profiler (off by default) ----
struct KernelStat {
    std::string name;
    long long calls = 0;
    double ms = 0.0, flops = 0.0, bytes = 0.0;
};
void profile_enable(bool enable);
bool profile_enabled();
void profile_add_flops(const char *name, double flops);
std::vector<KernelStat> profile_collect();
// frees the profiler's device clock slots and event pool (re-created on demand)
void release_process_resources();
// while one lives, launches made by this thread are not timed (no events created)
struct ProfileSuspend {
    ProfileSuspend();
    ~ProfileSuspend();
    bool prev;
};

// ---- launchers (all asynchronous on `st`) ----
// x32 (FP32 mode, optional): N complex FP32 of scratch; with several entries
// the FP64 input is converted into it once and every entry's first stage
// reads the FP32 copy (the values each stage would have converted itself)
void launch_prog_stages(const ProgView &p, const double2 *in, hipStream_t st, float2 *x32 = nullptr);
// tile autotuner: time every admissible register tile of each tiled stage of p
// and keep the fastest (process-wide table, keyed by the stage's shape)
void tune_prog_stages(const ProgView &p, const double2 *in, hipStream_t st);
size_t tile_table_size();
void tile_table_save(const char *path);
int tile_table_load(const char *path);
void tile_table_clear();
void launch_prog_sum(const ProgView &p, const double2 *in, double2 *out_single, hipStream_t st);
void launch_prog_contract(const ProgView &p, const double2 *A, hipStream_t st);

// Y[l,i,r] = sum_j M[i,j] X[l,j,r] (transM: M[j,i]); X has (L, n_in, R), Y (L, n_out, R)
void launch_mode_product(const double2 *X, double2 *Y, const double2 *M, int64_t L, int n_in, int n_out,
                         int64_t R, int transM, hipStream_t st);
// out[m,n] = sum_{l,r} conj(A[l,m,r]) B[l,n,r] for (L, nA, R) and (L, nB, R)
void launch_contract(const double2 *A, const double2 *B, double2 *out, int64_t L, int nA, int nB,
                     int64_t R, double2 *part, hipStream_t st);
void launch_qr(double2 *A, int64_t L, int n, int64_t R, double2 *Rout, int transR, hipStream_t st,
               const int *gate = nullptr);
void launch_qr_multi(double2 *A, int64_t L, int n, int64_t R, double2 *Rout, int transR, const QRWork &q,
                     hipStream_t st);
// The same factors as the Householder kernels (LAPACK convention) for full-rank
// matrices away from the zero-snap, by Cholesky QR applied twice and the signs
// of the reflectors read off an LU factorisation of the leading block; sets
// *q.cq_state to 1 when the matrix is outside that range, so that the
// Householder kernels launched next with q.gate = q.cq_state do the work.
// Returns false (nothing launched) when the shape is not covered.
bool launch_qr_chol(double2 *A, int64_t L, int n, int64_t R, double2 *Rout, int transR, const QRWork &q,
                    hipStream_t st);
constexpr int CQR_BLOCKS_MAX = 256;
constexpr int CQR_TILE = 64;  // rows per LDS tile
// the same reflectors in one cooperative launch (grid-wide barriers between columns);
// returns false (nothing launched) when the grid cannot be co-resident
bool launch_qr_coop(double2 *A, int64_t L, int n, int64_t R, double2 *Rout, int transR, QRWork &q,
                    hipStream_t st);
void launch_small_solve(const SmallSolveArgs &a, hipStream_t st);
// independent fused solves in one launch (work-group b takes d_args[b]; h_args
// is the host copy of the same array, for the launch shape)
void launch_small_solve_group(const SmallSolveArgs *d_args, const std::vector<SmallSolveArgs> &h_args,
                              hipStream_t st);
void launch_copy(double2 *dst, const double2 *src, int64_t n, hipStream_t st);
void launch_combine(const CombJob *jobs, const CombSrc *srcs, int n_jobs, int max_n2, hipStream_t st);

// ---- subspace expansion pieces ----
// out[g * n + j] = sum_{l,r} op(A[l, j, r]) B[g * bstride + l * R + r] for g < groups
// (op: conj when conjA), through partial sums in `part`.
void launch_ts_contract(const double2 *A, int64_t L, int n, int64_t R, int conjA, const double2 *B,
                        int64_t bstride, int groups, double2 *out, double2 *part, hipStream_t st);
// out[g * L * R + l * R + r] = base[...] - sum_j op(A[l, j, r]) S[g * n + j] (base NULL: no base,
// the sum itself); op: conj when conjA
void launch_ts_expand(const double2 *A, int64_t L, int n, int64_t R, int conjA, const double2 *S, int groups,
                      const double2 *base, int negate, double2 *out, hipStream_t st);
// Y[l, j, r] (slot size n_new) from X[l, j, r] (slot size n_old): copied for j < min(n_old, n_new),
// beyond n_old taken from the vectors V (vector j - n_old at V + (j - n_old) * vstride, element l * R + r,
// conjugated when conjV) or zero when V is NULL
void launch_repack(const double2 *X, double2 *Y, int64_t L, int n_old, int n_new, int64_t R, const double2 *V,
                   int64_t vstride, int conjV, hipStream_t st);
// seeded complex start vector: re, im uniform in [-1, 1) from SplitMix64(seed + 2 i), (seed + 2 i + 1)
void launch_seed_vector(double2 *v, int64_t N, uint64_t seed, hipStream_t st);
// singular value decomposition of the real upper-bidiagonal matrix with diagonal alpha[0..n) and
// superdiagonal beta[0..n-1), n read from nptr and at most 48 (one-sided Jacobi); s (descending),
// U and V (n x n, column j belongs to s[j], row-major with leading dimension nmax)
void launch_bidiag_svd(const double *alpha, const double *beta, const int *nptr, int nmax, double *s, double *U,
                       double *V, hipStream_t st);
// out[c * N + i] = sum_{q < n} W[q * ldw + c] V[q * N + i] for c < ncols (W real), n read from nptr
void launch_basis_combine(const double2 *V, int64_t N, const int *nptr, const double *W, int ldw, int ncols,
                          double2 *out, hipStream_t st);
// n = dimension of the Golub-Kahan-Lanczos bidiagonal after m steps (breakdown flags of both bases)
void launch_gkl_count(const int *meffP, const int *meffQ, const double *alpha0, int m, int *n, hipStream_t st);
// dst[i] = src[i] for i < count (doubles), device to device in stream order
void launch_copy_scalars(double *dst, const double *src, int count, hipStream_t st);
void launch_transpose(double2 *dst, const double2 *src, int n, hipStream_t st);

// multi-kernel Krylov pieces
void launch_krylov_start(const double2 *x, int64_t N, const BigKrylov &k, hipStream_t st);
void launch_krylov_orth(const BigKrylov &k, int64_t N, int j, int mmax, hipStream_t st);
// the same orthonormalisation with one pass over the basis for the dots and one
// for the update (Gram-matrix form of the second Gram-Schmidt pass); needs
// k.G, k.refine and k.part of VEC_BLOCKS * (2 mmax + 4) * 2 doubles
void launch_krylov_orth1(const BigKrylov &k, int64_t N, int j, int mmax, hipStream_t st);
void launch_krylov_finish(const BigKrylov &k, int64_t N, int m, int mmax, double tau, double tol,
                          int hermitian, double2 *x, SolveStat *stat, hipStream_t st);
// Ground-state form of the finish: x <- the Ritz vector of the lowest Ritz
// value of the m-dimensional Lanczos matrix (unit norm), stat->eval the value,
// stat->err the residual estimate |beta_m y_m| relative to max(1, |value|)
void launch_krylov_ground(const BigKrylov &k, int64_t N, int m, int mmax, double2 *x, SolveStat *stat,
                          hipStream_t st);

}  // namespace ttn
