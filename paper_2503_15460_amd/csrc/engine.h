// Host orchestration of the one-site TDVP sweep on one GPU.
#pragma once

#include <hip/hip_runtime.h>

#include <functional>
#include <string>
#include <unordered_map>
#include <vector>

#include "kernels.h"
#include "ttn_internal.h"

namespace ttn {

// Grouped operator program on one node tensor (host tables + device copies).
struct Prog {
    Geom g{};
    std::vector<DevEntry> ents;
    std::vector<int> gptr{0}, gent;
    std::vector<double2 *> gdst;
    int n_groups = 0, max_nf = 0, contract_slot = -1;
    int64_t flops = 0;  // algorithmic flops of one application (8 per complex MAC)
    double sflops[MAXF] = {0}, sbytes[MAXF] = {0};  // per stage launch
    int snmin[MAXF] = {0}, snmax[MAXF] = {0};        // factor dims at each stage
    int stile[MAXF] = {0};                           // 1: every factor of the stage is dense, n <= 64
    DevEntry *d_ent = nullptr;
    int *d_gptr = nullptr, *d_gent = nullptr;
    double2 **d_gdst = nullptr;
    int capdims[MAXD] = {0};  // slot dims at the bond capacity (buffers are sized for them)
    // merged entries: their factor matrices are recombined before every use
    std::vector<double2 *> comb_bufs;  // one per summed factor, sized for the capacity
    std::vector<CombJob> cjobs;
    std::vector<CombSrc> csrcs;
    int comb_max_n2 = 0;
    CombJob *d_cjobs = nullptr;
    CombSrc *d_csrcs = nullptr;
    // pair-operator form (empty: staged application); device buffers are sized
    // for the capacity at the first plan and reused by later plans
    std::vector<PairPass> pair;
    std::vector<double> pair_flops;       // algorithmic flops of each pass
    std::vector<float2 *> pair_w;         // per child slot (null: not allocated)
    std::vector<unsigned short *> pair_wb;  // BF16x3 hi / lo parts per child slot
    std::vector<PairTerm *> pair_dterms;  // per child slot
    std::vector<int> pair_cap_terms;
};

class Engine {
public:
    Engine(const Tree &t, const ttn_options &o);
    ~Engine();

    void set_sop(const SopInput &s);
    // New coefficients for the terms of the operator in place (same operators
    // and terms); returns true if the compiled structure changed and the
    // operator was rebuilt, false if only values were replaced.
    bool set_coefficients(const double *coeff, int n_terms);
    void set_product_state(const double *leaf_vecs);
    void set_state(const double *buf, size_t bytes);
    void get_state(double *buf, size_t bytes);
    size_t state_bytes() const;
    void step(double dt, int n_steps);
    // split form of one step for instances advanced together (batches)
    void enqueue_step(double dt);
    void finish_step(double dt);
    void set_stream(hipStream_t s);
    // lockstep batches: the operations of one step as a schedule (snapshot
    // already enqueued); fused solves met while defer_fused is set are left in
    // `deferred` for a grouped launch; finish_record enqueues the statistics
    std::vector<std::function<void()>> record_step(double dt);
    void finish_record();
    bool defer_fused = false;
    std::vector<SmallSolveArgs> deferred;
    void check_ready(double dt) const;
    hipStream_t stream() const { return st; }
    std::vector<double> observe(int kind, int n, const int32_t *op_ids, const double *vecs);
    double krylov_tolerance() const;  // local exponential error target (option or precision default)
    // n one-site ground-state sweeps (DMRG on trees); returns <Psi|G|Psi> / <Psi|Psi>
    double ground_sweeps(int n, int *unconverged);
    void apply_root_heff(const double *x, double *y);
    void info(int32_t *bonds, int64_t *counters);
    size_t workspace_need() const { return ws_need; }
    int64_t graph_captures() const { return counters_graph_captures; }
    int step_solves(int max, int32_t *node, int32_t *fwd, int32_t *matvecs) const;

    Tree t;
    ttn_options opt;

private:
    hipStream_t st = nullptr;
    bool have_sop = false, have_state = false;
    bool adaptive = false;  // subspace expansion on (spawn_tol > 0)
    bool graph_mode = false;  // steps replayed from captured hipGraphs (use_graph)
    bool ground = false;      // inside ground_sweeps: node solves are lowest-eigenvector solves, no bond steps
    // large QRs take the Cholesky route first (TTN_CHOLQR=0 in the environment:
    // Householder kernels only)
    bool cholqr = true;
    // FP32 effective generators of large nodes in the pair-operator form
    // (TTN_PAIR_OPS=0 in the environment: staged products only)
    bool pair_ops = true;
    // multi-kernel Krylov: two classical Gram-Schmidt passes per iteration
    // instead of the Gram-matrix form (TTN_KRYLOV_CGS2=1)
    bool krylov_cgs2 = false;
    int64_t pair_min_n = 1 << 18;  // node size from which the pair form is considered (TTN_PAIR_MIN_N)
    float2 *pair_x32 = nullptr;    // scratch (FP32 modes): complex FP32 copy of a pair-form or first-stage input
    // pair GEMMs shared evenly by the resident work-groups, cut tiles summed
    // from pair_ws: 1 (default) the FP32 form, 2 (TTN_PAIR_SPLIT=2) also the
    // BF16x3 form (which the hardware's own dispatch of one work-group per
    // tile balances as well: not bound by its matrix cores), 0 neither
    int pair_split = 1;
    int pair_slots = 0;  // work-groups sharing it (0: the device's capacity; TTN_PAIR_SLOTS, rounded down to 8s)
    // FP32 pair GEMM: four kappa per thread and 16-byte staging where the
    // parent dimension allows (TTN_PAIR_V4=0: one kappa per thread)
    bool pair_v4 = true;
    float *pair_ws = nullptr;
    // FP32 mode: dense stages with factors of 24..64 on the FP32 matrix cores
    // (TTN_MODE_MFMA32=0 in the environment: the vector-ALU tiled kernel)
    bool mode_mfma32 = true;
    // FP64 mode: dense stages with factors of 16..64 on the FP64 matrix cores
    // (TTN_MODE_MFMA64=0: the vector-ALU tiled kernel)
    bool mode_mfma64 = true;
    hipStream_t own_stream = nullptr;
    struct GraphEntry {
        std::vector<int64_t> key;  // Krylov dimension hints and dt of the captured step
        hipGraphExec_t exec;
        int n_solves;
    };
    std::vector<GraphEntry> graphs;
    int64_t counters_graph_captures = 0;
    SopInput sop;
    TreeOp op;
    // state (allocated at construction)
    std::vector<double2 *> A, Aalt, A0;
    double2 *state_mem = nullptr;
    // environments and programs (allocated by set_sop)
    std::vector<double2 *> spo, mf, U;
    std::vector<std::vector<int>> ulo, uhi;  // band of each leaf channel operator
    std::vector<Prog> heffP, spoP, bondP;
    std::vector<std::vector<Prog>> mfP;
    std::vector<void *> sop_allocs;
    // bytes last written to every host-written device table (program tables,
    // leaf operators, pair terms); in staged mode (coefficient updates)
    // unchanged tables are skipped and the rest copied asynchronously from
    // pinned staging chunks, which the next update reuses after its first sync
    std::unordered_map<const void *, std::string> shadow;
    bool staged = false;
    std::vector<std::pair<char *, size_t>> stage_chunks;
    size_t stage_cur = 0, stage_off = 0;
    void h2d(void *dst, const void *src, size_t bytes);
    char *stage_alloc(size_t bytes);
    double2 *tmp = nullptr, *gsum = nullptr, *cpart = nullptr;
    unsigned short *mprep = nullptr;  // BF16x3 split factors
    double2 *Rbuf = nullptr, *Cbuf = nullptr, *smallV = nullptr, *obs = nullptr, *snapshot = nullptr;
    int64_t obs_elems = 0;
    BigKrylov bk{};
    QRWork qrw{};
    int64_t bigN = 0;
    SolveStat *d_stats = nullptr;
    SolveStat *h_stats = nullptr;  // pinned host copy
    unsigned *h_flags = nullptr;   // pinned: [0] failure flag of the cooperative QR barrier
    int n_stats = 0;
    hipEvent_t step_done = nullptr;
    std::vector<int> m_hint;     // per solve index in the step schedule
    std::vector<int> solve_node; // node (forward) or bond-owner (backward) per solve index
    std::vector<char> solve_fwd, solve_small;
    int solve_idx = 0;
    int mmax = 40;
    int64_t counters[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    size_t ws_need = 0;  // scratch bytes of the current operator (workspace size)
    // subspace expansion: two-site programs of each bond (by the child node):
    // OT = outside factors transposed (grouped by bond channel), OC = outside
    // factors conjugated (entry inputs by channel), B = below factors (entry
    // inputs by channel), BH = below factors conjugate-transposed (grouped)
    struct TwoSite {
        Prog OT, OC, B, BH;
        std::vector<int> chans;
    };
    std::vector<TwoSite> tsP;
    std::vector<int> snap_bond;
    int gkl_m = 40;                       // largest Golub-Kahan-Lanczos dimension
    double2 *ts_in = nullptr, *ts_s = nullptr, *ts_w1 = nullptr, *ts_w2 = nullptr, *ts_out = nullptr;
    double2 *ts_R = nullptr, *ts_part = nullptr;
    double *gkl_sc = nullptr;             // alpha[64] beta[64] s[64] U[64*64] V[64*64]
    int *gkl_n = nullptr;
    BigKrylov gkP{}, gkQ{};
    uint64_t spawn_calls = 0;

    void *dalloc(size_t bytes);
    void free_sop();
    void put_leaf_ops(int c);  // leaf channel operators of leaf c and their bands into U[c]
    Geom geom_of(const std::vector<int> &dims) const;
    void upload(Prog &p);
    void merge_entries(Prog &p);
    void prep(const Prog &p);
    ProgView view(const Prog &p) const;
    void build_programs();
    void build_node_programs(int z);
    int capdim(const Prog &p, int slot) const;
    void rebuild_all_spos();

    // sweep pieces
    void sweep_S(int z, double h);
    void sweep_Sstar(int z, double h);
    void forward(int z, double tau);
    void backward(int c, double2 *C, double tau);
    void expm_prog(const Prog &p, double2 *x, double tau, int node, bool fwd);
    bool use_fused(const Prog &p) const;
    void qr_slot(int z, int s, double2 *Rout, int transR);
    void qr_any(double2 *X, const Geom &g, int s, double2 *Rout, int transR);
    // subspace expansion
    bool spawn(int z, int k, double h, bool below);
    void build_two_site(int z, int k);
    void apply_R(int z, int k, const double2 *Qc, const double2 *Qo, const double2 *q, double2 *p);
    void apply_RH(int z, int k, const double2 *Qc, const double2 *Qo, const double2 *y, double2 *w);
    void project_out(const double2 *Q, int64_t L, int n, int64_t R, int conjQ, double2 *x);
    void resize_psi0(int c, int nb_new);
    void transform_factors(Prog &p, int mode);
    void absorb(int z, int s, const double2 *M, int transM);
    void build_spo(int c);
    void build_mf(int z, int k);
    void apply_prog(const Prog &p, const double2 *in, double2 *out);
    // one application of an effective-generator program after prep (pair
    // GEMMs or staged products and the group sum)
    void launch_apply(const Prog &p, const ProgView &v, const double2 *in, double2 *out);
    void plan_pairs(Prog &h, int z);
    void sync_check(const char *where);
    void save_snapshot();
    void restore_snapshot();
    void enqueue_sweep(double dt);
    void enqueue_sweep_body(double dt);
    void enqueue_stats();
    void emit(std::function<void()> op);
    std::vector<std::function<void()>> *rec = nullptr;  // schedule being recorded (lockstep batches)
    void drop_graphs();
};

void debug_qr(int64_t rows, int cols, const double *m, int variant, double *q_out, double *r_out);

}  // namespace ttn
