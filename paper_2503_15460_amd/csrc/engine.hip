// Host orchestration of the one-site TDVP projector-splitting sweep on one GPU.
//
// Paper: pyTTN (arXiv 2503.15460), Sec. II C.  One step is the symmetric
// sweep S(dt/2) followed by its mirror S*(dt/2), with the two root forward
// half steps merged:
//   S(z):  for each child c (increasing id): QR of A^z along c's bond, absorb R
//          into c, rebuild the mean fields of c, recurse into c (leaf: forward
//          step), QR of A^c along its parent bond, rebuild the SPOs of c,
//          backward bond step C <- exp(+i h K) C, absorb C into A^z; then the
//          forward step of z.
//   S*(z): forward step of z; for each child in decreasing id: QR of A^z,
//          rebuild the mean fields of c, backward bond step on R^T, absorb into
//          c, recurse, QR of A^c, rebuild the SPOs of c, absorb R into A^z.
// All arithmetic runs in the kernels of kernels.hip on one HIP stream; the host
// only enqueues work and reads back one small statistics array per step.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <cstdio>
#include <cstdlib>
#include <functional>
#include <map>
#include <set>

#include "engine.h"

namespace ttn {

static_assert(MAX_CHILDREN + 1 <= MAXD, "node tensors must fit the slot arrays");
static_assert(MAX_CHILDREN + 1 <= MAXF, "operator entries must fit the factor arrays");

#define HIPCHK(x)                                                                                  \
    do {                                                                                           \
        hipError_t e_ = (x);                                                                       \
        if (e_ != hipSuccess) throw Error(TTN_E_DEVICE, std::string(#x) + ": " + hipGetErrorString(e_)); \
    } while (0)

static inline double2 to_d2(cplx c) { return make_double2(c.real(), c.imag()); }

Engine::Engine(const Tree &tr, const ttn_options &o) : t(tr), opt(o) {
    HIPCHK(hipSetDevice(opt.device));
    st = (hipStream_t)opt.hip_stream;
    mmax = opt.krylov_mmax > 0 ? std::min(opt.krylov_mmax, 40) : 40;
    if (mmax < 3) mmax = 3;
    for (int z = 0; z < t.n; ++z)
        if (z != t.root && t.cap[z] > 64) throw Error(TTN_E_DIMS, "bond dimensions above 64 are not supported");
    adaptive = opt.spawn_tol > 0.0;
    graph_mode = opt.use_graph != 0;
    if (const char *e = getenv("TTN_CHOLQR")) cholqr = atoi(e) != 0;
    if (const char *e = getenv("TTN_PAIR_OPS")) pair_ops = atoi(e) != 0;
    if (const char *e = getenv("TTN_KRYLOV_CGS2")) krylov_cgs2 = atoi(e) != 0;
    if (const char *e = getenv("TTN_MODE_MFMA32")) mode_mfma32 = atoi(e) != 0;
    if (const char *e = getenv("TTN_MODE_MFMA64")) mode_mfma64 = atoi(e) != 0;
    if (const char *e = getenv("TTN_PAIR_SPLIT")) pair_split = std::max(0, std::min(2, atoi(e)));
    if (const char *e = getenv("TTN_PAIR_SLOTS")) pair_slots = std::max(0, atoi(e));
    if (const char *e = getenv("TTN_PAIR_V4")) pair_v4 = atoi(e) != 0;
    if (const char *e = getenv("TTN_PAIR_MIN_N")) pair_min_n = std::max<int64_t>(1, atoll(e));
    if (graph_mode && !st) {  // the null stream cannot be captured: a stream of the handle's own
        HIPCHK(hipStreamCreateWithFlags(&own_stream, hipStreamNonBlocking));
        st = own_stream;
    }
    // node tensors are allocated for the bond capacity (bonds may grow)
    int64_t tot = 0;
    for (int z = 0; z < t.n; ++z) tot += t.capsize[z];
    HIPCHK(hipMalloc(&state_mem, sizeof(double2) * 3 * tot));
    HIPCHK(hipMemset(state_mem, 0, sizeof(double2) * 3 * tot));
    counters[5] += (int64_t)sizeof(double2) * 3 * tot;
    A.resize(t.n);
    Aalt.resize(t.n);
    A0.resize(t.n);
    int64_t off = 0;
    for (int z = 0; z < t.n; ++z) {
        A[z] = state_mem + off;
        Aalt[z] = state_mem + tot + off;
        A0[z] = state_mem + 2 * tot + off;
        off += t.capsize[z];
    }
    HIPCHK(hipEventCreateWithFlags(&step_done, hipEventDisableTiming));
}

Engine::~Engine() {
    drop_graphs();
    free_sop();
    if (own_stream) (void)hipStreamDestroy(own_stream);
    if (h_stats) (void)hipHostFree(h_stats);
    if (h_flags) (void)hipHostFree(h_flags);
    if (step_done) (void)hipEventDestroy(step_done);
    if (state_mem) (void)hipFree(state_mem);
    for (auto &c : stage_chunks) (void)hipHostFree(c.first);
}

// Copy of a host-written device table (see `shadow`).
void Engine::h2d(void *dst, const void *src, size_t bytes) {
    std::string &sh = shadow[dst];
    if (staged && sh.size() == bytes && std::memcmp(sh.data(), src, bytes) == 0) return;
    sh.assign((const char *)src, bytes);
    if (!staged) {
        HIPCHK(hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice));
        return;
    }
    char *p = stage_alloc(bytes);
    std::memcpy(p, src, bytes);
    HIPCHK(hipMemcpyAsync(dst, p, bytes, hipMemcpyHostToDevice, st));
}

// Pinned staging space for one asynchronous copy (1 MiB chunks, kept).
char *Engine::stage_alloc(size_t bytes) {
    bytes = (bytes + 255) / 256 * 256;
    while (stage_cur < stage_chunks.size() && stage_off + bytes > stage_chunks[stage_cur].second) {
        ++stage_cur;
        stage_off = 0;
    }
    if (stage_cur == stage_chunks.size()) {
        const size_t cap = std::max<size_t>(bytes, (size_t)1 << 20);
        void *p = nullptr;
        HIPCHK(hipHostMalloc(&p, cap, hipHostMallocDefault));
        stage_chunks.push_back({(char *)p, cap});
        stage_off = 0;
    }
    char *p = stage_chunks[stage_cur].first + stage_off;
    stage_off += bytes;
    return p;
}

void Engine::set_stream(hipStream_t s) {
    HIPCHK(hipStreamSynchronize(st));
    st = s;
}

void *Engine::dalloc(size_t bytes) {
    void *p = nullptr;
    if (bytes == 0) bytes = 16;
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) throw Error(TTN_E_OOM, std::string("hipMalloc failed: ") + hipGetErrorString(e));
    // recycled device memory holds stale values: every buffer starts at zero
    e = hipMemset(p, 0, bytes);
    if (e != hipSuccess) {
        (void)hipFree(p);
        throw Error(TTN_E_DEVICE, std::string("hipMemset failed: ") + hipGetErrorString(e));
    }
    sop_allocs.push_back(p);
    counters[5] += (int64_t)bytes;
    return p;
}

void Engine::free_sop() {
    drop_graphs();
    have_sop = false;
    for (void *p : sop_allocs) (void)hipFree(p);
    sop_allocs.clear();
    shadow.clear();  // freed addresses may come back for other tables
    heffP.clear();
    spoP.clear();
    bondP.clear();
    mfP.clear();
    tsP.clear();
}

Geom Engine::geom_of(const std::vector<int> &dims) const {
    Geom g{};
    g.D = (int)dims.size();
    int64_t N = 1;
    for (int s = 0; s < g.D; ++s) {
        g.dims[s] = dims[s];
        N *= dims[s];
    }
    g.N = N;
    for (int s = 0; s < g.D; ++s) {
        int64_t L = 1, R = 1;
        for (int q = 0; q < s; ++q) L *= dims[q];
        for (int q = s + 1; q < g.D; ++q) R *= dims[q];
        g.L[s] = L;
        g.R[s] = R;
    }
    return g;
}

// Clear the host tables of a program, keeping its device tables and buffers.
static void reset_host(Prog &p) {
    p.ents.clear();
    p.gptr.assign(1, 0);
    p.gent.clear();
    p.gdst.clear();
    p.cjobs.clear();
    p.csrcs.clear();
    p.comb_max_n2 = 0;
}

// Dimension of `slot` of the program's node tensor at the bond capacity.
int Engine::capdim(const Prog &p, int slot) const { return p.capdims[slot]; }

// Device tables of a program are allocated at its first upload; later uploads
// (after a bond changed size) copy into the same tables, whose sizes do not
// change (the entry structure of a node does not depend on the bonds).
void Engine::upload(Prog &p) {
    auto put = [&](auto *&dptr, const auto &vec) {
        using T = std::remove_reference_t<decltype(vec[0])>;
        if (!dptr) dptr = (std::remove_const_t<T> *)dalloc(sizeof(T) * std::max<size_t>(1, vec.size()));
        if (!vec.empty()) h2d((void *)dptr, vec.data(), sizeof(T) * vec.size());
    };
    put(p.d_ent, p.ents);
    put(p.d_gptr, p.gptr);
    put(p.d_gent, p.gent);
    put(p.d_gdst, p.gdst);
    if (!p.cjobs.empty()) {
        put(p.d_cjobs, p.cjobs);
        put(p.d_csrcs, p.csrcs);
    }
}

// Entries of one group that carry the same factors on every slot but one are
// summed into a single entry whose factor on that slot is the coefficient-
// weighted sum of theirs (the node form (B) + (C) of the hierarchical SOP:
// sum_e c_e (x)_f M_ef = (x)_{f != s} M_f (x) (sum_e c_e M_es) when the other
// factors coincide).  The summed factors are recombined on the device before
// every use of the program (prep), since the environments they are made of
// change during the sweep.
void Engine::merge_entries(Prog &p) {
    const int ne = (int)p.ents.size();
    if (ne < 2) return;
    std::vector<MergeItem> items(ne);
    for (int e = 0; e < ne; ++e) {
        const DevEntry &E = p.ents[e];
        items[e].group = E.group;
        items[e].nf = E.nf;
        for (int f = 0; f < E.nf; ++f) {
            items[e].slot[f] = E.slot[f];
            items[e].id[f] = (int64_t)(intptr_t)E.M[f];
        }
    }
    const std::vector<MergeSet> plan = plan_entry_merge(items);
    if (plan.empty()) return;
    std::vector<char> used(ne, 0);
    std::vector<DevEntry> out;
    p.cjobs.clear();
    p.csrcs.clear();
    p.comb_max_n2 = 0;
    if (p.comb_bufs.empty()) {  // one buffer per summed factor, at the capacity's size
        for (auto &m : plan) {
            const int n = capdim(p, p.ents[m.members[0]].slot[m.f]);
            p.comb_bufs.push_back((double2 *)dalloc(sizeof(double2) * (size_t)n * n));
        }
    }
    if (p.comb_bufs.size() != plan.size()) throw Error(TTN_E_STATE, "internal: merge plan changed");
    size_t qi = 0;
    for (auto &m : plan) {
        const int f = m.f;
        DevEntry d = p.ents[m.members[0]];
        const int n = p.g.dims[d.slot[f]];
        d.coef = make_double2(1.0, 0.0);
        int lo = 0, hi = 0;
        bool dense = false;
        CombJob j{};
        j.dst = p.comb_bufs[qi++];
        j.n2 = n * n;
        j.first = (int)p.csrcs.size();
        j.count = (int)m.members.size();
        for (int e : m.members) {
            used[e] = 1;
            const DevEntry &E = p.ents[e];
            if (E.lo[f] < 0 || E.hi[f] < 0) dense = true;  // unset band: dense
            lo = std::max(lo, E.lo[f]);
            hi = std::max(hi, E.hi[f]);
            p.csrcs.push_back({E.coef, E.M[f]});
        }
        d.lo[f] = dense ? -1 : lo;
        d.hi[f] = dense ? -1 : hi;
        d.M[f] = j.dst;
        p.cjobs.push_back(j);
        p.comb_max_n2 = std::max(p.comb_max_n2, j.n2);
        out.push_back(d);
    }
    for (int e = 0; e < ne; ++e)
        if (!used[e]) out.push_back(p.ents[e]);
    p.ents.swap(out);
}

void Engine::prep(const Prog &p) {
    if (!p.cjobs.empty()) launch_combine(p.d_cjobs, p.d_csrcs, (int)p.cjobs.size(), p.comb_max_n2, st);
    for (const PairPass &pp : p.pair) {
        launch_pair_build(pp, st);
        if (pp.Wb) launch_pair_split(pp, st);
    }
}

ProgView Engine::view(const Prog &p) const {
    ProgView v{};
    v.g = p.g;
    v.ent = p.d_ent;
    v.n_ent = (int)p.ents.size();
    v.max_nf = p.max_nf;
    v.gptr = p.d_gptr;
    v.gent = p.d_gent;
    v.n_groups = p.n_groups;
    v.gdst = p.d_gdst;
    v.contract_slot = p.contract_slot;
    v.tmp = tmp;
    v.gsum = gsum;
    v.cpart = cpart;
    v.f32 = (opt.precision == TTN_FP32 || opt.precision == TTN_BF16X3) ? 1 : 0;
    v.bf16x3 = opt.precision == TTN_BF16X3 ? 1 : 0;
    v.mprep = mprep;
    v.mfma32 = mode_mfma32 ? 1 : 0;
    v.mfma64 = mode_mfma64 ? 1 : 0;
    for (int f = 0; f < MAXF; ++f) {
        v.sflops[f] = p.sflops[f];
        // FP32 temporaries: stage 0 reads FP64 and writes FP32, later stages FP32 both ways
        v.sbytes[f] = v.f32 ? p.sbytes[f] * (f == 0 ? 0.75 : 0.5) : p.sbytes[f];
        v.snmin[f] = p.snmin[f];
        v.snmax[f] = p.snmax[f];
        v.stile[f] = p.stile[f];
    }
    return v;
}

// An entry with every factor band unset (finish_groups makes unset bands dense).
static DevEntry blank_entry() {
    DevEntry de{};
    for (int f = 0; f < MAXF; ++f) de.lo[f] = de.hi[f] = -1;
    return de;
}

// Finalise group tables of a program from the per-entry group ids.
static void finish_groups(Prog &p, const std::vector<double2 *> &dst_by_group) {
    p.n_groups = (int)dst_by_group.size();
    p.gdst = dst_by_group;
    p.gptr.assign(p.n_groups + 1, 0);
    for (auto &e : p.ents) p.gptr[e.group + 1]++;
    for (int g = 0; g < p.n_groups; ++g) p.gptr[g + 1] += p.gptr[g];
    p.gent.assign(p.ents.size(), 0);
    std::vector<int> fill(p.gptr.begin(), p.gptr.end() - 1);
    for (size_t e = 0; e < p.ents.size(); ++e) p.gent[fill[p.ents[e].group]++] = (int)e;
    p.max_nf = 0;
    p.flops = 0;
    for (int f = 0; f < MAXF; ++f) {
        p.sflops[f] = p.sbytes[f] = 0.0;
        p.snmin[f] = 1 << 30;
        p.snmax[f] = 0;
        p.stile[f] = 1;
    }
    for (auto &e : p.ents) {
        p.max_nf = std::max(p.max_nf, e.nf);
        for (int f = 0; f < e.nf; ++f) {
            const int n = p.g.dims[e.slot[f]];
            p.snmin[f] = std::min(p.snmin[f], n);
            p.snmax[f] = std::max(p.snmax[f], n);
            if (e.lo[f] < 0 || e.lo[f] > n - 1) e.lo[f] = n - 1;  // unset: dense
            if (e.hi[f] < 0 || e.hi[f] > n - 1) e.hi[f] = n - 1;
            if (n > 64 || e.lo[f] < n - 1 || e.hi[f] < n - 1) p.stile[f] = 0;
            // algorithmic work of a banded factor: the band only
            const int w = std::min(n, e.lo[f] + e.hi[f] + 1);
            p.flops += 8 * p.g.N * w;
            p.sflops[f] += 8.0 * p.g.N * w;
            p.sbytes[f] += 16.0 * (2.0 * p.g.N + (double)n * w);
        }
    }
}

void Engine::build_programs() {
    const int n = t.n;
    heffP.assign(n, Prog{});
    spoP.assign(n, Prog{});
    bondP.assign(n, Prog{});
    mfP.assign(n, {});
    int64_t total_entries = 0;
    for (int z = 0; z < n; ++z) {
        total_entries += (int64_t)op.entries[z].size();
        build_node_programs(z);
    }
    counters[6] = total_entries;
}

// Host tables of every program of node z (effective generator, SPO rebuild,
// bond generator of the bond above z, mean-field rebuilds of z's children) for
// the current bonds, uploaded into the node's device tables.
void Engine::build_node_programs(int z) {
    const int n = t.n;
    (void)n;
    auto child_M = [&](int z, int k, int ch) -> const double2 * {
        if (t.local_dim[z] > 0) {
            int d = t.local_dim[z];
            return U[z] + (size_t)ch * d * d;
        }
        int c = t.kids[z][k];
        int nc = t.bond[c];
        return spo[c] + (size_t)ch * nc * nc;
    };
    // band of a child factor (leaf operators may be banded; SPOs are dense)
    auto child_band = [&](DevEntry &de, int f, int z, int ch) {
        if (t.local_dim[z] > 0 && ch < (int)ulo[z].size()) {
            de.lo[f] = ulo[z][ch];
            de.hi[f] = uhi[z][ch];
        }
    };
    auto parent_M = [&](int z, int ch) -> const double2 * {
        int np = t.bond[z];
        return mf[z] + (size_t)ch * np * np;
    };
    {
        const auto &ents = op.entries[z];
        const int D = (int)t.dims[z].size();
        const int nk = D - 1;
        const bool root = z == t.root;
        // effective generator of the node
        Prog &h = heffP[z];
        reset_host(h);
        h.g = geom_of(t.dims[z]);
        for (int q = 0; q < D; ++q) h.capdims[q] = t.capdims[z][q];
        for (auto &e : ents) {
            DevEntry de = blank_entry();
            de.coef = to_d2(e.coef);
            int nf = 0;
            for (int k = 0; k < nk; ++k)
                if (e.slot[k] >= 1) {
                    de.slot[nf] = k;
                    child_band(de, nf, z, e.slot[k]);
                    de.M[nf++] = child_M(z, k, e.slot[k]);
                }
            if (!root && e.bp != 1) {
                de.slot[nf] = D - 1;
                de.M[nf++] = parent_M(z, e.bp);
            }
            de.nf = nf;
            de.group = 0;
            h.ents.push_back(de);
        }
        merge_entries(h);
        finish_groups(h, {nullptr});
        upload(h);
        plan_pairs(h, z);
        if (!root) {
            // SPO rebuild: groups by own-bond channel (>= 1), children factors only
            Prog &s = spoP[z];
            reset_host(s);
            s.g = h.g;
            for (int q = 0; q < D; ++q) s.capdims[q] = t.capdims[z][q];
            s.contract_slot = D - 1;
            std::map<int, int> gid;
            std::vector<double2 *> dst;
            const int np = t.bond[z];
            for (auto &e : ents) {
                if (e.bp < 1) continue;
                if (!gid.count(e.bp)) {
                    gid[e.bp] = (int)dst.size();
                    dst.push_back(spo[z] + (size_t)e.bp * np * np);
                }
                DevEntry de = blank_entry();
                de.coef = to_d2(e.coef);
                int nf = 0;
                for (int k = 0; k < nk; ++k)
                    if (e.slot[k] >= 1) {
                        de.slot[nf] = k;
                        child_band(de, nf, z, e.slot[k]);
                        de.M[nf++] = child_M(z, k, e.slot[k]);
                    }
                de.nf = nf;
                de.group = gid[e.bp];
                s.ents.push_back(de);
            }
            merge_entries(s);
            finish_groups(s, dst);
            upload(s);
            // backward bond generator K(C) = sum_b U_b C O_b^T on the bond above z
            Prog &b = bondP[z];
            reset_host(b);
            b.g = geom_of({np, np});
            b.capdims[0] = b.capdims[1] = t.cap[z];
            const double2 *Sb = spo[z], *Mb = mf[z];
            if (op.outside_used[z]) {
                DevEntry de = blank_entry();
                de.coef = make_double2(1.0, 0.0);
                de.nf = 1;
                de.slot[0] = 1;
                de.M[0] = Mb;
                b.ents.push_back(de);
            }
            if (op.inside_used[z]) {
                DevEntry de = blank_entry();
                de.coef = make_double2(1.0, 0.0);
                de.nf = 1;
                de.slot[0] = 0;
                de.M[0] = Sb + (size_t)np * np;
                b.ents.push_back(de);
            }
            for (int ch = 2; ch < op.n_ch[z]; ++ch) {
                DevEntry de = blank_entry();
                de.coef = make_double2(1.0, 0.0);
                de.nf = 2;
                de.slot[0] = 0;
                de.M[0] = Sb + (size_t)ch * np * np;
                de.slot[1] = 1;
                de.M[1] = Mb + (size_t)ch * np * np;
                b.ents.push_back(de);
            }
            finish_groups(b, {nullptr});
            upload(b);
        }
        // mean-field rebuilds of every child
        if (t.local_dim[z] == 0) {
            if ((int)mfP[z].size() != nk) mfP[z].assign(nk, Prog{});
            for (int k = 0; k < nk; ++k) {
                const int c = t.kids[z][k];
                const int nc = t.bond[c];
                Prog &m = mfP[z][k];
                reset_host(m);
                m.g = h.g;
                for (int q = 0; q < D; ++q) m.capdims[q] = t.capdims[z][q];
                m.contract_slot = k;
                std::map<int, int> gid;
                std::vector<double2 *> dst;
                for (auto &e : ents) {
                    int ch;
                    if (e.slot[k] == -1) {
                        if (!op.outside_used[c]) continue;
                        ch = 0;
                    } else if (e.slot[k] == 1) {
                        continue;  // inside channel: identity mean field
                    } else {
                        ch = e.slot[k];
                    }
                    if (!gid.count(ch)) {
                        gid[ch] = (int)dst.size();
                        dst.push_back(mf[c] + (size_t)ch * nc * nc);
                    }
                    DevEntry de = blank_entry();
                    de.coef = to_d2(e.coef);
                    int nf = 0;
                    for (int j = 0; j < nk; ++j)
                        if (j != k && e.slot[j] >= 1) {
                            de.slot[nf] = j;
                            child_band(de, nf, z, e.slot[j]);
                            de.M[nf++] = child_M(z, j, e.slot[j]);
                        }
                    if (!root && e.bp != 1) {
                        de.slot[nf] = D - 1;
                        de.M[nf++] = parent_M(z, e.bp);
                    }
                    de.nf = nf;
                    de.group = gid[ch];
                    m.ents.push_back(de);
                }
                merge_entries(m);
                finish_groups(m, dst);
                upload(m);
            }
        }
    }
}

// Leaf channel operators of leaf c (channel 0, the identity, left empty) and
// the band of each; U[c] is allocated on the first call and overwritten after.
void Engine::put_leaf_ops(int c) {
    const int d = t.local_dim[c];
    const int li = t.leaf_index[c];
    std::vector<double2> hu((size_t)op.n_ch[c] * d * d, make_double2(0.0, 0.0));
    for (int ch = 1; ch < op.n_ch[c]; ++ch)
        if (ch < (int)op.leafU[li].size())
            for (size_t q = 0; q < op.leafU[li][ch].size(); ++q) hu[(size_t)ch * d * d + q] = to_d2(op.leafU[li][ch][q]);
    // band of every channel operator (exact zeros outside i - lo <= j <= i + hi)
    ulo[c].assign(op.n_ch[c], d - 1);
    uhi[c].assign(op.n_ch[c], d - 1);
    for (int ch = 1; ch < op.n_ch[c]; ++ch) {
        int lo = 0, hi = 0;
        for (int i = 0; i < d; ++i)
            for (int j = 0; j < d; ++j) {
                const double2 v = hu[(size_t)ch * d * d + (size_t)i * d + j];
                if (v.x != 0.0 || v.y != 0.0) {
                    lo = std::max(lo, i - j);
                    hi = std::max(hi, j - i);
                }
            }
        ulo[c][ch] = lo;
        uhi[c][ch] = hi;
    }
    if (!U[c]) U[c] = (double2 *)dalloc(sizeof(double2) * hu.size());
    h2d(U[c], hu.data(), sizeof(double2) * hu.size());
}

void Engine::set_sop(const SopInput &s) {
    if (opt.hermitian && !sop_is_hermitian(s))
        throw Error(TTN_E_INVALID, "hermitian=1 but the SOP generator is not Hermitian");
    TreeOp newop = compile_tree_operator(t, s);
    HIPCHK(hipStreamSynchronize(st));
    free_sop();
    sop = s;
    op = std::move(newop);
    const int n = t.n;
    spo.assign(n, nullptr);
    mf.assign(n, nullptr);
    U.assign(n, nullptr);
    ulo.assign(n, {});
    uhi.assign(n, {});
    for (int c = 0; c < n; ++c) {
        if (c == t.root) continue;
        const size_t nb = t.cap[c];  // environments sized for the bond capacity
        const size_t bytes = sizeof(double2) * op.n_ch[c] * nb * nb;
        spo[c] = (double2 *)dalloc(bytes);
        mf[c] = (double2 *)dalloc(bytes);
        HIPCHK(hipMemset(spo[c], 0, bytes));
        HIPCHK(hipMemset(mf[c], 0, bytes));
        if (t.local_dim[c] > 0) put_leaf_ops(c);
    }
    build_programs();
    // scratch sizes
    // every size at the bond capacity (bonds may grow)
    int64_t tmp_e = 1, gsum_e = 1, cpart_e = 1, maxN = 1, maxb2 = 1;
    auto capN = [](const Prog &p) {
        int64_t v = 1;
        for (int q = 0; q < p.g.D; ++q) v *= p.capdims[q];
        return v;
    };
    auto fused_at = [](const Prog &p, int64_t N) {
        return N <= SMALL_MAX && (p.g.D == 2 || (int64_t)p.ents.size() * N <= SMALL_SEQ_WORK);
    };
    auto acc = [&](const Prog &p) {
        const int64_t N = capN(p);
        tmp_e = std::max<int64_t>(tmp_e, 2 * (int64_t)p.ents.size() * N);
        gsum_e = std::max<int64_t>(gsum_e, (int64_t)p.n_groups * N);
        if (p.contract_slot >= 0) {
            int nn = p.capdims[p.contract_slot];
            cpart_e = std::max<int64_t>(cpart_e, (int64_t)p.n_groups * 64 * nn * nn);
        }
    };
    bigN = 0;
    for (int z = 0; z < n; ++z) {
        acc(heffP[z]);
        maxN = std::max<int64_t>(maxN, t.capsize[z]);
        if (!fused_at(heffP[z], t.capsize[z])) bigN = std::max<int64_t>(bigN, t.capsize[z]);
        if (z != t.root) {
            acc(spoP[z]);
            acc(bondP[z]);
            int64_t b2 = (int64_t)t.cap[z] * t.cap[z];
            maxb2 = std::max(maxb2, b2);
            if (!fused_at(bondP[z], b2)) bigN = std::max<int64_t>(bigN, b2);
        }
        for (auto &m : mfP[z]) acc(m);
    }
    // subspace expansion: the two-site programs and vectors of every bond
    int64_t ts_v = 1, ts_no = 1, ts_nb = 1;
    int ts_g = 1;
    if (adaptive) {
        tsP.assign(n, TwoSite{});
        for (int c = 0; c < n; ++c) {
            if (c == t.root) continue;
            const int z = t.parent[c];
            const int64_t no = t.capsize[z] / t.cap[c], nbel = t.capsize[c] / t.cap[c];
            ts_no = std::max(ts_no, no);
            ts_nb = std::max(ts_nb, nbel);
            ts_g = std::max(ts_g, op.n_ch[c]);
            tmp_e = std::max<int64_t>(tmp_e, 2 * (int64_t)op.entries[z].size() * no);
            tmp_e = std::max<int64_t>(tmp_e, 2 * (int64_t)op.entries[c].size() * nbel);
            gsum_e = std::max<int64_t>(gsum_e, (int64_t)op.n_ch[c] * std::max(no, nbel));
        }
        ts_v = std::max(ts_no, ts_nb);
        gkl_m = std::min(40, mmax);
    }
    cpart_e = std::max<int64_t>(cpart_e, 64 * 64 * 64);
    // scratch: every buffer below is either allocated here or carved from the
    // caller's workspace (256-byte aligned pieces, zeroed)
    std::vector<std::pair<void **, size_t>> want;
    auto need = [&](auto **ptr, size_t bytes) { want.push_back({(void **)ptr, bytes < 16 ? 16 : bytes}); };
    need(&tmp, sizeof(double2) * tmp_e);
    mprep = nullptr;
    if (opt.precision == TTN_BF16X3) {  // split factors of the matrix-core stages
        size_t ents = 1;
        for (int z = 0; z < n; ++z) {
            ents = std::max(ents, heffP[z].ents.size());
            if (z != t.root) ents = std::max(ents, std::max(spoP[z].ents.size(), bondP[z].ents.size()));
            for (auto &m : mfP[z]) ents = std::max(ents, m.ents.size());
        }
        need(&mprep, sizeof(unsigned short) * ents * 2 * 128 * 128);
    }
    need(&gsum, sizeof(double2) * gsum_e);
    need(&cpart, sizeof(double2) * cpart_e);
    need(&Rbuf, sizeof(double2) * maxb2);
    need(&Cbuf, sizeof(double2) * maxb2);
    need(&smallV, sizeof(double2) * (SMALL_MMAX + 2) * SMALL_MAX);
    int64_t mats = 0;
    for (int z = 0; z < n; ++z) {
        mats += (int64_t)t.cap[z] * t.cap[z];
        if (t.local_dim[z] > 0) mats += (int64_t)t.local_dim[z] * t.local_dim[z];
    }
    obs_elems = 2 * maxN + mats + 64;
    need(&obs, sizeof(double2) * obs_elems);
    bk = BigKrylov{};
    if (bigN > 0) {
        need(&bk.V, sizeof(double2) * (mmax + 1) * bigN);
        need(&bk.Hm, sizeof(double2) * (mmax + 1) * mmax);
        need(&bk.h, sizeof(double2) * (mmax + 1));
        need(&bk.y, sizeof(double2) * (mmax + 1));
        need(&bk.part, sizeof(double) * VEC_BLOCKS * (2 * mmax + 4) * 2);
        need(&bk.scal, sizeof(double) * 4);
        need(&bk.meff, sizeof(int) * 4);
        need(&bk.counter, sizeof(unsigned) * 4);
        need(&bk.G, sizeof(double2) * (mmax + 1) * (mmax + 1));
        need(&bk.refine, sizeof(int) * 4);
    }
    {  // copy of the state taken at the start of every step (restored on failure)
        int64_t tot = 0;
        for (int z = 0; z < n; ++z) tot += t.capsize[z];
        need(&snapshot, sizeof(double2) * tot);
    }
    if (adaptive) {  // subspace expansion vectors, Krylov bases and the bidiagonal's SVD
        need(&ts_in, sizeof(double2) * ts_g * ts_v);
        need(&ts_s, sizeof(double2) * ts_g * 64);
        need(&ts_w1, sizeof(double2) * ts_v);
        need(&ts_w2, sizeof(double2) * ts_v);
        need(&ts_out, sizeof(double2) * 64 * ts_v);
        need(&ts_R, sizeof(double2) * 64 * 64);
        need(&ts_part, sizeof(double2) * 64 * 64 * std::max(ts_g, 1));
        need(&gkl_sc, sizeof(double) * (192 + 2 * 64 * 64));
        need(&gkl_n, sizeof(int) * 4);
        for (BigKrylov *k : {&gkP, &gkQ}) {
            const int64_t N = k == &gkP ? ts_nb : ts_no;
            *k = BigKrylov{};
            need(&k->V, sizeof(double2) * (gkl_m + 1) * N);
            need(&k->Hm, sizeof(double2) * (gkl_m + 1) * gkl_m);
            need(&k->h, sizeof(double2) * (gkl_m + 1));
            need(&k->y, sizeof(double2) * (gkl_m + 1));
            need(&k->part, sizeof(double) * VEC_BLOCKS * (gkl_m + 2) * 2);
            need(&k->scal, sizeof(double) * 4);
            need(&k->meff, sizeof(int) * 4);
            need(&k->counter, sizeof(unsigned) * 4);
        }
    }
    // many-work-group QR scratch
    need(&qrw.tau, sizeof(double2) * 64);
    need(&qrw.scl, sizeof(double2) * 64);
    need(&qrw.diag, sizeof(double2) * 64);
    need(&qrw.snapped, sizeof(int) * 64);
    need(&qrw.w, sizeof(double2) * 64 * 64);
    need(&qrw.rowi, sizeof(double2) * 64);
    need(&qrw.part, sizeof(double) * QRM_BLOCKS_MAX * (2 + 2 * 64));
    need(&qrw.S, sizeof(double2) * QRM_BLOCKS_MAX * 64 * 63 / 2);
    need(&qrw.K, sizeof(double2) * 64 * 64);
    need(&qrw.thr, sizeof(double) * 4);
    need(&qrw.counter, sizeof(unsigned) * 4);
    need(&qrw.cpart, sizeof(double) * 2 * QRM_BLOCKS_MAX * QRC_REC);
    need(&qrw.bar, sizeof(unsigned) * 192);
    qrw.bar_base = 0;
    // complex FP32 copy of the input of pair-form applications
    // complex FP32 copy of an input (FP32 modes): pair-form applications and
    // the shared first-stage input of the staged programs
    pair_x32 = nullptr;
    pair_ws = nullptr;
    if (opt.precision == TTN_FP32 || opt.precision == TTN_BF16X3) need(&pair_x32, sizeof(float2) * maxN);
    // cut tiles of the shared pair-GEMM schedule (FP32 form; BF16x3 form with TTN_PAIR_SPLIT=2)
    if (pair_split > 0) {
        size_t ws = 0;
        for (int z = 0; z < n; ++z)
            if (!heffP[z].pair.empty() && (!heffP[z].pair[0].Wb || pair_split > 1))
                ws = std::max(ws, pair_gemm_ws_bytes(pair_slots, heffP[z].pair[0].Wb ? 1 : 0));
        if (ws) need(&pair_ws, ws);
    }
    // Cholesky route of the QR: Gram partials, small matrices, first-pass factor
    need(&qrw.cq_part, sizeof(double2) * CQR_BLOCKS_MAX * 64 * 64);
    need(&qrw.cq_G, sizeof(double2) * 64 * 64);
    need(&qrw.cq_R1, sizeof(double2) * 64 * 64);
    need(&qrw.cq_R1inv, sizeof(double2) * 64 * 64);
    need(&qrw.cq_M, sizeof(double2) * 64 * 64);
    need(&qrw.cq_Y, sizeof(double2) * maxN);
    qrw.cq_ycap = maxN;
    need(&qrw.cq_scal, sizeof(double) * 4);
    need(&qrw.cq_state, sizeof(int) * 4);
    need(&qrw.cq_counter, sizeof(unsigned) * 4);
    const int n_solves = (2 * n - 1) + 2 * (n - 1);
    need(&d_stats, sizeof(SolveStat) * n_solves);
    size_t total = 0;
    for (auto &w : want) total += (w.second + 255) / 256 * 256;
    ws_need = total;
    if (opt.workspace) {
        if (total > opt.workspace_bytes)
            throw Error(TTN_E_OOM, "workspace too small: the operator needs " + std::to_string(total) +
                                       " bytes of scratch, the workspace has " + std::to_string(opt.workspace_bytes));
        char *base = (char *)opt.workspace;
        HIPCHK(hipMemset(base, 0, total));
        size_t off = 0;
        for (auto &w : want) {
            *w.first = base + off;
            off += (w.second + 255) / 256 * 256;
        }
    } else {
        for (auto &w : want) *w.first = dalloc(w.second);
    }
    // pinned, so that the per-step statistics copy stays asynchronous
    if (h_stats) (void)hipHostFree(h_stats);
    h_stats = nullptr;
    n_stats = n_solves;
    HIPCHK(hipHostMalloc((void **)&h_stats, sizeof(SolveStat) * n_solves, hipHostMallocDefault));
    std::memset(h_stats, 0, sizeof(SolveStat) * n_solves);
    if (!h_flags) HIPCHK(hipHostMalloc((void **)&h_flags, sizeof(unsigned) * 4, hipHostMallocDefault));
    std::memset(h_flags, 0, sizeof(unsigned) * 4);
    m_hint.assign(n_solves, 0);
    solve_node.assign(n_solves, -1);
    solve_fwd.assign(n_solves, 0);
    solve_small.assign(n_solves, 0);
    have_sop = true;
    if (opt.autotune) {  // register tiles of every staged program, timed on the programs themselves
        for (int z = 0; z < n; ++z) {
            auto tune = [&](const Prog &p, const double2 *in) {
                prep(p);
                tune_prog_stages(view(p), in, st);
            };
            if (!use_fused(heffP[z])) tune(heffP[z], A[z]);
            if (z != t.root) {
                tune(spoP[z], A[z]);
                if (!use_fused(bondP[z])) tune(bondP[z], Cbuf);
            }
            for (auto &m : mfP[z]) tune(m, A[z]);
        }
        sync_check("autotune");
    }
    if (have_state) rebuild_all_spos();
    HIPCHK(hipStreamSynchronize(st));
}

// Time-dependent coefficients (Sec. II B): the same terms with new c_r.  The
// operator is compiled again on the host; when its structure is unchanged,
// the leaf channel operators and the program tables (entry coefficients,
// combination weights, pair-operator terms) are rewritten in place, with no
// device allocation, and the environments are rebuilt from the state.
bool Engine::set_coefficients(const double *coeff, int n_terms) {
    if (!have_sop) throw Error(TTN_E_STATE, "no SOP generator set");
    if (!coeff || n_terms != sop.n_terms)
        throw Error(TTN_E_INVALID, "set_coefficients needs the " + std::to_string(sop.n_terms) +
                                       " coefficients of the terms in place");
    SopInput s = sop;
    for (int r = 0; r < n_terms; ++r) {
        const cplx c(coeff[2 * r], coeff[2 * r + 1]);
        if (!std::isfinite(c.real()) || !std::isfinite(c.imag()))
            throw Error(TTN_E_INVALID, "non-finite coefficient in term " + std::to_string(r));
        s.coeff[r] = c;
    }
    if (opt.hermitian && !sop_is_hermitian(s))
        throw Error(TTN_E_INVALID, "hermitian=1 but the SOP generator with these coefficients is not Hermitian");
    TreeOp newop = compile_tree_operator(t, s);
    if (!same_tree_operator_structure(op, newop)) {
        set_sop(s);
        return true;
    }
    // kernels in flight read the tables rewritten below, and earlier staged
    // copies read the staging chunks reused below
    HIPCHK(hipStreamSynchronize(st));
    sop = std::move(s);
    op = std::move(newop);
    const size_t n_alloc = sop_allocs.size();
    const auto lo0 = ulo, hi0 = uhi;
    stage_cur = stage_off = 0;
    struct Staged {
        bool &f;
        ~Staged() { f = false; }
    } staged_guard{staged};
    staged = true;  // tables whose bytes did not change are skipped, the rest copied on the stream
    for (int c = 0; c < t.n; ++c)
        if (c != t.root && t.local_dim[c] > 0) put_leaf_ops(c);
    // step graphs read the rewritten tables through their device pointers; the
    // launch sequence itself depends on the values only through the bands of
    // the leaf channel operators (banded or dense stage kernels)
    if (ulo != lo0 || uhi != hi0) drop_graphs();
    for (int z = 0; z < t.n; ++z) build_node_programs(z);
    if (sop_allocs.size() != n_alloc) throw Error(TTN_E_STATE, "internal: coefficient update allocated");
    if (have_state) rebuild_all_spos();
    HIPCHK(hipStreamSynchronize(st));
    return false;
}

// ------------------------------------------------------------------ state
size_t Engine::state_bytes() const {
    size_t s = 0;
    for (int z = 0; z < t.n; ++z) s += (size_t)t.size[z];
    return s * sizeof(double2);
}

void Engine::set_product_state(const double *leaf_vecs) {
    if (!leaf_vecs) throw Error(TTN_E_INVALID, "null leaf vectors");
    std::vector<std::vector<double2>> host(t.n);
    size_t off = 0;
    for (int z = 0; z < t.n; ++z) {
        const auto &dims = t.dims[z];
        std::vector<double2> T((size_t)t.size[z], make_double2(0.0, 0.0));
        if (t.local_dim[z] > 0) {
            const int d = dims[0], nb = dims[1];
            const size_t li = (size_t)t.leaf_index[z];
            (void)li;
            // vectors are concatenated in leaf-id order
            std::vector<cplx> v(d);
            double nr = 0.0;
            for (int i = 0; i < d; ++i) {
                v[i] = cplx(leaf_vecs[2 * (off + i)], leaf_vecs[2 * (off + i) + 1]);
                nr += std::norm(v[i]);
            }
            off += d;
            nr = std::sqrt(nr);
            if (!(nr > 0.0) || !std::isfinite(nr)) throw Error(TTN_E_INVALID, "zero or non-finite leaf vector");
            std::vector<std::vector<cplx>> cols;
            std::vector<cplx> q0(d);
            for (int i = 0; i < d; ++i) q0[i] = v[i] / nr;
            cols.push_back(q0);
            int j = 0;
            while ((int)cols.size() < nb && j < d) {
                std::vector<cplx> e(d, cplx(0.0));
                e[j] = 1.0;
                for (auto &q : cols) {  // modified Gram-Schmidt
                    cplx dot(0.0);
                    for (int i = 0; i < d; ++i) dot += std::conj(q[i]) * e[i];
                    for (int i = 0; i < d; ++i) e[i] -= dot * q[i];
                }
                double en = 0.0;
                for (int i = 0; i < d; ++i) en += std::norm(e[i]);
                en = std::sqrt(en);
                if (en > 1e-6) {
                    for (int i = 0; i < d; ++i) e[i] /= en;
                    cols.push_back(e);
                }
                ++j;
            }
            for (int c = 0; c < (int)cols.size(); ++c)
                for (int i = 0; i < d; ++i) T[(size_t)i * nb + c] = to_d2(cols[c][i]);
        } else {
            const int np = dims.back();
            const int64_t rows = t.size[z] / np;
            for (int c = 0; c < np && c < rows; ++c) T[(size_t)c * np + c] = make_double2(1.0, 0.0);
        }
        host[z] = std::move(T);
    }
    for (int z = 0; z < t.n; ++z) {
        HIPCHK(hipMemcpyAsync(A[z], host[z].data(), sizeof(double2) * t.size[z], hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(A0[z], A[z], sizeof(double2) * t.size[z], hipMemcpyDeviceToDevice, st));
    }
    have_state = true;
    if (have_sop) rebuild_all_spos();
    HIPCHK(hipStreamSynchronize(st));
}

void Engine::set_state(const double *buf, size_t bytes) {
    if (!buf || bytes != state_bytes()) throw Error(TTN_E_DIMS, "state buffer size mismatch");
    size_t off = 0;
    for (int z = 0; z < t.n; ++z) {
        HIPCHK(hipMemcpyAsync(A[z], buf + 2 * off, sizeof(double2) * t.size[z], hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(A0[z], A[z], sizeof(double2) * t.size[z], hipMemcpyDeviceToDevice, st));
        off += t.size[z];
    }
    have_state = true;
    if (have_sop) rebuild_all_spos();
    HIPCHK(hipStreamSynchronize(st));
}

void Engine::get_state(double *buf, size_t bytes) {
    if (!buf || bytes != state_bytes()) throw Error(TTN_E_DIMS, "state buffer size mismatch");
    size_t off = 0;
    for (int z = 0; z < t.n; ++z) {
        HIPCHK(hipMemcpyAsync(buf + 2 * off, A[z], sizeof(double2) * t.size[z], hipMemcpyDeviceToHost, st));
        off += t.size[z];
    }
    HIPCHK(hipStreamSynchronize(st));
}

void Engine::rebuild_all_spos() {
    for (int c : t.postorder)
        if (c != t.root) build_spo(c);
}

// ------------------------------------------------------------ building blocks
void Engine::apply_prog(const Prog &p, const double2 *in, double2 *out) {
    prep(p);
    ProgView v = view(p);
    launch_apply(p, v, in, out);
}

void Engine::launch_apply(const Prog &p, const ProgView &v, const double2 *in, double2 *out) {
    if (!p.pair.empty()) {
        if (!pair_x32) throw Error(TTN_E_STATE, "internal: pair-form scratch not allocated");
        if (p.pair[0].Wb) {  // BF16x3: hi and lo parts of the input (4 + 4 bytes per element)
            unsigned *xh = reinterpret_cast<unsigned *>(pair_x32), *xl = xh + p.g.N;
            launch_to_bf16x2(in, xh, xl, p.g.N, st);
            for (size_t i = 0; i < p.pair.size(); ++i)
                launch_pair_gemm_bf(p.pair[i], xh, xl, out, i > 0 ? 1 : 0, p.pair_flops[i],
                                    pair_split > 1 ? pair_ws : nullptr, pair_slots, st);
        } else {
            launch_to_f32(in, pair_x32, p.g.N, st);
            for (size_t i = 0; i < p.pair.size(); ++i)
                launch_pair_gemm(p.pair[i], pair_x32, out, i > 0 ? 1 : 0, p.pair_flops[i], pair_ws, pair_slots, st);
        }
        return;
    }
    launch_prog_stages(v, in, st, pair_x32);
    launch_prog_sum(v, in, out, st);
}

// Pair-operator form of node z's effective generator in the FP32 mode: when
// every product carries at most one child factor besides the parent factor,
// the products of child slot k make up W_k = sum_e c_e F_e (x) P_e on the
// index pair (k, parent), applied as one GEMM on the matrix cores; products
// with the parent factor alone (or none) join the pass with the most products.
// Taken for large nodes when each dense pair operator costs at most twice the
// flops of the products it replaces.
void Engine::plan_pairs(Prog &h, int z) {
    h.pair.clear();
    h.pair_flops.clear();
    if ((opt.precision != TTN_FP32 && opt.precision != TTN_BF16X3) || !pair_ops || z == t.root || t.local_dim[z] > 0)
        return;
    const int D = h.g.D, P = D - 1;
    int64_t ncap = 1;
    for (int q = 0; q < D; ++q) ncap *= h.capdims[q];
    if (ncap < pair_min_n || h.n_groups != 1 || h.contract_slot >= 0 || P < 1) return;
    std::vector<std::vector<PairTerm>> per(P);
    std::vector<double> work(P, 0.0), wcur(P, 0.0);  // summed factor dims (capacity / current)
    std::vector<PairTerm> loose;
    double loose_work = 0.0, loose_cur = 0.0;
    for (const DevEntry &e : h.ents) {
        if (e.src != 0) return;
        int k = -1;
        const double2 *F = nullptr, *Pm = nullptr;
        for (int f = 0; f < e.nf; ++f) {
            if (e.slot[f] == P) {
                Pm = e.M[f];
            } else if (k < 0) {
                k = e.slot[f];
                F = e.M[f];
            } else {
                return;  // two child factors: no pair form
            }
        }
        const double w = (F ? h.capdims[k] : 0) + (Pm ? h.capdims[P] : 0);
        const double wc = (F ? h.g.dims[k] : 0) + (Pm ? h.g.dims[P] : 0);
        if (k < 0) {
            loose.push_back({e.coef, nullptr, Pm});
            loose_work += w;
            loose_cur += wc;
        } else {
            per[k].push_back({e.coef, F, Pm});
            work[k] += w;
            wcur[k] += wc;
        }
    }
    int home = -1;
    for (int k = 0; k < P; ++k)
        if (!per[k].empty() && (home < 0 || per[k].size() > per[home].size())) home = k;
    if (home < 0) {
        if (loose.empty()) return;
        home = 0;
    }
    for (auto &x : loose) per[home].push_back(x);
    work[home] += loose_work;
    wcur[home] += loose_cur;
    for (int k = 0; k < P; ++k) {
        if (per[k].empty()) continue;
        const double qcap = (double)h.capdims[k] * h.capdims[P];
        if (qcap > 4096 || qcap > 2.0 * work[k]) return;
    }
    if ((int)h.pair_w.size() != P) {
        h.pair_w.assign(P, nullptr);
        h.pair_wb.assign(P, nullptr);
        h.pair_dterms.assign(P, nullptr);
        h.pair_cap_terms.assign(P, 0);
    }
    // BF16x3 form of the GEMM where the parent dimension keeps 32-kappa chunks
    // inside one child index (else the FP32 form serves the BF16x3 mode)
    const bool bf = opt.precision == TTN_BF16X3 && h.capdims[P] % 32 == 0 && h.g.dims[P] % 32 == 0;
    for (int k = 0; k < P; ++k) {
        if (per[k].empty()) continue;
        const int64_t qcap = (int64_t)h.capdims[k] * h.capdims[P];
        if (!h.pair_w[k]) h.pair_w[k] = (float2 *)dalloc(sizeof(float2) * qcap * qcap);
        if (bf && !h.pair_wb[k]) h.pair_wb[k] = (unsigned short *)dalloc(sizeof(unsigned short) * 8 * qcap * qcap);
        if (h.pair_cap_terms[k] < (int)per[k].size()) {
            if (h.pair_dterms[k]) throw Error(TTN_E_STATE, "internal: pair-operator terms grew");
            h.pair_dterms[k] = (PairTerm *)dalloc(sizeof(PairTerm) * per[k].size());
            h.pair_cap_terms[k] = (int)per[k].size();
        }
        h2d(h.pair_dterms[k], per[k].data(), sizeof(PairTerm) * per[k].size());
        PairPass pp{};
        pp.nk = h.g.dims[k];
        pp.np = h.g.dims[P];
        pp.L = h.g.L[k];
        pp.Mid = h.g.R[k] / h.g.dims[P];
        pp.W = h.pair_w[k];
        pp.terms = h.pair_dterms[k];
        pp.n_terms = (int)per[k].size();
        pp.Wb = bf ? h.pair_wb[k] : nullptr;
        pp.v4 = (pair_v4 && pp.np % 4 == 0) ? 1 : 0;
        h.pair.push_back(pp);
        h.pair_flops.push_back(8.0 * (double)h.g.N * wcur[k]);
    }
}

void Engine::build_spo(int c) {
    const Prog &p = spoP[c];
    if (p.n_groups == 0) return;
    prep(p);
    ProgView v = view(p);
    launch_prog_stages(v, A[c], st, pair_x32);
    launch_prog_sum(v, A[c], nullptr, st);
    launch_prog_contract(v, A[c], st);
}

void Engine::build_mf(int z, int k) {
    const Prog &p = mfP[z][k];
    if (p.n_groups == 0) return;
    prep(p);
    ProgView v = view(p);
    launch_prog_stages(v, A[z], st, pair_x32);
    launch_prog_sum(v, A[z], nullptr, st);
    launch_prog_contract(v, A[z], st);
}

void Engine::qr_slot(int z, int s, double2 *Rout, int transR) { qr_any(A[z], heffP[z].g, s, Rout, transR); }

void Engine::qr_any(double2 *X, const Geom &g, int s, double2 *Rout, int transR) {
    // wide factors of mid-size tensors also leave the single work-group kernel:
    // its column loop is sequential on one compute unit
    const bool coop = g.N >= QR_MULTI_MIN || (g.N >= 4096 && g.dims[s] >= 16);
    // large matrices first take the Cholesky route; the Householder kernels
    // behind it run only when the matrix is outside its range (device flag)
    qrw.gate = nullptr;
    if (coop && cholqr && launch_qr_chol(X, g.L[s], g.dims[s], g.R[s], Rout, transR, qrw, st)) qrw.gate = qrw.cq_state;
    if (coop && !graph_mode && launch_qr_coop(X, g.L[s], g.dims[s], g.R[s], Rout, transR, qrw, st)) return;
    if (g.N >= QR_MULTI_MIN) launch_qr_multi(X, g.L[s], g.dims[s], g.R[s], Rout, transR, qrw, st);
    else launch_qr(X, g.L[s], g.dims[s], g.R[s], Rout, transR, st, qrw.gate);
}

void Engine::absorb(int z, int s, const double2 *M, int transM) {
    const Geom g = heffP[z].g;
    launch_mode_product(A[z], Aalt[z], M, g.L[s], g.dims[s], g.dims[s], g.R[s], transM, st);
    std::swap(A[z], Aalt[z]);
}

// The fused one-work-group solver takes two-slot problems and problems with
// few entries (its generic matvec applies entries one after the other); all
// other local exponentials use the multi-kernel Krylov path.
bool Engine::use_fused(const Prog &p) const {
    return p.g.N <= SMALL_MAX && (p.g.D == 2 || (int64_t)p.ents.size() * p.g.N <= SMALL_SEQ_WORK);
}

// Relative error target of the local exponentials: the option, else 1e-13 in
// FP64 and 1e-10 in the FP32 modes.  A looser FP32 target (1e-8, still below
// the ~1e-7 relative rounding of the FP32 contractions) saves about 9 % of the
// matrix-vector products on the exciton tree but let a multi-kernel solve of
// a seeded spin-boson tree (79 nodes, bonds up to 40) fail at the Krylov limit
// within three steps, where 1e-10 converges.
double Engine::krylov_tolerance() const {
    if (opt.krylov_tol > 0) return opt.krylov_tol;
    return opt.precision == TTN_FP64 ? 1e-13 : 1e-10;
}

void Engine::expm_prog(const Prog &p, double2 *x, double tau, int node, bool fwd) {
    const int si = solve_idx++;
    if (si >= n_stats) throw Error(TTN_E_STATE, "internal: solve index overflow");
    solve_node[si] = node;
    solve_fwd[si] = fwd ? 1 : 0;
    const bool fused = use_fused(p);
    solve_small[si] = fused ? 1 : 0;
    SolveStat *stat = d_stats + si;
    const double tol = krylov_tolerance();
    prep(p);
    if (fused) {
        SmallSolveArgs a{};
        a.g = p.g;
        a.ent = p.d_ent;
        a.n_ent = (int)p.ents.size();
        a.x = x;
        a.V = smallV;
        a.tau = tau;
        a.tol = tol;
        a.mmax = std::min(mmax, SMALL_MMAX);
        a.hermitian = opt.hermitian;
        a.m_hint = m_hint[si] > 0 ? m_hint[si] : 8;
        a.stat = stat;
        a.ground = ground ? 1 : 0;
        // two-slot problems use the batched matvec when its temporaries fit in LDS
        int nA = 0;
        for (auto &e : p.ents)
            if (e.nf >= 1 && e.slot[e.nf - 1] == 1) ++nA;
        a.nA = nA;
        a.batched = (p.g.D == 2 && (int)p.ents.size() <= SMALL_MAXENT && p.g.dims[0] * p.g.dims[0] <= SMALL_UB &&
                     small_solve_lds_bytes(p.g.N, a.mmax, 1, nA) + SMALL_STATIC_LDS <= 160 * 1024)
                        ? 1
                        : 0;
        // LDS beyond the solver's own data: first the factor matrices (read on
        // every matvec), then the Krylov basis, each when it fits
        size_t lds = small_solve_lds_bytes(p.g.N, a.mmax, a.batched, nA) + SMALL_STATIC_LDS;
        a.mlds = 0;
        a.mlds_elems = 0;
        if (a.batched) {
            int64_t elems = 0;
            for (auto &e : p.ents) {
                if (e.nf >= 1 && e.slot[0] == 0) elems += (int64_t)p.g.dims[0] * p.g.dims[0];
                if (e.nf >= 1 && e.slot[e.nf - 1] == 1) elems += (int64_t)p.g.dims[1] * p.g.dims[1];
            }
            if (lds + sizeof(double2) * (size_t)elems <= 160 * 1024) {
                a.mlds = 1;
                a.mlds_elems = (int)elems;
                lds += sizeof(double2) * (size_t)elems;
            }
        }
        a.vlds = lds + small_solve_vlds_bytes(p.g.N, a.mmax) <= 160 * 1024 ? 1 : 0;
        if (defer_fused) deferred.push_back(a);  // launched with other instances' solves
        else launch_small_solve(a, st);
    } else {
        if (!bk.V) throw Error(TTN_E_STATE, "internal: Krylov scratch not allocated");
        if (ground) {  // one Lanczos pass of the largest dimension, then the lowest Ritz pair
            const int64_t N = p.g.N;
            const int m = (int)std::min<int64_t>(mmax, N);
            launch_krylov_start(x, N, bk, st);
            ProgView v = view(p);
            for (int j = 0; j < m; ++j) {
                launch_apply(p, v, bk.V + (size_t)j * N, bk.V + (size_t)(j + 1) * N);
                if (krylov_cgs2) launch_krylov_orth(bk, N, j, mmax, st);
                else launch_krylov_orth1(bk, N, j, mmax, st);
            }
            launch_krylov_ground(bk, N, m, mmax, x, stat, st);
            return;
        }
        int m = m_hint[si] > 0 ? m_hint[si] : 20;
        m = std::max(3, std::min(m, mmax));
        m = (int)std::min<int64_t>(m, p.g.N);
        m_hint[si] = m;
        const int64_t N = p.g.N;
        launch_krylov_start(x, N, bk, st);
        ProgView v = view(p);
        for (int j = 0; j < m; ++j) {
            launch_apply(p, v, bk.V + (size_t)j * N, bk.V + (size_t)(j + 1) * N);
            if (krylov_cgs2) launch_krylov_orth(bk, N, j, mmax, st);
            else launch_krylov_orth1(bk, N, j, mmax, st);
        }
        launch_krylov_finish(bk, N, m, mmax, tau, tol, opt.hermitian, x, stat, st);
    }
}

void Engine::forward(int z, double tau) { expm_prog(heffP[z], A[z], tau, z, true); }

void Engine::backward(int c, double2 *C, double tau) {
    if (ground) return;  // ground-state sweeps: the bond factor is absorbed unchanged
    expm_prog(bondP[c], C, -tau, c, false);
}

// ------------------------------------------------------ subspace expansion
// Paper Sec. II D: when the sweep crosses the bond between node z and its
// k-th child c, the bond is widened by new functions with zero coefficients
// along the dominant singular vectors of the two-site residual
//   R = (1 - P_c) X (1 - P_o^T),  X = the two-site projection of G Psi,
// matricised (indices below c) x (indices outside c), P_c the projector on the
// columns of A^c and P_o on the columns of A^z along k.  X acts at one-site
// cost through the bond's channels: the compiled operator splits G on this
// bond as sum_b S_b (x) M_b, where S_b (below c) is the channel-b combination
// of c's node entries and M_b (outside c) that of z's entries carrying channel
// b on slot k, so X w = sum_b S_b A^c A^z^T M_b^T w.  The singular pairs come
// from a Golub-Kahan-Lanczos bidiagonalisation with full re-orthogonalisation.

// Replace every factor of p by its transformed copy (mode 1: transpose, 2:
// conjugate, 3: conjugate transpose), recomputed by prep() before each use.
void Engine::transform_factors(Prog &p, int mode) {
    std::map<const double2 *, double2 *> done;
    std::vector<std::pair<const double2 *, int>> order;
    for (auto &e : p.ents)
        for (int f = 0; f < e.nf; ++f)
            if (!done.count(e.M[f])) {
                done[e.M[f]] = nullptr;
                order.push_back({e.M[f], p.g.dims[e.slot[f]]});
            }
    if (p.comb_bufs.empty()) {
        for (auto &o : order) {
            (void)o;
            p.comb_bufs.push_back((double2 *)dalloc(sizeof(double2) * 64 * 64));
        }
    }
    if (p.comb_bufs.size() != order.size()) throw Error(TTN_E_STATE, "internal: two-site factor count changed");
    for (size_t q = 0; q < order.size(); ++q) {
        CombJob j{};
        j.dst = p.comb_bufs[q];
        j.n = order[q].second;
        j.n2 = j.n * j.n;
        j.first = (int)p.csrcs.size();
        j.count = 1;
        j.mode = mode;
        p.csrcs.push_back({make_double2(1.0, 0.0), order[q].first});
        p.cjobs.push_back(j);
        p.comb_max_n2 = std::max(p.comb_max_n2, j.n2);
        done[order[q].first] = j.dst;
    }
    for (auto &e : p.ents)
        for (int f = 0; f < e.nf; ++f) {
            e.M[f] = done[e.M[f]];
            if (mode & 1) std::swap(e.lo[f], e.hi[f]);  // the band of the transpose
        }
}

// Host tables of the four two-site programs of the bond above c = kids[z][k]
// for the current bonds (device tables allocated at the first build).
void Engine::build_two_site(int z, int k) {
    const int c = t.kids[z][k];
    TwoSite &T = tsP[c];
    const int D = (int)t.dims[z].size();
    const bool root = z == t.root;
    const int np = t.bond[z];
    std::set<int> cb, zb;
    for (auto &e : op.entries[c]) cb.insert(e.bp);
    for (auto &e : op.entries[z]) zb.insert(e.slot[k] == -1 ? 0 : e.slot[k]);
    T.chans.clear();
    for (int b : cb)
        if (zb.count(b)) T.chans.push_back(b);
    std::map<int, int> gid;
    for (size_t g = 0; g < T.chans.size(); ++g) gid[T.chans[g]] = (int)g;
    const int G = (int)T.chans.size();
    // outside geometry: z's slots with slot k of size 1; below geometry: c's
    // slots with the parent slot of size 1
    std::vector<int> dw = t.dims[z], dv = t.dims[c];
    dw[k] = 1;
    dv.back() = 1;
    std::vector<int> cw = t.capdims[z], cv = t.capdims[c];
    cw[k] = 1;
    cv.back() = 1;
    auto setg = [&](Prog &p, const std::vector<int> &d, const std::vector<int> &cd) {
        reset_host(p);
        p.g = geom_of(d);
        for (size_t q = 0; q < cd.size(); ++q) p.capdims[q] = cd[q];
    };
    setg(T.OT, dw, cw);
    setg(T.OC, dw, cw);
    setg(T.B, dv, cv);
    setg(T.BH, dv, cv);
    for (auto &e : op.entries[z]) {
        const int b = e.slot[k] == -1 ? 0 : e.slot[k];
        if (!gid.count(b)) continue;
        DevEntry de = blank_entry();
        de.coef = to_d2(e.coef);
        int nf = 0;
        for (int j = 0; j < D - 1; ++j)
            if (j != k && e.slot[j] >= 1) {
                const int cj = t.kids[z][j];
                de.slot[nf] = j;
                de.M[nf++] = spo[cj] + (size_t)e.slot[j] * t.bond[cj] * t.bond[cj];
            }
        if (!root && e.bp != 1) {
            de.slot[nf] = D - 1;
            de.M[nf++] = mf[z] + (size_t)e.bp * np * np;
        }
        de.nf = nf;
        DevEntry a = de, o = de;
        a.group = gid[b];  // X: outside factors transposed, outputs by channel
        T.OT.ents.push_back(a);
        o.group = 0;  // X^dag: conjugated factors, each entry reads its channel's input
        o.src = gid[b];
        o.coef.y = -o.coef.y;
        T.OC.ents.push_back(o);
    }
    const bool leaf = t.local_dim[c] > 0;
    const int d = t.local_dim[c];
    for (auto &e : op.entries[c]) {
        if (!gid.count(e.bp)) continue;
        DevEntry de = blank_entry();
        de.coef = to_d2(e.coef);
        int nf = 0;
        if (leaf) {
            if (e.slot[0] >= 1) {
                de.slot[0] = 0;
                if (e.slot[0] < (int)ulo[c].size()) {
                    de.lo[0] = ulo[c][e.slot[0]];
                    de.hi[0] = uhi[c][e.slot[0]];
                }
                de.M[nf++] = U[c] + (size_t)e.slot[0] * d * d;
            }
        } else {
            for (int j = 0; j < (int)t.kids[c].size(); ++j)
                if (e.slot[j] >= 1) {
                    const int cj = t.kids[c][j];
                    de.slot[nf] = j;
                    de.M[nf++] = spo[cj] + (size_t)e.slot[j] * t.bond[cj] * t.bond[cj];
                }
        }
        de.nf = nf;
        DevEntry a = de, h = de;
        a.group = 0;  // X: below factors, each entry reads its channel's input
        a.src = gid[e.bp];
        T.B.ents.push_back(a);
        h.group = gid[e.bp];  // X^dag: conjugate-transposed factors, outputs by channel
        h.coef.y = -h.coef.y;
        T.BH.ents.push_back(h);
    }
    transform_factors(T.OT, 1);
    transform_factors(T.OC, 2);
    transform_factors(T.BH, 3);
    finish_groups(T.OT, std::vector<double2 *>(G, nullptr));
    finish_groups(T.OC, {nullptr});
    finish_groups(T.B, {nullptr});
    finish_groups(T.BH, std::vector<double2 *>(G, nullptr));
    upload(T.OT);
    upload(T.OC);
    upload(T.B);
    upload(T.BH);
}

// x <- x - Q op(Q)^H... : with the columns of the (L, n, R) tensor Q along its
// middle index, x <- x - Q (Q^H x) (conjQ = 0) or x - conj(Q) (Q^T x) (conjQ = 1)
void Engine::project_out(const double2 *Q, int64_t L, int n, int64_t R, int conjQ, double2 *x) {
    launch_ts_contract(Q, L, n, R, conjQ ? 0 : 1, x, 0, 1, ts_s, ts_part, st);
    launch_ts_expand(Q, L, n, R, conjQ ? 1 : 0, ts_s, 1, x, 1, x, st);
}

// p = R q (q outside c, p below c)
void Engine::apply_R(int z, int k, const double2 *Qc, const double2 *Qo, const double2 *q, double2 *p) {
    const int c = t.kids[z][k];
    TwoSite &T = tsP[c];
    const Geom gz = heffP[z].g;
    const int nb = t.bond[c];
    const int64_t no = t.size[z] / nb, nbel = t.size[c] / nb;
    const int G = (int)T.chans.size();
    launch_copy(ts_w1, q, no, st);
    project_out(Qo, gz.L[k], nb, gz.R[k], 1, ts_w1);  // (1 - P_o^T) q
    ProgView vo = view(T.OT);
    vo.f32 = vo.bf16x3 = 0;
    launch_prog_stages(vo, ts_w1, st);
    launch_prog_sum(vo, ts_w1, nullptr, st);  // u_b = M_b^T q', channel sums
    launch_ts_contract(A[z], gz.L[k], nb, gz.R[k], 0, gsum, no, G, ts_s, ts_part, st);   // A^z^T u_b
    launch_ts_expand(A[c], nbel, nb, 1, 0, ts_s, G, nullptr, 0, ts_in, st);            // A^c (.)
    ProgView vb = view(T.B);
    vb.f32 = vb.bf16x3 = 0;
    vb.in_stride = nbel;
    launch_prog_stages(vb, ts_in, st);
    launch_prog_sum(vb, ts_in, p, st);  // sum_b S_b v_b
    project_out(Qc, nbel, nb, 1, 0, p);  // (1 - P_c) y
}

// w = R^dag y (y below c, w outside c)
void Engine::apply_RH(int z, int k, const double2 *Qc, const double2 *Qo, const double2 *y, double2 *w) {
    const int c = t.kids[z][k];
    TwoSite &T = tsP[c];
    const Geom gz = heffP[z].g;
    const int nb = t.bond[c];
    const int64_t nbel = t.size[c] / nb;
    const int G = (int)T.chans.size();
    launch_copy(ts_w2, y, nbel, st);
    project_out(Qc, nbel, nb, 1, 0, ts_w2);  // (1 - P_c) y
    ProgView vh = view(T.BH);
    vh.f32 = vh.bf16x3 = 0;
    launch_prog_stages(vh, ts_w2, st);
    launch_prog_sum(vh, ts_w2, nullptr, st);  // S_b^dag y', channel sums
    launch_ts_contract(A[c], nbel, nb, 1, 1, gsum, nbel, G, ts_s, ts_part, st);           // A^c^dag (.)
    launch_ts_expand(A[z], gz.L[k], nb, gz.R[k], 1, ts_s, G, nullptr, 0, ts_in, st);     // conj(A^z) (.)
    ProgView vc = view(T.OC);
    vc.f32 = vc.bf16x3 = 0;
    vc.in_stride = t.size[z] / nb;
    launch_prog_stages(vc, ts_in, st);
    launch_prog_sum(vc, ts_in, w, st);  // sum_b conj(M_b) q_b
    project_out(Qo, gz.L[k], nb, gz.R[k], 1, w);  // (1 - conj(P_o)) w
}

// Zero-pad (or truncate the zero padding of) Psi(0) along the bond above c.
void Engine::resize_psi0(int c, int nb_new) {
    const int z = t.parent[c];
    const int k = (int)(std::find(t.kids[z].begin(), t.kids[z].end(), c) - t.kids[z].begin());
    const int nb = t.bond[c];
    const Geom gz = geom_of(t.dims[z]);
    const int64_t nbel = t.size[c] / nb;
    launch_repack(A0[c], Aalt[c], nbel, nb, nb_new, 1, nullptr, 0, 0, st);
    launch_copy(A0[c], Aalt[c], nbel * nb_new, st);
    launch_repack(A0[z], Aalt[z], gz.L[k], nb, nb_new, gz.R[k], nullptr, 0, 0, st);
    launch_copy(A0[z], Aalt[z], gz.L[k] * nb_new * gz.R[k], st);
}

// One expansion attempt at the bond above c = kids[z][k] with substep h.
// below: centre at c, new functions of c (left singular vectors); otherwise
// centre at z, new single hole functions of c (conjugated right singular
// vectors).  Returns true when the bond grew (programs of z and c rebuilt).
bool Engine::spawn(int z, int k, double h, bool below) {
    const int c = t.kids[z][k];
    const int nb = t.bond[c];
    const int64_t no = t.size[z] / nb, nbel = t.size[c] / nb;
    const int room = (int)std::min<int64_t>({(int64_t)t.cap[c], nbel, no}) - nb;
    if (room <= 0) return false;
    build_two_site(z, k);
    for (Prog *p : {&tsP[c].OT, &tsP[c].OC, &tsP[c].BH}) prep(*p);
    const Geom gz = heffP[z].g, gc = heffP[c].g;
    // orthonormal bases of the two spans: the isometry where there is one, the
    // Householder Q of a copy of the centre tensor otherwise
    const double2 *Qc = A[c], *Qo = A[z];
    if (below) {
        launch_copy(Aalt[c], A[c], t.size[c], st);
        qr_any(Aalt[c], gc, gc.D - 1, ts_R, 0);
        Qc = Aalt[c];
    } else {
        launch_copy(Aalt[z], A[z], t.size[z], st);
        qr_any(Aalt[z], gz, k, ts_R, 0);
        Qo = Aalt[z];
    }
    const int m = (int)std::min<int64_t>({(int64_t)gkl_m, nbel, no});
    double *alpha = gkl_sc, *beta = gkl_sc + 64, *sv = gkl_sc + 128, *Ub = gkl_sc + 192, *Vb = Ub + 64 * 64;
    BigKrylov P = gkP, Q = gkQ;
    // start in the row space of R: q_0 = R^dag u for a seeded u below c
    launch_seed_vector(ts_out, nbel, opt.seed + 0x5851F42D4C957F2Dull * (++spawn_calls), st);
    apply_RH(z, k, Qc, Qo, ts_out, ts_w1);
    launch_krylov_start(ts_w1, no, Q, st);
    for (int j = 0; j < m; ++j) {
        double2 *pj = P.V + (size_t)j * nbel;
        apply_R(z, k, Qc, Qo, Q.V + (size_t)j * no, pj);
        if (j == 0) {
            launch_krylov_start(pj, nbel, P, st);  // alpha_0
            launch_copy_scalars(alpha, P.scal, 1, st);
        } else {
            launch_krylov_orth(P, nbel, j - 1, gkl_m, st);  // alpha_j
            launch_copy_scalars(alpha + j, P.scal + 1, 1, st);
        }
        if (j == m - 1) break;
        apply_RH(z, k, Qc, Qo, pj, Q.V + (size_t)(j + 1) * no);
        launch_krylov_orth(Q, no, j, gkl_m, st);  // beta_j
        launch_copy_scalars(beta + j, Q.scal + 1, 1, st);
    }
    launch_gkl_count(P.meff, Q.meff, alpha, m, gkl_n, st);
    launch_bidiag_svd(alpha, beta, gkl_n, 64, sv, Ub, Vb, st);
    double hs[65];
    int hn = 0;
    HIPCHK(hipMemcpyAsync(hs, sv, sizeof(double) * 64, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(&hn, gkl_n, sizeof(int), hipMemcpyDeviceToHost, st));
    sync_check("subspace expansion");
    int take = 0;
    while (take < std::min(room, hn) && std::fabs(h) * hs[take] >= opt.spawn_tol) ++take;
    if (take == 0) return false;
    if (below) {
        launch_basis_combine(P.V, nbel, gkl_n, Ub, 64, take, ts_out, st);
        launch_repack(A[c], Aalt[c], nbel, nb, nb + take, 1, ts_out, nbel, 0, st);
        launch_repack(A[z], Aalt[z], gz.L[k], nb, nb + take, gz.R[k], nullptr, 0, 0, st);
    } else {
        launch_basis_combine(Q.V, no, gkl_n, Vb, 64, take, ts_out, st);
        launch_repack(A[z], Aalt[z], gz.L[k], nb, nb + take, gz.R[k], ts_out, no, 1, st);
        launch_repack(A[c], Aalt[c], nbel, nb, nb + take, 1, nullptr, 0, 0, st);
    }
    std::swap(A[c], Aalt[c]);
    std::swap(A[z], Aalt[z]);
    resize_psi0(c, nb + take);
    t.bond[c] = nb + take;
    t.update_dims();
    build_node_programs(z);
    build_node_programs(c);
    return true;
}

// ------------------------------------------------------------------ sweep
// Each operation of the sweep goes through emit(): run at once, or, while a
// schedule is recorded (batches advanced in lockstep), appended to it.  The
// solve operations are separate entries, so the j-th entries of several
// instances' schedules can share one grouped launch of the fused solver.
void Engine::emit(std::function<void()> op) {
    if (rec) rec->push_back(std::move(op));
    else op();
}

void Engine::sweep_S(int z, double h) {
    const auto &kids = t.kids[z];
    for (int k = 0; k < (int)kids.size(); ++k) {
        const int c = kids[k];
        const int pc = (int)t.dims[c].size() - 1;
        emit([=] {
            qr_slot(z, k, Rbuf, 0);  // gauge down
            absorb(c, pc, Rbuf, 0);
            build_mf(z, k);
        });
        if (t.local_dim[c] > 0) emit([=] { forward(c, h); });
        else sweep_S(c, h);
        emit([=] {
            const int nb0 = t.bond[c];
            const bool grew = adaptive && spawn(z, k, h, true);  // centre at c: new functions of c
            if (grew) build_mf(z, k);
            const int pcn = (int)t.dims[c].size() - 1;
            qr_slot(c, pcn, Cbuf, 0);  // up: backward bond step
            // the new functions enter with zero coefficients: the bond matrix's
            // block on them (the unit block the QR gives the orthonormal new
            // columns) is exactly zero, so that rounding in the bond generator
            // cannot carry its norm into the state
            if (grew) launch_zero_tail(Cbuf, t.bond[c], nb0, st);
            build_spo(c);
        });
        emit([=] { backward(c, Cbuf, h); });
        emit([=] { absorb(z, k, Cbuf, 0); });
    }
    if (z != t.root) emit([=] { forward(z, h); });
}

void Engine::sweep_Sstar(int z, double h) {
    if (z != t.root) emit([=] { forward(z, h); });
    const auto &kids = t.kids[z];
    for (int k = (int)kids.size() - 1; k >= 0; --k) {
        const int c = kids[k];
        emit([=] {
            const int nb0 = t.bond[c];
            const bool grew = adaptive && spawn(z, k, h, false);  // centre at z: new hole functions of c
            if (grew) build_spo(c);
            qr_slot(z, k, Cbuf, 1);  // down: backward bond step on R^T
            if (grew) launch_zero_tail(Cbuf, t.bond[c], nb0, st);  // zero coefficients of the new functions
            build_mf(z, k);
        });
        emit([=] { backward(c, Cbuf, h); });
        emit([=] {
            const int pc = (int)t.dims[c].size() - 1;
            absorb(c, pc, Cbuf, 1);
        });
        if (t.local_dim[c] > 0) emit([=] { forward(c, h); });
        else sweep_Sstar(c, h);
        emit([=] {
            const int pc = (int)t.dims[c].size() - 1;
            qr_slot(c, pc, Rbuf, 0);  // gauge up
            build_spo(c);
            absorb(z, k, Rbuf, 0);
        });
    }
}

void Engine::sync_check(const char *where) {
    hipError_t e = hipStreamSynchronize(st);
    if (e == hipSuccess) e = hipGetLastError();
    if (e != hipSuccess) throw Error(TTN_E_DEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

void Engine::check_ready(double dt) const {
    if (!have_sop || !have_state) throw Error(TTN_E_STATE, "ttn_step needs ttn_set_sop and a state");
    if (!std::isfinite(dt)) throw Error(TTN_E_INVALID, "dt must be finite");
}

void Engine::save_snapshot() {
    if (!snapshot) return;
    snap_bond = t.bond;
    int64_t off = 0;
    for (int z = 0; z < t.n; ++z) {
        launch_copy(snapshot + off, A[z], t.size[z], st);
        off += t.size[z];
    }
}

void Engine::restore_snapshot() {
    if (adaptive && snap_bond != t.bond) {
        // bonds grown during the failed step: Psi(0) loses its zero padding, the
        // bonds and every program go back to the state of the snapshot
        for (int c = 0; c < t.n; ++c)
            if (c != t.root && t.bond[c] != snap_bond[c]) {
                resize_psi0(c, snap_bond[c]);
                t.bond[c] = snap_bond[c];
                t.update_dims();
            }
        for (int z = 0; z < t.n; ++z) build_node_programs(z);
    }
    int64_t off = 0;
    for (int z = 0; z < t.n; ++z) {
        launch_copy(A[z], snapshot + off, t.size[z], st);
        off += t.size[z];
    }
    rebuild_all_spos();
}

// Enqueue one sweep and the asynchronous copy of its solve statistics; nothing
// here waits for the device.
void Engine::enqueue_sweep(double dt) {
    enqueue_sweep_body(dt);
    HIPCHK(hipEventRecord(step_done, st));
}

void Engine::enqueue_sweep_body(double dt) {
    solve_idx = 0;
    const double h = 0.5 * dt;
    sweep_S(t.root, h);
    emit([=] { forward(t.root, dt); });
    sweep_Sstar(t.root, h);
    enqueue_stats();
}

void Engine::enqueue_stats() {
    HIPCHK(hipMemcpyAsync(h_stats, d_stats, sizeof(SolveStat) * solve_idx, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(h_flags, qrw.bar + 128, sizeof(unsigned), hipMemcpyDeviceToHost, st));
}

// Lockstep form of enqueue_step for batches: the snapshot is enqueued and the
// sweep's operations are returned as a schedule instead of being run.
std::vector<std::function<void()>> Engine::record_step(double dt) {
    check_ready(dt);
    if (adaptive) throw Error(TTN_E_INVALID, "lockstep batches do not take subspace expansion");
    save_snapshot();
    std::vector<std::function<void()>> ops;
    rec = &ops;
    solve_idx = 0;
    const double h = 0.5 * dt;
    try {
        sweep_S(t.root, h);
        emit([=] { forward(t.root, dt); });
        sweep_Sstar(t.root, h);
    } catch (...) {
        rec = nullptr;
        throw;
    }
    rec = nullptr;
    return ops;
}

void Engine::finish_record() {
    enqueue_stats();
    HIPCHK(hipEventRecord(step_done, st));
}

void Engine::enqueue_step(double dt) {
    check_ready(dt);
    if (!graph_mode || profile_enabled()) {
        save_snapshot();
        enqueue_sweep(dt);
        return;
    }
    // hipGraph form: the launch sequence of a step (snapshot, sweep, statistics
    // copy) depends only on dt and the Krylov dimension hints, so it is
    // captured once per such key and replayed; the host-side bookkeeping of a
    // sweep (solve indices, the even number of buffer swaps per node) comes out
    // the same as in the capture
    // key: dt and the Krylov dimensions of the multi-kernel solves (they fix the
    // launch sequence); the fused solver's hint only says when it first checks
    // convergence, so a replay keeps the hint of its capture
    std::vector<int64_t> key;
    for (size_t i = 0; i < m_hint.size(); ++i) key.push_back(solve_small[i] ? -1 : m_hint[i]);
    int64_t dbits;
    std::memcpy(&dbits, &dt, sizeof dbits);
    key.push_back(dbits);
    GraphEntry *ge = nullptr;
    for (auto &g : graphs)
        if (g.key == key) ge = &g;
    if (!ge) {
        HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
        hipGraph_t graph = nullptr;
        try {
            save_snapshot();
            enqueue_sweep_body(dt);
        } catch (...) {
            (void)hipStreamEndCapture(st, &graph);
            if (graph) (void)hipGraphDestroy(graph);
            throw;
        }
        HIPCHK(hipStreamEndCapture(st, &graph));
        hipGraphExec_t exec = nullptr;
        hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) throw Error(TTN_E_DEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
        if (graphs.size() >= 8) {  // keep the most recent keys
            (void)hipGraphExecDestroy(graphs.front().exec);
            graphs.erase(graphs.begin());
        }
        graphs.push_back({key, exec, solve_idx});
        ge = &graphs.back();
        ++counters_graph_captures;
    }
    solve_idx = ge->n_solves;
    HIPCHK(hipGraphLaunch(ge->exec, st));
    HIPCHK(hipEventRecord(step_done, st));
}

void Engine::drop_graphs() {
    for (auto &g : graphs) (void)hipGraphExecDestroy(g.exec);
    graphs.clear();
}

// Wait for the enqueued sweep, update the Krylov dimension hints and, if a
// multi-kernel solve missed its tolerance, restore the snapshot and run the
// sweep again (synchronously) with larger dimensions.
void Engine::finish_step(double dt) {
    const double tol = krylov_tolerance();
    while (true) {
        hipError_t e = hipEventSynchronize(step_done);
        if (e == hipSuccess) e = hipGetLastError();
        if (e != hipSuccess) throw Error(TTN_E_DEVICE, std::string("ttn_step: ") + hipGetErrorString(e));
        if (h_flags[0]) throw Error(TTN_E_DEVICE, "grid-wide barrier of the cooperative QR timed out");
        bool redo = false;
        for (int i = 0; i < solve_idx; ++i) {
            const SolveStat &q = h_stats[i];
            if (solve_small[i]) {
                if (q.fail) {
                    char msg[256];
                    const int zn = solve_node[i];
                    const int64_t Nn = solve_fwd[i] ? t.size[zn] : (int64_t)t.bond[zn] * t.bond[zn];
                    snprintf(msg, sizeof msg,
                             "local exponential did not converge (fused solver; %s solve %d at node %d, "
                             "N=%lld, m=%d, matvecs=%d, err=%.3g)",
                             solve_fwd[i] ? "forward" : "backward", i, zn, (long long)Nn, q.m, q.matvecs, q.err);
                    restore_snapshot();
                    sync_check("restore");
                    throw Error(TTN_E_NOCONV, msg);
                }
                m_hint[i] = q.m;
            } else {
                if (q.fail) {
                    if (m_hint[i] >= mmax) {
                        restore_snapshot();
                        sync_check("restore");
                        throw Error(TTN_E_NOCONV, "local exponential did not converge at the Krylov limit");
                    }
                    m_hint[i] = std::min(mmax, m_hint[i] + 6);
                    redo = true;
                } else if (q.err_lo <= 1e-3 * tol) {
                    // lower the prediction only with a wide margin at two dimensions
                    // less: a failed prediction costs a whole step
                    m_hint[i] = std::max(3, m_hint[i] - 1);
                }
            }
        }
        if (!redo) break;
        ++counters[7];
        restore_snapshot();
        enqueue_sweep(dt);
    }
    if (profile_enabled()) {  // H_eff work done inside the fused solver launches
        double f = 0.0;
        for (int i = 0; i < solve_idx; ++i)
            if (solve_small[i]) {
                const Prog &p = solve_fwd[i] ? heffP[solve_node[i]] : bondP[solve_node[i]];
                f += (double)h_stats[i].matvecs * (double)p.flops;
            }
        profile_add_flops("k_small_solve", f);
    }
    ++counters[0];
    for (int i = 0; i < solve_idx; ++i) {
        const int z = solve_node[i];
        const Prog &p = solve_fwd[i] ? heffP[z] : bondP[z];
        if (solve_fwd[i]) ++counters[1];
        else ++counters[2];
        counters[3] += h_stats[i].matvecs;
        counters[4] += (int64_t)h_stats[i].matvecs * p.flops;
    }
}

void Engine::step(double dt, int n_steps) {
    for (int s = 0; s < n_steps; ++s) {
        enqueue_step(dt);
        finish_step(dt);
    }
}

// ------------------------------------------------------ ground state
// One-site ground-state sweeps (Sec. II C: the single-site machinery also
// serves ground-state optimisation, DMRG on trees): the traversal of the
// time-evolution sweep, S, the root, S*, with every node's local step replaced
// by the lowest eigenvector of the same local effective generator and the
// R factor of every gauge move absorbed unchanged (no backward bond step).
double Engine::ground_sweeps(int n, int *unconverged) {
    if (!have_sop || !have_state) throw Error(TTN_E_STATE, "the ground-state sweep needs ttn_set_sop and a state");
    if (n < 1) throw Error(TTN_E_INVALID, "n_sweeps must be at least 1");
    if (!opt.hermitian) throw Error(TTN_E_INVALID, "the ground-state sweep needs a Hermitian generator");
    if (adaptive) throw Error(TTN_E_INVALID, "the ground-state sweep does not take subspace expansion");
    int bad = 0;
    ground = true;
    try {
        for (int s = 0; s < n; ++s) {
            solve_idx = 0;
            sweep_S(t.root, 0.0);
            forward(t.root, 0.0);
            sweep_Sstar(t.root, 0.0);
            HIPCHK(hipMemcpyAsync(h_stats, d_stats, sizeof(SolveStat) * solve_idx, hipMemcpyDeviceToHost, st));
            sync_check("ground-state sweep");
            for (int i = 0; i < solve_idx; ++i) {  // matvec and H_eff flop counters as for a time step
                bad += h_stats[i].fail;
                const Prog &p = heffP[solve_node[i]];
                ++counters[1];
                counters[3] += h_stats[i].matvecs;
                counters[4] += (int64_t)h_stats[i].matvecs * p.flops;
            }
        }
    } catch (...) {
        ground = false;
        throw;
    }
    ground = false;
    if (unconverged) *unconverged = bad;
    const std::vector<double> e = observe(TTN_OBS_ENERGY, 0, nullptr, nullptr);
    const std::vector<double> nn = observe(TTN_OBS_NORM, 0, nullptr, nullptr);
    return e[0] / nn[0];
}

// ------------------------------------------------------------ observables
std::vector<double> Engine::observe(int kind, int n, const int32_t *op_ids, const double *vecs) {
    if (!have_state) throw Error(TTN_E_STATE, "no state");
    const int root = t.root;
    if (!obs) throw Error(TTN_E_STATE, "ttn_observe needs ttn_set_sop first");
    int64_t maxN = 0;
    for (int z = 0; z < t.n; ++z) maxN = std::max<int64_t>(maxN, t.size[z]);
    double2 *buf0 = obs, *buf1 = obs + maxN;
    double2 *mats = obs + 2 * maxN;
    std::vector<double2 *> Mc(t.n, nullptr);
    {
        int64_t off = 0;
        for (int z = 0; z < t.n; ++z) {
            Mc[z] = mats + off;
            off += (int64_t)t.bond[z] * t.bond[z];
        }
    }
    double2 *opbuf = nullptr;  // operator uploads, after the node matrices
    {
        int64_t off = 0;
        for (int z = 0; z < t.n; ++z) off += (int64_t)t.bond[z] * t.bond[z];
        opbuf = mats + off;
    }
    auto fetch = [&](const double2 *p, int64_t cnt) {
        std::vector<double2> h(cnt);
        HIPCHK(hipMemcpyAsync(h.data(), p, sizeof(double2) * cnt, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        return h;
    };
    std::vector<double> out(2, 0.0);
    // host staging of uploads: kept until the final fetch synchronises the stream
    std::vector<std::vector<double2>> staging;
    if (kind == TTN_OBS_NORM) {
        auto a = fetch(A[root], t.size[root]);
        double s = 0.0;
        for (auto &v : a) s += v.x * v.x + v.y * v.y;
        out[0] = s;
        return out;
    }
    if (kind == TTN_OBS_ENERGY) {
        if (!have_sop) throw Error(TTN_E_STATE, "no SOP");
        apply_prog(heffP[root], A[root], buf0);
        auto a = fetch(A[root], t.size[root]);
        auto b = fetch(buf0, t.size[root]);
        cplx s(0.0);
        for (size_t i = 0; i < a.size(); ++i) s += std::conj(cplx(a[i].x, a[i].y)) * cplx(b[i].x, b[i].y);
        out[0] = s.real();
        out[1] = s.imag();
        return out;
    }
    if (kind == TTN_OBS_EXPECT || kind == TTN_OBS_OVERLAP_T0) {
        std::vector<char> need(t.n, 0);
        std::vector<const std::vector<cplx> *> leafop(t.n, nullptr);
        const bool ov = kind == TTN_OBS_OVERLAP_T0;
        if (ov) {
            std::fill(need.begin(), need.end(), 1);
        } else {
            if (n < 0 || (n > 0 && !op_ids)) throw Error(TTN_E_INVALID, "bad op ids");
            for (int i = 0; i < n; ++i) {
                int o = op_ids[i];
                if (o < 0 || o >= sop.n_ops) throw Error(TTN_E_INVALID, "op id out of range");
                int l = sop.op_leaf[o];
                if (leafop[l]) throw Error(TTN_E_INVALID, "two operators on one leaf");
                leafop[l] = &sop.op_mat[o];
                for (int w = l; w != -1; w = t.parent[w]) need[w] = 1;
            }
            need[root] = 1;
        }
        int64_t opoff = 0;
        for (int c : t.postorder) {
            if (!need[c]) continue;
            const Geom g = geom_of(t.dims[c]);
            const int D = g.D;
            const double2 *bra = ov ? A0[c] : A[c];
            const double2 *cur = A[c];
            double2 *bufs[2] = {buf0, buf1};
            int pp = 0;
            if (t.local_dim[c] > 0) {
                if (leafop[c]) {
                    const int d = t.local_dim[c];
                    staging.emplace_back(d * d);
                    std::vector<double2> &hm = staging.back();
                    for (int q = 0; q < d * d; ++q) hm[q] = to_d2((*leafop[c])[q]);
                    double2 *dm = opbuf + opoff;
                    opoff += d * d;
                    HIPCHK(hipMemcpyAsync(dm, hm.data(), sizeof(double2) * d * d, hipMemcpyHostToDevice, st));
                    launch_mode_product(cur, bufs[pp], dm, 1, d, d, g.R[0], 0, st);
                    cur = bufs[pp];
                    pp ^= 1;
                }
            } else {
                for (int k = 0; k < D - 1; ++k) {
                    const int kid = t.kids[c][k];
                    if (!need[kid]) continue;
                    launch_mode_product(cur, bufs[pp], Mc[kid], g.L[k], g.dims[k], g.dims[k], g.R[k], 0, st);
                    cur = bufs[pp];
                    pp ^= 1;
                }
            }
            const int np = g.dims[D - 1];
            launch_contract(bra, cur, Mc[c], g.N / np, np, np, 1, cpart, st);
        }
        auto r = fetch(Mc[root], 1);
        out[0] = r[0].x;
        out[1] = r[0].y;
        return out;
    }
    if (kind == TTN_OBS_BILINEAR) {
        if (!vecs) throw Error(TTN_E_INVALID, "null vectors");
        // per node: vector over the parent index
        int64_t voff = 0;
        std::vector<int64_t> leafoff(t.n, 0);
        for (int z = 0; z < t.n; ++z)
            if (t.local_dim[z] > 0) {
                leafoff[z] = voff;
                voff += t.local_dim[z];
            }
        int64_t opoff = 0;
        for (int c : t.postorder) {
            const Geom g = geom_of(t.dims[c]);
            const int D = g.D;
            std::vector<int> dims(t.dims[c].begin(), t.dims[c].end());
            const double2 *cur = A[c];
            double2 *bufs[2] = {buf0, buf1};
            int pp = 0;
            auto shrink = [&](int k, const double2 *vecM) {
                int64_t L = 1, R = 1;
                for (int q = 0; q < k; ++q) L *= dims[q];
                for (int q = k + 1; q < D; ++q) R *= dims[q];
                launch_mode_product(cur, bufs[pp], vecM, L, dims[k], 1, R, 0, st);
                dims[k] = 1;
                cur = bufs[pp];
                pp ^= 1;
            };
            if (t.local_dim[c] > 0) {
                const int d = t.local_dim[c];
                staging.emplace_back(d);
                std::vector<double2> &hv = staging.back();
                for (int i = 0; i < d; ++i)
                    hv[i] = make_double2(vecs[2 * (leafoff[c] + i)], vecs[2 * (leafoff[c] + i) + 1]);
                double2 *dv = opbuf + opoff;
                opoff += d;
                HIPCHK(hipMemcpyAsync(dv, hv.data(), sizeof(double2) * d, hipMemcpyHostToDevice, st));
                shrink(0, dv);
            } else {
                for (int k = 0; k < D - 1; ++k) shrink(k, Mc[t.kids[c][k]]);
            }
            launch_copy(Mc[c], cur, dims[D - 1], st);
        }
        auto r = fetch(Mc[root], 1);
        out[0] = r[0].x;
        out[1] = r[0].y;
        return out;
    }
    throw Error(TTN_E_INVALID, "unknown observable kind");
}

void Engine::apply_root_heff(const double *x, double *y) {
    if (!have_sop || !have_state) throw Error(TTN_E_STATE, "needs SOP and state");
    const int64_t N = t.size[t.root];
    HIPCHK(hipMemcpyAsync(obs, x, sizeof(double2) * N, hipMemcpyHostToDevice, st));
    apply_prog(heffP[t.root], obs, obs + N);
    HIPCHK(hipMemcpyAsync(y, obs + N, sizeof(double2) * N, hipMemcpyDeviceToHost, st));
    sync_check("apply_root_heff");
}

void debug_qr(int64_t rows, int cols, const double *m, int variant, double *q_out, double *r_out) {
    if (rows < cols || cols < 1 || cols > 64) throw Error(TTN_E_INVALID, "QR shape out of range");
    if (variant < 0 || variant > 4) throw Error(TTN_E_INVALID, "QR variant out of range");
    const size_t nm = (size_t)rows * cols;
    std::vector<void *> mem;
    auto alloc = [&](size_t bytes) {
        void *p = nullptr;
        HIPCHK(hipMalloc(&p, bytes < 16 ? 16 : bytes));
        mem.push_back(p);
        return p;
    };
    try {
        double2 *A = (double2 *)alloc(sizeof(double2) * nm);
        double2 *Rd = (double2 *)alloc(sizeof(double2) * cols * cols);
        HIPCHK(hipMemcpy(A, m, sizeof(double2) * nm, hipMemcpyHostToDevice));
        if (variant == 0) {
            launch_qr(A, rows, cols, 1, Rd, 0, nullptr);
        } else {
            QRWork q{};
            q.tau = (double2 *)alloc(sizeof(double2) * 64);
            q.scl = (double2 *)alloc(sizeof(double2) * 64);
            q.diag = (double2 *)alloc(sizeof(double2) * 64);
            q.snapped = (int *)alloc(sizeof(int) * 64);
            q.w = (double2 *)alloc(sizeof(double2) * 64 * 64);
            q.rowi = (double2 *)alloc(sizeof(double2) * 64);
            q.part = (double *)alloc(sizeof(double) * QRM_BLOCKS_MAX * (2 + 2 * 64));
            q.S = (double2 *)alloc(sizeof(double2) * QRM_BLOCKS_MAX * 64 * 63 / 2);
            q.K = (double2 *)alloc(sizeof(double2) * 64 * 64);
            q.thr = (double *)alloc(sizeof(double) * 4);
            q.counter = (unsigned *)alloc(sizeof(unsigned) * 4);
            HIPCHK(hipMemset(q.counter, 0, sizeof(unsigned) * 4));
            q.cpart = (double *)alloc(sizeof(double) * 2 * QRM_BLOCKS_MAX * QRC_REC);
            q.bar = (unsigned *)alloc(sizeof(unsigned) * 192);
            HIPCHK(hipMemset(q.bar, 0, sizeof(unsigned) * 192));
            if (variant >= 3) {  // Cholesky route (3: Householder kernels behind it, 4: alone)
                q.cq_part = (double2 *)alloc(sizeof(double2) * CQR_BLOCKS_MAX * 64 * 64);
                q.cq_G = (double2 *)alloc(sizeof(double2) * 64 * 64);
                q.cq_R1 = (double2 *)alloc(sizeof(double2) * 64 * 64);
                q.cq_R1inv = (double2 *)alloc(sizeof(double2) * 64 * 64);
                q.cq_M = (double2 *)alloc(sizeof(double2) * 64 * 64);
                q.cq_Y = (double2 *)alloc(sizeof(double2) * nm);
                q.cq_ycap = (int64_t)nm;
                q.cq_scal = (double *)alloc(sizeof(double) * 4);
                q.cq_state = (int *)alloc(sizeof(int) * 4);
                q.cq_counter = (unsigned *)alloc(sizeof(unsigned) * 4);
                HIPCHK(hipMemset(q.cq_counter, 0, sizeof(unsigned) * 4));
                if (!launch_qr_chol(A, rows, cols, 1, Rd, 0, q, nullptr))
                    throw Error(TTN_E_INVALID, "QR shape outside the Cholesky route");
                if (variant == 4) {
                    int state = 1;
                    HIPCHK(hipMemcpy(&state, q.cq_state, sizeof(int), hipMemcpyDeviceToHost));
                    if (state != 0) throw Error(TTN_E_NOCONV, "matrix outside the range of the Cholesky route");
                } else {
                    q.gate = q.cq_state;
                    launch_qr_multi(A, rows, cols, 1, Rd, 0, q, nullptr);
                }
            } else if (variant == 1) launch_qr_multi(A, rows, cols, 1, Rd, 0, q, nullptr);
            else if (!launch_qr_coop(A, rows, cols, 1, Rd, 0, q, nullptr))
                throw Error(TTN_E_INVALID, "cooperative QR grid cannot be co-resident");
            if (variant == 2) {
                unsigned flag = 0;
                HIPCHK(hipMemcpy(&flag, q.bar + 128, sizeof(unsigned), hipMemcpyDeviceToHost));
                if (flag) throw Error(TTN_E_DEVICE, "grid-wide barrier of the cooperative QR timed out");
            }
        }
        HIPCHK(hipDeviceSynchronize());
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpy(q_out, A, sizeof(double2) * nm, hipMemcpyDeviceToHost));
        HIPCHK(hipMemcpy(r_out, Rd, sizeof(double2) * cols * cols, hipMemcpyDeviceToHost));
    } catch (...) {
        for (void *p : mem) (void)hipFree(p);
        throw;
    }
    for (void *p : mem) (void)hipFree(p);
}

int Engine::step_solves(int max, int32_t *node, int32_t *fwd, int32_t *matvecs) const {
    if (counters[0] == 0 || !h_stats) throw Error(TTN_E_STATE, "no completed step");
    for (int i = 0; i < solve_idx && i < max; ++i) {
        if (node) node[i] = solve_node[i];
        if (fwd) fwd[i] = solve_fwd[i];
        if (matvecs) matvecs[i] = h_stats[i].matvecs;
    }
    return solve_idx;
}

void Engine::info(int32_t *bonds, int64_t *ctr) {
    if (bonds)
        for (int z = 0; z < t.n; ++z) bonds[z] = z == t.root ? 1 : t.bond[z];
    if (ctr)
        for (int i = 0; i < 8; ++i) ctr[i] = counters[i];
}

}  // namespace ttn
