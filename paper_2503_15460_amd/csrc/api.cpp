// C boundary of the library: argument checks, handle management and the
// conversion of exceptions into ttn_status codes.
#include <cmath>
#include <cstdint>
#include <cstring>
#include <functional>
#include <vector>
#include <memory>
#include <string>

#include "engine.h"
#include "ttn.h"
#include "ttn_debug.h"
#include "ttn_internal.h"

struct ttn_ctx {
    std::unique_ptr<ttn::Engine> eng;
    std::string err;
    bool dead = false;
    struct ttn_batch_ctx *batch = nullptr;  // batch the handle currently belongs to
};

// Instances advanced together: each instance runs on one of the batch's HIP
// streams (round robin), so the sweeps of different instances overlap on the
// device while the host enqueues them one after the other.
struct ttn_batch_ctx {
    std::vector<ttn_t> insts;
    std::vector<hipStream_t> own;      // each instance's stream before joining
    std::vector<hipStream_t> streams;  // created by the batch, default priority
    std::string err;
    // lockstep: every instance on streams[0]; layer j of a step runs the j-th
    // operation of every instance's sweep, its fused solves as one launch
    bool lockstep = false;
    ttn::SmallSolveArgs *h_args = nullptr, *d_args = nullptr;  // pinned host / device argument arrays
    size_t args_cap = 0;
    ~ttn_batch_ctx() {
        if (h_args) (void)hipHostFree(h_args);
        if (d_args) (void)hipFree(d_args);
    }
};

namespace {
thread_local std::string g_err;

// A sweep that stops on anything but a library error (a failed launch, a host
// allocation) has been partly applied: report it as a device error, which
// makes the handle unusable.
template <class F>
void sweep_guard(F &&f) {
    try {
        f();
    } catch (const ttn::Error &) {
        throw;
    } catch (const std::exception &e) {
        throw ttn::Error(TTN_E_DEVICE, std::string("sweep aborted: ") + e.what());
    }
}

template <class F>
ttn_status guard(ttn_t h, F &&f) {
    try {
        if (h && h->dead) throw ttn::Error(TTN_E_DEVICE, "handle unusable after a device error");
        f();
        return TTN_OK;
    } catch (const ttn::Error &e) {
        if (h) {
            h->err = e.what();
            if (e.code == TTN_E_DEVICE) h->dead = true;
        }
        g_err = e.what();
        return e.code;
    } catch (const std::bad_alloc &) {
        g_err = "host allocation failed";
        if (h) h->err = g_err;
        return TTN_E_OOM;
    } catch (const std::exception &e) {
        g_err = e.what();
        if (h) h->err = g_err;
        return TTN_E_INVALID;
    }
}
}  // namespace

extern "C" {

void ttn_default_options(ttn_options *opt) {
    if (!opt) return;
    std::memset(opt, 0, sizeof(*opt));
    opt->precision = TTN_FP64;
    opt->krylov_tol = 0.0;
    opt->krylov_mmax = 40;
    opt->hermitian = 1;
}

ttn_status ttn_create(int32_t n_nodes, const int32_t *parent, const int32_t *local_dim, const int32_t *bond_dim,
                      const ttn_options *opt, ttn_t *out) {
    if (!out) {
        g_err = "null output handle";
        return TTN_E_INVALID;
    }
    *out = nullptr;
    return guard(nullptr, [&] {
        ttn_options o;
        ttn_default_options(&o);
        if (opt) o = *opt;
        if (o.precision != TTN_FP64 && o.precision != TTN_FP32 && o.precision != TTN_BF16X3)
            throw ttn::Error(TTN_E_INVALID, "precision must be TTN_FP64, TTN_FP32 or TTN_BF16X3");
        if (o.use_graph != 0 && o.use_graph != 1) throw ttn::Error(TTN_E_INVALID, "use_graph must be 0 or 1");
        if (o.use_graph && o.spawn_tol > 0.0)
            throw ttn::Error(TTN_E_INVALID, "use_graph cannot be combined with subspace expansion");
        if (o.autotune != 0 && o.autotune != 1) throw ttn::Error(TTN_E_INVALID, "autotune must be 0 or 1");
        if (o.workspace && ((uintptr_t)o.workspace % 256 != 0))
            throw ttn::Error(TTN_E_INVALID, "workspace must be 256-byte aligned");
        if (!(o.spawn_tol >= 0.0) || !std::isfinite(o.spawn_tol))
            throw ttn::Error(TTN_E_INVALID, "spawn_tol must be finite and >= 0");
        ttn::Tree t = ttn::build_tree(n_nodes, parent, local_dim, bond_dim, o.bond_max);
        o.bond_max = nullptr;  // copied into the tree; no caller pointer is kept
        auto h = std::make_unique<ttn_ctx>();
        h->eng = std::make_unique<ttn::Engine>(t, o);
        *out = h.release();
    });
}

ttn_status ttn_set_sop(ttn_t h, int32_t n_ops, const int32_t *op_leaf, const int64_t *op_offset,
                       const double *op_data, int32_t n_terms, const double *coeff, const int64_t *term_ptr,
                       const int32_t *term_ops) {
    if (!h) return TTN_E_INVALID;
    return guard(h, [&] {
        ttn::SopInput s = ttn::read_sop(h->eng->t, n_ops, op_leaf, op_offset, op_data, n_terms, coeff, term_ptr,
                                        term_ops);
        h->eng->set_sop(s);
    });
}

ttn_status ttn_set_coefficients(ttn_t h, int32_t n_terms, const double *coeff, int32_t *rebuilt) {
    if (!h) return TTN_E_INVALID;
    return guard(h, [&] {
        const bool r = h->eng->set_coefficients(coeff, n_terms);
        if (rebuilt) *rebuilt = r ? 1 : 0;
    });
}

ttn_status ttn_set_product_state(ttn_t h, const double *leaf_vecs) {
    if (!h) return TTN_E_INVALID;
    return guard(h, [&] { h->eng->set_product_state(leaf_vecs); });
}

ttn_status ttn_step(ttn_t h, double dt, int32_t n_steps) {
    if (!h) return TTN_E_INVALID;
    return guard(h, [&] {
        if (n_steps < 0) throw ttn::Error(TTN_E_INVALID, "negative step count");
        sweep_guard([&] { h->eng->step(dt, n_steps); });
    });
}

ttn_status ttn_ground_sweeps(ttn_t h, int32_t n_sweeps, double *energy, int32_t *unconverged) {
    if (!h) return TTN_E_INVALID;
    return guard(h, [&] {
        if (!energy) throw ttn::Error(TTN_E_INVALID, "null output");
        if (h->batch) throw ttn::Error(TTN_E_INVALID, "the handle belongs to a batch");
        int bad = 0;
        double e = 0.0;
        sweep_guard([&] { e = h->eng->ground_sweeps(n_sweeps, &bad); });
        *energy = e;
        if (unconverged) *unconverged = bad;
    });
}

ttn_status ttn_batch_create(int32_t n, ttn_t const *insts, int32_t n_streams, ttn_batch_t *out) {
    if (!out) {
        g_err = "null output handle";
        return TTN_E_INVALID;
    }
    *out = nullptr;
    return guard(nullptr, [&] {
        if (n < 1 || !insts) throw ttn::Error(TTN_E_INVALID, "empty batch");
        for (int32_t i = 0; i < n; ++i) {
            if (!insts[i]) throw ttn::Error(TTN_E_INVALID, "null instance handle");
            if (insts[i]->dead) throw ttn::Error(TTN_E_DEVICE, "instance unusable after a device error");
            if (insts[i]->batch) throw ttn::Error(TTN_E_INVALID, "instance already belongs to a batch");
            for (int32_t j = 0; j < i; ++j)
                if (insts[j] == insts[i]) throw ttn::Error(TTN_E_INVALID, "instance listed twice");
            if (insts[i]->eng->opt.device != insts[0]->eng->opt.device)
                throw ttn::Error(TTN_E_INVALID, "instances on different devices");
        }
        int ns = n_streams > 0 ? n_streams : 8;
        if (ns > n) ns = n;
        if (ns > 64) ns = 64;
        auto b = std::make_unique<ttn_batch_ctx>();
        hipError_t e = hipSetDevice(insts[0]->eng->opt.device);
        for (int i = 0; i < ns && e == hipSuccess; ++i) {
            hipStream_t s = nullptr;
            e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
            if (e == hipSuccess) b->streams.push_back(s);
        }
        if (e != hipSuccess) {
            for (auto s : b->streams) (void)hipStreamDestroy(s);
            throw ttn::Error(TTN_E_DEVICE, std::string("hipStreamCreate: ") + hipGetErrorString(e));
        }
        for (int32_t i = 0; i < n; ++i) {
            b->insts.push_back(insts[i]);
            b->own.push_back(insts[i]->eng->stream());
            insts[i]->eng->set_stream(b->streams[i % ns]);
            insts[i]->batch = b.get();
        }
        *out = b.release();
    });
}

ttn_status ttn_batch_set_lockstep(ttn_batch_t b, int32_t on) {
    if (!b) return TTN_E_INVALID;
    return guard(nullptr, [&] {
        for (auto *h : b->insts)
            if (h->dead) throw ttn::Error(TTN_E_DEVICE, "instance unusable after a device error");
        b->lockstep = on != 0;
        for (size_t i = 0; i < b->insts.size(); ++i)
            b->insts[i]->eng->set_stream(b->lockstep ? b->streams[0] : b->streams[i % b->streams.size()]);
    });
}

// One lockstep step of every instance: the schedules are recorded, then run
// layer by layer; each layer's fused solves go out as one grouped launch.
static void lockstep_step(ttn_batch_t b, const double *dt, int &cur) {
    const int n = (int)b->insts.size();
    std::vector<std::vector<std::function<void()>>> sched(n);
    size_t L = 0;
    for (cur = 0; cur < n; ++cur) {
        sweep_guard([&] { sched[cur] = b->insts[cur]->eng->record_step(dt[cur]); });
        L = std::max(L, sched[cur].size());
    }
    const size_t need = L * (size_t)n;
    if (need > b->args_cap) {
        if (b->h_args) (void)hipHostFree(b->h_args);
        if (b->d_args) (void)hipFree(b->d_args);
        b->h_args = b->d_args = nullptr;
        b->args_cap = 0;
        if (hipHostMalloc((void **)&b->h_args, sizeof(ttn::SmallSolveArgs) * need, hipHostMallocDefault) !=
                hipSuccess ||
            hipMalloc((void **)&b->d_args, sizeof(ttn::SmallSolveArgs) * need) != hipSuccess)
            throw ttn::Error(TTN_E_OOM, "lockstep argument arrays");
        b->args_cap = need;
    }
    hipStream_t st = b->streams[0];
    size_t used = 0;
    std::vector<ttn::SmallSolveArgs> grp;
    std::vector<size_t> pos(n, 0);
    // layer j: every instance runs its operations up to and including its j-th
    // fused local exponential, whose launch is deferred; then the layer's
    // exponentials go out together
    for (size_t j = 0; j < L; ++j) {
        grp.clear();
        bool any = false;
        for (cur = 0; cur < n; ++cur) {
            ttn::Engine &e = *b->insts[cur]->eng;
            e.defer_fused = true;
            e.deferred.clear();
            while (pos[cur] < sched[cur].size() && e.deferred.empty()) {
                sweep_guard([&] { sched[cur][pos[cur]](); });
                ++pos[cur];
                any = true;
            }
            e.defer_fused = false;
            grp.insert(grp.end(), e.deferred.begin(), e.deferred.end());
        }
        cur = -1;
        if (!any) break;
        if (grp.empty()) continue;
        std::memcpy(b->h_args + used, grp.data(), sizeof(ttn::SmallSolveArgs) * grp.size());
        if (hipMemcpyAsync(b->d_args + used, b->h_args + used, sizeof(ttn::SmallSolveArgs) * grp.size(),
                           hipMemcpyHostToDevice, st) != hipSuccess)
            throw ttn::Error(TTN_E_DEVICE, "lockstep argument upload");
        sweep_guard([&] { ttn::launch_small_solve_group(b->d_args + used, grp, st); });
        used += grp.size();
    }
    for (cur = 0; cur < n; ++cur) sweep_guard([&] { b->insts[cur]->eng->finish_record(); });
}

ttn_status ttn_batch_step(ttn_batch_t b, const double *dt, int32_t n_steps) {
    if (!b) return TTN_E_INVALID;
    const int n = (int)b->insts.size();
    int cur = -1;  // instance being handled when an error is raised
    ttn_status rc = guard(nullptr, [&] {
        if (!dt) throw ttn::Error(TTN_E_INVALID, "null time steps");
        if (n_steps < 0) throw ttn::Error(TTN_E_INVALID, "negative step count");
        for (int i = 0; i < n; ++i)
            if (b->insts[i]->dead) throw ttn::Error(TTN_E_DEVICE, "instance unusable after a device error");
        for (cur = 0; cur < n; ++cur) b->insts[cur]->eng->check_ready(dt[cur]);
        for (int s = 0; s < n_steps; ++s) {
            if (b->lockstep) {
                try {
                    lockstep_step(b, dt, cur);
                } catch (const ttn::Error &e) {
                    if (e.code == TTN_E_DEVICE)  // schedules of every instance may be half run
                        for (auto *h : b->insts) h->dead = true;
                    throw;
                }
            } else {
                for (cur = 0; cur < n; ++cur) sweep_guard([&] { b->insts[cur]->eng->enqueue_step(dt[cur]); });
            }
            // finish every instance (each one's bookkeeping stays consistent), then report the first error
            int bad = -1;
            ttn_status bad_code = TTN_OK;
            std::string bad_msg;
            for (int i = 0; i < n; ++i) {
                try {
                    sweep_guard([&] { b->insts[i]->eng->finish_step(dt[i]); });
                } catch (const ttn::Error &e) {
                    if (bad < 0) {
                        bad = i;
                        bad_code = e.code;
                        bad_msg = e.what();
                    }
                }
            }
            if (bad >= 0) {
                cur = bad;
                throw ttn::Error(bad_code, bad_msg);
            }
        }
        cur = -1;
    });
    if (rc != TTN_OK) {
        b->err = g_err;
        if (cur >= 0 && cur < n) {
            b->err = "instance " + std::to_string(cur) + ": " + g_err;
            b->insts[cur]->err = g_err;
            if (rc == TTN_E_DEVICE) b->insts[cur]->dead = true;
        }
        // leave every instance idle: drain whatever was enqueued
        for (auto s : b->streams) (void)hipStreamSynchronize(s);
    }
    return rc;
}

const char *ttn_batch_last_error(ttn_batch_t b) { return b ? b->err.c_str() : g_err.c_str(); }

void ttn_batch_destroy(ttn_batch_t b) {
    if (!b) return;
    for (size_t i = 0; i < b->insts.size(); ++i) {
        try {
            b->insts[i]->eng->set_stream(b->own[i]);
        } catch (...) {
        }
        b->insts[i]->batch = nullptr;
    }
    for (auto s : b->streams) (void)hipStreamDestroy(s);
    delete b;
}

ttn_status ttn_observe(ttn_t h, int32_t kind, int32_t n, const int32_t *op_ids, const double *vecs, double *out) {
    if (!h) return TTN_E_INVALID;
    return guard(h, [&] {
        if (!out) throw ttn::Error(TTN_E_INVALID, "null output");
        auto r = h->eng->observe(kind, n, op_ids, vecs);
        out[0] = r[0];
        out[1] = r[1];
    });
}

ttn_status ttn_apply_root_heff(ttn_t h, const double *x, double *y) {
    if (!h) return TTN_E_INVALID;
    return guard(h, [&] {
        if (!x || !y) throw ttn::Error(TTN_E_INVALID, "null buffer");
        h->eng->apply_root_heff(x, y);
    });
}

ttn_status ttn_get_info(ttn_t h, int32_t *effective_bond_dim, int64_t *counters) {
    if (!h) return TTN_E_INVALID;
    return guard(h, [&] { h->eng->info(effective_bond_dim, counters); });
}

ttn_status ttn_get_step_solves(ttn_t h, int32_t max_solves, int32_t *node, int32_t *forward, int32_t *matvecs,
                               int32_t *n_solves) {
    if (!h) return TTN_E_INVALID;
    return guard(h, [&] {
        const int n = h->eng->step_solves(max_solves, node, forward, matvecs);
        if (n_solves) *n_solves = n;
    });
}

ttn_status ttn_debug_graph_captures(ttn_t h, int64_t *captures) {
    if (!h || !captures) return TTN_E_INVALID;
    *captures = h->eng->graph_captures();
    return TTN_OK;
}

ttn_status ttn_workspace_size(ttn_t h, size_t *bytes) {
    if (!h || !bytes) return TTN_E_INVALID;
    *bytes = h->eng->workspace_need();
    return TTN_OK;
}

ttn_status ttn_tile_table_save(const char *path) {
    return guard(nullptr, [&] {
        if (!path) throw ttn::Error(TTN_E_INVALID, "null path");
        try {
            ttn::tile_table_save(path);
        } catch (const std::runtime_error &e) {
            throw ttn::Error(TTN_E_INVALID, e.what());
        }
    });
}

ttn_status ttn_tile_table_load(const char *path, int32_t *n_loaded) {
    return guard(nullptr, [&] {
        if (!path) throw ttn::Error(TTN_E_INVALID, "null path");
        int n = 0;
        try {
            n = ttn::tile_table_load(path);
        } catch (const std::runtime_error &e) {
            throw ttn::Error(TTN_E_INVALID, e.what());
        }
        if (n_loaded) *n_loaded = n;
    });
}

ttn_status ttn_tile_table_size(int64_t *n_entries) {
    if (!n_entries) return TTN_E_INVALID;
    *n_entries = (int64_t)ttn::tile_table_size();
    return TTN_OK;
}

void ttn_tile_table_clear(void) { ttn::tile_table_clear(); }

void ttn_release_process_resources(void) {
    try {
        ttn::release_process_resources();
    } catch (...) {
    }
}

ttn_status ttn_state_size(ttn_t h, size_t *bytes) {
    if (!h || !bytes) return TTN_E_INVALID;
    return guard(h, [&] { *bytes = h->eng->state_bytes(); });
}

ttn_status ttn_get_state(ttn_t h, double *buf, size_t bytes) {
    if (!h) return TTN_E_INVALID;
    return guard(h, [&] { h->eng->get_state(buf, bytes); });
}

ttn_status ttn_set_state(ttn_t h, const double *buf, size_t bytes) {
    if (!h) return TTN_E_INVALID;
    return guard(h, [&] { h->eng->set_state(buf, bytes); });
}

ttn_status ttn_profile_begin(void) {
    return guard(nullptr, [&] { ttn::profile_enable(true); });
}

ttn_status ttn_profile_end(ttn_kernel_stat *rows, int32_t max_rows, int32_t *n_rows) {
    return guard(nullptr, [&] {
        auto st = ttn::profile_collect();
        ttn::profile_enable(false);
        int32_t k = 0;
        for (auto &r : st) {
            if (rows && k < max_rows) {
                std::memset(rows[k].name, 0, sizeof(rows[k].name));
                std::strncpy(rows[k].name, r.name.c_str(), sizeof(rows[k].name) - 1);
                rows[k].calls = r.calls;
                rows[k].total_ms = r.ms;
                rows[k].flops = r.flops;
                rows[k].bytes = r.bytes;
            }
            ++k;
        }
        if (n_rows) *n_rows = k;
    });
}

const char *ttn_last_error(ttn_t h) {
    if (h) return h->err.c_str();
    return g_err.c_str();
}

void ttn_destroy(ttn_t h) {
    if (!h) return;
    try {
        if (h->batch) {  // leave the batch first
            ttn_batch_ctx *b = h->batch;
            for (size_t i = 0; i < b->insts.size(); ++i)
                if (b->insts[i] == h) {
                    b->insts.erase(b->insts.begin() + i);
                    b->own.erase(b->own.begin() + i);
                    break;
                }
            (void)hipStreamSynchronize(h->eng->stream());
        }
        delete h;
    } catch (...) {
    }
}

ttn_status ttn_debug_clamp_bonds(int32_t n_nodes, const int32_t *parent, const int32_t *local_dim,
                                 const int32_t *bond_dim, int32_t *effective) {
    return guard(nullptr, [&] {
        if (!effective) throw ttn::Error(TTN_E_INVALID, "null output");
        ttn::Tree t = ttn::build_tree(n_nodes, parent, local_dim, bond_dim);
        for (int z = 0; z < t.n; ++z) effective[z] = z == t.root ? 1 : t.bond[z];
    });
}

ttn_status ttn_debug_dense_tree_operator(int32_t n_nodes, const int32_t *parent, const int32_t *local_dim,
                                         int32_t n_ops, const int32_t *op_leaf, const int64_t *op_offset,
                                         const double *op_data, int32_t n_terms, const double *coeff,
                                         const int64_t *term_ptr, const int32_t *term_ops, int64_t max_dim,
                                         double *out, int64_t *n_entries) {
    return guard(nullptr, [&] {
        std::vector<int32_t> ones(n_nodes > 0 ? n_nodes : 1, 1);
        ttn::Tree t = ttn::build_tree(n_nodes, parent, local_dim, ones.data());
        ttn::SopInput s = ttn::read_sop(t, n_ops, op_leaf, op_offset, op_data, n_terms, coeff, term_ptr, term_ops);
        ttn::TreeOp op = ttn::compile_tree_operator(t, s);
        if (n_entries) {
            int64_t cnt = 0;
            for (auto &e : op.entries) cnt += (int64_t)e.size();
            *n_entries = cnt;
        }
        using ttn::cplx;
        using Mat = std::vector<cplx>;
        auto kron = [](const Mat &a, int64_t da, const Mat &b, int64_t db) {
            Mat c((size_t)(da * db * da * db));
            for (int64_t i = 0; i < da; ++i)
                for (int64_t j = 0; j < da; ++j)
                    for (int64_t k = 0; k < db; ++k)
                        for (int64_t l = 0; l < db; ++l)
                            c[(size_t)((i * db + k) * (da * db) + j * db + l)] = a[i * da + j] * b[k * db + l];
            return c;
        };
        auto eye = [](int64_t d) {
            Mat m((size_t)(d * d), cplx(0));
            for (int64_t i = 0; i < d; ++i) m[i * d + i] = 1.0;
            return m;
        };
        std::vector<int64_t> dim(t.n, 1);
        for (int z : t.postorder) {
            if (t.local_dim[z] > 0) dim[z] = t.local_dim[z];
            else
                for (int c : t.kids[z]) dim[z] *= dim[c];
            if (dim[z] > max_dim) throw ttn::Error(TTN_E_INVALID, "dense dimension exceeds max_dim");
        }
        // dense bond operators U^c_b over the subtree of c (channel 0 = identity)
        std::vector<std::vector<Mat>> Ub(t.n);
        auto node_sum = [&](int z, const std::vector<ttn::OpEntry> &ents, int want_bp, bool all) {
            Mat acc((size_t)(dim[z] * dim[z]), cplx(0));
            for (auto &e : ents) {
                if (!all && e.bp != want_bp) continue;
                Mat m{cplx(1.0)};
                int64_t dm = 1;
                for (size_t k = 0; k < t.kids[z].size(); ++k) {
                    int c = t.kids[z][k];
                    const Mat &f = e.slot[k] >= 1 ? Ub[c][e.slot[k]] : eye(dim[c]);
                    m = kron(m, dm, f, dim[c]);
                    dm *= dim[c];
                }
                for (size_t q = 0; q < acc.size(); ++q) acc[q] += e.coef * m[q];
            }
            return acc;
        };
        for (int z : t.postorder) {
            if (z == t.root) continue;
            Ub[z].assign(op.n_ch[z], Mat());
            Ub[z][0] = eye(dim[z]);
            if (t.local_dim[z] > 0) {
                int li = t.leaf_index[z];
                for (int b = 1; b < op.n_ch[z]; ++b)
                    Ub[z][b] = op.leafU[li][b].empty() ? Mat((size_t)(dim[z] * dim[z]), cplx(0)) : op.leafU[li][b];
            } else {
                for (int b = 1; b < op.n_ch[z]; ++b) Ub[z][b] = node_sum(z, op.entries[z], b, false);
            }
        }
        const int64_t D = dim[t.root];
        Mat G = node_sum(t.root, op.entries[t.root], 0, true);
        for (int64_t q = 0; q < D * D; ++q) {
            out[2 * q] = G[q].real();
            out[2 * q + 1] = G[q].imag();
        }
    });
}

ttn_status ttn_debug_hermiticity_defect(int32_t n_nodes, const int32_t *parent, const int32_t *local_dim,
                                        int32_t n_ops, const int32_t *op_leaf, const int64_t *op_offset,
                                        const double *op_data, int32_t n_terms, const double *coeff,
                                        const int64_t *term_ptr, const int32_t *term_ops, double *defect) {
    return guard(nullptr, [&] {
        if (!defect) throw ttn::Error(TTN_E_INVALID, "null output");
        std::vector<int32_t> ones(n_nodes > 0 ? n_nodes : 1, 1);
        ttn::Tree t = ttn::build_tree(n_nodes, parent, local_dim, ones.data());
        ttn::SopInput s = ttn::read_sop(t, n_ops, op_leaf, op_offset, op_data, n_terms, coeff, term_ptr, term_ops);
        *defect = ttn::sop_hermiticity_defect(s, 1e-12);
    });
}

ttn_status ttn_debug_tree_operator_stats(int32_t n_nodes, const int32_t *parent, const int32_t *local_dim,
                                         int32_t n_ops, const int32_t *op_leaf, const int64_t *op_offset,
                                         const double *op_data, int32_t n_terms, const double *coeff,
                                         const int64_t *term_ptr, const int32_t *term_ops, int32_t *n_channels,
                                         int32_t *n_entries, int32_t *n_merged, int32_t *n_sop_terms) {
    return guard(nullptr, [&] {
        std::vector<int32_t> ones(n_nodes > 0 ? n_nodes : 1, 1);
        ttn::Tree t = ttn::build_tree(n_nodes, parent, local_dim, ones.data());
        ttn::SopInput s = ttn::read_sop(t, n_ops, op_leaf, op_offset, op_data, n_terms, coeff, term_ptr, term_ops);
        ttn::TreeOp op = ttn::compile_tree_operator(t, s);
        // leaves below every node
        std::vector<std::vector<char>> below(t.n, std::vector<char>(t.n, 0));
        for (int z : t.postorder) {
            if (t.local_dim[z] > 0) below[z][z] = 1;
            for (int c : t.kids[z])
                for (int l = 0; l < t.n; ++l) below[z][l] |= below[c][l];
        }
        for (int z = 0; z < t.n; ++z) {
            if (n_channels) n_channels[z] = op.n_ch[z];
            if (n_entries) n_entries[z] = (int32_t)op.entries[z].size();
            if (n_merged) {  // the effective generator's products, as the engine builds them
                const int D = (int)t.dims[z].size();
                std::vector<ttn::MergeItem> items;
                for (auto &e : op.entries[z]) {
                    ttn::MergeItem it;
                    for (int k = 0; k < D - 1; ++k)
                        if (e.slot[k] >= 1) {
                            it.slot[it.nf] = k;
                            it.id[it.nf++] = (int64_t)k << 32 | e.slot[k];
                        }
                    if (z != t.root && e.bp != 1) {
                        it.slot[it.nf] = D - 1;
                        it.id[it.nf++] = (int64_t)(D - 1) << 32 | e.bp;
                    }
                    items.push_back(it);
                }
                int cnt = (int)items.size();
                for (auto &m : ttn::plan_entry_merge(items)) cnt -= (int)m.members.size() - 1;
                n_merged[z] = cnt;
            }
            if (n_sop_terms) {
                int cnt = 0;
                if (z != t.root)
                    for (int r = 0; r < s.n_terms; ++r) {
                        bool in = false, out = false;
                        for (int o : s.term_ops[r]) (below[z][s.op_leaf[o]] ? in : out) = true;
                        if (in && out) ++cnt;
                    }
                n_sop_terms[z] = cnt;
            }
        }
    });
}

ttn_status ttn_debug_qr(int64_t rows, int32_t cols, const double *m, int32_t variant, double *q_out,
                        double *r_out) {
    return guard(nullptr, [&] {
        if (!m || !q_out || !r_out) throw ttn::Error(TTN_E_INVALID, "null buffer");
        ttn::debug_qr(rows, cols, m, variant, q_out, r_out);
    });
}

}  // extern "C"
