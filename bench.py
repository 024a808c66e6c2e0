#!/usr/bin/env python3
"""Throughput of the one-site TDVP sweep on one MI355X.

Headline workload: the synthetic 10-state / 120-mode donor-acceptor exciton
model (seed 3; 120 modes paired into 60 composite leaves of 36-144 levels,
1500 SOP terms; tree R(E, A1, A2), A(B, B, B), B(C, C), C(5 leaves), bonds
8/32/48/64: node tensors up to 48 x 48 x 48 x 64 = 7.08M elements), dt 0.5 fs,
from the product state |0>|vac>.  One step = one symmetric projector-splitting
sweep (ttn_step(dt)).  The metric is sweeps per second with the state resident
on the GPU in the FP32-mixed form (effective-generator and environment
contractions in complex FP32; QR, Krylov and the projected exponential in
FP64) against the FP64 form, with the H_eff flop rate and the error of every
population and of a(t) against FP64 from a seeded full-rank start.

Prints ONE JSON line.  A separate profiled sweep (dispatch-stamped HIP events
per launch; the cooperative QR from its own clock readings) gives the
dominant kernel's average launch duration and its roofline numbers; the
oracle (CPU) is timed on a bounded sample of the same workload.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6    # MI355X dense FP64 (matrix = vector)
PEAK_FP32_TFLOPS = 157.3   # MI355X dense FP32 (matrix = vector)
PEAK_BF16_TFLOPS = 2500.0  # MI355X dense bf16 matrix
PEAK_HBM_GBS = 8000.0      # MI355X HBM3E

HEADLINE = "fp32"  # the FP32-mixed form
PRECISIONS = {"fp64": 0, "fp32": 1, "bf16x3": 2}

# Compute peak of each kernel family: plain FMA code runs at the vector rate of
# its precision (256 CUs x 2.4 GHz x 128 (FP64) or 256 (FP32) flop/clk/CU);
# the BF16x3 stage and the BF16x3 pair-operator GEMM run on the bf16 matrix
# cores (their algorithmic flops count one complex product as 8 flops, while
# the hardware issues three bf16 products for it), the FP32 stage, the FP32
# environment contraction and the FP32 pair-operator GEMM on the FP32 matrix
# cores (whose dense peak equals the FP32 vector peak), the FP64 stage and the
# QR's Gram matrix on the FP64 matrix cores (dense peak equal to the FP64
# vector peak).  First match wins.
KERNEL_PEAK = [("k_mode_mfma32", "mfma", PEAK_FP32_TFLOPS), ("k_mode_mfma64", "mfma", PEAK_FP64_TFLOPS),
               ("k_contract_mfma", "mfma", PEAK_FP32_TFLOPS), ("k_cqr_gram_mfma", "mfma", PEAK_FP64_TFLOPS),
               ("k_mode_mfma", "mfma", PEAK_BF16_TFLOPS),
               ("k_pair_gemm_bf", "mfma", PEAK_BF16_TFLOPS), ("k_pair_gemm", "mfma", PEAK_FP32_TFLOPS),
               ("_f32", "alu", PEAK_FP32_TFLOPS)]


# second kernels that finish the work of a launch of the first
COMPANION = {"k_pair_gemm": "k_pair_fixup", "k_pair_gemm_bf": "k_pair_fixup"}


def kernel_peak(name: str):
    for key, bound, peak in KERNEL_PEAK:
        if key in name:
            return bound, peak
    return "alu", PEAK_FP64_TFLOPS


def roofline(stats, steps: int, workload: str):
    """Roofline numbers of the kernel with the largest total time: algorithmic
    flops and bytes per launch (the library's model of each launch) over the
    average launch duration, against the compute peak of its precision or the
    HBM peak, whichever bounds it at its arithmetic intensity.  A kernel with
    a companion pass (the pair GEMM's sum of cut tiles) is charged that pass's
    time too."""
    top = max(stats, key=lambda r: r["total_ms"])
    extra_ms = sum(r["total_ms"] for r in stats if r["name"] == COMPANION.get(top["name"]))
    avg_s = (top["total_ms"] + extra_ms) / 1e3 / top["calls"]
    flops = top["flops"] / top["calls"]
    byts = top["bytes"] / top["calls"]
    bound, peak = kernel_peak(top["name"])
    ridge = peak * 1e12 / (PEAK_HBM_GBS * 1e9)
    intensity = flops / byts if byts > 0 else float("inf")
    if flops > 0 and intensity >= ridge:
        ach = flops / avg_s / 1e12
        r = dict(bound=bound, achieved=ach, peak=peak, unit="TFLOP/s", frac=ach / peak)
    else:
        ach = byts / avg_s / 1e9
        r = dict(bound="hbm", achieved=ach, peak=PEAK_HBM_GBS, unit="GB/s", frac=ach / PEAK_HBM_GBS)
    r.update(kernel=top["name"], avg_launch_us=avg_s * 1e6, companion_ms=extra_ms, flops_per_launch=flops,
             bytes_per_launch=byts,
             launches_per_step=top["calls"] / steps, traffic=measured_traffic(top["name"], workload))
    return r


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 PMC summary
    (FETCH_SIZE and WRITE_SIZE, each scaled by the same counter's reading for a
    plain copy kernel of known size), or None when there is none or the kernel
    sources changed after the counters were taken (SHA-256 of kernels.hip)."""
    safe = "".join(ch if ch.isalnum() or ch == "_" else "_" for ch in kernel).strip("_")
    path = os.path.join(ROOT, "profiles", f"{safe}_{workload}_hbm_traffic.md")
    src = os.path.join(ROOT, "paper_2503_15460_amd", "csrc", "kernels.hip")
    if not os.path.exists(path):
        return None
    rec = None
    for line in open(path):
        if line.startswith("traffic: "):
            rec = json.loads(line[len("traffic: "):])
    if not rec or hashlib.sha256(open(src, "rb").read()).hexdigest() != rec.get("kernels_hip_sha256"):
        return None
    return rec["bytes_per_launch"]


def timed_run(T, p, precision, steps, warmup, keep=False):
    """`warmup` then `steps` timed sweeps from the product state; returns a dict
    (and the open handle when keep)."""
    import torch
    g = T.TTN.from_problem(p, precision=precision)
    g.set_product_state(p.init_vecs)
    g.step(p.dt, warmup)
    torch.cuda.synchronize()
    c0 = g.counters()
    t0 = time.perf_counter()
    g.step(p.dt, steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    c1 = g.counters()
    out = {"value": steps / el, "unit": "sweeps/s", "ms_per_step": 1e3 * el / steps,
           "heff_tflops": (c1["heff_flops"] - c0["heff_flops"]) / el / 1e12,
           "matvecs_per_step": (c1["matvecs"] - c0["matvecs"]) / steps, "redo_steps": c1["redo"] - c0["redo"],
           "device_gib": c1["device_bytes"] / 2**30}
    if keep:
        return out, g
    g.close()
    return out


def profiled_sweep(T, g, p, steps=1):
    import torch
    T.profile_begin()
    g.step(p.dt, steps)
    torch.cuda.synchronize()
    return T.profile_end()


def stage_rate(stats, precision):
    """Rate of the H_eff / environment stage kernels of a profiled sweep."""
    names = {0: ("k_mode_mfma64", "k_mode_tile"), 1: ("k_pair_gemm", "k_mode_mfma32", "k_mode_tile"),
             2: ("k_pair_gemm_bf", "k_mode_mfma")}[precision]
    name = "+".join(names)
    # BF16x3: the bf16 stage only (not the FP32 / FP64 ones, whose names share the prefix)
    rows = [r for r in stats if r["name"].startswith(names)
            and not (precision == 2 and ("mfma32" in r["name"] or "mfma64" in r["name"]))]
    ms = sum(r["total_ms"] for r in rows)
    fl = sum(r["flops"] for r in rows)
    if ms <= 0:
        return None
    peak = {0: PEAK_FP64_TFLOPS, 1: PEAK_FP32_TFLOPS, 2: PEAK_BF16_TFLOPS}[precision]
    return {"kernel": name, "tflops": fl / ms / 1e9, "frac": fl / ms / 1e9 / peak, "peak_tflops": peak,
            "share_of_sweep_kernel_time": ms / sum(r["total_ms"] for r in stats)}


def error_vs_fp64(T, p, obs, precisions, steps, seed):
    """Largest difference of each observable between each mixed form and FP64
    over `steps` sweeps from a seeded full-rank isometric state (from the
    product state, the rank-deficient first QRs amplify rounding of any
    precision and say nothing about the contractions)."""
    from workloads import random_isometric_state
    bonds = T.clamp_bonds(p.parent, p.local_dim, p.bond_dim)
    st = random_isometric_state(p.parent, p.local_dim, bonds, seed=seed)
    runs = {}
    for name in ["fp64"] + list(precisions):
        g = T.TTN.from_problem(p, precision=PRECISIONS[name])
        g.set_state(st)
        rows = []
        for k in range(steps):
            t0 = time.perf_counter()
            g.step(p.dt)
            rows.append([g.expect(p.observables[o]) for o in obs] + [g.overlap_t0()])
            print(f"bench.py: {p.name} {name} from a full-rank state, sweep {k + 1}/{steps}: "
                  f"{time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
        runs[name] = np.array(rows)
        g.close()
    out = {"start": f"seeded full-rank isometric state (seed {seed})", "steps": steps,
           "observables": list(obs) + ["a(t)"]}
    for name in precisions:
        d = np.abs(runs[name] - runs["fp64"]).max(axis=0)
        out[name] = {"max_abs": float(d.max()), "per_observable": [float(x) for x in d]}
    return out


def cpu_oracle_sample(p, a_matvecs_per_step: float, a_node: int, n_terms_sample: int, threads: int):
    """The oracle on the host: its effective-generator application at an A node
    (7.08M elements) is the sweep's dominant local operation.  A sample of its
    per-term products (the code path Oracle.heff runs for every crossing term,
    on random environment matrices of the right shapes) is timed, scaled to the
    node's full term list and to the A-node matvecs of one sweep; all other work
    of the sweep is left out, so the rate is an upper bound on the oracle's."""
    from threadpoolctl import threadpool_limits

    from oracle import Oracle
    o = Oracle(p)
    kids = o.kids[a_node]
    pax = len(kids)
    # the terms Oracle.heff applies one by one at this node: touching it, not
    # lying inside one child (those are summed into the child's inside channel)
    crossing = [r for r in range(len(o.terms))
                if o.touches(r, a_node) and not any(o.inside(r, c) for c in kids)]
    rng = np.random.default_rng(0)
    shp = o.shape(a_node)
    X = rng.normal(size=shp) + 1j * rng.normal(size=shp)
    sample = sorted(rng.choice(len(crossing), size=min(n_terms_sample, len(crossing)), replace=False))
    facs = []
    for i in sample:
        r = crossing[i]
        f = {k: rng.normal(size=(shp[k], shp[k])) + 0j for k, c in enumerate(kids) if o.touches(r, c)}
        if o.touches_outside(r, a_node):
            f[pax] = rng.normal(size=(shp[pax], shp[pax])) + 0j
        facs.append((r, f))
    with threadpool_limits(limits=threads):
        o._apply_factors(X, facs[0][1])  # warm-up
        t0 = time.perf_counter()
        for r, f in facs:
            _ = o.coef[r] * o._apply_factors(X, f)
        el = time.perf_counter() - t0
    per_term = el / len(facs)
    t_matvec = per_term * len(crossing)
    t_step = t_matvec * a_matvecs_per_step
    return {"value": 1.0 / t_step, "unit": "sweeps/s", "cores": threads, "kind": "oracle",
            "sample": (f"{len(facs)} of the {len(crossing)} per-term products of the oracle's H_eff application at "
                       f"an A node ({int(np.prod(shp))} elements), {el:.1f} s, scaled to the full term list and to "
                       f"the {a_matvecs_per_step:.0f} A-node matvecs of one sweep (all other work left out: an "
                       f"upper bound on the oracle's rate)"),
            "seconds_per_step_estimate": t_step}


def oracle_step(p, coef_at=None, threads: int = 16):
    """The oracle on the host: one whole step of p from its product state
    (coefficients at the step's midpoint when they depend on time), timed at
    `threads` BLAS threads (at most the host's)."""
    from threadpoolctl import threadpool_limits

    from oracle import Oracle
    threads = max(1, min(threads, os.cpu_count() or 1))
    o = Oracle(p)
    o.set_product_state(p.init_vecs)
    with threadpool_limits(limits=threads):
        t0 = time.perf_counter()
        if coef_at is None:
            o.step(p.dt)
        else:
            o.step_td(p.dt, coef_at)
        el = time.perf_counter() - t0
    return {"value": 1.0 / el, "unit": "sweeps/s", "cores": threads, "kind": "oracle",
            "sample": f"one whole step from the product state, {el:.1f} s"}


def launch_summary(stats, steps: int, wall_ms_per_step: float):
    """Launch-level view of a profiled sweep: launches and summed kernel time
    per step, the fraction of the (unprofiled) wall time the kernels fill, and
    the three kernels with the largest total time."""
    launches = sum(r["calls"] for r in stats) / steps
    busy = sum(r["total_ms"] for r in stats) / steps
    top = sorted(stats, key=lambda r: -r["total_ms"])[:3]
    return {"launches_per_step": launches, "kernel_ms_per_step": busy,
            "kernel_busy_frac": busy / wall_ms_per_step if wall_ms_per_step > 0 else None,
            "avg_launch_us": 1e3 * busy / launches if launches else None,
            "top": [{"kernel": r["name"], "ms_per_step": r["total_ms"] / steps, "calls_per_step": r["calls"] / steps}
                    for r in top]}


def vibronic_line(T, steps, warmup):
    """Secondary line: the 2-state / 24-mode vibronic model (bonds 8/16/20) in
    FP64 and FP32-mixed."""
    from workloads import vibronic_problem
    p = vibronic_problem()
    out = {"workload": "vibronic24: 2 states x 24 modes (d 8-32), ~150 SOP terms, tree R(E,M,M) M(L,L,L) "
                       "L(4 modes), bonds 8/16/20, dt 0.5 fs, product initial state"}
    out["fp64"], g = timed_run(T, p, 0, steps, warmup, keep=True)
    st = profiled_sweep(T, g, p, 2)
    out["fp64"]["roofline"] = roofline(st, 2, "vibronic24")
    g.close()
    out["fp32"] = timed_run(T, p, 1, steps, warmup)
    out["fp32"]["error_vs_fp64"] = error_vs_fp64(T, p, ["P0", "P1"], ["fp32"], 5, 2)
    return out


def heom_line(T, steps: int):
    """HEOM spin-boson (Debye bath, K = 16 poles, 32 auxiliary modes x 10
    levels, bonds 10-48, Arnoldi): FP64 and FP32 sweeps/s and the FP32
    difference of <sigma_z> and Tr rho_S against FP64."""
    from workloads import heom_sbm_problem
    p = heom_sbm_problem()
    S = p.leaf_names["S"]

    def obs(g):
        out = []
        for key in ("bra_sz", "bra_tr"):
            bra = {z: np.eye(p.local_dim[z])[0].astype(np.complex128) for z in p.leaves()}
            bra[S] = p.meta[key]
            out.append(g.bilinear(bra))
        return np.array(out)
    out, vals = {}, {}
    for name in ("fp64", "fp32"):
        out[name], g = timed_run(T, p, PRECISIONS[name], steps, 1, keep=True)
        vals[name] = obs(g)
        g.close()
    out["sigma_z_trace_fp64"] = [float(vals["fp64"][0].real), float(vals["fp64"][1].real)]
    out["fp32_max_abs_diff_vs_fp64"] = float(np.abs(vals["fp64"] - vals["fp32"]).max())
    out["workload"] = (f"heom_sbm: eps 0.5, Delta 1, Debye lambda 0.2 gamma 1 T 1, 16 poles, 32 auxiliary modes x "
                       f"10 levels, binary tree, bonds 10-48, non-Hermitian (Arnoldi), dt 0.0075, {1 + steps} sweeps")
    return out


def pseudomode_line(T, steps: int):
    """Quasi-Lindblad pseudomode spin-boson (the same Debye bath as the HEOM
    line with 8 poles, each pseudomode and its tilde partner one leaf of 5 x 5
    levels, bonds 16-32, Arnoldi): FP64 and FP32 sweeps/s, <sigma_z> and
    Tr rho_S (the boson trace) after the sweeps."""
    from workloads import pseudomode_sbm_problem
    p = pseudomode_sbm_problem(K=8, levels=5, bonds=(16, 24, 32))
    S = p.leaf_names["S"]

    def obs(g):
        out = []
        for key in ("bra_sz", "bra_tr"):
            bra = {z: p.meta["bra_bath"] for z in p.leaves()}
            bra[S] = p.meta[key]
            out.append(g.bilinear(bra))
        return np.array(out)
    out, vals = {}, {}
    for name in ("fp64", "fp32"):
        out[name], g = timed_run(T, p, PRECISIONS[name], steps, 1, keep=True)
        vals[name] = obs(g)
        if name == "fp64":
            try:
                st = profiled_sweep(T, g, p, 1)
                out[name]["launches"] = launch_summary(st, 1, out[name]["ms_per_step"])
                out[name]["roofline"] = roofline(st, 1, "pseudomode_sbm")
            except Exception as e:  # context only: the line keeps its timings
                out[name]["launches"] = {"error": str(e)}
        g.close()
    try:
        out["cpu_baseline"] = oracle_step(p)
    except Exception as e:
        out["cpu_baseline"] = {"error": str(e)}
    out["sigma_z_trace_fp64"] = [float(vals["fp64"][0].real), float(vals["fp64"][1].real)]
    out["fp32_max_abs_diff_vs_fp64"] = float(np.abs(vals["fp64"] - vals["fp32"]).max())
    out["workload"] = ("pseudomode_sbm: eps 0.5, Delta 1, Debye lambda 0.2 gamma 1 T 1, 8 poles as quasi-Lindblad "
                       "pseudomodes (leaf = mode and tilde partner, 5 x 5 levels), binary tree, bonds 16-32, "
                       f"non-Hermitian (Arnoldi), dt 0.0075, {1 + steps} sweeps")
    return out


def ipchain_line(T, steps: int):
    """Interaction-picture chain spin-boson (Ohmic, alpha 0.5, w_c 5, 64 chain
    modes of 8 levels, bonds 8-24): time-dependent couplings G_l(t) set at
    every step's midpoint through ttn_set_coefficients.  FP64 and FP32 sweeps/s
    with the coefficient updates inside the timed region (FP32 also with step
    graphs), the share of the time spent in the updates, and <sigma_z>."""
    import torch
    from workloads import ipchain_coefficients, ipchain_sbm_problem
    p = ipchain_sbm_problem(n_modes=64, d=8, bonds=(8, 16, 24), eps=0.0, delta=1.0, alpha=0.5, wc=5.0, dt=0.02)
    coef = lambda t: ipchain_coefficients(p, t)  # noqa: E731
    out = {}
    for name, prec, graph in (("fp64", T.TTN_FP64, False), ("fp32", T.TTN_FP32, False),
                              ("fp32_graph", T.TTN_FP32, True)):
        g = T.TTN(p.parent, p.local_dim, p.bond_dim, precision=prec, hermitian=True, use_graph=graph)
        g.set_sop_problem(p)
        g.set_product_state(p.init_vecs)
        t = g.step_td(p.dt, coef, 0.0, 2)  # step graphs: the second step settles the capture key
        torch.cuda.synchronize()
        upd = 0.0
        t0 = time.perf_counter()
        for _ in range(steps):
            u0 = time.perf_counter()
            g.set_coefficients(coef(t + 0.5 * p.dt))
            upd += time.perf_counter() - u0
            g.step(p.dt)
            t += p.dt
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        out[name] = {"value": steps / el, "unit": "sweeps/s", "ms_per_step": 1e3 * el / steps,
                     "coefficient_update_ms": 1e3 * upd / steps,
                     "sigma_z": float(g.expect(p.observables["sz"]).real)}
        if graph:
            out[name]["graph_captures"] = g.graph_captures()
        if name == "fp64":
            try:
                g.set_coefficients(coef(t + 0.5 * p.dt))
                st = profiled_sweep(T, g, p, 1)
                out[name]["launches"] = launch_summary(st, 1, out[name]["ms_per_step"] - out[name]["coefficient_update_ms"])
                out[name]["roofline"] = roofline(st, 1, "ipchain_sbm")
            except Exception as e:  # context only: the line keeps its timings
                out[name]["launches"] = {"error": str(e)}
        g.close()
    try:
        out["cpu_baseline"] = oracle_step(p, coef)
    except Exception as e:
        out["cpu_baseline"] = {"error": str(e)}
    out["workload"] = ("ipchain_sbm: eps 0, Delta 1, Ohmic alpha 0.5 w_c 5 (Gauss rule to 10 w_c), 64 chain modes "
                       "of 8 levels in a balanced binary tree beside the spin, bonds 8-24, dt 0.02, couplings "
                       f"G_l(t) at every step's midpoint, {2 + steps} steps")
    return out


def batch_line(T, n_inst: int, steps: int, warmup: int):
    """Uneven spin-boson instances (8-64 modes, 6-16 levels, bonds 8-48): one
    at a time in FP64 against one batch in FP32-mixed on several streams, and
    in lockstep sweep layers (one grouped launch of the fused solver per layer)
    with and without step graphs."""
    import torch
    from workloads import batch_sbm_problems
    allp = batch_sbm_problems(seed=5)
    stride = max(1, len(allp) // n_inst)
    probs = allp[::stride][:n_inst]  # spread over the seeded sizes
    dts = np.array([p.dt for p in probs])
    n_inst = len(probs)
    res = {}
    for name, prec, mode, graph in (("sequential_fp64", 0, None, False), ("streams_fp32", 1, "streams", False),
                                    ("lockstep_fp32", 1, "lockstep", False), ("streams_graph_fp32", 1, "streams", True)):
        gs = []
        for p in probs:
            g = T.TTN(p.parent, p.local_dim, p.bond_dim, precision=prec, use_graph=graph)
            g.set_sop_problem(p)
            g.set_product_state(p.init_vecs)
            gs.append(g)
        b = None
        if mode is not None:
            b = T.TTNBatch(gs, lockstep=(mode == "lockstep"))
            b.step(dts, warmup)
        else:
            for i, (g, p) in enumerate(zip(gs, probs)):
                g.step(p.dt, warmup)
                if (i + 1) % 64 == 0:
                    print(f"bench.py: batch, {name}: {i + 1} of {n_inst} instances warmed up", file=sys.stderr,
                          flush=True)
        torch.cuda.synchronize()
        print(f"bench.py: batch of {n_inst} instances, {name}: warm-up done", file=sys.stderr, flush=True)
        t0 = time.perf_counter()
        if b is not None:
            b.step(dts, steps)
        else:
            for i, (g, p) in enumerate(zip(gs, probs)):
                g.step(p.dt, steps)
                if (i + 1) % 64 == 0:
                    print(f"bench.py: batch, {name}: {i + 1} of {n_inst} instances stepped", file=sys.stderr,
                          flush=True)
        torch.cuda.synchronize()
        res[name] = n_inst * steps / (time.perf_counter() - t0)
        print(f"bench.py: batch of {n_inst} instances, {name}: {res[name]:.1f} instance-sweeps/s", file=sys.stderr,
              flush=True)
        if b is not None:
            b.close()
        for g in gs:
            g.close()
    best = max(res["streams_fp32"], res["lockstep_fp32"], res["streams_graph_fp32"])
    return {"unit": "instance-sweeps/s", **res, "speedup_best_fp32_vs_sequential_fp64": best / res["sequential_fp64"],
            "note": "streams_graph_fp32: step graphs (use_graph) on several streams",
            "workload": f"{len(probs)} of the 256 seeded uneven spin-boson instances (seed 5, every {stride}th), "
                        f"{warmup} warm-up and {steps} timed sweeps each"}


def ground_line(T, sweeps: int):
    """One-site ground-state sweeps (DMRG on trees, Sec. II C) on the vibronic
    model from its product state, FP64 and FP32-mixed: sweeps/s and the energy
    after every sweep (exact-diagonalisation parity is in the tests, on trees
    small enough for the dense generator)."""
    import torch
    from workloads import vibronic_problem
    p = vibronic_problem()
    out = {"workload": "vibronic24 ground state: one-site sweeps (S, root, S*) with Lanczos lowest-eigenvector "
                       f"node solves and no bond steps, {sweeps} sweeps from the product state"}
    for name in ("fp64", "fp32"):
        g = T.TTN.from_problem(p, precision=PRECISIONS[name])
        g.set_product_state(p.init_vecs)
        es, per = [], []
        for k in range(sweeps):
            t0 = time.perf_counter()
            e = g.ground_sweeps(1)
            torch.cuda.synchronize()
            per.append(time.perf_counter() - t0)
            es.append(e)
        out[name] = {"unit": "sweeps/s", "value": (sweeps - 1) / sum(per[1:]), "energy_per_sweep_eV": es,
                     "norm_minus_1": g.norm2() - 1.0}
        print(f"bench.py: vibronic24 ground state {name}: {1e3 * sum(per[1:]) / (sweeps - 1):.0f} ms/sweep, "
              f"energy {es[-1]:.10f}", file=sys.stderr, flush=True)
        g.close()
    out["fp32_energy_minus_fp64"] = out["fp32"]["energy_per_sweep_eV"][-1] - out["fp64"]["energy_per_sweep_eV"][-1]
    return out


def adaptive_line(T, steps: int):
    """The exciton workload with subspace expansion (Sec. II D) from bonds of 8
    (spawning tolerance 1e-6, bonds up to 8/32/48/64 per layer), FP32-mixed:
    sweeps/s and how the bonds grew."""
    import torch
    from workloads import exciton_problem
    p = exciton_problem()
    start = np.minimum(np.asarray(p.bond_dim), 8)
    g = T.TTN(p.parent, p.local_dim, start, precision=PRECISIONS["fp32"], spawn_tol=1e-6, bond_max=p.bond_dim,
              seed=3)
    g.set_sop_problem(p)
    g.set_product_state(p.init_vecs)
    b0 = int(g.bonds().sum())
    per = []
    for k in range(steps):
        t0 = time.perf_counter()
        g.step(p.dt)
        torch.cuda.synchronize()
        per.append(time.perf_counter() - t0)
        print(f"bench.py: exciton10x120 with subspace expansion, sweep {k + 1}/{steps}: {per[-1]:.1f} s, bond sum "
              f"{int(g.bonds().sum())}", file=sys.stderr, flush=True)
    b = g.bonds()
    out = {"unit": "sweeps/s", "value": steps / sum(per), "seconds_per_sweep": per, "bond_sum_start": b0,
           "bond_sum_end": int(b.sum()), "largest_bond": int(b.max()), "norm_minus_1": g.norm2() - 1.0,
           "workload": "exciton10x120 from bonds of 8, spawning tolerance 1e-6 (|dt/2| sigma), FP32-mixed, "
                       f"{steps} sweeps from the product state"}
    g.close()
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--error-steps", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-error", action="store_true", help="skip the error runs from a full-rank start")
    ap.add_argument("--no-extra", action="store_true", help="skip the secondary workloads")
    ap.add_argument("--only", choices=list(PRECISIONS), help="time one precision only (profiling runs)")
    ap.add_argument("--batch-instances", type=int, default=16)
    ap.add_argument("--batch-steps", type=int, default=2)
    ap.add_argument("--batch-warmup", type=int, default=1)
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: the sweep runs on one GPU only (the sweep of one tree is sequential; "
              "see the design notes for how instances would shard); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2503_15460_amd as T
    from workloads import exciton_problem

    torch.cuda.init()
    torch.zeros(1, device="cuda:0")
    p = exciton_problem()
    names = [args.only] if args.only else ["fp64", "fp32", "bf16x3"]
    runs, rooflines, a_matvecs = {}, {}, None
    for name in names:
        prec = PRECISIONS[name]
        r, g = timed_run(T, p, prec, args.steps, args.warmup, keep=True)
        print(f"bench.py: exciton10x120 {name}: {r['ms_per_step']:.0f} ms/sweep", file=sys.stderr, flush=True)
        st = profiled_sweep(T, g, p)
        r["stage"] = stage_rate(st, prec)
        rooflines[name] = roofline(st, 1, "exciton10x120")
        r["top_kernels"] = [{k: v for k, v in x.items()} for x in sorted(st, key=lambda x: -x["total_ms"])[:12]]
        if name == "fp64" or a_matvecs is None:
            node, fwd, mv = g.step_solves()
            root = [z for z in range(p.n_nodes) if p.parent[z] < 0][0]
            a_nodes = [z for z in range(p.n_nodes) if p.parent[z] == root and p.local_dim[z] == 0]
            a_matvecs = (float(sum(m for z, f, m in zip(node, fwd, mv) if f and z in a_nodes)) / len(a_nodes),
                         a_nodes[0])
        g.close()
        runs[name] = r
    head = args.only or HEADLINE
    hr = runs[head]
    peak = {"fp64": PEAK_FP64_TFLOPS, "fp32": PEAK_FP32_TFLOPS, "bf16x3": PEAK_BF16_TFLOPS}
    config = {
        "workload": ("exciton10x120: 10 electronic states x 120 modes paired into 60 composite leaves (d 36-144), "
                     "1500 SOP terms, tree R(E,A1,A2) A(B,B,B) B(C,C) C(5 leaves), bonds 8/32/48/64 (node tensors "
                     "up to 48x48x48x64), dt 0.5 fs, product initial state, fixed bonds"),
        "precision": {"fp64": "FP64", "fp32": "FP32-mixed: H_eff / environment contractions complex FP32, "
                      "QR / Krylov / projected exponential FP64",
                      "bf16x3": "BF16x3-mixed: as FP32-mixed, dense stages on bf16 matrix cores with hi/lo split"}[head],
        "heff_tflops": hr["heff_tflops"], "heff_frac_peak": hr["heff_tflops"] / peak[head],
        "runs": runs,
    }
    if "fp64" in runs and head != "fp64":
        config["speedup_vs_fp64"] = hr["value"] / runs["fp64"]["value"]
    if not args.no_error and not args.only:
        config["error_vs_fp64"] = error_vs_fp64(T, p, [f"P{k}" for k in range(10)], ["fp32", "bf16x3"],
                                                args.error_steps, 3)
    out = {
        "metric": "TDVP sweeps/s + H_eff TFLOP/s (% MFMA peak), FP32-mixed vs FP64 at stated err",
        "value": hr["value"],
        "unit": "sweeps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": hr["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "c128", "fp32": "c64+c128", "bf16x3": "bf16x3+c128"}[head],
        "data": "synthetic (seeded 10-state 120-mode exciton model standing in for P3HT:PCBM)",
        "config": config,
        "roofline": rooflines[head],
    }
    if not args.no_extra:
        # context lines: a failure there is recorded and the headline still printed
        for key, fn in (("vibronic24", lambda: vibronic_line(T, 30, 3)),
                        ("heom_sbm", lambda: heom_line(T, 3)),
                        ("pseudomode_sbm", lambda: pseudomode_line(T, 3)),
                        ("ipchain_sbm", lambda: ipchain_line(T, 5)),
                        ("exciton10x120_adaptive", lambda: adaptive_line(T, 3)),
                        ("vibronic24_ground_state", lambda: ground_line(T, 6)),
                        ("batched_instances", lambda: batch_line(T, args.batch_instances, args.batch_steps, args.batch_warmup))):
            try:
                t0 = time.perf_counter()
                config[key] = fn()
                print(f"bench.py: {key} line done in {time.perf_counter() - t0:.0f} s", file=sys.stderr, flush=True)
            except (T.TTNError, RuntimeError, MemoryError) as e:
                config[key] = {"error": str(e)}
                print(f"bench.py: {key} failed: {e}", file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        # samples of about 10 s of host work each (0.05-0.1 s per product)
        cb = cpu_oracle_sample(p, a_matvecs[0], a_matvecs[1], 120, threads)
        one = cpu_oracle_sample(p, a_matvecs[0], a_matvecs[1], 60, 1)
        cb["value_1_thread"] = one["value"]
        cb["sample_1_thread"] = one["sample"]
        out["cpu_baseline"] = cb
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
