#!/usr/bin/env python3
"""Throughput of the one-site TDVP sweep on one MI355X.

Workload: the synthetic 2-state / 24-mode vibronic-coupling model (seed 2;
3-layer tree R(E, M1, M2), M(L, L, L), L(4 modes), bonds 8/16/20, mode bases
8-32 levels, ~150 SOP terms), complex128, dt = 0.5 fs, from the product state
|s=1>|0...0>.  One step = one symmetric projector-splitting sweep
(ttn_step(dt)); the metric is sweeps per second with the state resident on
the GPU, plus the H_eff flop rate.

Prints ONE JSON line.  A separate short pass with the library's launch
profiler (dispatch-stamped HIP events per launch; the cooperative QR from its
own clock readings) gives the dominant kernel's average launch duration and
its roofline numbers; the oracle (CPU) is timed on a one-step sample of the
same workload.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6   # MI355X dense FP64 (matrix = vector)
PEAK_HBM_GBS = 8000.0     # MI355X HBM3E
PEAK_FP32_TFLOPS = 157.3  # MI355X dense FP32 (matrix = vector)
PEAK_BF16_TFLOPS = 2500.0  # MI355X dense bf16 matrix

# Kernels whose arithmetic is plain FP64 vector FMA code (no matrix-core
# instructions): their compute peak is the FP64 vector rate, 256 CUs x 2.4 GHz
# x 128 flop/clk/CU = 78.6 TFLOP/s.
ALU_KERNELS = {"k_small_solve", "k_mode_stage", "k_group_sum", "k_contract_part", "k_kry_orth", "k_qr",
               "k_qrm_step", "k_qrm_finish", "k_mode_single"}


def roofline(stats):
    """Roofline numbers of the kernel with the largest total time."""
    top = max(stats, key=lambda r: r["total_ms"])
    avg_s = top["total_ms"] / 1e3 / top["calls"]
    flops = top["flops"] / top["calls"]
    byts = top["bytes"] / top["calls"]
    intensity = flops / byts if byts > 0 else float("inf")
    ridge = PEAK_FP64_TFLOPS * 1e12 / (PEAK_HBM_GBS * 1e9)
    if flops > 0 and intensity >= ridge:
        ach = flops / avg_s / 1e12
        bound = "alu" if top["name"] in ALU_KERNELS else "mfma"
        r = dict(bound=bound, achieved=ach, peak=PEAK_FP64_TFLOPS, unit="TFLOP/s", frac=ach / PEAK_FP64_TFLOPS)
    else:
        ach = byts / avg_s / 1e9
        r = dict(bound="hbm", achieved=ach, peak=PEAK_HBM_GBS, unit="GB/s", frac=ach / PEAK_HBM_GBS)
    r.update(kernel=top["name"], avg_launch_us=avg_s * 1e6, flops_per_launch=flops, bytes_per_launch=byts,
             launches_per_step=None, traffic=None)
    return r


def measured_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 PMC summary
    (FETCH_SIZE and WRITE_SIZE, each scaled by the same counter's reading for a
    plain copy kernel of known size), or None when there is none or the kernel
    sources changed after the counters were taken (SHA-256 of kernels.hip)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"{kernel}_vibronic24_hbm_traffic.md")
    src = os.path.join(ROOT, "paper_2503_15460_amd", "csrc", "kernels.hip")
    if not os.path.exists(path):
        return None
    rec = None
    for line in open(path):
        if line.startswith("traffic: "):
            rec = json.loads(line[len("traffic: "):])
    if not rec:
        return None
    if hashlib.sha256(open(src, "rb").read()).hexdigest() != rec.get("kernels_hip_sha256"):
        return None
    return rec["bytes_per_launch"]


def timed_run(T, p, precision, steps, warmup):
    """Sweeps of the workload from its product state; returns (handle, seconds, counters before, after)."""
    import torch
    g = T.TTN.from_problem(p, precision=precision)
    g.set_product_state(p.init_vecs)
    g.step(p.dt, warmup)
    torch.cuda.synchronize()
    c0 = g.counters()
    t0 = time.perf_counter()
    g.step(p.dt, steps)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    return g, elapsed, c0, g.counters()


def fp32_error(T, p, steps: int):
    """Largest difference of populations and autocorrelation between the FP32
    and FP64 modes over `steps` sweeps from a seeded full-rank state (from the
    product state, rounding-size differences are amplified by the
    rank-deficient first QRs and say nothing about the FP32 contractions)."""
    from workloads import random_isometric_state
    runs = []
    for prec in (T.TTN_FP64, T.TTN_FP32):
        g = T.TTN.from_problem(p, precision=prec)
        st = random_isometric_state(p.parent, p.local_dim, g.bonds(), seed=2)
        g.set_state(st)
        obs = []
        for _ in range(steps):
            g.step(p.dt)
            obs += [g.expect(p.observables["P0"]), g.expect(p.observables["P1"]), g.overlap_t0()]
        runs.append(np.array(obs))
        g.close()
    return {"max_abs": float(np.abs(runs[0] - runs[1]).max()), "observables": "P0, P1, a(t)",
            "start": "seeded full-rank isometric state", "steps": steps}


def exciton_run(T, steps: int):
    """The 10-state / 120-mode exciton model (bonds 32-64), FP64 and FP32 modes:
    sweeps/s, H_eff flop rate and the FP32 population error against FP64."""
    import torch
    from workloads import exciton_problem
    p = exciton_problem()
    out, pops = {}, {}
    for prec, name in ((T.TTN_FP64, "fp64"), (T.TTN_FP32, "fp32"), (T.TTN_BF16X3, "bf16x3")):
        g, el, c0, c1 = timed_run(T, p, prec, steps, 1)
        pops[name] = np.array([g.expect(p.observables[f"P{k}"]).real for k in range(10)])
        T.profile_begin()
        g.step(p.dt)
        torch.cuda.synchronize()
        st = T.profile_end()
        kname = "k_mode_mfma" if prec == T.TTN_BF16X3 else "k_mode_tile"
        tile = [r for r in st if r["name"].startswith(kname)]
        tms = sum(r["total_ms"] for r in tile)
        tfl = sum(r["flops"] for r in tile)
        peak = {T.TTN_FP64: PEAK_FP64_TFLOPS, T.TTN_FP32: PEAK_FP32_TFLOPS, T.TTN_BF16X3: PEAK_BF16_TFLOPS}[prec]
        out[name] = {"value": steps / el, "unit": "sweeps/s", "ms_per_step": 1e3 * el / steps,
                     "heff_tflops": (c1["heff_flops"] - c0["heff_flops"]) / el / 1e12,
                     "stage_kernel": kname,
                     "stage_tflops": tfl / tms / 1e9 if tms > 0 else None,
                     "stage_frac": (tfl / tms / 1e9) / peak if tms > 0 else None,
                     "stage_peak_tflops": peak,
                     "device_gib": c1["device_bytes"] / 2**30}
        g.close()
    out["fp32_max_abs_population_diff_vs_fp64"] = float(np.abs(pops["fp64"] - pops["fp32"]).max())
    out["bf16x3_max_abs_population_diff_vs_fp64"] = float(np.abs(pops["fp64"] - pops["bf16x3"]).max())
    out["note"] = ("stage_tflops counts algorithmic complex flops (8 per MAC); BF16x3 executes three bf16 "
                   "matrix-core products per real product and its peak is the dense bf16 one. Product-state "
                   "start: population differences include the rank-deficient-QR amplification of rounding")
    out["workload"] = ("exciton10x120: 10 states, 120 modes in 60 composite leaves (d 36-144), 1500 SOP terms, "
                       "tree R(E,A,A) A(B,B,B) B(C,C) C(5 leaves), bonds 8/32/48/64, dt 0.5 fs, product start, "
                       f"{1 + steps} sweeps")
    return out


def heom_run(T, steps: int):
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
    for prec, name in ((T.TTN_FP64, "fp64"), (T.TTN_FP32, "fp32")):
        g, el, c0, c1 = timed_run(T, p, prec, steps, 1)
        vals[name] = obs(g)
        out[name] = {"value": steps / el, "unit": "sweeps/s", "ms_per_step": 1e3 * el / steps,
                     "heff_tflops": (c1["heff_flops"] - c0["heff_flops"]) / el / 1e12}
        g.close()
    out["sigma_z_trace_fp64"] = [float(vals["fp64"][0].real), float(vals["fp64"][1].real)]
    out["fp32_max_abs_diff_vs_fp64"] = float(np.abs(vals["fp64"] - vals["fp32"]).max())
    out["workload"] = (f"heom_sbm: eps 0.5, Delta 1, Debye lambda 0.2 gamma 1 T 1, 16 poles, 32 auxiliary modes x "
                       f"10 levels, binary tree, bonds 10-48, non-Hermitian (Arnoldi), dt 0.0075, {1 + steps} sweeps")
    return out


def batch_run(T, n_inst: int, steps: int):
    """Uneven spin-boson instances (8-64 modes, 6-16 levels, bonds 8-48): one
    at a time in FP64 against one batch (FP64 and FP32) on 8 streams."""
    import torch
    from workloads import batch_sbm_problems
    probs = batch_sbm_problems(seed=5, n_inst=n_inst)
    dts = np.array([p.dt for p in probs])
    res = {}
    for prec, name in ((T.TTN_FP64, "fp64"), (T.TTN_FP32, "fp32")):
        gs = []
        for p in probs:
            g = T.TTN.from_problem(p, precision=prec)
            g.set_product_state(p.init_vecs)
            g.step(p.dt)
            gs.append(g)
        torch.cuda.synchronize()
        if prec == T.TTN_FP64:
            t0 = time.perf_counter()
            for g, p in zip(gs, probs):
                g.step(p.dt, steps)
            torch.cuda.synchronize()
            res["sequential_fp64"] = n_inst * steps / (time.perf_counter() - t0)
        b = T.TTNBatch(gs, n_streams=8)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b.step(dts, steps)
        torch.cuda.synchronize()
        res[f"batched_{name}"] = n_inst * steps / (time.perf_counter() - t0)
        b.close()
        for g in gs:
            g.close()
    return {"unit": "instance-sweeps/s", **res,
            "speedup_batched_fp32_vs_sequential_fp64": res["batched_fp32"] / res["sequential_fp64"],
            "workload": f"{n_inst} of the 256 seeded uneven spin-boson instances (seed 5), {steps} timed sweeps each"}


def cpu_baseline(problem, steps: int):
    """The oracle (numpy complex128) on the host cores: seconds for `steps` sweeps."""
    from oracle import Oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    o = Oracle(problem)
    o.set_product_state(problem.init_vecs)
    t0 = time.perf_counter()
    for _ in range(steps):
        o.step(problem.dt)
    dt = time.perf_counter() - t0
    return dict(value=steps / dt, unit="sweeps/s", cores=threads, kind="oracle",
                sample=f"{steps} sweep(s) of the same 24-mode vibronic workload from the product state")


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--profile-steps", type=int, default=2)
    ap.add_argument("--cpu-steps", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true", help="skip the FP32-contraction comparison run")
    ap.add_argument("--no-extra", action="store_true", help="skip the exciton and batched-instance lines")
    ap.add_argument("--batch-instances", type=int, default=8)
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: the sweep runs on one GPU only (the sweep of one tree is sequential; "
              "see the design notes for how instances would shard); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2503_15460_amd as T
    from workloads import vibronic_problem

    torch.cuda.init()
    torch.zeros(1, device="cuda:0")
    p = vibronic_problem()
    g, elapsed, c0, c1 = timed_run(T, p, T.TTN_FP64, args.steps, args.warmup)
    sweeps_per_s = args.steps / elapsed
    heff_tflops = (c1["heff_flops"] - c0["heff_flops"]) / elapsed / 1e12
    pops = [g.expect(p.observables[k]).real for k in ("P0", "P1")]

    # profiled pass (separate from the timed region)
    T.profile_begin()
    g.step(p.dt, args.profile_steps)
    torch.cuda.synchronize()
    stats = T.profile_end()
    roof = roofline(stats)
    top = roof["kernel"]
    roof["launches_per_step"] = next(r["calls"] for r in stats if r["name"] == top) / args.profile_steps
    roof["traffic"] = measured_traffic(top)
    # the H_eff stage kernel of the same pass against its own (HBM) roofline
    tile = [r for r in stats if r["name"] == "k_mode_tile"]
    stage_roof = None
    if tile:
        r = tile[0]
        s_avg = r["total_ms"] / 1e3 / r["calls"]
        gbs = r["bytes"] / r["calls"] / s_avg / 1e9
        stage_roof = {"kernel": "k_mode_tile", "bound": "hbm", "achieved_gbs": gbs, "peak_gbs": PEAK_HBM_GBS,
                      "frac": gbs / PEAK_HBM_GBS, "tflops": r["flops"] / r["calls"] / s_avg / 1e12,
                      "avg_launch_us": s_avg * 1e6, "launches_per_step": r["calls"] / args.profile_steps}

    # the same run with the FP32 contraction mode (same steps from the same start)
    fp32 = None
    if not args.no_fp32:
        g32, el32, d0, d1 = timed_run(T, p, T.TTN_FP32, args.steps, args.warmup)
        g32.close()
        fp32 = {"value": args.steps / el32, "unit": "sweeps/s", "ms_per_step": 1e3 * el32 / args.steps,
                "heff_tflops": (d1["heff_flops"] - d0["heff_flops"]) / el32 / 1e12,
                "error_vs_fp64": fp32_error(T, p, steps=5)}

    out = {
        "metric": "TDVP sweeps/s + H_eff TFLOP/s (% MFMA peak), FP32-mixed vs FP64 at stated err",
        "value": sweeps_per_s,
        "unit": "sweeps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c128",
        "data": "synthetic (seeded 2-state 24-mode vibronic model standing in for pyrazine)",
        "config": {"workload": "vibronic24: 2 states x 24 modes (d 8-32), ~150 SOP terms, tree R(E,M,M) M(L,L,L) "
                               "L(4 modes), bonds 8/16/20, dt 0.5 fs, product initial state, FP64",
                   "precision": "fp64", "heff_tflops": heff_tflops,
                   "heff_frac_fp64_peak": heff_tflops / PEAK_FP64_TFLOPS,
                   "populations_after": pops, "redo_steps": c1["redo"] - c0["redo"],
                   "fp32_mixed": fp32, "heff_stage_roofline": stage_roof},
        "roofline": roof,
        "kernels": sorted(({k: (v if k != "name" else v) for k, v in r.items()} for r in stats),
                          key=lambda r: -r["total_ms"])[:8],
    }
    if not args.no_extra:
        # the other workloads are context lines: a failure there is recorded, and
        # the headline line is still printed
        for key, fn in (("exciton10x120", lambda: exciton_run(T, 1)), ("heom_sbm", lambda: heom_run(T, 3)),
                        ("batched_instances", lambda: batch_run(T, args.batch_instances, 1))):
            try:
                out["config"][key] = fn()
            except (T.TTNError, RuntimeError, MemoryError) as e:
                out["config"][key] = {"error": str(e)}
                print(f"bench.py: {key} failed: {e}", file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(p, args.cpu_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
