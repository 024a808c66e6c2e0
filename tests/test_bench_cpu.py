"""Host logic of bench.py: roofline classification, the PMC traffic record,
the one-GPU guard (no GPU needed)."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _row(name, calls, ms, flops, byts):
    return {"name": name, "calls": calls, "total_ms": ms, "flops": flops, "bytes": byts}


def test_roofline_takes_the_kernel_with_the_largest_total_time():
    stats = [_row("k_mode_tile", 100, 2.0, 1e9, 3e8), _row("k_qr_coop", 10, 3.0, 1.2e8, 2.2e7)]
    r = bench.roofline(stats, 2, "vibronic24")
    assert r["kernel"] == "k_qr_coop" and r["launches_per_step"] == 5
    assert abs(r["avg_launch_us"] - 300.0) < 1e-9
    # intensity 5.5 flop/B is below the FP64 ridge (78.6 TF / 8 TB/s = 9.8): HBM bound
    assert r["bound"] == "hbm" and r["unit"] == "GB/s"
    assert abs(r["achieved"] - 2.2e6 / 300e-6 / 1e9) < 1e-9
    assert abs(r["frac"] - r["achieved"] / bench.PEAK_HBM_GBS) < 1e-15


def test_roofline_charges_the_pair_gemm_its_fixup_pass():
    """The cut tiles of the shared pair-GEMM schedule are summed by a second
    kernel: its time counts towards the GEMM's launch duration."""
    stats = [_row("k_pair_gemm", 10, 10.0, 1e12, 1e9), _row("k_pair_fixup", 10, 0.5, 0.0, 1e8)]
    r = bench.roofline(stats, 1, "x")
    assert r["kernel"] == "k_pair_gemm" and abs(r["avg_launch_us"] - 1050.0) < 1e-9
    assert abs(r["achieved"] - 1e11 / 1.05e-3 / 1e12) < 1e-9


def test_roofline_compute_bound_classes():
    # no modelled bytes: compute bound; plain FP64 vector code reports "alu" at the FP64 peak
    r = bench.roofline([_row("k_small_solve", 10, 1.0, 1e7, 0.0)], 1, "x")
    assert r["bound"] == "alu" and r["unit"] == "TFLOP/s" and r["peak"] == bench.PEAK_FP64_TFLOPS
    # FP32 vector code against the FP32 peak, the bf16 matrix-core stage against the bf16 peak
    r = bench.roofline([_row("k_mode_tile_f32", 10, 1.0, 1e10, 1e7)], 1, "x")
    assert r["bound"] == "alu" and r["peak"] == bench.PEAK_FP32_TFLOPS
    r = bench.roofline([_row("k_mode_mfma", 10, 1.0, 1e11, 1e7)], 1, "x")
    assert r["bound"] == "mfma" and r["peak"] == bench.PEAK_BF16_TFLOPS
    # the FP32 matrix-core stage against the FP32 peak (its name extends the bf16 stage's)
    r = bench.roofline([_row("k_mode_mfma32", 10, 1.0, 1e11, 1e7)], 1, "x")
    assert r["bound"] == "mfma" and r["peak"] == bench.PEAK_FP32_TFLOPS
    r = bench.roofline([_row("k_contract_mfma", 10, 1.0, 1e11, 1e7)], 1, "x")
    assert r["bound"] == "mfma" and r["peak"] == bench.PEAK_FP32_TFLOPS
    # the FP64 matrix-core stage against the FP64 peak
    r = bench.roofline([_row("k_mode_mfma64", 10, 1.0, 1e11, 1e7)], 1, "x")
    assert r["bound"] == "mfma" and r["peak"] == bench.PEAK_FP64_TFLOPS
    # the pair-operator GEMMs: FP32 matrix cores, and bf16 matrix cores in the BF16x3 form
    r = bench.roofline([_row("k_pair_gemm", 10, 1.0, 1e11, 1e7)], 1, "x")
    assert r["bound"] == "mfma" and r["peak"] == bench.PEAK_FP32_TFLOPS
    r = bench.roofline([_row("k_pair_gemm_bf", 10, 1.0, 1e12, 1e7)], 1, "x")
    assert r["bound"] == "mfma" and r["peak"] == bench.PEAK_BF16_TFLOPS
    # below the bf16 ridge (312 flop/B) the same kernel is HBM bound
    r = bench.roofline([_row("k_mode_mfma", 10, 1.0, 1e9, 1e7)], 1, "x")
    assert r["bound"] == "hbm"


def test_traffic_record_follows_the_kernel_sources():
    import hashlib
    src = os.path.join(ROOT, "paper_2503_15460_amd", "csrc", "kernels.hip")
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    found = 0
    for fn in sorted(os.listdir(os.path.join(ROOT, "profiles"))):
        if not fn.endswith("_hbm_traffic.md"):
            continue
        rec = None
        for line in open(os.path.join(ROOT, "profiles", fn)):
            if line.startswith("traffic: "):
                rec = json.loads(line[len("traffic: "):])
        assert rec is not None, fn
        workload = rec["workload"]
        got = bench.measured_traffic(rec["kernel"], workload)
        assert got == (rec["bytes_per_launch"] if sha == rec["kernels_hip_sha256"] else None)
        assert abs(rec["bytes_per_launch"] - rec["fetch_bytes_per_launch"] - rec["write_bytes_per_launch"]) <= 1
        found += 1
    assert found >= 1
    assert bench.measured_traffic("no_such_kernel", "vibronic24") is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_launch_summary():
    stats = [_row("k_small_solve", 40, 20.0, 0.0, 0.0), _row("k_mode_tile", 200, 10.0, 0.0, 0.0),
             _row("k_qr", 100, 5.0, 0.0, 0.0), _row("k_copy", 10, 1.0, 0.0, 0.0)]
    s = bench.launch_summary(stats, 2, 50.0)
    assert s["launches_per_step"] == 175 and abs(s["kernel_ms_per_step"] - 18.0) < 1e-12
    assert abs(s["kernel_busy_frac"] - 18.0 / 50.0) < 1e-12
    assert abs(s["avg_launch_us"] - 1e3 * 18.0 / 175) < 1e-9
    assert [t["kernel"] for t in s["top"]] == ["k_small_solve", "k_mode_tile", "k_qr"]


def test_oracle_step_baseline():
    """The oracle leg of the context lines: one whole step, also with
    time-dependent coefficients, reported as a rate with its thread count."""
    from workloads import ipchain_coefficients, ipchain_sbm_problem, sbm_problem
    r = bench.oracle_step(sbm_problem(n_modes=2, d=3, bond=2), threads=1)
    assert r["kind"] == "oracle" and r["cores"] == 1 and r["value"] > 0 and r["unit"] == "sweeps/s"
    p = ipchain_sbm_problem(n_modes=2, d=3, bonds=(2, 2, 2))
    r = bench.oracle_step(p, lambda t: ipchain_coefficients(p, t), threads=2)
    assert r["value"] > 0 and r["cores"] == min(2, os.cpu_count())
