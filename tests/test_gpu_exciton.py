"""Exciton-model trees on the GPU against the oracle: nodes with five composite
leaves (6 tensor slots), one-child nodes and a 3-state electronic leaf; the
FP64 path to 1e-10, the FP32 and BF16x3 modes to 1e-4 on populations and the
autocorrelation (full-rank starts)."""
import numpy as np
import pytest

from oracle import Oracle
from workloads import exciton_problem, random_isometric_state

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def T():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2503_15460_amd as mod
    return mod


def _obs(src, p):
    return np.array([src.expect(p.observables[f"P{k}"]) for k in range(3)] + [src.overlap_t0()])


def _reference(p, st, n):
    o = Oracle(p)
    o.set_state(st)
    out = []
    for _ in range(n):
        o.step(p.dt)
        out.append(_obs(o, p))
    return np.array(out)


def _run(T, p, st, n, precision):
    g = T.TTN.from_problem(p, precision=precision)
    g.set_state(st)
    T.profile_begin()
    out = []
    for _ in range(n):
        g.step(p.dt)
        out.append(_obs(g, p))
    names = {r["name"] for r in T.profile_end()}
    g.close()
    return np.array(out), names


def test_exciton_tree_fp64_parity(T):
    p = exciton_problem(n_states=3, n_modes=40, dmin=2, dmax=3, leaf_bond=3, c_bond=6, b_bond=8, a_bond=10,
                        n_inter=8)
    st = random_isometric_state(p.parent, p.local_dim, Oracle(p).bond, seed=12)
    ref = _reference(p, st, 3)
    got, _ = _run(T, p, st, 3, T.TTN_FP64)
    assert np.abs(got - ref).max() < 1e-10


def test_exciton_tree_mixed_precisions(T):
    """Bonds of 24: the two-child nodes' stages qualify for the matrix cores
    (BF16x3 stage in that mode, FP32 stage in the FP32 mode)."""
    p = exciton_problem(n_states=3, n_modes=40, dmin=2, dmax=3, leaf_bond=3, c_bond=24, b_bond=24, a_bond=24,
                        n_inter=8)
    st = random_isometric_state(p.parent, p.local_dim, Oracle(p).bond, seed=13)
    ref = _reference(p, st, 2)
    got, _ = _run(T, p, st, 2, T.TTN_FP64)
    assert np.abs(got - ref).max() < 1e-10
    for prec in (T.TTN_FP32, T.TTN_BF16X3):
        got, names = _run(T, p, st, 2, prec)
        err = np.abs(got - ref).max()
        print(f"precision {prec}: max error {err:.2e}")
        assert err < 1e-4
        assert ("k_mode_mfma" in names) == (prec == T.TTN_BF16X3)
        assert ("k_mode_mfma32" in names) == (prec == T.TTN_FP32)


def _obs10(src, p):
    return np.array([src.expect(p.observables[f"P{k}"]) for k in range(10)] + [src.overlap_t0()])


@pytest.mark.parametrize("prec,tol", [(0, 1e-10), (1, 1e-4), (2, 1e-4)])
def test_c3_shaped_tree_parity(T, prec, tol):
    """The exciton workload's tree at reduced size (10 states, 60 modes in 30
    composite leaves, five-leaf C nodes, B(C, C), A1(B, B), A2(B), bonds
    4/24/28/32: every stage factor of 24..32 qualifies for the matrix cores in
    BF16x3; 735 SOP terms), three sweeps from a seeded full-rank state against
    the stored oracle run, per precision: all ten populations and a(t) after
    every sweep (FP64 to 1e-10, FP32 and BF16x3 contractions to 1e-4), FP64
    also element-wise on sampled entries of every node tensor."""
    import golden_refs as G
    p = G.maker.c3_shaped()
    bonds = T.clamp_bonds(p.parent, p.local_dim, p.bond_dim)
    st = random_isometric_state(p.parent, p.local_dim, bonds, seed=31)
    rec = G.reference("c3_shaped", p, bonds, st)
    ref = G.observables(rec)
    g = T.TTN.from_problem(p, precision=prec)
    g.set_state(st)
    T.profile_begin()
    got = []
    for _ in range(3):
        g.step(p.dt)
        got.append(_obs10(g, p))
    names = {r["name"] for r in T.profile_end()}
    got = np.array(got)
    err = np.abs(got - ref).max(axis=0)
    print(f"precision {prec}: max error per observable (P0..P9, a(t)) {np.array2string(err, precision=1)}")
    assert err.max() < tol
    assert ("k_mode_mfma" in names) == (prec == T.TTN_BF16X3)
    assert ("k_mode_mfma32" in names) == (prec == T.TTN_FP32)
    if prec == T.TTN_FP64:
        terr = G.tensor_sample_error(rec, g.get_state())
        print(f"node tensors (sampled) within {terr:.2e}")
        assert terr < 1e-10
    g.close()


@pytest.mark.parametrize("prec,dtol", [(1, 1e-6), (2, 1e-5)])
def test_pair_operator_form_on_the_c3_shaped_tree(T, monkeypatch, prec, dtol):
    """Effective generators in the pair-operator form (each child slot's
    products summed into one dense operator on the pair (child, parent) and
    applied as a GEMM on the matrix cores: FP32, or BF16x3 where the parent
    dimension is a multiple of 32), switched on for every eligible node of the
    C3-shaped tree by lowering the node-size threshold: three sweeps from the
    seeded full-rank state against the stored oracle run (1e-4, as the other
    mixed-precision contractions) and against the staged products of the same
    precision mode (1e-6 FP32, 1e-5 BF16x3)."""
    import golden_refs as G
    p = G.maker.c3_shaped()
    bonds = T.clamp_bonds(p.parent, p.local_dim, p.bond_dim)
    st = random_isometric_state(p.parent, p.local_dim, bonds, seed=31)
    ref = G.observables(G.reference("c3_shaped", p, bonds, st))
    runs = {}
    for form, env in (("pair", {"TTN_PAIR_MIN_N": "1"}), ("staged", {"TTN_PAIR_OPS": "0"})):
        for k, v in env.items():
            monkeypatch.setenv(k, v)
        g = T.TTN.from_problem(p, precision=prec)
        for k in env:
            monkeypatch.delenv(k)
        g.set_state(st)
        T.profile_begin()
        got = []
        for _ in range(3):
            g.step(p.dt)
            got.append(_obs10(g, p))
        names = {r["name"] for r in T.profile_end()}
        runs[form] = np.array(got)
        assert ("k_pair_gemm" in names) == (form == "pair")
        # the A nodes (parent dimension 32) take the BF16x3 GEMM in that mode
        assert ("k_pair_gemm_bf" in names) == (form == "pair" and prec == T.TTN_BF16X3)
        g.close()
    err = np.abs(runs["pair"] - ref).max()
    diff = np.abs(runs["pair"] - runs["staged"]).max()
    print(f"pair form, precision {prec}: max error vs oracle {err:.2e}, vs staged products {diff:.2e}")
    assert err < 1e-4
    assert diff < dtol


def test_pair_gemm_staging_forms_agree_bit_for_bit(T, monkeypatch):
    """The FP32 pair GEMM stages its operands either four kappa at a time with
    16-byte loads and stores (parent dimension a multiple of 4, the default)
    or one at a time (TTN_PAIR_V4=0, and any other parent dimension): the same
    values reach LDS and the matrix cores take them in the same order, so two
    sweeps of the C3-shaped tree in the pair form give identical node tensors."""
    import golden_refs as G
    p = G.maker.c3_shaped()
    bonds = T.clamp_bonds(p.parent, p.local_dim, p.bond_dim)
    st = random_isometric_state(p.parent, p.local_dim, bonds, seed=31)
    states = []
    for flag in ("1", "0"):
        monkeypatch.setenv("TTN_PAIR_MIN_N", "1")
        monkeypatch.setenv("TTN_PAIR_V4", flag)
        g = T.TTN.from_problem(p, precision=T.TTN_FP32)
        monkeypatch.delenv("TTN_PAIR_MIN_N")
        monkeypatch.delenv("TTN_PAIR_V4")
        g.set_state(st)
        T.profile_begin()
        g.step(p.dt, 2)
        assert "k_pair_gemm" in {r["name"] for r in T.profile_end()}
        states.append(g.get_state())
        g.close()
    for a, b in zip(*states):
        assert np.array_equal(a, b)


def test_shared_pair_gemm_schedule_at_full_size(T, monkeypatch):
    """The exciton workload at full size (the configuration bench.py times),
    one sweep from a seeded full-rank state: the A nodes' pair GEMMs (864
    tiles each, FP32 and BF16x3 forms) shared evenly by the resident
    work-groups (the FP32 default; TTN_PAIR_SPLIT=2 for BF16x3), tiles cut
    between two of them summed by k_pair_fixup, against one work-group per tile
    (TTN_PAIR_SPLIT=0, the BF16x3 default): populations and a(t) agree to
    1e-6 (FP32) and 1e-5 (BF16x3) (FP32 sums of the cut tiles in two parts)
    and all stay within 1e-4 of the FP64 sweep (whose kernels are pinned to
    the oracle on the smaller trees)."""
    p = exciton_problem()
    bonds = T.clamp_bonds(p.parent, p.local_dim, p.bond_dim)
    st = random_isometric_state(p.parent, p.local_dim, bonds, seed=41)
    runs = {}
    for form, prec, env in (("fp64", T.TTN_FP64, {}), ("shared", T.TTN_FP32, {}),
                            ("tiles", T.TTN_FP32, {"TTN_PAIR_SPLIT": "0"}), ("bf_shared", T.TTN_BF16X3, {"TTN_PAIR_SPLIT": "2"}),
                            ("bf_tiles", T.TTN_BF16X3, {})):
        for k, v in env.items():
            monkeypatch.setenv(k, v)
        g = T.TTN.from_problem(p, precision=prec)
        for k in env:
            monkeypatch.delenv(k)
        g.set_state(st)
        T.profile_begin()
        g.step(p.dt)
        names = {r["name"] for r in T.profile_end()}
        runs[form] = _obs10(g, p)
        if prec != T.TTN_FP64:
            assert ("k_pair_gemm" if prec == T.TTN_FP32 else "k_pair_gemm_bf") in names
            assert ("k_pair_fixup" in names) == form.endswith("shared")
        g.close()
    for form in ("shared", "tiles", "bf_shared", "bf_tiles"):
        err = np.abs(runs[form] - runs["fp64"]).max()
        print(f"pair GEMM, {form}: max difference from the FP64 sweep {err:.2e}")
        assert err < 1e-4
    for a, b, tol in (("shared", "tiles", 1e-6), ("bf_shared", "bf_tiles", 1e-5)):
        diff = np.abs(runs[a] - runs[b]).max()
        print(f"{a} schedule vs one work-group per tile: {diff:.2e}")
        assert diff < tol


def test_fp32_matrix_core_stages_on_the_c3_shaped_tree(T, monkeypatch):
    """FP32 mode, staged products: the dense stages with factors of 24..32
    (k_mode_mfma32) and the environment contractions with bonds of 16..64
    (k_contract_mfma) on the FP32 matrix cores against the same work on the
    vector ALUs (k_mode_tile_f32, k_contract_part_f32; TTN_MODE_MFMA32=0):
    three sweeps from the seeded full-rank state agree to 1e-6 (FP32
    accumulation in a different order), and both stay within 1e-4 of the
    stored oracle run."""
    import golden_refs as G
    p = G.maker.c3_shaped()
    bonds = T.clamp_bonds(p.parent, p.local_dim, p.bond_dim)
    st = random_isometric_state(p.parent, p.local_dim, bonds, seed=31)
    ref = G.observables(G.reference("c3_shaped", p, bonds, st))
    runs = {}
    for form, flag in (("mfma", "1"), ("valu", "0")):
        monkeypatch.setenv("TTN_PAIR_OPS", "0")
        monkeypatch.setenv("TTN_MODE_MFMA32", flag)
        g = T.TTN.from_problem(p, precision=T.TTN_FP32)
        monkeypatch.delenv("TTN_PAIR_OPS")
        monkeypatch.delenv("TTN_MODE_MFMA32")
        g.set_state(st)
        T.profile_begin()
        got = []
        for _ in range(3):
            g.step(p.dt)
            got.append(_obs10(g, p))
        names = {r["name"] for r in T.profile_end()}
        runs[form] = np.array(got)
        assert ("k_mode_mfma32" in names) == (form == "mfma")
        assert ("k_contract_mfma" in names) == (form == "mfma")
        g.close()
    for form in runs:
        err = np.abs(runs[form] - ref).max()
        print(f"FP32 stages on {form}: max error vs oracle {err:.2e}")
        assert err < 1e-4
    diff = np.abs(runs["mfma"] - runs["valu"]).max()
    print(f"matrix-core vs vector-ALU stages: {diff:.2e}")
    assert diff < 1e-6


def test_fp64_matrix_core_stages_on_the_c3_shaped_tree(T, monkeypatch):
    """FP64 mode: the dense stages with factors of 16..64 on the FP64 matrix
    cores (k_mode_mfma64) against the same stages on the vector ALUs
    (k_mode_tile, TTN_MODE_MFMA64=0): three sweeps from the seeded full-rank
    state agree to 1e-12 (FP64 accumulation in a different order), both stay
    within 1e-10 of the stored oracle run, and so do sampled entries of every
    node tensor."""
    import golden_refs as G
    p = G.maker.c3_shaped()
    bonds = T.clamp_bonds(p.parent, p.local_dim, p.bond_dim)
    st = random_isometric_state(p.parent, p.local_dim, bonds, seed=31)
    rec = G.reference("c3_shaped", p, bonds, st)
    ref = G.observables(rec)
    runs = {}
    for form, flag in (("mfma", "1"), ("valu", "0")):
        monkeypatch.setenv("TTN_MODE_MFMA64", flag)
        g = T.TTN.from_problem(p, precision=T.TTN_FP64)
        monkeypatch.delenv("TTN_MODE_MFMA64")
        g.set_state(st)
        T.profile_begin()
        got = []
        for _ in range(3):
            g.step(p.dt)
            got.append(_obs10(g, p))
        names = {r["name"] for r in T.profile_end()}
        runs[form] = np.array(got)
        assert ("k_mode_mfma64" in names) == (form == "mfma")
        terr = G.tensor_sample_error(rec, g.get_state())
        err = np.abs(runs[form] - ref).max()
        print(f"FP64 stages on {form}: max error vs oracle {err:.2e}, node tensors (sampled) {terr:.2e}")
        assert err < 1e-10 and terr < 1e-10
        g.close()
    diff = np.abs(runs["mfma"] - runs["valu"]).max()
    print(f"matrix-core vs vector-ALU stages: {diff:.2e}")
    assert diff < 1e-12


def test_exciton10x120_full_size_properties(T):
    """The full exciton workload (10 states, 120 modes, bonds 8/32/48/64,
    1500 SOP terms: nodes of 7.08M elements, the sizes bench.py times), one
    sweep from the product state. The oracle cannot run this size, so the
    checks are properties that hold at any size: the FP64 sweep keeps the norm
    and the energy (time-independent Hermitian generator), and the BF16x3 mode
    (FP64 QR and Krylov around bf16 matrix-core stages) and the FP32 mode (the
    timed configuration: pair-operator GEMM shared by the resident work-groups,
    FP32 matrix-core stages) keep the norm and stay within the rounding floor
    of product-state starts (3e-3) of the FP64 populations."""
    p = exciton_problem()
    g = T.TTN.from_problem(p, precision=T.TTN_FP64)
    g.set_product_state(p.init_vecs)
    e0 = g.energy()
    g.step(p.dt)
    ref = _obs(g, p)
    assert abs(g.norm2() - 1.0) < 1e-10
    assert abs(g.energy() - e0) < 1e-9 * abs(e0)
    g.close()
    for prec, label in ((T.TTN_FP32, "FP32"), (T.TTN_BF16X3, "BF16x3")):
        g = T.TTN.from_problem(p, precision=prec)
        g.set_product_state(p.init_vecs)
        T.profile_begin()
        g.step(p.dt)
        names = {r["name"] for r in T.profile_end()}
        got = _obs(g, p)
        assert abs(g.norm2() - 1.0) < 1e-9
        g.close()
        err = np.abs(got - ref).max()
        print(f"{label} vs FP64 after one sweep: {err:.2e}")
        assert err < 3e-3
        if prec == T.TTN_FP32:  # the A nodes' 864 GEMM tiles exceed the resident work-groups: cut tiles
            assert {"k_pair_gemm", "k_pair_fixup", "k_mode_mfma32"} <= names
