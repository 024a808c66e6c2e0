"""FP32 contraction mode against the FP64 oracle.

In TTN_FP32 mode the operator stages, group sums and environment contractions
run in complex FP32 with FP32 accumulation, everything else (QR, Krylov
orthogonalisation, projected exponential, fused small solver) in FP64.  The
target error on observables is 1e-4; complex FP32 rounding (2^-24 ~ 6e-8 per
operation, summed over channels and contraction lengths of a few hundred)
puts a single contraction at ~1e-6 relative, which is what the brute-force
H_eff test bounds.
"""
import numpy as np
import pytest

from oracle import Oracle
from workloads import heom_sbm_problem, random_isometric_state, sbm_problem, vibronic_problem

pytestmark = pytest.mark.gpu

OBS_TOL = 1e-4


@pytest.fixture(scope="module")
def T():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2503_15460_amd as mod
    return mod


def _pair(T, p, state=None, **kw):
    g = T.TTN.from_problem(p, precision=T.TTN_FP32, **kw)
    o = Oracle(p)
    if state is None:
        g.set_product_state(p.init_vecs)
        o.set_product_state(p.init_vecs)
    else:
        g.set_state(state)
        o.set_state(state)
    return g, o


def test_fp32_root_heff_brute(T):
    """Root H_eff from FP32 environments and FP32 stages, relative error ~1e-6."""
    p = sbm_problem(n_modes=8, d=6, bond=16, alpha=0.3)
    o0 = Oracle(p)
    st = random_isometric_state(p.parent, p.local_dim, o0.bond, seed=31)
    g, o = _pair(T, p, state=st)
    rng = np.random.default_rng(2)
    shp = o.A[o.root].shape
    x = rng.normal(size=shp) + 1j * rng.normal(size=shp)
    y = g.apply_root_heff(x.reshape(-1)).reshape(shp)
    ref = o.heff(o.root, x)
    rel = np.abs(y - ref).max() / np.abs(ref).max()
    assert 1e-9 < rel < 1e-5  # FP32 rounding is visible, and small


def test_fp32_big_path_spin_boson(T):
    p = sbm_problem(n_modes=8, d=6, bond=16, alpha=0.3, dt=0.05)
    o0 = Oracle(p)
    assert max(int(np.prod(o0.shape(z))) for z in range(p.n_nodes)) > 1024
    st = random_isometric_state(p.parent, p.local_dim, o0.bond, seed=5)
    g, o = _pair(T, p, state=st)
    err = 0.0
    for _ in range(6):
        g.step(p.dt)
        o.step(p.dt)
        err = max(err, abs(g.expect(p.observables["sz"]) - o.expect(p.observables["sz"])))
    assert err < OBS_TOL
    assert abs(g.norm2() - 1.0) < 1e-10  # unitary steps stay unitary in FP64 Krylov


def _vib():
    return vibronic_problem(n_modes=8, dmin=4, dmax=6, leaf_bond=4, l_bond=6, m_bond=8, dt=0.5)


def _vib_err(g, o, p, n):
    err = 0.0
    for _ in range(n):
        g.step(p.dt)
        o.step(p.dt)
        for name in ("P0", "P1"):
            err = max(err, abs(g.expect(p.observables[name]) - o.expect(p.observables[name])))
        err = max(err, abs(g.overlap_t0() - o.overlap_t0()))
    return err


def test_fp32_vibronic_random_state(T):
    p = _vib()
    st = random_isometric_state(p.parent, p.local_dim, Oracle(p).bond, seed=8)
    g, o = _pair(T, p, state=st)
    assert _vib_err(g, o, p, 6) < OBS_TOL


# From a product state the first QRs are rank deficient and FP32-size noise
# picks the completion of the empty columns: the oracle itself, with 1e-7
# relative noise injected before every QR, moves its populations by ~3e-3 over
# these 6 steps (tests/test_oracle_pins.py measures it).  No FP32 contraction
# path can do better than that floor on this start.
FP32_PRODUCT_FLOOR = 3e-3


def test_fp32_vibronic_product_state(T):
    p = _vib()
    g, o = _pair(T, p)
    assert _vib_err(g, o, p, 6) < FP32_PRODUCT_FLOOR


def test_fp32_heom_arnoldi(T):
    p = heom_sbm_problem(K=8, levels=4, bonds=(4, 8, 16, 24), dt=0.05)
    g, o = _pair(T, p, hermitian=False)
    S = p.leaf_names["S"]

    def obs(src):
        out = []
        for key in ("bra_sz", "bra_tr"):
            bra = {z: np.eye(p.local_dim[z])[0].astype(np.complex128) for z in p.leaves()}
            bra[S] = p.meta[key]
            out.append(src.bilinear(bra))
        return np.array(out)
    for _ in range(3):
        g.step(p.dt)
        o.step(p.dt)
        assert np.abs(obs(g) - obs(o)).max() < OBS_TOL


# ----------------------------------------------------------- BF16x3 on MFMA
def test_bf16x3_spin_boson_bond32(T):
    """Bond-32 spin-boson (nodes of 32^3 elements): the dense stages run on the
    matrix cores (the BF16x3 kernel, or the FP32 kernel in the FP32 mode;
    checked through the launch profiler) and the observables stay within 1e-4
    of the FP64 oracle."""
    p = sbm_problem(n_modes=8, d=8, bond=32, alpha=0.3, dt=0.05)
    o = Oracle(p)
    st = random_isometric_state(p.parent, p.local_dim, o.bond, seed=6)
    o.set_state(st)
    ref = []
    for _ in range(3):
        o.step(p.dt)
        ref.append(o.expect(p.observables["sz"]))
    for prec in (T.TTN_FP32, T.TTN_BF16X3):
        g = T.TTN.from_problem(p, precision=prec)
        g.set_state(st)
        T.profile_begin()
        g.step(p.dt)
        names = {r["name"] for r in T.profile_end()}
        assert ("k_mode_mfma" in names) == (prec == T.TTN_BF16X3)
        assert ("k_mode_mfma32" in names) == (prec == T.TTN_FP32)
        got = [g.expect(p.observables["sz"])]
        for _ in range(2):
            g.step(p.dt)
            got.append(g.expect(p.observables["sz"]))
        err = np.abs(np.array(got) - np.array(ref)).max()
        print(f"precision {prec}: max |d<sz>| = {err:.2e}")
        assert err < OBS_TOL
        assert abs(g.norm2() - 1.0) < 1e-9
        g.close()
