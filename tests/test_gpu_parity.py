"""GPU parity: the HIP path (through the C boundary) against the CPU oracle.

Tolerances: the FP64 path must reproduce the oracle's observables to 1e-10
absolute (the unitary observables are O(1)); the measured rounding jitter of
the oracle itself on these runs is ~1e-13, and both sides stop their local
Krylov exponentials at a 1e-13 relative error estimate.
"""
import numpy as np
import pytest

from oracle import Oracle
from oracle.ttn_oracle import full_state
from workloads import heom_sbm_problem, random_isometric_state, sbm_problem, vibronic_problem

pytestmark = pytest.mark.gpu

TOL = 1e-10


@pytest.fixture(scope="module")
def T():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2503_15460_amd as mod
    return mod


def _pair(T, p, bond=None, state=None, **kw):
    g = T.TTN.from_problem(p, bond_dim=bond, **kw)
    o = Oracle(p, bond_dim=bond)
    assert np.array_equal(g.bonds(), o.bond)
    if state is None:
        g.set_product_state(p.init_vecs)
        o.set_product_state(p.init_vecs)
    else:
        g.set_state(state)
        o.set_state(state)
    return g, o


def _gauge_free_overlap(a_tensors, b_tensors, o):
    return o._contract(a_tensors, b_tensors, {})


def _tensor_error(g_tensors, o_tensors):
    """Largest element-wise difference of the node tensors, relative to each
    node's largest element.  From a full-rank start both sides take the same
    Householder gauge, so this bounds the state error linearly (an overlap
    |<g|o>| - 1 is quadratic in it)."""
    return max(float(np.abs(a - b).max() / np.abs(b).max()) for a, b in zip(g_tensors, o_tensors))


def test_root_heff_brute(T):
    """H_eff at the root (children SPOs from the env kernels) equals the oracle's."""
    p = sbm_problem(n_modes=4, d=6, bond=4, alpha=0.4)
    o0 = Oracle(p)
    st = random_isometric_state(p.parent, p.local_dim, o0.bond, seed=21)
    g, o = _pair(T, p, state=st)
    rng = np.random.default_rng(1)
    shp = o.A[o.root].shape
    x = rng.normal(size=shp) + 1j * rng.normal(size=shp)
    y = g.apply_root_heff(x.reshape(-1)).reshape(shp)
    ref = o.heff(o.root, x)
    assert np.abs(y - ref).max() < 1e-12 * np.abs(ref).max()


def test_observables_match(T):
    p = sbm_problem(n_modes=4, d=6, bond=4, alpha=0.4)
    o0 = Oracle(p)
    st = random_isometric_state(p.parent, p.local_dim, o0.bond, seed=22)
    g, o = _pair(T, p, state=st)
    assert abs(g.norm2() - o.norm2()) < 1e-12
    assert abs(g.energy() - o.energy()) < 1e-12
    for name in ("sz", "sx"):
        assert abs(g.expect(p.observables[name]) - o.expect(p.observables[name])) < 1e-12
    b1 = p.leaf_names["b1"]
    S = p.leaf_names["S"]
    ids = [p.observables["sz"][0], p.op_leaf.index(b1) if b1 in p.op_leaf else None]
    ids = [i for i in ids if i is not None]
    assert abs(g.expect(ids) - o.expect(ids)) < 1e-12
    vecs = {z: np.random.default_rng(z).normal(size=p.local_dim[z]) + 0j for z in p.leaves()}
    assert abs(g.bilinear(vecs) - o.bilinear(vecs)) < 1e-12
    g.step(p.dt, 3)
    for _ in range(3):
        o.step(p.dt)
    assert abs(g.overlap_t0() - o.overlap_t0()) < 1e-11


def test_sbm4_product_state_parity(T):
    """Spin-boson, 4 modes x 8 levels, binary tree, bond 4, 100 steps dt = 0.05."""
    p = sbm_problem(n_modes=4, d=8, bond=4)
    g, o = _pair(T, p)
    sz_g, sz_o = [], []
    for _ in range(100):
        g.step(p.dt)
        o.step(p.dt)
        sz_g.append(g.expect(p.observables["sz"]))
        sz_o.append(o.expect(p.observables["sz"]))
    sz_g, sz_o = np.array(sz_g), np.array(sz_o)
    assert np.abs(sz_g - sz_o).max() < TOL
    assert abs(g.norm2() - 1.0) < 1e-12
    # gauge-free comparison: the dense wavefunctions agree
    psi_g = full_state(p.parent, p.local_dim, g.get_state())
    psi_o = o.dense_state()
    assert np.abs(psi_g - psi_o).max() < TOL
    c = g.counters()
    assert c["steps"] == 100 and c["forward_solves"] == 100 * (2 * p.n_nodes - 1)
    assert c["backward_solves"] == 100 * 2 * (p.n_nodes - 1)


def test_big_path_random_state_parity(T):
    """Nodes above the fused-solver size exercise the multi-kernel Krylov path."""
    p = sbm_problem(n_modes=8, d=6, bond=16, alpha=0.3, dt=0.05)
    o0 = Oracle(p)
    assert max(int(np.prod(o0.shape(z))) for z in range(p.n_nodes)) > 1024
    st = random_isometric_state(p.parent, p.local_dim, o0.bond, seed=5)
    g, o = _pair(T, p, state=st)
    e0 = o.energy()
    for _ in range(4):
        g.step(p.dt)
        o.step(p.dt)
        assert abs(g.expect(p.observables["sz"]) - o.expect(p.observables["sz"])) < TOL
    assert abs(g.energy() - e0) < 1e-9 * abs(e0)
    assert _tensor_error(g.get_state(), o.state()) < 1e-10


def _vib():
    return vibronic_problem(n_modes=8, dmin=4, dmax=6, leaf_bond=4, l_bond=6, m_bond=8, dt=0.5)


def test_vibronic24_full_size_sweep(T):
    """The full-size vibronic workload (2 states x 24 modes, d 8-32, bonds
    8/16/20, FP64), three sweeps from a seeded full-rank state against the
    stored oracle run: populations and the autocorrelation to 1e-10 after
    every sweep, and sampled entries of every node tensor (64 per node,
    relative to the node's largest sample) to 1e-10."""
    import golden_refs as G
    p = vibronic_problem()
    bonds = T.clamp_bonds(p.parent, p.local_dim, p.bond_dim)
    st = random_isometric_state(p.parent, p.local_dim, bonds, seed=24)
    rec = G.reference("vibronic24_full_rank", p, bonds, st)  # the oracle's run, stored
    ref = G.observables(rec)
    g = T.TTN.from_problem(p)
    g.set_state(st)
    for s in range(3):
        g.step(p.dt)
        got = np.array([g.expect(p.observables["P0"]), g.expect(p.observables["P1"]), g.overlap_t0()])
        assert np.abs(got - ref[s]).max() < TOL
    err = G.tensor_sample_error(rec, g.get_state())
    print(f"vibronic24 after 3 sweeps: node tensors (sampled) within {err:.2e} of the oracle")
    assert err < 1e-10
    assert abs(g.norm2() - rec["norm2"]) < TOL


def test_reduced_vibronic_random_state_parity(T):
    """Vibronic 2-state model, 8 modes, 3-layer tree (nodes with 3 and 4
    children, both Krylov paths), full-rank start: strict FP64 parity."""
    p = _vib()
    st = random_isometric_state(p.parent, p.local_dim, Oracle(p).bond, seed=8)
    g, o = _pair(T, p, state=st)
    for s in range(6):
        g.step(p.dt)
        o.step(p.dt)
        for name in ("P0", "P1"):
            assert abs(g.expect(p.observables[name]) - o.expect(p.observables[name])) < TOL
        assert abs(g.overlap_t0() - o.overlap_t0()) < TOL
    assert _tensor_error(g.get_state(), o.state()) < 1e-10


# Product-state starts pass through rank-deficient QRs whose small singular
# values amplify rounding differences; the oracle's own floor for this run,
# measured by injecting 1e-16 relative noise before every QR, is below 1e-8.
JTOL_VIB = 1e-7


def test_reduced_vibronic_product_state_parity(T):
    p = _vib()
    g, o = _pair(T, p)
    for s in range(6):
        g.step(p.dt)
        o.step(p.dt)
        for name in ("P0", "P1"):
            assert abs(g.expect(p.observables[name]) - o.expect(p.observables[name])) < JTOL_VIB
        assert abs(g.overlap_t0() - o.overlap_t0()) < JTOL_VIB


def test_negative_dt_reverses(T):
    p = sbm_problem(n_modes=4, d=6, bond=4, alpha=0.3)
    o0 = Oracle(p)
    st = random_isometric_state(p.parent, p.local_dim, o0.bond, seed=9)
    g, o = _pair(T, p, state=st)
    g.step(p.dt, 10)
    ref = g.get_state()
    g.step(p.dt, 5)
    g.step(-p.dt, 5)
    back = full_state(p.parent, p.local_dim, g.get_state())
    assert np.abs(back - full_state(p.parent, p.local_dim, ref)).max() < 1e-11


def test_degenerate_cases(T):
    """Smallest tree (root with two leaves, complete bonds): 20 sweeps equal the
    exact propagator exp(-i G t) psi0 and the oracle; a sweep with dt = 0
    leaves the state unchanged (up to rounding, the gauge may flip signs) and
    zero sweeps leave the tensors bit for bit."""
    from scipy.linalg import expm
    from oracle import dense_sop
    p = sbm_problem(n_modes=1, d=3, bond=4, dt=0.05)
    g, o = _pair(T, p)
    psi0 = full_state(p.parent, p.local_dim, g.get_state())
    for _ in range(20):
        g.step(p.dt)
        o.step(p.dt)
    exact = expm(-1j * 20 * p.dt * dense_sop(p)) @ psi0
    assert np.abs(full_state(p.parent, p.local_dim, g.get_state()) - exact).max() < 1e-10
    assert abs(g.expect(p.observables["sz"]) - o.expect(p.observables["sz"])) < TOL
    before = g.get_state()
    g.step(0.0)
    after = full_state(p.parent, p.local_dim, g.get_state())
    assert np.abs(after - full_state(p.parent, p.local_dim, before)).max() < 1e-13
    before = g.get_state()
    g.step(p.dt, 0)
    for bad in ((float("nan"), 1), (float("inf"), 1), (p.dt, -1)):
        with pytest.raises(T.TTNError) as e:
            g.step(*bad)
        assert "E_INVALID" in str(e.value)
    for x, y in zip(before, g.get_state()):
        assert np.array_equal(x, y)


def test_checkpoint_resume(T):
    """ttn_get_state / ttn_set_state as checkpoint and resume: a fresh handle
    loaded with the saved tensors continues the run (environments are rebuilt
    from the tensors; only the Krylov dimension hints start afresh, so the
    two runs agree to the Krylov tolerance, not bit for bit)."""
    p = _vib()
    st = random_isometric_state(p.parent, p.local_dim, Oracle(p).bond, seed=17)
    g = T.TTN.from_problem(p)
    g.set_state(st)
    g.step(p.dt, 4)
    saved = g.get_state()
    g.step(p.dt, 4)
    h = T.TTN.from_problem(p)
    h.set_state(saved)
    h.step(p.dt, 4)
    for name in ("P0", "P1"):
        assert abs(g.expect(p.observables[name]) - h.expect(p.observables[name])) < 1e-11
    assert _tensor_error(h.get_state(), g.get_state()) < 1e-11
    g.close()
    h.close()


def test_non_hermitian_rejected_with_lanczos(T):
    p = heom_sbm_problem(K=1, levels=3)
    with pytest.raises(T.TTNError) as e:
        T.TTN.from_problem(p, hermitian=True)
    assert "E_INVALID" in str(e.value)


def test_state_errors(T):
    p = sbm_problem(n_modes=2, d=3, bond=2)
    g = T.TTN(p.parent, p.local_dim, p.bond_dim)
    with pytest.raises(T.TTNError) as e:
        g.step(0.1)
    assert "E_STATE" in str(e.value)
    g.set_sop_problem(p)
    with pytest.raises(T.TTNError):
        g.set_state([np.zeros(1)])


def _heom_obs(src, p):
    S = p.leaf_names["S"]
    out = []
    for key in ("bra_sz", "bra_tr"):
        bra = {z: np.eye(p.local_dim[z])[0].astype(np.complex128) for z in p.leaves()}
        bra[S] = p.meta[key]
        out.append(src.bilinear(bra))
    return np.array(out)


@pytest.mark.parametrize("K,levels,bonds,n_steps,tol", [
    # fused one-work-group Arnoldi on every node; oracle floor J ~ 6e-11
    (4, 6, (6, 8, 12, 16), 10, 1e-9),
    # nodes of up to 6144 elements on the multi-kernel Arnoldi path; J ~ 1e-11
    (8, 4, (4, 8, 16, 24), 3, 1e-10),
])
def test_heom_arnoldi_parity(T, K, levels, bonds, n_steps, tol):
    """HEOM spin-boson (non-Hermitian generator, Arnoldi exponentials) from the
    physical product state: <sigma_z> and Tr rho_S against the oracle."""
    p = heom_sbm_problem(K=K, levels=levels, bonds=bonds, dt=0.05)
    g, o = _pair(T, p, hermitian=False)
    for _ in range(n_steps):
        g.step(p.dt)
        o.step(p.dt)
        assert np.abs(_heom_obs(g, p) - _heom_obs(o, p)).max() < tol
    assert abs(_heom_obs(g, p)[1] - 1.0) < tol


def test_heom_full_size_sweep(T):
    """The benchmarked HEOM workload (16 Debye poles, 32 auxiliary modes x 10
    levels, bonds 10-48, dt 0.0075, Arnoldi): one sweep from the physical
    product state, <sigma_z> and Tr rho_S against the oracle."""
    p = heom_sbm_problem()
    g, o = _pair(T, p, hermitian=False)
    g.step(p.dt)
    o.step(p.dt)
    d = np.abs(_heom_obs(g, p) - _heom_obs(o, p)).max()
    print(f"full-size HEOM sweep: max difference {d:.2e}")
    assert d < TOL


@pytest.mark.parametrize("bond", [4, 16])  # fused solver only / also the multi-kernel path
def test_noconv_restores_state(T, bond):
    """A Krylov limit far too small for the step: TTN_E_NOCONV, and the state
    is the one before the failed step (the step is not half applied)."""
    p = sbm_problem(n_modes=8 if bond == 16 else 4, d=6, bond=bond, alpha=0.3)
    st = random_isometric_state(p.parent, p.local_dim, Oracle(p).bond, seed=3)
    g = T.TTN.from_problem(p, krylov_mmax=6)
    g.set_state(st)
    g.step(1e-5)  # converges within the limit
    before = g.get_state()
    with pytest.raises(T.TTNError) as e:
        g.step(50.0)
    assert "E_NOCONV" in str(e.value)
    after = g.get_state()
    for x, y in zip(before, after):
        assert np.array_equal(x, y)
    g.step(1e-5)  # the handle stays usable
