"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: exact
propagation of the dense generator, closed-form dynamics, conservation laws,
time reversibility, brute-force projections of the dense operator, and the
LAPACK Householder convention.
"""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import Oracle, dense_sop, householder_qr_lapack
from oracle.ttn_oracle import contract_except, full_state, mode_product, clamp_bonds
from workloads import heom_sbm_problem, random_isometric_state, sbm_problem, vibronic_problem
from workloads.models import SIGMA, boson_ops


def run_sz(o, p, n):
    out = []
    for _ in range(n):
        o.step(p.dt)
        out.append(o.expect(p.observables["sz"]))
    return np.array(out)


# ------------------------------------------------------------------ QR
@pytest.mark.parametrize("shape", [(7, 4), (16, 16), (40, 8)])
def test_numpy_qr_is_lapack_householder(shape):
    """numpy.linalg.qr follows the zgeqr2/zung2r convention the library implements."""
    rng = np.random.default_rng(1)
    M = rng.normal(size=shape) + 1j * rng.normal(size=shape)
    for variant in range(3):
        X = M.copy()
        if variant == 1:  # exactly rank deficient columns
            X[:, 1] = 0
            X[2:, 2] = 0
        if variant == 2:  # a real column with zeros below the diagonal
            X[:, 0] = 0
            X[0, 0] = 2.0
        Q1, R1 = np.linalg.qr(X)
        Q2, R2 = householder_qr_lapack(X)
        assert np.abs(Q1 - Q2).max() < 1e-13
        assert np.abs(R1 - R2).max() < 1e-13
        assert np.abs(Q2.conj().T @ Q2 - np.eye(Q2.shape[1])).max() < 1e-13
        assert np.abs(Q2 @ R2 - X).max() < 1e-13


def test_householder_exact_zero_column_gives_unit_completion():
    """x = 0 and real alpha give tau = 0: the completion column is a unit vector."""
    X = np.zeros((5, 3), dtype=np.complex128)
    X[0, 0] = 1.0
    Q, R = householder_qr_lapack(X)
    assert np.array_equal(Q, np.eye(5, 3))
    assert R[0, 0] == 1.0 and np.count_nonzero(R) == 1


# -------------------------------------------------------------- clamp
def test_bond_clamp():
    p = sbm_problem(n_modes=4, d=8, bond=4)
    b = clamp_bonds(p.parent, p.local_dim, p.bond_dim)
    # R(S, B); B(B1, B2); Bi(b, b): spin bond 2, B bond limited by outside (2)
    assert b.tolist() == [1, 2, 2, 4, 4, 4, 4, 4, 4]
    p2 = sbm_problem(n_modes=2, d=3, bond=100)
    b2 = clamp_bonds(p2.parent, p2.local_dim, p2.bond_dim)
    assert b2.tolist() == [1, 2, 2, 3, 3]


# ----------------------------------------------------- P1: full bonds
@pytest.mark.parametrize("n_modes,d", [(2, 4), (3, 3)])
def test_full_bond_tdvp_is_exact(n_modes, d):
    """With every bond at its clamp maximum the sweep reproduces exp(-iGt)."""
    p = sbm_problem(n_modes=n_modes, d=d, bond=10_000, alpha=0.5, dt=0.05)
    o = Oracle(p)
    o.set_product_state(p.init_vecs)
    G = dense_sop(p)
    psi0 = o.dense_state()
    nst = 12
    for _ in range(nst):
        o.step(p.dt)
    exact = sla.expm(-1j * G * p.dt * nst) @ psi0
    assert np.abs(o.dense_state() - exact).max() < 1e-11


def test_full_bond_random_state_is_exact():
    p = sbm_problem(n_modes=3, d=3, bond=10_000, alpha=0.8, dt=0.1)
    o = Oracle(p)
    o.set_state(random_isometric_state(p.parent, p.local_dim, o.bond, seed=3))
    G = dense_sop(p)
    psi0 = o.dense_state()
    for _ in range(5):
        o.step(p.dt)
    exact = sla.expm(-1j * G * p.dt * 5) @ psi0
    assert np.abs(o.dense_state() - exact).max() < 1e-11


# --------------------------------------------- P2: uncoupled closed form
def test_uncoupled_modes_closed_form():
    eps, delta = 0.5, 1.0
    p = sbm_problem(n_modes=4, d=6, bond=3, eps=eps, delta=delta, coupling_scale=0.0,
                    mode_init=[1.0, 1.0], dt=0.05)
    # <a_k> observables
    a_ops = []
    for k in range(4):
        leaf = p.leaf_names[f"b{k}"]
        a_ops.append(p.add_op(leaf, boson_ops(6)["a"]))
    o = Oracle(p)
    o.set_product_state(p.init_vecs)
    w = p.meta["omega"]
    Om = np.hypot(eps, delta)
    for s in range(1, 41):
        o.step(p.dt)
        t = s * p.dt
        sz = o.expect(p.observables["sz"]).real
        assert abs(sz - (1 - 2 * (delta / Om) ** 2 * np.sin(Om * t / 2) ** 2)) < 1e-11
        for k in range(4):
            ak = o.expect([a_ops[k]])
            assert abs(ak - 0.5 * np.exp(-1j * w[k] * t)) < 1e-11


# --------------------------------------------- P3: independent boson
def test_independent_boson_coherence():
    """Delta = 0: rho_updn(t) = rho_updn(0) e^{-i eps t} exp(-4 sum (g/w)^2 (1 - cos w t))."""
    eps = 0.5
    p = sbm_problem(n_modes=2, d=10, bond=10_000, eps=eps, delta=0.0, alpha=0.02,
                    spin_init=np.array([1, 1]) / np.sqrt(2), dt=0.05)
    S = p.leaf_names["S"]
    lower = p.add_op(S, np.array([[0, 0], [1, 0]], dtype=np.complex128))  # |dn><up|
    o = Oracle(p)
    o.set_product_state(p.init_vecs)
    g, w = p.meta["g"], p.meta["omega"]
    assert 4 * np.max((g / w) ** 2) < 0.05
    G = dense_sop(p)
    psi0 = o.dense_state()
    for s in range(1, 21):
        o.step(p.dt)
        t = s * p.dt
        rho = o.expect([lower])
        closed = 0.5 * np.exp(-1j * eps * t) * np.exp(-4 * np.sum((g / w) ** 2 * (1 - np.cos(w * t))))
        assert abs(rho - closed) < 1e-6  # Fock truncation error only
    exact = sla.expm(-1j * G * p.dt * 20) @ psi0
    assert np.abs(o.dense_state() - exact).max() < 1e-11


# ------------------------------------------ P4-P6: conservation laws
@pytest.fixture(scope="module")
def sbm4_run():
    p = sbm_problem(n_modes=4, d=8, bond=4)
    o = Oracle(p)
    o.set_product_state(p.init_vecs)
    e0 = o.energy()
    for _ in range(100):
        o.step(p.dt)
    return p, o, e0


def test_norm_conserved(sbm4_run):
    p, o, _ = sbm4_run
    assert abs(o.norm2() - 1.0) < 1e-12


def test_energy_conserved(sbm4_run):
    p, o, e0 = sbm4_run
    assert abs(o.energy() - e0) / abs(e0) < 1e-11


def test_sbm_underdamped(sbm4_run):
    """alpha = 0.1 is in the underdamped regime (Sec. V A): <sz> changes sign."""
    p = sbm_problem(n_modes=4, d=8, bond=4)
    o = Oracle(p)
    o.set_product_state(p.init_vecs)
    sz = run_sz(o, p, 100).real
    assert sz.min() < -0.3 and sz[-1] > sz.min() + 0.2


def test_time_reversibility():
    p = sbm_problem(n_modes=4, d=6, bond=4, alpha=0.3)
    o = Oracle(p)
    o.set_state(random_isometric_state(p.parent, p.local_dim, o.bond, seed=11))
    for _ in range(10):
        o.step(p.dt)
    ref = o.state()
    for _ in range(5):
        o.step(p.dt)
    for _ in range(5):
        o.step(-p.dt)
    ov = o.overlap(ref)
    assert abs(abs(ov) - 1.0) < 1e-11


# ------------------------------------ energy and a(t) against dense forms
def _dense_run(seed, n_steps):
    """Oracle on a small tree from a seeded full-rank state, with its dense
    state before and after ``n_steps`` steps and the dense generator."""
    p = sbm_problem(n_modes=3, d=4, bond=3, alpha=0.4, dt=0.07)
    o = Oracle(p)
    o.set_state(random_isometric_state(p.parent, p.local_dim, o.bond, seed=seed))
    psi0 = o.dense_state()
    for _ in range(n_steps):
        o.step(p.dt)
    return p, o, psi0, o.dense_state(), dense_sop(p)


def test_energy_is_the_dense_expectation_value():
    """<Psi|G|Psi> from the tree contraction equals psi^H G psi of the dense state
    (every SOP term with its coefficient; Sec. II B 1)."""
    p, o, _, psi, G = _dense_run(21, 4)
    ref = np.vdot(psi, G @ psi)
    e = o.energy()
    assert abs(e - ref) < 1e-12 * max(1.0, abs(ref))
    # a non-Hermitian generator (complex coefficients): the raw value, complex
    q = sbm_problem(n_modes=3, d=4, bond=3, alpha=0.4)
    q.coeff = [c * (1.0 + 0.3j * ((i % 3) - 1)) for i, c in enumerate(q.coeff)]
    oq = Oracle(q, hermitian=False)
    oq.set_state(random_isometric_state(q.parent, q.local_dim, oq.bond, seed=22))
    psi_q = oq.dense_state()
    ref_q = np.vdot(psi_q, dense_sop(q) @ psi_q)
    assert abs(ref_q.imag) > 1e-3
    assert abs(oq.energy() - ref_q) < 1e-12 * max(1.0, abs(ref_q))


def test_overlap_t0_is_the_dense_autocorrelation():
    """a(t) = <Psi(0)|Psi(t)> (Sec. IV A) as a complex number: bra conjugated,
    the phase of the propagated state kept."""
    p, o, psi0, psi, G = _dense_run(23, 6)
    ref = np.vdot(psi0, psi)
    a = o.overlap_t0()
    assert abs(ref) < 0.999 and abs(ref.imag) > 1e-3  # a phase that a conjugation error would flip
    assert abs(a - ref) < 1e-12
    # and against exact propagation: at full bonds the sweep is exact
    q = sbm_problem(n_modes=2, d=4, bond=10_000, alpha=0.5, dt=0.05)
    oq = Oracle(q)
    oq.set_state(random_isometric_state(q.parent, q.local_dim, oq.bond, seed=24))
    phi0 = oq.dense_state()
    for _ in range(8):
        oq.step(q.dt)
    exact = np.vdot(phi0, sla.expm(-1j * dense_sop(q) * q.dt * 8) @ phi0)
    assert abs(oq.overlap_t0() - exact) < 1e-11


def test_krylov_substepping_matches_dense_expm():
    """A Krylov space too small for the step forces the halving branch; the
    sub-stepped result is still exp(-i tau G) v (Hermitian and not)."""
    from oracle import expm_krylov
    rng = np.random.default_rng(5)
    n = 200
    A = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))
    A /= np.linalg.norm(A, 2)
    v = rng.normal(size=n) + 1j * rng.normal(size=n)
    for herm, G, tau in ((True, A + A.conj().T, 2.0), (False, A, 2.0)):
        cnt = [0]
        y = expm_krylov(lambda x: G @ x, v, tau, hermitian=herm, tol=1e-13, mmax=8, dense_max=0, counter=cnt)
        # one solve of dimension <= 8 cannot reach 1e-13 at this |tau G|: it sub-stepped
        assert cnt[0] > 8 * 4
        assert np.abs(y - sla.expm(-1j * tau * G) @ v).max() < 1e-11 * np.linalg.norm(v)


# ------------------------------------------- P7: brute-force projections
def _embedding(o, z):
    """Dense V with psi = V vec(A^z) for the current tensors (A^z varied)."""
    shp = o.A[z].shape
    n = int(np.prod(shp))
    cols = []
    saved = o.A[z]
    for j in range(n):
        e = np.zeros(n, dtype=np.complex128)
        e[j] = 1.0
        o.A[z] = e.reshape(shp)
        cols.append(full_state(o.parent, o.local_dim, o.A))
    o.A[z] = saved
    return np.stack(cols, axis=1)


def _move_centre_down(o, path):
    """Gauge-shift the centre from the root along ``path`` (list of nodes), building MFs."""
    z = o.root
    for c in path:
        k = o.kids[z].index(c)
        Q, R = o.qr_along(o.A[z], k)
        o.A[z] = Q
        o.A[c] = mode_product(o.A[c], R, o.A[c].ndim - 1)
        o.build_mf(z, k)
        z = c


def test_heff_keff_brute_force():
    p = sbm_problem(n_modes=4, d=3, bond=3, alpha=0.4)
    p.term_ops.append([p.observables["sx"][0], p.add_op(p.leaf_names["b1"], boson_ops(3)["q2"]),
                       p.add_op(p.leaf_names["b2"], boson_ops(3)["q"])])
    p.coeff = np.append(p.coeff, 0.3 - 0.1j)
    o = Oracle(p, hermitian=False)
    o.set_state(random_isometric_state(p.parent, p.local_dim, o.bond, seed=5))
    G = dense_sop(p)
    rng = np.random.default_rng(0)
    # root
    V = _embedding(o, o.root)
    X = rng.normal(size=o.A[o.root].shape) + 1j * rng.normal(size=o.A[o.root].shape)
    ref = (V.conj().T @ G @ V @ X.reshape(-1)).reshape(X.shape)
    assert np.abs(o.heff(o.root, X) - ref).max() < 1e-12
    # an interior node and a leaf deeper in the tree
    B = o.kids[o.root][1]
    B1 = o.kids[B][0]
    leaf = o.kids[B1][1]
    _move_centre_down(o, [B, B1, leaf])
    for z in (leaf,):
        V = _embedding(o, z)
        X = rng.normal(size=o.A[z].shape) + 1j * rng.normal(size=o.A[z].shape)
        ref = (V.conj().T @ G @ V @ X.reshape(-1)).reshape(X.shape)
        assert np.abs(o.heff(z, X) - ref).max() < 1e-12
    # bond above the leaf: centre matrix C between leaf (SPF) and B1 (SHF)
    pax = o.A[leaf].ndim - 1
    Q, R = o.qr_along(o.A[leaf], pax)
    o.A[leaf] = Q
    o.build_spo(leaf)
    k = o.kids[B1].index(leaf)
    base = o.A[B1].copy()
    n = R.shape[0]
    cols = []
    for j in range(n * n):
        e = np.zeros(n * n, dtype=np.complex128)
        e[j] = 1.0
        o.A[B1] = mode_product(base, e.reshape(n, n), k)
        cols.append(full_state(o.parent, o.local_dim, o.A))
    o.A[B1] = base
    Ve = np.stack(cols, axis=1)
    C = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))
    ref = (Ve.conj().T @ G @ Ve @ C.reshape(-1)).reshape(n, n)
    assert np.abs(o.keff(leaf, C) - ref).max() < 1e-12
    # interior node B1 as centre: absorb C back and move down from B to B1 state
    o2 = Oracle(p, hermitian=False)
    o2.set_state(random_isometric_state(p.parent, p.local_dim, o2.bond, seed=6))
    _move_centre_down(o2, [B, B1])
    V = _embedding(o2, B1)
    X = rng.normal(size=o2.A[B1].shape) + 1j * rng.normal(size=o2.A[B1].shape)
    ref = (V.conj().T @ G @ V @ X.reshape(-1)).reshape(X.shape)
    assert np.abs(o2.heff(B1, X) - ref).max() < 1e-12


# ------------------------------------------------ Krylov vs dense
def test_lanczos_matches_dense_expm():
    p = sbm_problem(n_modes=4, d=8, bond=4)
    a = Oracle(p, dense_max=0)
    b = Oracle(p, dense_max=10_000)
    for o in (a, b):
        o.set_product_state(p.init_vecs)
        for _ in range(10):
            o.step(p.dt)
    assert abs(a.expect(p.observables["sz"]) - b.expect(p.observables["sz"])) < 1e-12
    assert abs(abs(a.overlap(b.state())) - 1) < 1e-12


def test_arnoldi_matches_dense_expm():
    from oracle import expm_krylov
    rng = np.random.default_rng(3)
    n = 300
    G = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))
    G /= np.linalg.norm(G, 2)
    v = rng.normal(size=n) + 1j * rng.normal(size=n)
    y = expm_krylov(lambda x: G @ x, v, 0.7, hermitian=False, tol=1e-13)
    assert np.abs(y - sla.expm(-0.7j * G) @ v).max() < 1e-11
    H = G + G.conj().T
    y = expm_krylov(lambda x: H @ x, v, 1.3, hermitian=True, tol=1e-13)
    assert np.abs(y - sla.expm(-1.3j * H) @ v).max() < 1e-11


# ---------------------------------------------------- QR zero-snap
def test_snap_qr_equals_lapack_without_tiny_columns():
    rng = np.random.default_rng(4)
    M = rng.normal(size=(30, 6)) + 1j * rng.normal(size=(30, 6))
    M[:, 2] = 0.0
    Q1, R1 = np.linalg.qr(M)
    Q2, R2 = householder_qr_lapack(M, snap=1e-12)
    assert np.abs(Q1 - Q2).max() < 1e-13 and np.abs(R1 - R2).max() < 1e-13


def test_snap_qr_ignores_noise_in_empty_columns():
    """Noise far below the snap level reproduces the exactly-zero completion."""
    rng = np.random.default_rng(5)
    M = np.zeros((12, 4), dtype=np.complex128)
    M[:, 0] = rng.normal(size=12)
    M[3, 2] = 0.7
    noisy = M + 1e-17 * (rng.normal(size=M.shape) + 1j * rng.normal(size=M.shape))
    Qa, Ra = householder_qr_lapack(M, snap=1e-12)
    Qb, Rb = householder_qr_lapack(noisy, snap=1e-12)
    assert np.abs(Qa - Qb).max() < 1e-12 and np.abs(Ra - Rb).max() < 1e-12
    Qc, _ = householder_qr_lapack(noisy, snap=0.0)
    assert np.abs(Qa - Qc).max() > 1e-3  # without the snap the noise picks the completion


# ---------------------------------------------------- jitter floor
def _noisy_traj(p, noise, n, obs, seed=0):
    rng = np.random.default_rng(seed)
    o = Oracle(p)
    base = o.qr_along

    def qr_along(A, axis):
        if noise:
            A = A + noise * np.abs(A).max() * (rng.normal(size=A.shape) + 1j * rng.normal(size=A.shape))
        return base(A, axis)
    o.qr_along = qr_along
    o.set_product_state(p.init_vecs)
    out = []
    for _ in range(n):
        o.step(p.dt)
        out.append([o.expect(p.observables[obs]), o.overlap_t0()])
    return np.array(out)


def test_jitter_floor_spin_boson():
    """Rounding-size noise (1e-16 relative, injected before every QR) moves the
    4-mode spin-boson product-state run by far less than the 1e-10 parity bar."""
    p = sbm_problem(n_modes=4, d=8, bond=4)
    a = _noisy_traj(p, 0.0, 40, "sz")
    b = _noisy_traj(p, 1e-16, 40, "sz")
    assert np.abs(a - b).max() < 1e-12


def test_fp32_noise_floor_vibronic_product_state():
    """FP32-size noise (1e-7 relative) before every QR moves the product-state
    vibronic run by ~3e-3: the floor of any FP32-contraction run from this start."""
    p = vibronic_problem(n_modes=8, dmin=4, dmax=6, leaf_bond=4, l_bond=6, m_bond=8, dt=0.5)
    a = _noisy_traj(p, 0.0, 6, "P1")
    b = _noisy_traj(p, 1e-7, 6, "P1")
    J32 = np.abs(a - b).max()
    assert 1e-3 < J32 < 1e-2


def test_jitter_floor_vibronic_product_state():
    """Product-state vibronic runs are sensitive to rounding through the small
    singular values of the first steps; the measured floor J bounds parity."""
    p = vibronic_problem(n_modes=8, dmin=4, dmax=6, leaf_bond=4, l_bond=6, m_bond=8, dt=0.5)
    a = _noisy_traj(p, 0.0, 6, "P1")
    b = _noisy_traj(p, 1e-16, 6, "P1")
    J = np.abs(a - b).max()
    assert J < 1e-8


# ---------------------------------------- P8: HEOM (non-Hermitian, Arnoldi)
def _heom_bra(p, sys_vec):
    S = p.leaf_names["S"]
    bra = {z: np.eye(p.local_dim[z])[0].astype(np.complex128) for z in p.leaves()}
    bra[S] = np.asarray(sys_vec, dtype=np.complex128)
    return bra


def test_heom_pure_dephasing_closed_form():
    """Delta = 0, one Debye pole, full bonds: the coherence follows
    rho_updn(0) e^{-i eps t} exp(-Gamma(t)), Gamma(t) = 4 Re sum_k alpha_k
    [t/nu_k - (1 - e^{-nu_k t})/nu_k^2] (second-order cumulant, exact for a
    Gaussian bath), and the trace stays 1 (Sec. II E 3)."""
    rho0 = 0.5 * np.ones((2, 2), dtype=np.complex128)
    p = heom_sbm_problem(K=1, levels=10, delta=0.0, rho0=rho0, bonds=(10_000,), dt=0.05)
    o = Oracle(p)
    assert not o.hermitian
    o.set_product_state(p.init_vecs)
    al, nu, eps = p.meta["alphas"], p.meta["nus"], p.meta["eps"]
    # Tr(O rho) = vec(O^T) . vec(rho): O = |dn><up| picks rho_updn
    coh = _heom_bra(p, [0, 1, 0, 0])
    tr = _heom_bra(p, p.meta["bra_tr"])
    for s in range(1, 21):
        o.step(p.dt)
        t = s * p.dt
        gam_t = 4.0 * np.real(np.sum(al * (t / nu - (1.0 - np.exp(-nu * t)) / nu ** 2)))
        ref = 0.5 * np.exp(-1j * eps * t) * np.exp(-gam_t)
        assert abs(o.bilinear(coh) - ref) < 1e-12
        assert abs(o.bilinear(tr) - 1.0) < 1e-13


def test_heom_two_poles_truncation_converges():
    """Two poles at 4 levels per auxiliary mode: the same closed form holds up
    to the hierarchy truncation (a wrong sign or scale in either pole's
    couplings moves the coherence by far more)."""
    rho0 = 0.5 * np.ones((2, 2), dtype=np.complex128)
    p = heom_sbm_problem(K=2, levels=4, delta=0.0, rho0=rho0, bonds=(10_000,), dt=0.1)
    G = dense_sop(p)
    o = Oracle(p)
    o.set_product_state(p.init_vecs)
    psi0 = o.dense_state()
    al, nu, eps = p.meta["alphas"], p.meta["nus"], p.meta["eps"]
    coh = _heom_bra(p, [0, 1, 0, 0])
    n = 8
    for s in range(1, n + 1):
        o.step(p.dt)
        t = s * p.dt
        gam_t = 4.0 * np.real(np.sum(al * (t / nu - (1.0 - np.exp(-nu * t)) / nu ** 2)))
        ref = 0.5 * np.exp(-1j * eps * t) * np.exp(-gam_t)
        assert abs(o.bilinear(coh) - ref) < 5e-5
    # and the full-bond sweep equals the exact propagation of the generator
    exact = sla.expm(-1j * G * p.dt * n) @ psi0
    assert np.abs(o.dense_state() - exact).max() < 1e-11


def test_heom_full_bond_arnoldi_is_exact():
    """Delta = 1 (no closed form): full-bond TDVP with Arnoldi equals expm."""
    p = heom_sbm_problem(K=1, levels=5, bonds=(10_000,), dt=0.05)
    G = dense_sop(p)
    assert np.abs(G - G.conj().T).max() > 0.1  # genuinely non-Hermitian
    o = Oracle(p)
    o.set_product_state(p.init_vecs)
    psi0 = o.dense_state()
    for _ in range(20):
        o.step(p.dt)
    exact = sla.expm(-1j * G * p.dt * 20) @ psi0
    assert np.abs(o.dense_state() - exact).max() < 1e-11
    tr = _heom_bra(p, p.meta["bra_tr"])
    assert abs(o.bilinear(tr) - 1.0) < 1e-12


def test_recorded_jitter_floors_bound_the_parity_tolerances():
    """The measured jitter floors J (tests/golden/jitter.json, written by
    tests/golden/measure_jitter.py from the oracle alone: BLAS thread count,
    1e-15 coefficient perturbations and 1e-16 noise before every QR) sit at
    least ten times below the FP64 parity tolerances the GPU tests use."""
    import json
    import os
    import test_gpu_parity as gp
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "jitter.json")
    rec = json.load(open(path))
    for name, r in rec.items():
        print(f"J({name}) = {r['J']:.2e}")
    assert max(1e-10, 10 * rec["sbm4_product_state_40_steps"]["J"]) <= gp.TOL
    assert max(1e-10, 10 * rec["reduced_vibronic_full_rank_6_steps"]["J"]) <= gp.TOL
    assert max(1e-10, 10 * rec["vibronic24_full_rank_3_steps"]["J"]) <= gp.TOL
    assert 10 * rec["reduced_vibronic_product_state_6_steps"]["J"] <= gp.JTOL_VIB
    import test_gpu_pseudomode as gpm
    import test_gpu_timedep as gtd
    assert max(1e-10, 10 * rec["ipchain_full_rank_20_steps"]["J"]) <= gtd.TOL_FULL_RANK
    assert 10 * rec["ipchain_product_state_20_steps"]["J"] <= gtd.TOL_PRODUCT
    assert max(1e-10, 10 * rec["pseudomode_product_state_6_steps"]["J"]) <= gpm.TOL_FP64
