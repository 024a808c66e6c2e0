"""Pins of the oracle's subspace expansion (Sec. II D), all on the CPU.

The spawned functions must reduce the squared error of the time derivative,
||(1 - P_T) G Psi||^2 with P_T the projector onto the one-site tangent space,
by exactly the sum of the spawned sigma_s^2.  The tangent space here is built
independently of the residual formula: the span of the state's derivatives
with respect to every node tensor, from dense vectors.
"""
import numpy as np
import pytest

from oracle import Oracle, dense_sop, full_state
from oracle.subspace import expand, move_centre_down, residual, spawn
from workloads import random_isometric_state, sbm_problem


def _node_derivatives(o, z):
    """Columns d Psi / d A^z (all other tensors fixed), dense."""
    shp = o.A[z].shape
    saved = o.A[z]
    cols = []
    for j in range(int(np.prod(shp))):
        e = np.zeros(int(np.prod(shp)), dtype=np.complex128)
        e[j] = 1.0
        o.A[z] = e.reshape(shp)
        cols.append(full_state(o.parent, o.local_dim, o.A))
    o.A[z] = saved
    return np.stack(cols, axis=1)


def _tdvp_error2(o, G):
    """||(1 - P_T) G Psi||^2: the part of the exact derivative the one-site TDVP misses."""
    D = np.concatenate([_node_derivatives(o, z) for z in range(o.n)], axis=1)
    U, s, _ = np.linalg.svd(D, full_matrices=False)
    U = U[:, : int(np.sum(s > 1e-10 * s[0]))]
    g = G @ full_state(o.parent, o.local_dim, o.A)
    return float(np.linalg.norm(g - U @ (U.conj().T @ g)) ** 2)


def _setup(bond, seed):
    p = sbm_problem(n_modes=4, d=3, bond=bond, alpha=0.4)
    o = Oracle(p)
    o.set_state(random_isometric_state(p.parent, p.local_dim, o.bond, seed=seed))
    return p, o, dense_sop(p)


def _names(o):
    B = o.kids[o.root][1]
    B1 = o.kids[B][0]
    return B, B1, o.kids[B1][1]


@pytest.mark.parametrize("which", ["interior", "leaf"])
def test_spawned_functions_remove_their_share_of_the_error(which):
    """Centre at z, new functions of the child c: E - E_aug = sum sigma_s^2."""
    p, o, G = _setup(bond=2, seed=3)
    B, B1, leaf = _names(o)
    if which == "interior":  # 4 x 4 children space, bond 2: two new functions
        move_centre_down(o, [B])
        z, c, n_new = B, B1, 2
    else:  # leaf of dimension 3, bond 2: one direction left
        move_centre_down(o, [B, B1])
        z, c, n_new = B1, leaf, 1
    k = o.kids[z].index(c)
    psi = full_state(o.parent, o.local_dim, o.A)
    e0 = _tdvp_error2(o, G)
    s, vecs = spawn(o, z, k, G, dt=1.0, eps_s=1e-8, chi_max=o.bond[c] + 2, centre="z", side="below")
    assert vecs.shape[1] == n_new and s[n_new - 1] > 1e-3 * s[0] > 0.0
    assert np.abs(vecs.conj().T @ o.A[c].reshape(vecs.shape[0], -1)).max() < 1e-12  # orthogonal to the old ones
    expand(o, z, k, vecs, side="below")
    assert np.abs(full_state(o.parent, o.local_dim, o.A) - psi).max() < 1e-14       # state unchanged
    e1 = _tdvp_error2(o, G)
    assert abs((e0 - e1) - np.sum(s[:n_new] ** 2)) < 1e-10 * e0


def test_spawned_hole_functions_remove_their_share_of_the_error():
    """Centre at c, new single hole functions of c: E - E_aug = sum sigma_s^2."""
    p, o, G = _setup(bond=2, seed=4)
    B, B1, _ = _names(o)
    move_centre_down(o, [B, B1])
    z, c = B, B1
    k = o.kids[z].index(c)
    psi = full_state(o.parent, o.local_dim, o.A)
    e0 = _tdvp_error2(o, G)
    s, vecs = spawn(o, z, k, G, dt=1.0, eps_s=0.0, chi_max=o.bond[c] + 1, centre="c", side="outside")
    assert vecs.shape[1] == 1 and s[0] > 0.0
    expand(o, z, k, vecs, side="outside")
    assert np.abs(full_state(o.parent, o.local_dim, o.A) - psi).max() < 1e-14
    e1 = _tdvp_error2(o, G)
    assert abs((e0 - e1) - s[0] ** 2) < 1e-10 * e0


def test_a_random_direction_gains_less_than_the_dominant_one():
    """Any other orthonormal new function removes at most sigma_0^2 (Delta's top eigenvalue)."""
    p, o, G = _setup(bond=2, seed=5)
    B, B1, _ = _names(o)
    move_centre_down(o, [B])
    k = o.kids[B].index(B1)
    s, _ = spawn(o, B, k, G, dt=1.0, eps_s=0.0, chi_max=o.bond[B1] + 1, centre="z", side="below")
    e0 = _tdvp_error2(o, G)
    Ac = o.A[B1].reshape(-1, o.A[B1].shape[-1])
    rng = np.random.default_rng(0)
    v = rng.normal(size=Ac.shape[0]) + 1j * rng.normal(size=Ac.shape[0])
    v -= Ac @ (Ac.conj().T @ v)
    v /= np.linalg.norm(v)
    expand(o, B, k, v[:, None], side="below")
    gain = e0 - _tdvp_error2(o, G)
    assert -1e-12 < gain < s[0] ** 2 * (1 + 1e-10)


def test_complete_bond_has_nothing_to_spawn():
    """A bond at its clamp maximum already spans the whole space below c: R = 0."""
    p, o, G = _setup(bond=100, seed=6)
    B, B1, _ = _names(o)
    move_centre_down(o, [B])
    k = o.kids[B].index(B1)
    assert o.bond[B1] == int(np.prod(o.A[B1].shape[:-1]))
    assert np.abs(residual(o, B, k, G, centre="z")).max() < 1e-12


def test_spawning_rule_threshold_and_cap():
    """dt sigma >= eps_S decides, in decreasing order, within chi_max."""
    p, o, G = _setup(bond=2, seed=7)
    B, B1, _ = _names(o)
    move_centre_down(o, [B])
    k = o.kids[B].index(B1)
    s, _ = spawn(o, B, k, G, dt=1.0, eps_s=0.0, chi_max=10, centre="z", side="below")
    dt = 0.05
    eps = dt * 0.5 * (s[0] + s[1])  # between the first two
    _, v = spawn(o, B, k, G, dt=dt, eps_s=eps, chi_max=10, centre="z", side="below")
    assert v.shape[1] == 1
    _, v = spawn(o, B, k, G, dt=dt, eps_s=0.0, chi_max=o.bond[B1], centre="z", side="below")
    assert v.shape[1] == 0


# ------------------------------------------- one-site-cost form vs the definition
def _configs():
    """(path of the centre from the root, z, child c, centre side) on the 4-mode tree."""
    def make(o):
        B, B1, leaf = _names(o)
        return [([B], B, B1, "z"), ([B, B1], B1, leaf, "z"), ([B, B1], B, B1, "c"),
                ([B, B1, leaf], B1, leaf, "c")]
    return make


def _centred(p, state, path):
    from oracle.ttn_oracle import mode_product
    o = Oracle(p, hermitian=False)
    o.set_state(state)
    z = o.root
    for c in path:  # gauge shift with mean fields, as the sweep does on its way down
        k = o.kids[z].index(c)
        Q, R = o.qr_along(o.A[z], k)
        o.A[z] = Q
        o.A[c] = mode_product(o.A[c], R, o.A[c].ndim - 1)
        o.build_mf(z, k)
        z = c
    return o


def _nonhermitian_sbm():
    from workloads.models import boson_ops
    p = sbm_problem(n_modes=4, d=3, bond=2, alpha=0.4)
    p.term_ops.append([p.observables["sx"][0], p.add_op(p.leaf_names["b1"], boson_ops(3)["q2"]),
                       p.add_op(p.leaf_names["b2"], boson_ops(3)["q"])])
    p.coeff = np.append(p.coeff, 0.3 - 0.1j)
    return p


@pytest.mark.parametrize("idx", range(4))
def test_one_site_cost_form_matches_the_definition(idx):
    """The two-site generator from the sweep's environments equals V2^dag G V2;
    R and R^dag applied through A^z and A^c equal the dense residual; the
    Golub-Kahan-Lanczos singular pairs (started in R's row space, nb steps)
    equal the dense SVD, singular vectors up to phase."""
    from oracle.subspace import ResidualOperator, heff2, krylov_singular, two_site_embedding
    p = _nonhermitian_sbm()
    G = dense_sop(p)
    st = random_isometric_state(p.parent, p.local_dim, Oracle(p).bond, seed=11)
    path, z, c, side = _configs()(Oracle(p))[idx]
    o = _centred(p, st, path)
    k = o.kids[z].index(c)
    rng = np.random.default_rng(idx)
    V2, below, outside = two_site_embedding(o, z, k)
    T = rng.normal(size=below + outside) + 1j * rng.normal(size=below + outside)
    ref = (V2.conj().T @ G @ V2 @ T.reshape(-1)).reshape(T.shape)
    assert np.abs(heff2(o, z, k, T) - ref).max() < 1e-12 * np.abs(ref).max()
    Rd = residual(o, z, k, G, side)
    op = ResidualOperator(o, z, k)
    w = rng.normal(size=op.no) + 1j * rng.normal(size=op.no)
    y = rng.normal(size=op.nb) + 1j * rng.normal(size=op.nb)
    scale = max(np.abs(Rd).max(), 1.0)
    assert np.abs(op.R(w) - Rd @ w).max() < 1e-12 * scale * np.abs(w).sum()
    assert np.abs(op.RH(y) - Rd.conj().T @ y).max() < 1e-12 * scale * np.abs(y).sum()
    U, s, Vh = np.linalg.svd(Rd)
    sk, L, Rv = krylov_singular(op, op.nb, rng.normal(size=op.nb) + 1j * rng.normal(size=op.nb))
    r = int(np.sum(s > 1e-10 * max(s[0], 1e-300)))
    assert len(sk) >= r
    assert np.abs(sk[:r] - s[:r]).max() < 1e-12 * max(s[0], 1.0)
    for i in range(r):  # simple singular values here: vectors agree up to a phase
        assert abs(abs(np.vdot(U[:, i], L[:, i])) - 1.0) < 1e-10
        assert abs(abs(np.vdot(Vh[i].conj(), Rv[:, i])) - 1.0) < 1e-10


# ------------------------------------------------------------ the adaptive sweep
def _exact_errors(p, runs, n_steps):
    from scipy.linalg import expm
    G = dense_sop(p)
    psi0 = full_state(p.parent, p.local_dim, runs[0].state())
    for _ in range(n_steps):
        for o in runs:
            o.step(p.dt)
    ex = expm(-1j * n_steps * p.dt * G) @ psi0
    return [float(np.linalg.norm(full_state(p.parent, p.local_dim, o.state()) - ex)) for o in runs]


def test_adaptive_sweep_without_spawning_is_the_fixed_sweep():
    from oracle.subspace import AdaptiveOracle
    p = sbm_problem(n_modes=4, d=3, bond=2, alpha=0.4, dt=0.05)
    a = Oracle(p)
    b = AdaptiveOracle(p, eps_s=np.inf, chi_max=100, seed=1)
    for o in (a, b):
        o.set_product_state(p.init_vecs)
        for _ in range(5):
            o.step(p.dt)
    assert b.spawned == 0
    for x, y in zip(a.state(), b.state()):
        assert np.array_equal(x, y)


def test_adaptive_sweep_converges_to_the_exact_propagator():
    """Spin-boson, 4 modes, bonds starting at 2 (below the complete bonds): with
    a small spawning tolerance the bonds grow and the run approaches
    exp(-i G t) psi0 (complete bonds make the sweep exact); a looser tolerance
    spawns less and lands in between; norm and energy stay conserved, every
    bond stays within chi_max and every non-root tensor an isometry."""
    from oracle.subspace import AdaptiveOracle
    p = sbm_problem(n_modes=4, d=3, bond=2, alpha=0.4, dt=0.05)
    fixed = Oracle(p)
    tight = AdaptiveOracle(p, eps_s=1e-8, chi_max=100, seed=1)
    loose = AdaptiveOracle(p, eps_s=1e-5, chi_max=100, seed=1)
    capped = AdaptiveOracle(p, eps_s=1e-8, chi_max=4, seed=1)
    runs = [fixed, tight, loose, capped]
    for o in runs:
        o.set_product_state(p.init_vecs)
    e0 = [o.energy() for o in runs]
    ef, et, el, ec = _exact_errors(p, runs, 20)
    assert et < 1e-5 and et < 1e-3 * ef
    assert et < el < ef
    assert tight.spawned > loose.spawned > 0
    assert max(capped.bond) <= 4 and ec < ef
    for o, e in zip(runs, e0):
        assert abs(o.norm2() - 1.0) < 1e-12
        assert abs(o.energy() - e) < 1e-12 * abs(e)
        for z in range(o.n):
            if z == o.root:
                continue
            M = o.A[z].reshape(-1, o.A[z].shape[-1])
            assert np.abs(M.conj().T @ M - np.eye(M.shape[1])).max() < 1e-12
