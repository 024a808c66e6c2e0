"""Pins of time-dependent coefficients (Sec. II B) on the interaction-picture
form of the spin-boson model (Sec. II E 2): the chain transformation of the
bath, the oracle's midpoint step against the product of dense midpoint
exponentials, its convergence at second order to the Schroedinger-picture
dynamics of the star model, and the chain basis against the star basis."""
import numpy as np
import scipy.linalg as sla

from oracle import Oracle, dense_sop, full_state
from oracle.ttn_oracle import leaf_order
from workloads import (chain_transform, ipchain_coefficients, ipchain_sbm_problem, sbm_problem)
from workloads.models import ohmic_discretisation


def _psi0(p):
    order = leaf_order(p.parent, p.local_dim)
    v = np.ones(1, dtype=np.complex128)
    for z in order:
        v = np.kron(v, p.init_vecs[z])
    return v


def _dense_at(p, coef):
    q = p.__class__(**{**p.__dict__, "coeff": np.asarray(coef)})
    return dense_sop(q)


def _midpoint_product(p, dt, n):
    psi = _psi0(p)
    for s in range(n):
        psi = sla.expm(-1j * dt * _dense_at(p, ipchain_coefficients(p, (s + 0.5) * dt))) @ psi
    return psi


def _sz_dense(p, psi):
    order = leaf_order(p.parent, p.local_dim)
    S = p.leaf_names["S"]
    op = np.ones((1, 1))
    for z in order:
        op = np.kron(op, np.diag([1.0, -1.0]) if z == S else np.eye(p.local_dim[z]))
    return float(np.vdot(psi, op @ psi).real)


def test_chain_transform():
    """V orthogonal, V^T diag(w) V tridiagonal with the returned on-site
    energies and hoppings, V[:, 0] = g / |g|; the time-dependent couplings keep
    sum_l |G_l(t)|^2 = |g|^2 and at t = 0 only the first chain mode couples."""
    w, g = ohmic_discretisation(12, 0.5, 5.0)
    V, eps, t, k0 = chain_transform(w, g)
    assert np.abs(V.T @ V - np.eye(12)).max() < 1e-12
    T = V.T @ np.diag(w) @ V
    ref = np.diag(eps) + np.diag(t, 1) + np.diag(t, -1)
    assert np.abs(T - ref).max() < 1e-11 * w.max()
    assert np.abs(V[:, 0] - g / np.linalg.norm(g)).max() < 1e-15
    p = ipchain_sbm_problem(n_modes=12, d=3)
    for tt in (0.0, 0.7, 3.1):
        G = ipchain_coefficients(p, tt)[2::2]
        assert abs(np.sum(np.abs(G) ** 2) - k0 ** 2) < 1e-12 * k0 ** 2
    G0 = ipchain_coefficients(p, 0.0)[2::2]
    assert abs(G0[0] - k0) < 1e-12 * k0 and np.abs(G0[1:]).max() < 1e-12 * k0


def test_midpoint_step_is_the_product_of_midpoint_exponentials():
    """Full bonds: each sweep with the coefficients frozen at the step midpoint
    is the exact exponential of G(t + dt/2), so n steps give the product of the
    n dense midpoint exponentials."""
    p = ipchain_sbm_problem(n_modes=3, d=4, bonds=(64, 64, 64), dt=0.05)
    o = Oracle(p)
    o.set_product_state(p.init_vecs)
    for s in range(5):
        o.step_td(p.dt, lambda t: ipchain_coefficients(p, t))
    ref = _midpoint_product(p, p.dt, 5)
    got = full_state(o.parent, o.local_dim, o.state())
    assert np.abs(got - ref).max() < 1e-11


def test_star_interaction_picture_converges_to_the_schroedinger_picture():
    """Star modes (V = 1): on the truncated Fock spaces the interaction picture
    is exact, psi_I(t) = exp(i H_B t) psi_S(t), with psi_S from the static star
    model.  The oracle's midpoint steps at full bonds converge to it at second
    order: halving dt divides the error by about 4 (a step at the left end of
    the interval would give first order, a wrong sign of the phase no
    convergence).  The midpoint step is symmetric, so the error has only even
    powers of dt and the Richardson combination (4 psi(dt/2) - psi(dt)) / 3 is
    fourth order (measured: 1.1e-3, then 4.7e-5)."""
    tend = 0.8
    ps = sbm_problem(n_modes=3, d=4, bond=64, eps=0.0, delta=1.0, alpha=0.5, wc=5.0)
    exact = sla.expm(-1j * tend * dense_sop(ps)) @ _psi0(ps)
    errs, states = [], []
    for n in (8, 16, 32):
        p = ipchain_sbm_problem(n_modes=3, d=4, bonds=(64, 64, 64), eps=0.0, delta=1.0, alpha=0.5, wc=5.0,
                                dt=tend / n, chain=False)
        assert np.allclose(p.meta["omega"], ps.meta["omega"]) and np.allclose(p.meta["g"], ps.meta["g"])
        order = leaf_order(p.parent, p.local_dim)
        phase = np.ones(1, dtype=np.complex128)
        for z in order:
            k = [k for k in range(3) if p.leaf_names[f"b{k}"] == z]
            ph = np.ones(p.local_dim[z], dtype=np.complex128) if not k else \
                np.exp(1j * p.meta["omega"][k[0]] * np.arange(p.local_dim[z]) * tend)
            phase = np.kron(phase, ph)
        o = Oracle(p)
        o.set_product_state(p.init_vecs)
        for _ in range(n):
            o.step_td(p.dt, lambda t: ipchain_coefficients(p, t))
        got = full_state(o.parent, o.local_dim, o.state())
        errs.append(np.abs(got - phase * exact).max())
        states.append(got)
    ref = phase * exact
    assert 3.5 < errs[0] / errs[1] < 4.5 and 3.5 < errs[1] / errs[2] < 4.5
    rich = [np.abs((4 * b - a) / 3 - ref).max() for a, b in zip(states, states[1:])]
    assert rich[1] < rich[0] / 12 and rich[1] < 1e-4


def test_chain_and_star_bases_agree_up_to_truncation():
    """The chain form is the star form in another mode basis: with the same
    midpoint steps their <sz>(t) differ only by the Fock truncation, which
    shrinks as the ladders grow."""
    diffs = []
    for d in (3, 5):
        r = []
        for chain in (True, False):
            p = ipchain_sbm_problem(n_modes=3, d=d, bonds=(64, 64, 64), eps=0.0, delta=1.0, alpha=0.3, wc=5.0,
                                    dt=0.05, chain=chain)
            r.append(_sz_dense(p, _midpoint_product(p, p.dt, 16)))
        diffs.append(abs(r[0] - r[1]))
    assert diffs[1] < diffs[0] / 5
    assert diffs[1] < 1e-3
