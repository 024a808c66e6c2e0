"""Pins of the oracle's one-site ground-state sweep (DMRG on trees) against
what the mathematics fixes: the closed-form ground state of uncoupled modes,
exact diagonalisation of the dense generator when the bonds can hold the
exact state, and the variational bound and monotone energies when they
cannot."""
import numpy as np

from oracle import dense_sop, full_state
from oracle.ground import GroundOracle
from workloads import random_isometric_state, sbm_problem, vibronic_problem
from workloads.models import boson_ops


def test_uncoupled_ground_closed_form():
    """No spin-bath coupling: G = eps/2 sz + delta/2 sx + sum w_k n_k, whose
    ground state is the spin's lower eigenvector times the bath vacuum, at
    energy -sqrt(eps^2 + delta^2) / 2 (the truncated ladders keep n_k's lowest
    eigenvalue 0)."""
    eps, delta = 0.5, 1.0
    p = sbm_problem(n_modes=4, d=5, bond=2, eps=eps, delta=delta, coupling_scale=0.0)
    n_ops = [p.add_op(p.leaf_names[f"b{k}"], boson_ops(5)["n"]) for k in range(4)]
    o = GroundOracle(p)
    o.set_state(random_isometric_state(p.parent, p.local_dim, o.bond, seed=4))
    for _ in range(3):
        e = o.sweep()
    Om = np.hypot(eps, delta)
    assert abs(e + Om / 2) < 1e-12
    assert abs(o.expect(p.observables["sz"]).real + eps / Om) < 1e-12
    for k in range(4):
        assert abs(o.expect([n_ops[k]])) < 1e-12


def test_full_bond_ground_state_is_exact():
    """Bonds as large as the tree allows (the clamp): the sweep reaches the
    lowest eigenvalue of the dense generator and its eigenvector (up to a
    phase; the ground state of this spin-boson model is nondegenerate)."""
    p = sbm_problem(n_modes=3, d=3, bond=16, alpha=0.3)
    G = dense_sop(p)
    w, V = np.linalg.eigh(G)
    assert w[1] - w[0] > 1e-3
    o = GroundOracle(p)
    o.set_state(random_isometric_state(p.parent, p.local_dim, o.bond, seed=5))
    for _ in range(4):
        e = o.sweep()
    assert abs(e - w[0]) < 1e-10
    psi = full_state(o.parent, o.local_dim, o.state())
    assert abs(abs(np.vdot(V[:, 0], psi)) - 1.0) < 1e-10


def test_truncated_bonds_are_variational_and_monotone():
    """Bonds too small for the exact state: every sweep's energy lies above the
    exact ground energy and no sweep raises it (each node update minimises
    the energy over that node's tensor with the rest fixed)."""
    p = vibronic_problem(n_modes=8, dmin=2, dmax=2, leaf_bond=2, l_bond=3, m_bond=3, seed=7)
    e0 = np.linalg.eigvalsh(dense_sop(p))[0]
    o = GroundOracle(p)
    o.set_state(random_isometric_state(p.parent, p.local_dim, o.bond, seed=6))
    energies = [o.sweep() for _ in range(4)]
    for a, b in zip(energies, energies[1:]):
        assert b <= a + 1e-12
    assert min(energies) >= e0 - 1e-12
    # the local eigenvalues are energies of normalised states: never below e0
    assert min(o.local_values) >= e0 - 1e-10
