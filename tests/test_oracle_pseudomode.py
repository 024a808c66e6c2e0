"""Pins of the quasi-Lindblad pseudomode generator (SI, equivalence of
free-pole HEOM and the generalised pseudomode method) and of the oracle on
it: trace preservation of the Liouville-space generator, the decoupled limit,
the equivalence with the free-pole HEOM generator for the same bath
correlation function, and the oracle's sweep at full bonds against the dense
exponential."""
import numpy as np
import scipy.linalg as sla

from oracle import Oracle, dense_sop
from oracle.ttn_oracle import leaf_order
from workloads import heom_sbm_problem, pseudomode_sbm_problem


def _prod(vs):
    v = np.ones(1, dtype=np.complex128)
    for x in vs:
        v = np.kron(v, x)
    return v


def _bra(p, system_vec, bath_vec):
    order = leaf_order(p.parent, p.local_dim)
    S = p.leaf_names["S"]
    return _prod([system_vec if z == S else bath_vec(z) for z in order])


def _dense_sz(p, bath_vec, times):
    G = dense_sop(p)
    order = leaf_order(p.parent, p.local_dim)
    psi0 = _prod([p.init_vecs[z] for z in order])
    b = _bra(p, p.meta["bra_sz"], bath_vec)
    return np.array([b @ sla.expm(-1j * t * G) @ psi0 for t in times])


def test_pseudomode_generator_preserves_the_trace():
    """The quasi-Lindblad equation preserves Tr rho, also with truncated
    ladders: the Liouville-space trace (vec(1) of the system times vec(1) of
    every pseudomode pair) is a left null vector of G."""
    p = pseudomode_sbm_problem(K=2, levels=4, bonds=(16, 16, 16))
    G = dense_sop(p)
    tr = _bra(p, p.meta["bra_tr"], lambda z: p.meta["bra_bath"])
    assert np.abs(tr @ G).max() < 1e-12 * np.abs(G).max()


def test_decoupled_pseudomodes_leave_the_rabi_dynamics():
    """V = M = 0: the spin evolves under L_s alone,
    <sz>(t) = 1 - 2 (Delta / Omega)^2 sin^2(Omega t / 2) from |up><up|."""
    eps, delta = 0.5, 1.0
    p = pseudomode_sbm_problem(K=2, levels=3, eps=eps, delta=delta, bonds=(9, 9, 9), coupling_scale=0.0)
    times = [0.3, 1.1, 2.5]
    got = _dense_sz(p, lambda z: p.meta["bra_bath"], times)
    Om = np.hypot(eps, delta)
    ref = [1 - 2 * (delta / Om) ** 2 * np.sin(Om * t / 2) ** 2 for t in times]
    assert np.abs(got - ref).max() < 1e-12


def test_pseudomode_equals_free_pole_heom():
    """Same Debye expansion (one pole): the pseudomode <sz>(t), read with the
    boson trace, equals the free-pole HEOM <sz>(t), read with the vacuum
    projection, up to the ladder truncation, and the difference shrinks as the
    ladders grow (the two forms are related by a similarity transformation of
    the auxiliary boson space)."""
    times = [0.5, 1.0, 2.0, 3.0]
    diffs = []
    for levels in (6, 8):
        pm = pseudomode_sbm_problem(K=1, levels=levels, bonds=(64, 64, 64))
        he = heom_sbm_problem(K=1, levels=levels, bonds=(64, 64, 64))

        def vac(z, q=he):
            v = np.zeros(q.local_dim[z], dtype=np.complex128)
            v[0] = 1.0
            return v
        a = _dense_sz(pm, lambda z: pm.meta["bra_bath"], times)
        b = _dense_sz(he, vac, times)
        diffs.append(np.abs(a - b).max())
    assert diffs[1] < 1e-6
    assert diffs[1] < diffs[0] / 10


def test_oracle_at_full_bonds_is_the_dense_exponential():
    """The oracle's Arnoldi sweep on the pseudomode generator, at bonds as
    large as the tree allows, reproduces exp(-i G t) psi0 (non-Hermitian
    generator: the full-bond projector-splitting sweep is exact)."""
    p = pseudomode_sbm_problem(K=2, levels=3, bonds=(64, 64, 64), dt=0.05)
    o = Oracle(p)
    o.set_product_state(p.init_vecs)
    G = dense_sop(p)
    order = leaf_order(p.parent, p.local_dim)
    psi0 = _prod([p.init_vecs[z] for z in order])
    from oracle import full_state
    for s in range(1, 6):
        o.step(p.dt)
        ref = sla.expm(-1j * s * p.dt * G) @ psi0
        got = full_state(o.parent, o.local_dim, o.state())
        assert np.abs(got - ref).max() < 1e-11
