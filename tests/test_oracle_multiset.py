"""Pins of the multi-set oracle (Sec. II A multi-set ansatz, one-site sweep of
Sec. II C with all sets evolved together at every node): exactness at full
bonds against the dense block generator, reduction to the single-set oracle
for one set, independent sets when the blocks do not couple, and the
conservation of norm and energy with truncated bonds."""
import numpy as np
import scipy.linalg as sla

from oracle import Oracle, full_state
from oracle.multiset import MultiSetOracle, dense_multiset
from workloads import multiset_vibronic_problem, random_isometric_state
from workloads.problem import Problem


def _block_problem(p, a):
    """The terms of block (a, a) with operators as a single-set problem, and
    the sum of its constant terms (a global phase for that set)."""
    keep = [r for r, ab in enumerate(p.meta["set_pair"]) if tuple(ab) == (a, a) and len(p.term_ops[r])]
    const = sum(p.coeff[r] for r, ab in enumerate(p.meta["set_pair"])
                if tuple(ab) == (a, a) and not len(p.term_ops[r]))
    q = Problem(**{**p.__dict__, "coeff": np.asarray([p.coeff[r] for r in keep]),
                   "term_ops": [p.term_ops[r] for r in keep], "meta": {}})
    return q, const


def _random_sets(p, o, seed):
    return [random_isometric_state(p.parent, p.local_dim, o.bond[a], seed=seed + a) for a in range(o.S)]


def test_full_bonds_equal_the_dense_block_exponential():
    """Bonds as large as the tree allows: every multi-set state is on the
    manifold and the sweep is exact, exp(-i G t) psi0 with G the dense block
    generator, from the state-0 product start (population moves to the other
    sets) and from random sets."""
    p = multiset_vibronic_problem(n_sets=3, n_modes=4, d=3, bonds=(9, 9), dt=0.1)
    G = dense_multiset(p)
    assert np.abs(G - G.conj().T).max() == 0.0
    for start in ("product", "random"):
        o = MultiSetOracle(p)
        if start == "product":
            o.set_product_state(p.init_vecs, p.meta["set_weights"])
        else:
            st = _random_sets(p, o, 3)
            for a in range(o.S):
                st[a][o.root] = st[a][o.root] / np.sqrt(o.S)
            o.set_state(st)
        psi0 = o.dense_state()
        for s in range(1, 5):
            o.step(p.dt)
            ref = sla.expm(-1j * s * p.dt * G) @ psi0
            assert np.abs(o.dense_state() - ref).max() < 1e-11  # the local solves' 1e-13 targets, summed
        if start == "product":
            assert o.populations()[1:].min() > 1e-4


def test_one_set_is_the_single_set_oracle():
    """One set and truncated bonds: the multi-set sweep is the single-set sweep
    (an independent implementation that aggregates inside and outside terms),
    the block's constant term a global phase."""
    p = multiset_vibronic_problem(n_sets=1, n_modes=4, d=4, bonds=(2, 3), dt=0.1, seed=2)
    q, const = _block_problem(p, 0)
    m = MultiSetOracle(p)
    o = Oracle(q)
    st = random_isometric_state(p.parent, p.local_dim, o.bond, seed=5)
    assert all((o.bond == b).all() for b in m.bond)
    m.set_state([st])
    o.set_state(st)
    for s in range(1, 6):
        m.step(p.dt)
        o.step(p.dt)
        ref = np.exp(-1j * const * s * p.dt) * full_state(o.parent, o.local_dim, o.state())
        assert np.abs(full_state(m.parent, m.local_dim, m.A[0]) - ref).max() < 1e-12


def test_uncoupled_sets_evolve_independently():
    """No off-diagonal blocks, truncated bonds: every set follows the
    single-set sweep of its own block, Psi^alpha(t) = exp(-i E_alpha t) times
    the single-set result."""
    p = multiset_vibronic_problem(n_sets=3, n_modes=4, d=4, bonds=(2, 3), dt=0.1, seed=4, coupled=False)
    m = MultiSetOracle(p)
    st = _random_sets(p, m, 7)
    m.set_state(st)
    singles = []
    for a in range(3):
        q, const = _block_problem(p, a)
        o = Oracle(q)
        o.set_state(st[a])
        singles.append((o, const))
    for s in range(1, 5):
        m.step(p.dt)
        for a, (o, const) in enumerate(singles):
            o.step(p.dt)
            ref = np.exp(-1j * const * s * p.dt) * full_state(o.parent, o.local_dim, o.state())
            assert np.abs(full_state(m.parent, m.local_dim, m.A[a]) - ref).max() < 1e-12


def test_norm_and_energy_are_conserved_with_truncated_bonds():
    """Coupled sets, bonds below the exact ones, from the state-0 product
    start: the norm (sum of the set populations) and <Psi|G|Psi> stay
    constant (the sweep is a composition of unitary substeps on a Hermitian
    generator)."""
    p = multiset_vibronic_problem(n_sets=3, n_modes=4, d=4, bonds=(2, 3), dt=0.1, seed=6)
    G = dense_multiset(p)
    m = MultiSetOracle(p)
    m.set_product_state(p.init_vecs, p.meta["set_weights"])
    psi = m.dense_state()
    e0 = np.vdot(psi, G @ psi).real
    for _ in range(20):
        m.step(p.dt)
        psi = m.dense_state()
        assert abs(np.vdot(psi, psi).real - 1.0) < 1e-12
        assert abs(np.vdot(psi, G @ psi).real - e0) < 1e-11 * max(1.0, abs(e0))
    assert m.populations()[1:].min() > 1e-4
