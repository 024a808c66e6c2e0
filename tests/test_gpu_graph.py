"""Steps replayed from captured hipGraphs (use_graph = 1) against ordinary
launches: every replay agrees with the eager run of the same instance (the
gauge QRs take the non-cooperative kernels in a graph, so agreement is to
rounding, not bit for bit), with the library's own eager work (observables,
state reads) and synchronisations between the replays; a batch of graph
instances agrees with the instances stepped alone."""
import numpy as np
import pytest

from oracle import Oracle
from workloads import batch_sbm_problems, random_isometric_state, sbm_problem, vibronic_problem

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def T():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2503_15460_amd as mod
    return mod


@pytest.mark.parametrize("make", [lambda: sbm_problem(n_modes=8, d=6, bond=16, alpha=0.3),
                                  lambda: vibronic_problem(n_modes=8, dmin=4, dmax=6, leaf_bond=4, l_bond=6,
                                                           m_bond=8, dt=0.5)])
def test_graph_replays_match_eager_steps(T, make):
    p = make()
    st = random_isometric_state(p.parent, p.local_dim, Oracle(p).bond, seed=41)
    obs = next(iter(p.observables))
    runs = {}
    for graph in (False, True):
        g = T.TTN(p.parent, p.local_dim, p.bond_dim, hermitian=p.hermitian, use_graph=graph)
        g.set_sop_problem(p)
        g.set_state(st)
        vals = []
        for _ in range(10):
            g.step(p.dt)
            vals.append([g.expect(p.observables[obs]), g.overlap_t0(), g.norm2()])
        runs[graph] = (np.array(vals), g.get_state(), g)
    err = np.abs(runs[True][0] - runs[False][0]).max()
    print(f"graph vs eager, 10 steps: {err:.2e}; captures {runs[True][2].graph_captures()}")
    assert err < 1e-12
    assert 1 <= runs[True][2].graph_captures() < 10  # later steps replay


def test_graph_batch_matches_instances_alone(T):
    probs = batch_sbm_problems(seed=11, n_inst=5, nmin=3, nmax=8, dmin=4, dmax=6, bmin=4, bmax=12)
    mk = lambda p, graph: T.TTN(p.parent, p.local_dim, p.bond_dim, use_graph=graph)  # noqa: E731
    batch, alone = [mk(p, True) for p in probs], [mk(p, False) for p in probs]
    for g, h, p in zip(batch, alone, probs):
        for x in (g, h):
            x.set_sop_problem(p)
            x.set_product_state(p.init_vecs)
    b = T.TTNBatch(batch, n_streams=3)
    for _ in range(4):
        b.step(np.array([p.dt for p in probs]))
        for h, p in zip(alone, probs):
            h.step(p.dt)
        for g, h, p in zip(batch, alone, probs):
            assert abs(g.expect(p.observables["sz"]) - h.expect(p.observables["sz"])) < 1e-12
    b.close()
