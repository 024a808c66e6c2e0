"""Batched instances (ttn_batch_*): uneven spin-boson instances advanced
together on several HIP streams give exactly the results of stepping each
instance alone (same kernels in the same order per instance)."""
import numpy as np
import pytest

from workloads import batch_sbm_problems, sbm_problem

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def T():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2503_15460_amd as mod
    return mod


def _make(T, p, precision):
    g = T.TTN.from_problem(p, precision=precision)
    g.set_product_state(p.init_vecs)
    return g


@pytest.mark.parametrize("precision", [0, 1])
def test_batch_equals_individual_steps(T, precision):
    probs = batch_sbm_problems(seed=11, n_inst=7, nmin=3, nmax=10, dmin=4, dmax=8, bmin=4, bmax=14)
    sizes = [max(int(np.prod(s)) for s in _make(T, p, precision).shapes()) for p in probs]
    assert max(sizes) > 1024 and min(sizes) <= 1024  # both Krylov paths among the instances
    batch = [_make(T, p, precision) for p in probs]
    alone = [_make(T, p, precision) for p in probs]
    dts = np.array([p.dt * (1.0 + 0.1 * i) for i, p in enumerate(probs)])
    b = T.TTNBatch(batch, n_streams=3)
    b.step(dts, 4)
    for g, dt in zip(alone, dts):
        g.step(dt, 4)
    for gb, ga, p in zip(batch, alone, probs):
        for x, y in zip(gb.get_state(), ga.get_state()):
            assert np.abs(x - y).max() <= 1e-13
        assert gb.counters()["steps"] == 4
        assert abs(gb.expect(p.observables["sz"]) - ga.expect(p.observables["sz"])) <= 1e-13
    b.close()
    # instances keep working on their own streams after the batch is gone
    batch[0].step(dts[0])
    alone[0].step(dts[0])
    assert abs(batch[0].expect(probs[0].observables["sz"]) - alone[0].expect(probs[0].observables["sz"])) <= 1e-13


def test_batch_errors(T):
    p = sbm_problem(n_modes=2, d=3, bond=2)
    ok = _make(T, p, 0)
    nostate = T.TTN.from_problem(p)
    b = T.TTNBatch([ok, nostate])
    with pytest.raises(T.TTNError) as e:
        b.step(p.dt)
    assert "E_STATE" in str(e.value) and "instance 1" in str(e.value)
    with pytest.raises(T.TTNError) as e:
        T.TTNBatch([ok])  # already in a batch
    assert "E_INVALID" in str(e.value)
    b.close()
    T.TTNBatch([ok]).close()
