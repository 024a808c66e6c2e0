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
def test_lockstep_batch_equals_individual_steps(T, precision):
    """Lockstep layers (one grouped launch of the fused solver per layer, all
    instances on one stream) give the results of stepping each instance
    alone.  The grouped work-group can be wider than an instance's own, which
    changes the reduction order only: FP64 agrees to 1e-12; with FP32
    contractions the rounding-size differences of the FP64 solves change
    FP32 roundings downstream, and the product-state start amplifies them
    (agreement to 1e-6)."""
    tol = 1e-12 if precision == 0 else 1e-6
    probs = batch_sbm_problems(seed=11, n_inst=7, nmin=3, nmax=10, dmin=4, dmax=8, bmin=4, bmax=14)
    batch = [_make(T, p, precision) for p in probs]
    alone = [_make(T, p, precision) for p in probs]
    dts = np.array([p.dt * (1.0 + 0.1 * i) for i, p in enumerate(probs)])
    b = T.TTNBatch(batch, lockstep=True)
    T.profile_begin()
    b.step(dts, 4)
    prof = {r["name"]: r for r in T.profile_end()}
    T.profile_begin()
    for g, dt in zip(alone, dts):
        g.step(dt, 4)
    prof_alone = {r["name"]: r for r in T.profile_end()}
    for gb, ga, p in zip(batch, alone, probs):
        assert gb.counters()["steps"] == 4
        assert abs(gb.expect(p.observables["sz"]) - ga.expect(p.observables["sz"])) <= tol
        assert abs(gb.overlap_t0() - ga.overlap_t0()) <= tol
    # the instances' fused solves went out together: far fewer launches
    print(f"fused-solver launches: {prof['k_small_solve']['calls']} lockstep, "
          f"{prof_alone['k_small_solve']['calls']} one instance at a time")
    assert prof["k_small_solve"]["calls"] < prof_alone["k_small_solve"]["calls"] / 2
    b.close()


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


@pytest.mark.parametrize("precision,tol", [(0, 1e-9), (1, 1e-4)])
def test_batch_of_seeded_instances_matches_oracle(T, precision, tol):
    """The three smallest instances of the 256-instance seeded batch (seed 5;
    uneven baths, cutoffs and bonds) stepped as one lockstep batch from |up>|0..0>
    match the stored oracle runs instance by instance after every step (FP64
    within 1e-9, FP32 contractions within 1e-4)."""
    import golden_refs as G
    picks = G.maker.c5_smallest()
    recs = []
    for i, p in picks:
        recs.append(G.reference(f"c5_instance_{i}", p, T.clamp_bonds(p.parent, p.local_dim, p.bond_dim)))
    gs = [_make(T, p, precision) for _, p in picks]
    b = T.TTNBatch(gs, lockstep=True)
    got = []
    for _ in range(3):
        b.step(np.array([p.dt for _, p in picks]))
        got.append([[g.expect(p.observables["sz"]), g.overlap_t0()] for g, (_, p) in zip(gs, picks)])
    got = np.array(got)  # (steps, instance, observable)
    for k, ((i, p), rec) in enumerate(zip(picks, recs)):
        err = np.abs(got[:, k, :] - G.observables(rec)).max()
        print(f"instance {i} ({p.meta['d']} levels, bond {p.meta['bond']}): max |d<sz>|, |d a(t)| {err:.2e}")
        assert err < tol
        assert abs(gs[k].norm2() - rec["norm2"]) < tol
    b.close()
