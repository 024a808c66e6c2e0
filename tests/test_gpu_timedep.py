"""Time-dependent coefficients (ttn_set_coefficients) on the GPU against the
oracle, on the interaction-picture chain form of the spin-boson model:
coefficients frozen at every step's midpoint, values rewritten in place while
the compiled structure stays, a rebuild when it changes, step graphs recorded
again, and the error paths."""
import numpy as np
import pytest

from oracle import Oracle, full_state
from workloads import ipchain_coefficients, ipchain_sbm_problem, random_isometric_state

pytestmark = pytest.mark.gpu

# FP64 bars: from a seeded full-rank state, and from the product state, whose
# rank-deficient factors pick their completion from rounding (the oracle's own
# floors, tests/golden/jitter.json: 2.4e-15 and 4.0e-8 over these 20 steps)
TOL_FULL_RANK = 1e-10
TOL_PRODUCT = 5e-7


@pytest.fixture(scope="module")
def T():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2503_15460_amd as mod
    return mod


def _problem():
    # 6 chain modes of 5 levels, bonds below the exact ones (5/8/10)
    return ipchain_sbm_problem(n_modes=6, d=5, bonds=(5, 8, 10), eps=0.0, delta=1.0, alpha=0.5, wc=5.0,
                               dt=0.05)


def _start(p, o, g, start):
    if start == "product":
        o.set_product_state(p.init_vecs)
        g.set_product_state(p.init_vecs)
    else:
        st = random_isometric_state(p.parent, p.local_dim, o.bond, seed=11)
        o.set_state(st)
        g.set_state(st)


@pytest.mark.parametrize("prec,start,tol", [(0, "random", TOL_FULL_RANK), (0, "product", TOL_PRODUCT),
                                             (1, "random", 1e-5)])
def test_timedep_parity(T, prec, start, tol):
    """20 midpoint steps: <sigma_z> after every step against the oracle, every
    coefficient change taken in place (no rebuild).  FP64 from a seeded
    full-rank state to 1e-10 and the full state vector at the end (1e-10
    relative); FP64 from the product state to 5e-7, ten times the oracle's
    own floor there (1e-16 noise before every QR moves <sigma_z> and a(t) by
    4e-8 over the 20 steps, as the rank-deficient factors of a product state
    pick their completion; measured on the GPU: 3e-10); FP32 contractions to
    1e-5."""
    p = _problem()
    o = Oracle(p)
    g = T.TTN.from_problem(p, precision=prec)
    _start(p, o, g, start)
    sz = p.observables["sz"]
    t = 0.0
    for s in range(20):
        rebuilt = g.set_coefficients(ipchain_coefficients(p, t + 0.5 * p.dt))
        assert not rebuilt
        g.step(p.dt)
        t += p.dt
        o.step_td(p.dt, lambda tt: ipchain_coefficients(p, tt))
        a, b = g.expect(sz), o.expect(sz)
        if s % 5 == 4:
            print(f"step {s}: <sz> GPU {a.real:.13f}, oracle {b.real:.13f}")
        assert abs(a - b) < tol
    if prec == T.TTN_FP64 and start == "random":
        x = full_state(p.parent, p.local_dim, g.get_state())
        y = full_state(p.parent, p.local_dim, o.state())
        d = np.abs(x - y).max() / np.abs(y).max()
        print(f"full state: relative difference {d:.2e}")
        assert d < 1e-10
    g.close()


def test_step_td_helper_and_structure_change(T):
    """From a seeded full-rank state: the binding's step_td equals the
    oracle's midpoint steps; a coefficient set to exactly zero (delta = 0 for
    two steps) changes the compiled structure and rebuilds the operator,
    setting it back rebuilds again, and through both the GPU follows the
    oracle to 1e-10."""
    p = _problem()
    o = Oracle(p)
    g = T.TTN.from_problem(p)
    _start(p, o, g, "random")
    sz = p.observables["sz"]

    def coef(tt, off=False):
        c = ipchain_coefficients(p, tt)
        if off:
            c[1] = 0.0
        return c
    t = g.step_td(p.dt, coef, 0.0, n_steps=3)
    for _ in range(3):
        o.step_td(p.dt, coef)
    assert abs(g.expect(sz) - o.expect(sz)) < 1e-10
    flags = []
    for s in range(5):
        off = s in (1, 2)
        flags.append(g.set_coefficients(coef(t + 0.5 * p.dt, off)))
        g.step(p.dt)
        t += p.dt
        o.step_td(p.dt, lambda tt: coef(tt, off))
        assert abs(g.expect(sz) - o.expect(sz)) < 1e-10
    print("rebuilt per step:", flags)
    assert flags == [False, True, False, True, False]
    assert abs(g.norm2() - 1.0) < 1e-12
    g.close()


def test_coefficient_changes_under_step_graphs(T):
    """use_graph handles: a coefficient change that keeps the structure and the
    bands of the leaf operators keeps the step graph, whose replays read the
    rewritten coefficient tables (stale values would move <sz> by far more
    than the bar), and the steps agree with ordinary launches to 1e-12
    (measured: bit for bit).  At most 2 captures over the 6 steps, as for a
    static generator (the key changes once, when the Krylov dimension hints
    settle after the first step); a graph dropped at every change would give
    6."""
    p = _problem()
    runs = {}
    for graph in (False, True):
        g = T.TTN(p.parent, p.local_dim, p.bond_dim, hermitian=True, use_graph=graph)
        g.set_sop_problem(p)
        g.set_state(random_isometric_state(p.parent, p.local_dim, g.bonds(), seed=11))
        vals = []
        t = 0.0
        for _ in range(6):
            t = g.step_td(p.dt, lambda tt: ipchain_coefficients(p, tt), t)
            vals.append(g.expect(p.observables["sz"]))
        runs[graph] = (np.array(vals), g)
    err = np.abs(runs[True][0] - runs[False][0]).max()
    print(f"graph vs eager with coefficient changes: {err:.2e}; captures {runs[True][1].graph_captures()}")
    assert err < 1e-12
    assert runs[True][1].graph_captures() <= 2
    for _, g in runs.values():
        g.close()


def test_set_coefficients_errors(T):
    p = _problem()
    g = T.TTN(p.parent, p.local_dim, p.bond_dim, hermitian=True)
    with pytest.raises(T.TTNError) as e:
        g.set_coefficients(p.coeff)  # no operator yet
    assert "E_STATE" in str(e.value)
    g.set_sop_problem(p)
    g.set_product_state(p.init_vecs)
    with pytest.raises(T.TTNError) as e:
        g.set_coefficients(p.coeff[:-1])
    assert "E_INVALID" in str(e.value)
    bad = p.coeff.copy()
    bad[2] = np.nan
    with pytest.raises(T.TTNError) as e:
        g.set_coefficients(bad)
    assert "E_INVALID" in str(e.value)
    nh = ipchain_coefficients(p, 0.3)
    nh[3] *= 2.0  # b^dag and b no longer conjugate: not Hermitian
    with pytest.raises(T.TTNError) as e:
        g.set_coefficients(nh)
    assert "E_INVALID" in str(e.value)
    # the operator in place is unchanged: a step equals the oracle's with the t = 0 coefficients
    o = Oracle(p)
    o.set_product_state(p.init_vecs)
    g.set_product_state(p.init_vecs)
    g.step(p.dt)
    o.step(p.dt)
    assert abs(g.expect(p.observables["sz"]) - o.expect(p.observables["sz"])) < 1e-10
    g.close()
