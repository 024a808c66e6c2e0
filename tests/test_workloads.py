"""Pins of the seeded input generators (bath discretisation, Debye expansion, models)."""
import numpy as np
import pytest
from scipy import integrate, special

from workloads import (batch_sbm_problems, exciton_problem, heom_sbm_problem, sbm_problem,
                       vibronic_problem)
from workloads.models import debye_matsubara, gauss_rule, ohmic_discretisation, ohmic_J


@pytest.mark.parametrize("n", [4, 16, 64])
def test_gauss_rule_moments(n):
    """The N-point rule integrates w^k J(w) exactly for k <= 2N-1 (Sec. II E 1)."""
    alpha, wc = 0.1, 5.0
    W = 10 * wc
    w, a = gauss_rule(lambda x: ohmic_J(x, alpha, wc), 0.0, W, n)
    for k in range(0, min(2 * n, 30)):
        # int_0^W (pi/2) alpha w^(k+1) e^(-w/wc) dw = (pi/2) alpha wc^(k+2) gamma(k+2, W/wc)
        exact = 0.5 * np.pi * alpha * wc ** (k + 2) * special.gamma(k + 2) * special.gammainc(k + 2, W / wc)
        got = np.sum(a * w ** k)
        assert abs(got - exact) <= 1e-10 * abs(exact), (k, got, exact)
    assert np.all(w > 0) and np.all(w < W) and np.all(a > 0)


def test_density_of_frequencies_reorganisation():
    """rho = J/w: every mode carries the same share of the reorganisation energy."""
    n, alpha, wc = 50, 0.2, 5.0
    w, g = ohmic_discretisation(n, alpha, wc, scheme="density")
    share = g ** 2 / w
    assert np.allclose(share, share[0], rtol=1e-12)
    lam_exact = (1 / np.pi) * integrate.quad(lambda x: ohmic_J(x, alpha, wc) / x, 0, 10 * wc)[0]
    assert abs(np.sum(share) - lam_exact) < 1e-12


def test_debye_matsubara_matches_correlation_integral():
    lam, gam, beta = 0.2, 1.0, 1.0
    a, nu = debye_matsubara(lam, gam, beta, 400)
    J = lambda w: 2 * lam * gam * w / (w * w + gam * gam)
    def jcoth(w):  # J(w) coth(beta w / 2), with its finite limit at w = 0
        return 4 * lam * gam / (beta * gam * gam) if w < 1e-12 else J(w) / np.tanh(beta * w / 2)
    for t in (0.5, 1.0, 2.0):
        re = integrate.quad(lambda w: jcoth(w) / np.pi, 0, np.inf, weight="cos", wvar=t)[0]
        im = -integrate.quad(lambda w: J(w) / np.pi, 0, np.inf, weight="sin", wvar=t)[0]
        c = np.sum(a * np.exp(-nu * t))
        assert abs(c.real - re) < 1e-7 and abs(c.imag - im) < 1e-7


def test_models_shapes():
    p = vibronic_problem()
    assert p.n_nodes == 34 and 140 <= p.n_terms <= 160
    assert all(8 <= p.local_dim[l] <= 32 for l in p.leaves() if l != p.leaf_names["E"])
    q = exciton_problem()
    assert 1400 <= q.n_terms <= 1600 and len(q.leaves()) == 61
    h = heom_sbm_problem()
    assert len(h.leaves()) == 33 and not h.hermitian and h.n_terms == 1 + 6 * 16
    b = batch_sbm_problems(n_inst=8)
    assert len(b) == 8
    s = sbm_problem()
    assert s.n_nodes == 9 and s.n_terms == 10


def test_models_deterministic():
    a, b = vibronic_problem(seed=2), vibronic_problem(seed=2)
    assert np.array_equal(a.coeff, b.coeff) and a.term_ops == b.term_ops
    c = vibronic_problem(seed=9)
    assert not np.array_equal(a.coeff[:60], c.coeff[:60])


def test_flat_sop_roundtrip():
    p = sbm_problem()
    op_leaf, off, data, coeff, tptr, tops = p.flat_sop()
    assert off[-1] * 2 == data.size and coeff.size == 2 * p.n_terms and tptr[-1] == tops.size
    m = data.view(np.complex128)[off[2]:off[3]]
    assert np.array_equal(m, p.op_mats[2].reshape(-1))
