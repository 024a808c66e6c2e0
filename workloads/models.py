"""Seeded synthetic models standing in for the paper's workloads.

The paper's benchmark models (the 24-mode pyrazine Hamiltonian of Sec. IV A and
the P3HT:PCBM exciton model of Sec. IV B) take their parameters from external
references that are not available here, so these generators draw synthetic
parameters of the same shape (number of states, modes, terms, tree depth and
bond dimensions) with ``numpy.random.default_rng(seed)`` in a fixed order.

* ``sbm_problem``: spin-boson model of Sec. III (star topology, ohmic bath,
  orthogonal-polynomial discretisation with omega_max = 10 omega_c).
* ``vibronic_problem``: 2-state / 24-mode quadratic vibronic-coupling model of
  the form used for pyrazine (Sec. IV A).
* ``exciton_problem``: 10-state / 120-mode linear vibronic exciton model with
  composite (mode-combined) leaves (Sec. IV B).
* ``heom_sbm_problem``: free-pole HEOM in bosonic-operator form for the
  spin-boson model with a Debye bath (Sec. II E 3).
* ``batch_sbm_problems``: many independent spin-boson instances of uneven size.
"""
from __future__ import annotations

import functools
from typing import Dict, List, Tuple

import numpy as np

from .problem import Problem, add_term, balanced_spec, empty_problem

HBAR_EV_FS = 0.6582119569  # eV fs


# --------------------------------------------------------------- operators
def boson_ops(d: int) -> Dict[str, np.ndarray]:
    """Truncated harmonic-oscillator operators in the number basis."""
    a = np.diag(np.sqrt(np.arange(1, d, dtype=np.float64)), k=1).astype(np.complex128)
    ad = a.T.copy()
    n = np.diag(np.arange(d, dtype=np.float64)).astype(np.complex128)
    q = (a + ad) / np.sqrt(2.0)
    # exact matrix elements of Q^2 inside the d-level space (needs level d)
    a1 = np.diag(np.sqrt(np.arange(1, d + 1, dtype=np.float64)), k=1)
    q1 = (a1 + a1.T) / np.sqrt(2.0)
    q2 = (q1 @ q1)[:d, :d].astype(np.complex128)
    return {"a": a, "adag": ad, "n": n, "q": q, "q2": q2, "x": a + ad,
            "nhalf": n + 0.5 * np.eye(d)}


SIGMA = {
    "z": np.array([[1, 0], [0, -1]], dtype=np.complex128),
    "x": np.array([[0, 1], [1, 0]], dtype=np.complex128),
    "y": np.array([[0, -1j], [1j, 0]], dtype=np.complex128),
    "up": np.array([[1, 0], [0, 0]], dtype=np.complex128),
    "dn": np.array([[0, 0], [0, 1]], dtype=np.complex128),
}


def _proj(n: int, s: int, t: int) -> np.ndarray:
    m = np.zeros((n, n), dtype=np.complex128)
    m[s, t] = 1.0
    return m


class _OpCache:
    """Deduplicates (leaf, name) -> operator id while building a problem."""

    def __init__(self, p: Problem):
        self.p = p
        self.ids: Dict[Tuple[int, str], int] = {}

    def __call__(self, leaf: int, name: str, mat: np.ndarray) -> int:
        key = (leaf, name)
        if key not in self.ids:
            self.ids[key] = self.p.add_op(leaf, mat)
        return self.ids[key]


# ------------------------------------------------------------ bath spectra
def ohmic_J(w, alpha: float, wc: float):
    """Ohmic spectral density with exponential cutoff (Sec. III)."""
    w = np.asarray(w, dtype=np.float64)
    return 0.5 * np.pi * alpha * w * np.exp(-w / wc)


@functools.lru_cache(maxsize=4)
def _legendre_grid(nquad: int):
    """Gauss-Legendre nodes and weights on [-1, 1] (computed once per size)."""
    x, w = np.polynomial.legendre.leggauss(nquad)
    x.flags.writeable = False
    w.flags.writeable = False
    return x, w


def gauss_rule(J, wmin: float, wmax: float, n: int, nquad: int = 4000):
    """N-point Gauss rule for the weight J(w) on [wmin, wmax] (Sec. II E 1).

    The recurrence coefficients of the orthonormal polynomials are obtained with
    the discretised Stieltjes (Lanczos) procedure on a fine Gauss-Legendre
    discretisation of the measure, then nodes and weights follow from the
    eigen-decomposition of the Jacobi matrix (Golub-Welsch).  Returns
    ``(nodes, weights)`` with ``sum weights_i F(nodes_i) ~ int F J``.
    """
    x, w = _legendre_grid(nquad)
    t = 0.5 * (wmax - wmin) * x + 0.5 * (wmax + wmin)
    wt = 0.5 * (wmax - wmin) * w * J(t)
    mu0 = wt.sum()
    q = np.sqrt(wt) / np.sqrt(mu0)
    alph = np.zeros(n)
    beta = np.zeros(n)
    Q = np.zeros((n, nquad))
    Q[0] = q
    for j in range(n):
        v = t * Q[j]
        alph[j] = Q[j] @ v
        v -= alph[j] * Q[j]
        if j > 0:
            v -= beta[j - 1] * Q[j - 1]
        v -= Q[: j + 1].T @ (Q[: j + 1] @ v)  # full re-orthogonalisation
        if j + 1 < n:
            beta[j] = np.linalg.norm(v)
            Q[j + 1] = v / beta[j]
    jac = np.diag(alph) + np.diag(beta[: n - 1], 1) + np.diag(beta[: n - 1], -1)
    ev, vec = np.linalg.eigh(jac)
    return ev, mu0 * vec[0] ** 2


def ohmic_discretisation(n: int, alpha: float, wc: float, wmax_factor: float = 10.0,
                         scheme: str = "gauss"):
    """Bath frequencies and couplings with J(w) = pi sum g_k^2 delta(w - w_k)."""
    wmax = wmax_factor * wc
    if scheme == "gauss":
        nodes, weights = gauss_rule(lambda w: ohmic_J(w, alpha, wc), 0.0, wmax, n)
        return nodes, np.sqrt(weights / np.pi)
    if scheme == "density":
        # density of frequencies rho = N J/w / int(J/w), mid-point rule
        k = np.arange(1, n + 1)
        s = 1.0 - np.exp(-wmax / wc)
        w = -wc * np.log(1.0 - (k - 0.5) / n * s)
        g = np.sqrt(alpha * w * wc * s / (2.0 * n))
        return w, g
    raise ValueError(scheme)


def debye_matsubara(lam: float, gam: float, beta: float, K: int):
    """Exponential expansion C(t) = sum_k alpha_k exp(-nu_k t) of a Debye bath.

    J(w) = 2 lam gam w / (w^2 + gam^2) with C(t) = (1/pi) int J(w) [coth(beta w/2)
    cos(w t) - i sin(w t)] dw; one Drude pole plus K-1 Matsubara poles.
    """
    alphas = [lam * gam * (1.0 / np.tan(beta * gam / 2.0) - 1j)]
    nus = [gam + 0j]
    for j in range(1, K):
        nj = 2.0 * np.pi * j / beta
        alphas.append(4.0 * lam * gam * nj / (beta * (nj * nj - gam * gam)) + 0j)
        nus.append(nj + 0j)
    return np.asarray(alphas, dtype=np.complex128), np.asarray(nus, dtype=np.complex128)


# ---------------------------------------------------------------- models
def sbm_problem(n_modes: int = 4, d: int = 8, bond: int = 4, eps: float = 0.5, delta: float = 1.0,
                alpha: float = 0.1, wc: float = 5.0, dt: float = 0.05, n_steps: int = 100,
                scheme: str = "gauss", coupling_scale: float = 1.0, spin_bond: int = None,
                mode_init=None, spin_init=None, name: str = "sbm") -> Problem:
    """Spin-boson model (Eq. for the star-topology SBM in Sec. III).

    ``G = eps/2 sz + delta/2 sx + sz sum_k g_k (a_k + a_k^dag) + sum_k w_k n_k``.
    Tree: ``R(S, B)`` with ``B`` a balanced binary tree over the bath leaves.
    """
    w, g = ohmic_discretisation(n_modes, alpha, wc, scheme=scheme)
    g = g * coupling_scale
    leaves = [("leaf", bond, d, f"b{k}") for k in range(n_modes)]
    bath = balanced_spec(leaves, lambda lev: bond, arity=2)
    spec = ("node", 1, [("leaf", spin_bond or bond, 2, "S"), bath])
    p = empty_problem(name, spec, dt=dt, n_steps=n_steps)
    op = _OpCache(p)
    S = p.leaf_names["S"]
    bo = boson_ops(d)
    add_term(p, eps / 2, [op(S, "sz", SIGMA["z"])])
    add_term(p, delta / 2, [op(S, "sx", SIGMA["x"])])
    for k in range(n_modes):
        b = p.leaf_names[f"b{k}"]
        if g[k] != 0.0:
            add_term(p, g[k], [op(S, "sz", SIGMA["z"]), op(b, "x", bo["x"])])
        add_term(p, w[k], [op(b, "n", bo["n"])])
    p.init_vecs[S] = np.asarray(spin_init if spin_init is not None else [1, 0], dtype=np.complex128)
    for k in range(n_modes):
        v = np.zeros(d, dtype=np.complex128)
        if mode_init is None:
            v[0] = 1.0
        else:
            v[: len(mode_init)] = mode_init
        p.init_vecs[p.leaf_names[f"b{k}"]] = v / np.linalg.norm(v)
    p.observables["sz"] = [op(S, "sz", SIGMA["z"])]
    p.observables["sx"] = [op(S, "sx", SIGMA["x"])]
    p.meta.update(dict(omega=w, g=g, eps=eps, delta=delta, alpha=alpha, wc=wc, d=d, bond=bond))
    return p


def vibronic_problem(seed: int = 2, n_modes: int = 24, dmin: int = 8, dmax: int = 32,
                     leaf_bond: int = 8, l_bond: int = 16, m_bond: int = 20,
                     dt: float = 0.5, n_steps: int = 2000, name: str = "vibronic24") -> Problem:
    """Synthetic 2-state quadratic vibronic-coupling model (form of Sec. IV A).

    Terms (all in eV, divided by hbar so that time is in fs): harmonic
    ``w_i (n_i + 1/2)``, gap ``-D sz``, intra-state linear ``|s><s| Q_i``,
    inter-state linear ``sx Q_i``, intra-state quadratic ``|s><s| Q_i^2`` and
    bilinear ``|s><s| Q_i Q_j`` / ``sx Q_i Q_j`` couplings.  Tree:
    ``R(E, M1, M2)``, ``M_j(L, L, L)``, ``L(4 modes)``.
    """
    rng = np.random.default_rng(seed)
    omega = rng.uniform(0.05, 0.4, n_modes)
    dims = rng.integers(dmin, dmax + 1, n_modes)
    gap = rng.uniform(0.2, 0.5)
    n_groups = n_modes // 4
    groups = [list(range(4 * g, 4 * g + 4)) for g in range(n_groups)]
    Ls = [("node", l_bond, [("leaf", leaf_bond, int(dims[i]), f"q{i}") for i in grp]) for grp in groups]
    half = n_groups // 2
    Ms = [("node", m_bond, Ls[:half]), ("node", m_bond, Ls[half:])]
    spec = ("node", 1, [("leaf", 2, 2, "E")] + Ms)
    p = empty_problem(name, spec, dt=dt, n_steps=n_steps)
    op = _OpCache(p)
    E = p.leaf_names["E"]
    P = [_proj(2, 0, 0), _proj(2, 1, 1)]
    c = 1.0 / HBAR_EV_FS
    qs = [p.leaf_names[f"q{i}"] for i in range(n_modes)]
    bos = [boson_ops(int(dims[i])) for i in range(n_modes)]
    for i in range(n_modes):
        add_term(p, c * omega[i], [op(qs[i], "nhalf", bos[i]["nhalf"])])
    add_term(p, -c * gap, [op(E, "sz", SIGMA["z"])])
    for s in range(2):
        kap = rng.normal(0.0, 0.05, n_modes)
        for i in range(n_modes):
            add_term(p, c * kap[i], [op(E, f"P{s}", P[s]), op(qs[i], "q", bos[i]["q"])])
    inter = rng.choice(n_modes, size=n_modes // 2, replace=False)
    lam = rng.normal(0.0, 0.05, len(inter))
    for k, i in enumerate(sorted(inter)):
        add_term(p, c * lam[k], [op(E, "sx", SIGMA["x"]), op(qs[i], "q", bos[i]["q"])])
    quad = rng.choice(n_modes, size=n_modes // 2, replace=False)
    for i in sorted(quad):
        for s in range(2):
            gq = float(np.clip(rng.normal(0.0, 0.05), -0.25 * omega[i], 0.25 * omega[i]))
            add_term(p, c * gq, [op(E, f"P{s}", P[s]), op(qs[i], "q2", bos[i]["q2"])])
    n_within_max = 6 * n_groups
    n_bil = min(40, n_modes * (n_modes - 1) // 4)
    n_within = min(3 * n_bil // 4, n_within_max)
    pairs = set()
    while len(pairs) < n_bil:
        if len(pairs) < n_within:
            grp = groups[rng.integers(n_groups)]
            i, j = sorted(rng.choice(grp, size=2, replace=False))
        else:
            i, j = sorted(rng.choice(n_modes, size=2, replace=False))
        pairs.add((int(i), int(j)))
    for (i, j) in sorted(pairs):
        kind = rng.integers(3)
        bound = 0.25 * np.sqrt(omega[i] * omega[j])
        cij = float(np.clip(rng.normal(0.0, 0.05), -bound, bound))
        eop = op(E, "sx", SIGMA["x"]) if kind == 2 else op(E, f"P{kind}", P[kind])
        add_term(p, c * cij, [eop, op(qs[i], "q", bos[i]["q"]), op(qs[j], "q", bos[j]["q"])])
    p.init_vecs[E] = np.array([0, 1], dtype=np.complex128)
    for i in range(n_modes):
        v = np.zeros(int(dims[i]), dtype=np.complex128)
        v[0] = 1.0
        p.init_vecs[qs[i]] = v
    p.observables["P0"] = [op(E, "P0", P[0])]
    p.observables["P1"] = [op(E, "P1", P[1])]
    p.meta.update(dict(omega=omega, dims=dims, gap=gap, units="eV/fs"))
    return p


def exciton_problem(seed: int = 3, n_states: int = 10, n_modes: int = 120, dmin: int = 6,
                    dmax: int = 12, leaf_bond: int = 8, c_bond: int = 32, b_bond: int = 48,
                    a_bond: int = 64, n_inter: int = 125, dt: float = 0.5, n_steps: int = 200,
                    name: str = "exciton10x120") -> Problem:
    """Synthetic donor-acceptor exciton model (form of Sec. IV B).

    ``n_states`` electronic states with a random real-symmetric coupling matrix,
    linear intra-state couplings for every (state, mode) pair and a number of
    inter-state linear couplings.  Modes are combined pairwise into composite
    leaves; tree ``R(E, A1, A2)``, ``A(B, B, B)``, ``B(C, C)``, ``C(5 leaves)``
    (scaled down proportionally when ``n_modes`` is smaller).
    """
    rng = np.random.default_rng(seed)
    omega = rng.uniform(0.05, 0.4, n_modes)
    dims = rng.integers(dmin, dmax + 1, n_modes)
    hel = rng.normal(0.0, 0.1, (n_states, n_states))
    hel = np.triu(hel) + np.triu(hel, 1).T
    n_pairs = n_modes // 2
    pair_leaf = []
    leaves_per_c = 5 if n_pairs % 5 == 0 else 1
    n_c = n_pairs // leaves_per_c
    cs = []
    for ci in range(n_c):
        kids = []
        for li in range(leaves_per_c):
            pi = ci * leaves_per_c + li
            da, db = int(dims[2 * pi]), int(dims[2 * pi + 1])
            kids.append(("leaf", leaf_bond, da * db, f"p{pi}"))
            pair_leaf.append(pi)
        cs.append(("node", c_bond, kids))
    # group C nodes into B nodes (2 each) and B nodes into two A nodes
    bs = [("node", b_bond, cs[i:i + 2]) for i in range(0, len(cs), 2)]
    half = (len(bs) + 1) // 2
    As = [("node", a_bond, bs[:half]), ("node", a_bond, bs[half:])]
    spec = ("node", 1, [("leaf", n_states, n_states, "E")] + As)
    p = empty_problem(name, spec, dt=dt, n_steps=n_steps)
    op = _OpCache(p)
    E = p.leaf_names["E"]
    c = 1.0 / HBAR_EV_FS

    def mode_op(k: int, name: str) -> int:
        pi = k // 2
        leaf = p.leaf_names[f"p{pi}"]
        da, db = int(dims[2 * pi]), int(dims[2 * pi + 1])
        if k % 2 == 0:
            mat = np.kron(boson_ops(da)[name], np.eye(db))
        else:
            mat = np.kron(np.eye(da), boson_ops(db)[name])
        return op(leaf, f"{name}{k % 2}", mat)

    for s in range(n_states):
        for t in range(s, n_states):
            m = _proj(n_states, s, t) + (_proj(n_states, t, s) if t != s else 0)
            add_term(p, c * hel[s, t], [op(E, f"h{s}_{t}", m)])
    for k in range(n_modes):
        add_term(p, c * omega[k], [mode_op(k, "nhalf")])
    for s in range(n_states):
        kap = rng.normal(0.0, 0.03, n_modes)
        for k in range(n_modes):
            add_term(p, c * kap[k], [op(E, f"P{s}", _proj(n_states, s, s)), mode_op(k, "q")])
    for _ in range(n_inter):
        s, t = sorted(rng.choice(n_states, size=2, replace=False))
        k = int(rng.integers(n_modes))
        m = _proj(n_states, s, t) + _proj(n_states, t, s)
        add_term(p, c * rng.normal(0.0, 0.03), [op(E, f"X{s}_{t}", m), mode_op(k, "q")])
    p.init_vecs[E] = np.eye(n_states, dtype=np.complex128)[0]
    for pi in range(n_pairs):
        leaf = p.leaf_names[f"p{pi}"]
        v = np.zeros(int(p.local_dim[leaf]), dtype=np.complex128)
        v[0] = 1.0
        p.init_vecs[leaf] = v
    for s in range(n_states):
        p.observables[f"P{s}"] = [op(E, f"P{s}", _proj(n_states, s, s))]
    p.meta.update(dict(omega=omega, dims=dims, hel=hel, units="eV/fs"))
    return p


def heom_sbm_problem(K: int = 16, levels: int = 10, eps: float = 0.5, delta: float = 1.0,
                     lam: float = 0.2, gam: float = 1.0, T: float = 1.0, bonds=(10, 16, 24, 32, 48),
                     dt: float = 0.0075, n_steps: int = 4000, rho0=None,
                     name: str = "heom_sbm") -> Problem:
    """Free-pole HEOM of the spin-boson model in bosonic-operator form.

    Generator ``G`` with ``d/dt |rho) = -i G |rho)`` (Eq. for the HEOM in
    operator form, Sec. II E 3, with the main text's scaling of the up/down
    couplings):
    ``G = L_s - i sum_k (nu_k n_k + nu_k^* nt_k)
          + sum_k [alpha_k/sqrt|alpha_k| S^L a_k^dag - alpha_k^*/sqrt|alpha_k| S^R at_k^dag]
          + sum_k sqrt|alpha_k| (S^L - S^R)(a_k + at_k)``
    with ``L_s = H_s^L - H_s^R``, row-major vec so ``X^L = X (x) 1`` and
    ``X^R = 1 (x) X^T``.  The system leaf is the 4-dim Liouville space; the
    2K auxiliary modes (m_k, n~_k adjacent) form a balanced binary subtree.
    ``rho0`` is the initial 2 x 2 system density matrix (default |up><up|).
    """
    beta = 1.0 / T
    alphas, nus = debye_matsubara(lam, gam, beta, K)
    n_aux = 2 * K
    leaves = [("leaf", bonds[0], levels, f"m{k}" if j == 0 else f"t{k}")
              for k in range(K) for j in range(2)]

    def bond_of(level):
        return bonds[min(level + 1, len(bonds) - 1)]
    bath = balanced_spec(leaves, bond_of, arity=2)
    spec = ("node", 1, [("leaf", 4, 4, "S"), bath])
    p = empty_problem(name, spec, dt=dt, n_steps=n_steps, hermitian=False)
    op = _OpCache(p)
    S = p.leaf_names["S"]
    I2 = np.eye(2, dtype=np.complex128)
    hs = 0.5 * eps * SIGMA["z"] + 0.5 * delta * SIGMA["x"]
    sop = SIGMA["z"]
    Ls = np.kron(hs, I2) - np.kron(I2, hs.T)
    SL = np.kron(sop, I2)
    SR = np.kron(I2, sop.T)
    add_term(p, 1.0, [op(S, "Ls", Ls)])
    bo = boson_ops(levels)
    for k in range(K):
        m = p.leaf_names[f"m{k}"]
        t = p.leaf_names[f"t{k}"]
        a = alphas[k]
        sa = np.sqrt(abs(a))
        add_term(p, -1j * nus[k], [op(m, "n", bo["n"])])
        add_term(p, -1j * np.conj(nus[k]), [op(t, "n", bo["n"])])
        add_term(p, a / sa, [op(S, "SL", SL), op(m, "adag", bo["adag"])])
        add_term(p, -np.conj(a) / sa, [op(S, "SR", SR), op(t, "adag", bo["adag"])])
        add_term(p, sa, [op(S, "Sm", SL - SR), op(m, "a", bo["a"])])
        add_term(p, sa, [op(S, "Sm", SL - SR), op(t, "a", bo["a"])])
    if rho0 is None:
        rho0 = np.array([[1, 0], [0, 0]], dtype=np.complex128)
    p.init_vecs[S] = np.asarray(rho0, dtype=np.complex128).reshape(-1)
    for k in range(n_aux):
        leaf = p.leaf_names[f"m{k // 2}" if k % 2 == 0 else f"t{k // 2}"]
        v = np.zeros(levels, dtype=np.complex128)
        v[0] = 1.0
        p.init_vecs[leaf] = v
    # bilinear observables: (b| rho) with b = vec(O^T) on S and vacuum on aux
    p.meta.update(dict(alphas=alphas, nus=nus, eps=eps, delta=delta, lam=lam, gam=gam, beta=beta,
                       K=K, levels=levels,
                       bra_sz=SIGMA["z"].T.reshape(-1).copy(), bra_tr=I2.reshape(-1).copy()))
    return p


def pseudomode_sbm_problem(K: int = 4, levels: int = 5, eps: float = 0.5, delta: float = 1.0,
                           lam: float = 0.2, gam: float = 1.0, T: float = 1.0, bonds=(16, 24, 32),
                           dt: float = 0.0075, n_steps: int = 400, rho0=None, coupling_scale: float = 1.0,
                           name: str = "pseudomode_sbm") -> Problem:
    """Quasi-Lindblad pseudomode form of the spin-boson model (SI, section on
    the equivalence of free-pole HEOM and the generalised pseudomode method).

    The bath correlation function C(t) = sum_k alpha_k exp(-nu_k t) of the
    Debye bath (the same expansion as ``heom_sbm_problem``) is written as
    sum_k (V_k - i M_k) exp(-(gamma_k + i E_k) t) (V_k + i M_k)^* with real
    V_k - i M_k = sqrt(alpha_k), gamma_k + i E_k = nu_k.  In the Liouville
    representation (ket index n and bra index m~ of every pseudomode, tilde
    operators acting from the right: a~ |n><m| = |n><m| a^dag) the generator
    G with d/dt |rho) = -i G |rho) is
    ``L_s + sum_k [2i gamma_k a_k a~_k - i (nu_k n_k + nu_k^* n~_k)]
          + sum_k 2i (M_k^* S^L a~_k + M_k S^R a_k)
          + sum_k [(V_k^* - i M_k^*) S^L a_k^dag - (V_k + i M_k) S^R a~_k^dag]
          + sum_k [(V_k - i M_k) S^L a_k - (V_k^* + i M_k^*) S^R a~_k]``
    with L_s = H_s^L - H_s^R and, for the row-major vec of the system's 2 x 2
    density matrix, X^L = X (x) 1 and X^R = 1 (x) X^T.  Each pseudomode and
    its tilde partner form one leaf of dimension levels^2 (index n levels + m),
    so that the boson trace vec(1) is a product over leaves; the K leaves form
    a balanced binary subtree beside the 4-dim system leaf.  ``coupling_scale``
    multiplies V_k and M_k (0: the spin decouples from the pseudomodes).
    """
    beta = 1.0 / T
    alphas, nus = debye_matsubara(lam, gam, beta, K)
    root_a = np.sqrt(alphas.astype(np.complex128))
    V = root_a.real * coupling_scale
    M = -root_a.imag * coupling_scale
    L = levels
    leaves = [("leaf", bonds[0], L * L, f"q{k}") for k in range(K)]

    def bond_of(level):
        return bonds[min(level + 1, len(bonds) - 1)]
    bath = balanced_spec(leaves, bond_of, arity=2)
    spec = ("node", 1, [("leaf", 4, 4, "S"), bath])
    p = empty_problem(name, spec, dt=dt, n_steps=n_steps, hermitian=False)
    op = _OpCache(p)
    S = p.leaf_names["S"]
    I2 = np.eye(2, dtype=np.complex128)
    hs = 0.5 * eps * SIGMA["z"] + 0.5 * delta * SIGMA["x"]
    sop = SIGMA["z"]
    SL = np.kron(sop, I2)
    SR = np.kron(I2, sop.T)
    add_term(p, 1.0, [op(S, "Ls", np.kron(hs, I2) - np.kron(I2, hs.T))])
    bo = boson_ops(L)
    IL = np.eye(L, dtype=np.complex128)
    a_, ad_, n_ = bo["a"], bo["adag"], bo["n"]
    pm = {"a": np.kron(a_, IL), "adag": np.kron(ad_, IL), "n": np.kron(n_, IL),
          "at": np.kron(IL, a_), "atdag": np.kron(IL, ad_), "nt": np.kron(IL, n_), "a_at": np.kron(a_, a_)}
    for k in range(K):
        q = p.leaf_names[f"q{k}"]
        g_k, nu = nus[k].real, nus[k]
        v, m = V[k], M[k]
        add_term(p, 2j * g_k, [op(q, "a_at", pm["a_at"])])
        add_term(p, -1j * nu, [op(q, "n", pm["n"])])
        add_term(p, -1j * np.conj(nu), [op(q, "nt", pm["nt"])])
        if v != 0.0 or m != 0.0:
            add_term(p, 2j * np.conj(m), [op(S, "SL", SL), op(q, "at", pm["at"])])
            add_term(p, 2j * m, [op(S, "SR", SR), op(q, "a", pm["a"])])
            add_term(p, np.conj(v) - 1j * np.conj(m), [op(S, "SL", SL), op(q, "adag", pm["adag"])])
            add_term(p, -(v + 1j * m), [op(S, "SR", SR), op(q, "atdag", pm["atdag"])])
            add_term(p, v - 1j * m, [op(S, "SL", SL), op(q, "a", pm["a"])])
            add_term(p, -(np.conj(v) + 1j * np.conj(m)), [op(S, "SR", SR), op(q, "at", pm["at"])])
    if rho0 is None:
        rho0 = np.array([[1, 0], [0, 0]], dtype=np.complex128)
    p.init_vecs[S] = np.asarray(rho0, dtype=np.complex128).reshape(-1)
    vac = np.zeros(L * L, dtype=np.complex128)
    vac[0] = 1.0  # |0><0|
    for k in range(K):
        p.init_vecs[p.leaf_names[f"q{k}"]] = vac.copy()
    # bilinear observables: (b| rho) with b = vec(O^T) on S and the boson trace vec(1) on every leaf
    p.meta.update(dict(alphas=alphas, nus=nus, V=V, M=M, eps=eps, delta=delta, lam=lam, gam=gam, beta=beta,
                       K=K, levels=L, bra_sz=SIGMA["z"].T.reshape(-1).copy(), bra_tr=I2.reshape(-1).copy(),
                       bra_bath=IL.reshape(-1).copy()))
    return p


def chain_transform(w, g):
    """Star-to-chain transformation of a harmonic bath (Sec. II E 2, chain form
    of the system-bath Hamiltonian): Lanczos tridiagonalisation of diag(w)
    started from g / |g|, with full re-orthogonalisation.

    Returns ``(V, eps, t, kappa0)`` with V real orthogonal (star mode
    a_k = sum_l V[k, l] b_l in terms of the chain modes b_l), V[:, 0] = g / kappa0,
    kappa0 = |g| and V^T diag(w) V tridiagonal with on-site energies eps and
    hoppings t.
    """
    w = np.asarray(w, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    n = len(w)
    kappa0 = float(np.linalg.norm(g))
    V = np.zeros((n, n))
    V[:, 0] = g / kappa0
    eps = np.zeros(n)
    t = np.zeros(max(n - 1, 0))
    for j in range(n):
        v = w * V[:, j]
        eps[j] = V[:, j] @ v
        for _ in range(2):  # projection on every earlier vector, twice
            v -= V[:, : j + 1] @ (V[:, : j + 1].T @ v)
        if j + 1 < n:
            t[j] = np.linalg.norm(v)
            V[:, j + 1] = v / t[j]
    return V, eps, t, kappa0


def ipchain_sbm_problem(n_modes: int = 8, d: int = 6, bonds=(8, 8, 8), eps: float = 0.0, delta: float = 1.0,
                        alpha: float = 0.5, wc: float = 5.0, dt: float = 0.02, n_steps: int = 200,
                        chain: bool = True, name: str = "ipchain_sbm") -> Problem:
    """Interaction-picture chain form of the spin-boson model (Sec. II E 2,
    equation for H_SB^ic(t)), a generator with time-dependent coefficients.

    The star model of ``sbm_problem`` (Ohmic bath, J(w) = pi sum g_k^2
    delta(w - w_k) from the Gauss rule of Sec. II E 1) is taken to the chain
    modes b_l = sum_k V[k, l] a_k of ``chain_transform`` and to the interaction
    picture of the bath Hamiltonian H_B = sum_k w_k n_k (in the chain basis the
    on-site and hopping terms), where H_B drops out and
    ``G(t) = eps/2 sz + delta/2 sx + sz sum_l [G_l(t) b_l^dag + G_l(t)^* b_l]``
    with ``G_l(t) = sum_k V[k, l] g_k exp(i w_k t)``; at t = 0 only the first
    chain mode couples, with kappa0 = |g|.  ``chain=False`` keeps the star
    modes (V = 1, G_k(t) = g_k exp(i w_k t)): on the truncated Fock spaces this
    is exactly the interaction picture of the truncated star model.

    Terms, in order: eps/2 sz, delta/2 sx, then per mode l the pair
    sz b_l^dag and sz b_l; ``ipchain_coefficients(p, t)`` gives all of their
    coefficients at time t (``p.coeff`` holds those at t = 0).  Tree: the spin
    leaf beside a balanced binary tree over the modes in chain order, bonds
    ``bonds[0]`` at the leaves and ``bonds[min(level + 1, -1)]`` above.
    """
    w, g = ohmic_discretisation(n_modes, alpha, wc)
    V, ceps, hop, kappa0 = chain_transform(w, g) if chain else (np.eye(n_modes), w, np.zeros(n_modes - 1),
                                                               float(np.linalg.norm(g)))

    def bond_of(level):
        return bonds[min(level + 1, len(bonds) - 1)]
    leaves = [("leaf", bonds[0], d, f"b{k}") for k in range(n_modes)]
    bath = balanced_spec(leaves, bond_of, arity=2)
    spec = ("node", 1, [("leaf", bonds[0], 2, "S"), bath])
    p = empty_problem(name, spec, dt=dt, n_steps=n_steps, hermitian=True)
    op = _OpCache(p)
    S = p.leaf_names["S"]
    bo = boson_ops(d)
    add_term(p, eps / 2, [op(S, "sz", SIGMA["z"])])
    add_term(p, delta / 2, [op(S, "sx", SIGMA["x"])])
    for k in range(n_modes):
        b = p.leaf_names[f"b{k}"]
        add_term(p, 1.0, [op(S, "sz", SIGMA["z"]), op(b, "adag", bo["adag"])])
        add_term(p, 1.0, [op(S, "sz", SIGMA["z"]), op(b, "a", bo["a"])])
    p.init_vecs[S] = np.array([1, 0], dtype=np.complex128)
    for k in range(n_modes):
        v = np.zeros(d, dtype=np.complex128)
        v[0] = 1.0
        p.init_vecs[p.leaf_names[f"b{k}"]] = v
    p.observables["sz"] = [op(S, "sz", SIGMA["z"])]
    p.observables["sx"] = [op(S, "sx", SIGMA["x"])]
    p.meta.update(dict(omega=w, g=g, V=V, chain_eps=ceps, chain_hop=hop, kappa0=kappa0, eps=eps, delta=delta,
                       alpha=alpha, wc=wc, d=d, chain=chain))
    p.coeff = ipchain_coefficients(p, 0.0)
    return p


def ipchain_coefficients(p: Problem, t: float) -> np.ndarray:
    """Coefficients of every term of ``ipchain_sbm_problem`` at time t."""
    m = p.meta
    G = m["V"].T @ (m["g"] * np.exp(1j * m["omega"] * t))
    c = np.empty(2 + 2 * len(G), dtype=np.complex128)
    c[0] = m["eps"] / 2
    c[1] = m["delta"] / 2
    c[2::2] = G
    c[3::2] = np.conj(G)
    return c


def multiset_vibronic_problem(n_sets: int = 3, n_modes: int = 4, d: int = 4, bonds=(4, 6), seed: int = 0,
                              coupled: bool = True, dt: float = 0.1, n_steps: int = 50,
                              name: str = "multiset_vibronic") -> Problem:
    """Seeded vibronic model for the multi-set ansatz of Sec. II A
    (|Psi> = sum_alpha |alpha> |Psi^alpha>, one tree tensor network of the
    same shape per electronic state alpha).

    ``G = sum_{alpha beta} |alpha><beta| (x) G_{alpha beta}`` on the modes with
    ``G_{alpha alpha} = E_alpha + sum_k w_k n_k + sum_k kappa_{alpha k} x_k``
    and, for alpha != beta, ``G_{alpha beta} = D_{alpha beta} + sum_k
    lambda_{alpha beta k} x_k`` (real symmetric couplings, so G is Hermitian);
    ``coupled=False`` drops the off-diagonal blocks.  The tree holds the modes
    only: a balanced binary tree with bonds ``bonds[0]`` at the leaves and
    ``bonds[1]`` above.  Every term lists its block in
    ``meta["set_pair"][r] = (alpha, beta)``; a term without operators is a
    constant of its block.  Start: alpha = 0 with every mode in its ground
    state (``meta["set_weights"]``: 1 for alpha = 0, else 0).
    """
    rng = np.random.default_rng(seed)
    w = rng.uniform(0.5, 1.5, n_modes)
    E = np.sort(rng.uniform(-0.5, 0.5, n_sets))
    kappa = rng.normal(0.0, 0.3, (n_sets, n_modes))
    D = rng.normal(0.0, 0.2, (n_sets, n_sets))
    lam = rng.normal(0.0, 0.1, (n_sets, n_sets, n_modes))
    leaves = [("leaf", bonds[0], d, f"q{k}") for k in range(n_modes)]
    top = balanced_spec(leaves, lambda lev: bonds[min(1, len(bonds) - 1)], arity=2)
    spec = ("node", 1, top[2]) if top[0] == "node" else ("node", 1, [top])
    p = empty_problem(name, spec, dt=dt, n_steps=n_steps, hermitian=True)
    op = _OpCache(p)
    bo = boson_ops(d)
    pairs = []

    def term(a, b, coef, ops):
        add_term(p, coef, ops)
        pairs.append((a, b))
    for a in range(n_sets):
        term(a, a, E[a], [])
        for k in range(n_modes):
            q = p.leaf_names[f"q{k}"]
            term(a, a, w[k], [op(q, "n", bo["n"])])
            term(a, a, kappa[a, k], [op(q, "x", bo["x"])])
    if coupled:
        for a in range(n_sets):
            for b in range(n_sets):
                if a == b:
                    continue
                lo, hi = min(a, b), max(a, b)
                term(a, b, D[lo, hi], [])
                for k in range(n_modes):
                    q = p.leaf_names[f"q{k}"]
                    term(a, b, lam[lo, hi, k], [op(q, "x", bo["x"])])
    vac = np.zeros(d, dtype=np.complex128)
    vac[0] = 1.0
    for k in range(n_modes):
        p.init_vecs[p.leaf_names[f"q{k}"]] = vac.copy()
    weights = np.zeros(n_sets, dtype=np.complex128)
    weights[0] = 1.0
    p.meta.update(dict(n_sets=n_sets, set_pair=pairs, set_weights=weights, omega=w, E=E, kappa=kappa))
    return p


def batch_sbm_problems(seed: int = 5, n_inst: int = 256, nmin: int = 8, nmax: int = 64,
                       dmin: int = 6, dmax: int = 16, bmin: int = 8, bmax: int = 48,
                       dt: float = 0.05, n_steps: int = 100) -> List[Problem]:
    """Many independent spin-boson instances of seeded uneven size."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n_inst):
        n = int(rng.integers(nmin, nmax + 1))
        d = int(rng.integers(dmin, dmax + 1))
        chi = int(rng.integers(bmin, bmax + 1))
        eps = float(rng.uniform(0.0, 1.0))
        delta = float(rng.uniform(0.5, 1.5))
        alpha = float(rng.uniform(0.05, 0.5))
        out.append(sbm_problem(n_modes=n, d=d, bond=chi, eps=eps, delta=delta, alpha=alpha,
                               wc=5.0, dt=dt, n_steps=n_steps, name=f"sbm_batch{i}"))
    return out


# ------------------------------------------------------------ test states
def random_isometric_state(parent, local_dim, bonds, seed: int) -> List[np.ndarray]:
    """Random TTN with every non-root node an isometry toward its parent.

    ``bonds`` must be feasible (each matricisation children x parent has at
    least as many rows as columns).  Node tensors have the children's indices
    first (in node-id order) and the parent index last; leaves are (d, n).
    """
    rng = np.random.default_rng(seed)
    parent = np.asarray(parent)
    n = len(parent)
    kids = [[c for c in range(n) if parent[c] == z] for z in range(n)]
    out = []
    for z in range(n):
        rows = [int(local_dim[z])] if local_dim[z] > 0 else [int(bonds[c]) for c in kids[z]]
        cols = int(bonds[z]) if parent[z] >= 0 else 1
        m = rng.normal(size=(int(np.prod(rows)), cols)) + 1j * rng.normal(size=(int(np.prod(rows)), cols))
        if parent[z] >= 0:
            q, _ = np.linalg.qr(m)
            t = q
        else:
            t = m / np.linalg.norm(m)
        out.append(np.ascontiguousarray(t.reshape(rows + [cols])))
    return out


# ------------------------------------------------------------- named configs
CONFIGS = {
    "sbm4": lambda: sbm_problem(n_modes=4, d=8, bond=4, name="sbm4"),
    "vibronic24": lambda: vibronic_problem(),
    "exciton10x120": lambda: exciton_problem(),
    "heom_sbm": lambda: heom_sbm_problem(),
}


def config_problem(name: str) -> Problem:
    return CONFIGS[name]()
