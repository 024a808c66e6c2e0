"""Measure the oracle's own rounding jitter floor J on the parity workloads and
write ``jitter.json`` beside this script.

J is the largest spread of the observables between runs of the oracle that
differ only in rounding: BLAS with one thread against all threads (summation
order), every SOP coefficient multiplied by (1 + 1e-15 u) with seeded u in
[-1, 1], and 1e-16 relative noise added to every tensor before each QR.  The
FP64 parity tolerance of a GPU test must not go below max(1e-10, 10 J).

Uses only the oracle and the seeded input generators:
    python tests/golden/measure_jitter.py            # every case
    python tests/golden/measure_jitter.py NAME ...   # these cases, the others kept
"""
import json
import os
import sys
import time

import numpy as np
from threadpoolctl import threadpool_limits

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import Oracle  # noqa: E402
from workloads import (ipchain_coefficients, ipchain_sbm_problem, pseudomode_sbm_problem,  # noqa: E402
                       random_isometric_state, sbm_problem, vibronic_problem)


def _observe(o, p, obs):
    # an observable is a key of p.observables or a function of (oracle, problem)
    return [o.expect(p.observables[k]) if isinstance(k, str) else k(o, p) for k in obs]


def trajectory(p, obs, n, state_seed=None, coeff_noise=0.0, qr_noise=0.0, seed=0, coef_at=None):
    """coef_at(p, t): time-dependent coefficients, set at every step's midpoint."""
    rng = np.random.default_rng(seed)
    u = 1.0
    if coeff_noise:
        u = 1.0 + coeff_noise * rng.uniform(-1, 1, len(p.coeff))
        p.coeff = np.asarray(p.coeff, dtype=np.complex128) * u
    o = Oracle(p)
    if qr_noise:
        base = o.qr_along

        def qr_along(A, axis):
            A = A + qr_noise * np.abs(A).max() * (rng.normal(size=A.shape) + 1j * rng.normal(size=A.shape))
            return base(A, axis)
        o.qr_along = qr_along
    if state_seed is None:
        o.set_product_state(p.init_vecs)
    else:
        o.set_state(random_isometric_state(p.parent, p.local_dim, o.bond, seed=state_seed))
    out = []
    for _ in range(n):
        if coef_at is None:
            o.step(p.dt)
        else:
            o.step_td(p.dt, lambda t: coef_at(p, t) * u)
        out.append(_observe(o, p, obs) + [o.overlap_t0()])
    return np.array(out)


def _pm_bilinear(key):
    def f(o, p):
        b = {z: p.meta["bra_bath"] for z in p.leaves()}
        b[p.leaf_names["S"]] = p.meta[key]
        return o.bilinear(b)
    f.__name__ = key
    return f


def _ipchain():
    return ipchain_sbm_problem(n_modes=6, d=5, bonds=(5, 8, 10), eps=0.0, delta=1.0, alpha=0.5, wc=5.0, dt=0.05)


CASES = {
    "sbm4_product_state_40_steps": (lambda: sbm_problem(n_modes=4, d=8, bond=4), ["sz"], 40, None),
    "reduced_vibronic_product_state_6_steps": (
        lambda: vibronic_problem(n_modes=8, dmin=4, dmax=6, leaf_bond=4, l_bond=6, m_bond=8, dt=0.5),
        ["P0", "P1"], 6, None),
    "reduced_vibronic_full_rank_6_steps": (
        lambda: vibronic_problem(n_modes=8, dmin=4, dmax=6, leaf_bond=4, l_bond=6, m_bond=8, dt=0.5),
        ["P0", "P1"], 6, 8),
    "vibronic24_full_rank_3_steps": (lambda: vibronic_problem(), ["P0", "P1"], 3, 24),
    # time-dependent coefficients: the interaction-picture chain case of the GPU parity test
    "ipchain_product_state_20_steps": (_ipchain, ["sz"], 20, None, ipchain_coefficients),
    "ipchain_full_rank_20_steps": (_ipchain, ["sz"], 20, 11, ipchain_coefficients),
    # the quasi-Lindblad pseudomode case of the GPU parity test (Arnoldi)
    "pseudomode_product_state_6_steps": (
        lambda: pseudomode_sbm_problem(K=4, levels=4, bonds=(16, 16, 16), dt=0.02),
        [_pm_bilinear("bra_sz"), _pm_bilinear("bra_tr")], 6, None),
}


def main(names):
    path = os.path.join(HERE, "jitter.json")
    res = json.load(open(path)) if names and os.path.exists(path) else {}
    for name, case in CASES.items():
        if names and name not in names:
            continue
        make, obs, n, seed = case[:4]
        td = case[4] if len(case) > 4 else None
        t0 = time.time()
        base = trajectory(make(), obs, n, seed, coef_at=td)
        with threadpool_limits(limits=1):
            one = trajectory(make(), obs, n, seed, coef_at=td)
        coeff = trajectory(make(), obs, n, seed, coeff_noise=1e-15, seed=1, coef_at=td)
        qr = trajectory(make(), obs, n, seed, qr_noise=1e-16, seed=2, coef_at=td)
        spread = {"blas_threads": float(np.abs(base - one).max()),
                  "coefficients_1e-15": float(np.abs(base - coeff).max()),
                  "qr_noise_1e-16": float(np.abs(base - qr).max())}
        res[name] = {"J": max(spread.values()), **spread,
                     "observables": [k if isinstance(k, str) else k.__name__ for k in obs] + ["a(t)"],
                     "steps": n,
                     "start": "product state" if seed is None else f"random isometric state, seed {seed}"}
        print(name, res[name], f"{time.time() - t0:.0f} s", flush=True)
    with open(path, "w") as f:
        json.dump(res, f, indent=1)


if __name__ == "__main__":
    unknown = [a for a in sys.argv[1:] if a not in CASES]
    if unknown:
        sys.exit(f"unknown cases {unknown}; known: {list(CASES)}")
    main(sys.argv[1:])
