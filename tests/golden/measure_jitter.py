"""Measure the oracle's own rounding jitter floor J on the parity workloads and
write ``jitter.json`` beside this script.

J is the largest spread of the observables between runs of the oracle that
differ only in rounding: BLAS with one thread against all threads (summation
order), every SOP coefficient multiplied by (1 + 1e-15 u) with seeded u in
[-1, 1], and 1e-16 relative noise added to every tensor before each QR.  The
FP64 parity tolerance of a GPU test must not go below max(1e-10, 10 J).

Uses only the oracle and the seeded input generators:
    python tests/golden/measure_jitter.py
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
from workloads import random_isometric_state, sbm_problem, vibronic_problem  # noqa: E402


def trajectory(p, obs, n, state_seed=None, coeff_noise=0.0, qr_noise=0.0, seed=0):
    rng = np.random.default_rng(seed)
    if coeff_noise:
        p.coeff = np.asarray(p.coeff, dtype=np.complex128) * (1.0 + coeff_noise * rng.uniform(-1, 1, len(p.coeff)))
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
        o.step(p.dt)
        out.append([o.expect(p.observables[k]) for k in obs] + [o.overlap_t0()])
    return np.array(out)


CASES = {
    "sbm4_product_state_40_steps": (lambda: sbm_problem(n_modes=4, d=8, bond=4), ["sz"], 40, None),
    "reduced_vibronic_product_state_6_steps": (
        lambda: vibronic_problem(n_modes=8, dmin=4, dmax=6, leaf_bond=4, l_bond=6, m_bond=8, dt=0.5),
        ["P0", "P1"], 6, None),
    "reduced_vibronic_full_rank_6_steps": (
        lambda: vibronic_problem(n_modes=8, dmin=4, dmax=6, leaf_bond=4, l_bond=6, m_bond=8, dt=0.5),
        ["P0", "P1"], 6, 8),
    "vibronic24_full_rank_3_steps": (lambda: vibronic_problem(), ["P0", "P1"], 3, 24),
}


def main():
    res = {}
    for name, (make, obs, n, seed) in CASES.items():
        t0 = time.time()
        base = trajectory(make(), obs, n, seed)
        with threadpool_limits(limits=1):
            one = trajectory(make(), obs, n, seed)
        coeff = trajectory(make(), obs, n, seed, coeff_noise=1e-15, seed=1)
        qr = trajectory(make(), obs, n, seed, qr_noise=1e-16, seed=2)
        spread = {"blas_threads": float(np.abs(base - one).max()),
                  "coefficients_1e-15": float(np.abs(base - coeff).max()),
                  "qr_noise_1e-16": float(np.abs(base - qr).max())}
        res[name] = {"J": max(spread.values()), **spread, "observables": obs + ["a(t)"], "steps": n,
                     "start": "product state" if seed is None else f"random isometric state, seed {seed}"}
        print(name, res[name], f"{time.time() - t0:.0f} s", flush=True)
    with open(os.path.join(HERE, "jitter.json"), "w") as f:
        json.dump(res, f, indent=1)


if __name__ == "__main__":
    main()
