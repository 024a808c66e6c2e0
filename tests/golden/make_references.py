"""Write ``references.json`` beside this script: oracle results for the GPU
parity tests whose oracle runs take minutes (so that the GPU test session
stays short).  Only the oracle and the seeded input generators are used:

    python tests/golden/make_references.py

Each case records a fingerprint of its inputs (SHA-256 of the SOP arrays, the
tree, the bonds and the start), the observables after every step, and, for
the element-wise checks, seeded samples of every node tensor of the final
state (SAMPLES flat indices per node, all of them for smaller nodes).
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import Oracle  # noqa: E402
from workloads import batch_sbm_problems, exciton_problem, random_isometric_state, vibronic_problem  # noqa: E402

SAMPLES = 64


def c3_shaped():
    """The exciton workload's tree at reduced size (10 states, 60 modes in 30
    composite leaves, five-leaf C nodes, B(C, C), A1(B, B), A2(B), bonds
    4/24/28/32, 735 SOP terms)."""
    return exciton_problem(n_states=10, n_modes=60, dmin=2, dmax=2, leaf_bond=4, c_bond=24, b_bond=28, a_bond=32,
                           n_inter=20)


def c5_smallest(k=3):
    """The k smallest instances (by total tensor size) of the 256-instance
    seeded spin-boson batch (seed 5), as (index, problem)."""
    probs = batch_sbm_problems(seed=5)
    sizes = []
    for i, p in enumerate(probs):
        o = Oracle(p)
        sizes.append((sum(int(np.prod(o.shape(z))) for z in range(o.n)), i))
    return [(i, probs[i]) for _, i in sorted(sizes)[:k]]


def fingerprint(p, bonds, state=None) -> str:
    h = hashlib.sha256()
    for a in p.flat_sop():
        h.update(np.ascontiguousarray(a).tobytes())
    for a in (p.parent, p.local_dim, bonds, p.flat_init()):
        h.update(np.ascontiguousarray(a).tobytes())
    h.update(repr(float(p.dt)).encode())
    if state is not None:
        for t in state:
            h.update(np.ascontiguousarray(t).tobytes())
    return h.hexdigest()


def sample_indices(size: int, node: int) -> np.ndarray:
    if size <= SAMPLES:
        return np.arange(size)
    return np.sort(np.random.default_rng(1000 + node).choice(size, SAMPLES, replace=False))


def cplx(a) -> list:
    a = np.asarray(a, dtype=np.complex128).reshape(-1)
    return [[float(x.real), float(x.imag)] for x in a]


def run_case(p, obs_names, n, state=None):
    o = Oracle(p)
    if state is None:
        o.set_product_state(p.init_vecs)
    else:
        o.set_state(state)
    obs = []
    for s in range(n):
        t0 = time.time()
        o.step(p.dt)
        obs.append(cplx([o.expect(p.observables[k]) for k in obs_names] + [o.overlap_t0()]))
        print(f"  step {s + 1}/{n}: {time.time() - t0:.0f} s", flush=True)
    samples = []
    for z, t in enumerate(o.state()):
        idx = sample_indices(t.size, z)
        samples.append({"idx": idx.tolist(), "val": cplx(t.reshape(-1)[idx])})
    return {"fingerprint": fingerprint(p, o.bond, state), "observables": obs_names + ["a(t)"], "obs": obs,
            "norm2": o.norm2(), "tensor_samples": samples}


def main():
    out = {}
    p = c3_shaped()
    st = random_isometric_state(p.parent, p.local_dim, Oracle(p).bond, seed=31)
    print("c3_shaped", flush=True)
    out["c3_shaped"] = run_case(p, [f"P{k}" for k in range(10)], 3, st)
    p = vibronic_problem()
    st = random_isometric_state(p.parent, p.local_dim, Oracle(p).bond, seed=24)
    print("vibronic24_full_rank", flush=True)
    out["vibronic24_full_rank"] = run_case(p, ["P0", "P1"], 3, st)
    for i, p in c5_smallest():
        print(f"c5_instance_{i}", flush=True)
        out[f"c5_instance_{i}"] = run_case(p, ["sz"], 3)
    with open(os.path.join(HERE, "references.json"), "w") as f:
        json.dump(out, f)


if __name__ == "__main__":
    main()
