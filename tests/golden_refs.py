"""Loading of the stored oracle references (tests/golden/references.json,
written by tests/golden/make_references.py from the oracle alone)."""
import importlib.util
import json
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_spec = importlib.util.spec_from_file_location("make_references", os.path.join(HERE, "golden", "make_references.py"))
maker = importlib.util.module_from_spec(_spec)
_spec.loader.exec_module(maker)
_cache = {}


def reference(name, p, bonds, state=None):
    """The stored case `name`, after checking that it was made from these inputs."""
    if not _cache:
        with open(os.path.join(HERE, "golden", "references.json")) as f:
            _cache.update(json.load(f))
    rec = _cache[name]
    assert rec["fingerprint"] == maker.fingerprint(p, bonds, state), \
        f"{name}: stored reference made from other inputs (rerun tests/golden/make_references.py)"
    return rec


def observables(rec) -> np.ndarray:
    """(steps, observables) complex array."""
    return np.array([[complex(a, b) for a, b in row] for row in rec["obs"]])


def tensor_sample_error(rec, tensors) -> float:
    """Largest difference at the stored sample positions of every node tensor,
    relative to the largest stored sample of that node."""
    err = 0.0
    for s, t in zip(rec["tensor_samples"], tensors):
        ref = np.array([complex(a, b) for a, b in s["val"]])
        got = np.asarray(t).reshape(-1)[np.asarray(s["idx"], dtype=np.int64)]
        err = max(err, float(np.abs(got - ref).max() / max(np.abs(ref).max(), 1e-300)))
    return err
