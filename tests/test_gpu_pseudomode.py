"""The quasi-Lindblad pseudomode generator (non-Hermitian, Arnoldi) on the GPU
against the oracle: <sigma_z> and Tr rho_S read with the boson trace after
every step, and the full state vector."""
import numpy as np
import pytest

from oracle import Oracle, full_state
from workloads import pseudomode_sbm_problem

pytestmark = pytest.mark.gpu

# FP64 bar; the oracle's own floor on this case (tests/golden/jitter.json,
# product state, 6 steps) is 4.1e-12
TOL_FP64 = 1e-10


@pytest.fixture(scope="module")
def T():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2503_15460_amd as mod
    return mod


def _bra(p, key):
    b = {z: p.meta["bra_bath"] for z in p.leaves()}
    b[p.leaf_names["S"]] = p.meta[key]
    return b


@pytest.mark.parametrize("prec,tol", [(0, TOL_FP64), (1, 1e-4)])
def test_pseudomode_parity(T, prec, tol):
    """Four pseudomodes of 4 x 4 levels (bonds 16/16/16, the multi-kernel and
    fused Arnoldi paths), 6 steps from |up><up| x vacuum: <sigma_z> and the
    trace against the oracle (FP64 1e-10, FP32 contractions 1e-4), the trace
    staying 1 (the generator preserves it), and in FP64 the full state vector
    (gauge-independent: single node tensors differ by a few 1e-10 in
    directions of small weight, where the QR gauge amplifies rounding by the
    inverse of the weight)."""
    p = pseudomode_sbm_problem(K=4, levels=4, bonds=(16, 16, 16), dt=0.02)
    o = Oracle(p)
    o.set_product_state(p.init_vecs)
    g = T.TTN.from_problem(p, precision=prec)
    g.set_product_state(p.init_vecs)
    for s in range(6):
        o.step(p.dt)
        g.step(p.dt)
        ref = np.array([o.bilinear(_bra(p, k)) for k in ("bra_sz", "bra_tr")])
        got = np.array([g.bilinear(_bra(p, k)) for k in ("bra_sz", "bra_tr")])
        print(f"step {s}: <sz> {got[0].real:.12f} (oracle {ref[0].real:.12f}), trace {got[1].real:.12f}")
        assert np.abs(got - ref).max() < tol
        assert abs(got[1] - 1.0) < tol
    if prec == T.TTN_FP64:
        a = full_state(p.parent, p.local_dim, g.get_state())
        b = full_state(p.parent, p.local_dim, o.state())
        d = np.abs(a - b).max() / np.abs(b).max()
        print(f"full state: relative difference {d:.2e}")
        assert d < 1e-10
    g.close()
