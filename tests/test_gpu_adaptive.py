"""Subspace expansion (bond adaptation, Sec. II D) on the GPU against the
oracle's adaptive sweep (oracle/subspace.py AdaptiveOracle): the same bonds
after every step (the spawn counts follow from the singular values of the
two-site residual and the threshold), the same observables, and the same dense
state, from a product state with small bonds on a spin-boson tree and on a
non-Hermitian (HEOM) generator with Arnoldi."""
import numpy as np
import pytest

from oracle.subspace import AdaptiveOracle
from oracle.ttn_oracle import full_state
from workloads import heom_sbm_problem, sbm_problem

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def T():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2503_15460_amd as mod
    return mod


def _heom_obs(g, p):
    S = p.leaf_names["S"]
    out = []
    for key in ("bra_sz", "bra_tr"):
        bra = {z: np.eye(p.local_dim[z])[0].astype(np.complex128) for z in p.leaves()}
        bra[S] = p.meta[key]
        out.append(g.bilinear(bra))
    return out


@pytest.mark.parametrize("case", ["sbm_1e-6", "sbm_1e-4", "heom_1e-6"])
def test_adaptive_sweep_matches_oracle(T, case):
    kind, eps = case.split("_")
    eps = float(eps)
    if kind == "sbm":
        p = sbm_problem(n_modes=4, d=4, bond=2, alpha=0.5, dt=0.05)
        chi, n_steps = 6, 8
        obs = lambda src: [src.expect(p.observables["sz"]), src.overlap_t0()]  # noqa: E731
    else:
        p = heom_sbm_problem(K=2, levels=3, bonds=(2, 2, 2, 2, 2), dt=0.05)
        chi, n_steps = 6, 6
        obs = lambda src: _heom_obs(src, p)  # noqa: E731
    o = AdaptiveOracle(p, eps_s=eps, chi_max=chi, seed=0)
    o.set_product_state(p.init_vecs)
    g = T.TTN(p.parent, p.local_dim, p.bond_dim, hermitian=p.hermitian, spawn_tol=eps,
              bond_max=[chi] * p.n_nodes, seed=7)
    g.set_sop_problem(p)
    g.set_product_state(p.init_vecs)
    grew = False
    for s in range(n_steps):
        o.step(p.dt)
        g.step(p.dt)
        b = g.bonds()
        grew |= bool((b > np.asarray(T.clamp_bonds(p.parent, p.local_dim, p.bond_dim))).any())
        assert b.tolist() == o.bond.tolist(), f"step {s}: bonds {b.tolist()} vs oracle {o.bond.tolist()}"
        err = max(abs(x - y) for x, y in zip(obs(g), obs(o)))
        print(f"{case} step {s}: bonds {b.tolist()}, max observable difference {err:.2e}", flush=True)
        assert err < 1e-9
    assert grew
    psi_g = full_state(p.parent, p.local_dim, g.get_state())
    assert np.abs(psi_g - o.dense_state()).max() < 1e-9


def test_adaptive_respects_bond_max_and_norm(T):
    """With a tolerance that spawns whatever the residual offers, no bond passes
    its maximum and the norm stays 1 (new functions enter with zero
    coefficients); a step that does not converge restores the bonds together
    with the state."""
    p = sbm_problem(n_modes=4, d=4, bond=2, alpha=0.8, dt=0.05)
    bmax = np.array([1, 2, 2, 3, 3, 3, 3, 3, 3], dtype=np.int32)
    g = T.TTN(p.parent, p.local_dim, p.bond_dim, spawn_tol=1e-14, bond_max=bmax, krylov_mmax=6)
    g.set_sop_problem(p)
    g.set_product_state(p.init_vecs)
    cap = T.clamp_bonds(p.parent, p.local_dim, bmax)
    start = g.bonds().copy()
    for _ in range(6):
        g.step(p.dt)
        assert (g.bonds() <= cap).all()
        assert abs(g.norm2() - 1.0) < 1e-12
    assert (g.bonds() > start).any()
    # a failed step (Krylov limit far too small) leaves bonds and state as they were
    h = T.TTN(p.parent, p.local_dim, p.bond_dim, spawn_tol=1e-14, bond_max=bmax, krylov_mmax=6)
    h.set_sop_problem(p)
    h.set_product_state(p.init_vecs)
    h.step(p.dt, 2)
    bonds, before = h.bonds().copy(), h.get_state()
    with pytest.raises(T.TTNError) as e:
        h.step(50.0)
    assert "E_NOCONV" in str(e.value)
    assert np.array_equal(h.bonds(), bonds)
    for x, y in zip(before, h.get_state()):
        assert np.array_equal(x, y)
    h.step(p.dt)  # still usable


def test_fp32_expansion_keeps_the_norm(T):
    """Subspace expansion in the FP32 mode on the exciton workload from bonds
    of 8 (two sweeps, the bond sum growing from 649 to ~1300): the new functions
    enter with zero coefficients, so the norm stays 1 to rounding (the bond
    matrix's unit block on the new functions, left by the QR, once carried
    ~1e-5 of norm into the state through FP32 rounding of the bond generator)."""
    import torch
    from workloads import exciton_problem
    p = exciton_problem()
    start = np.minimum(np.asarray(p.bond_dim), 8)
    g = T.TTN(p.parent, p.local_dim, start, precision=T.TTN_FP32, spawn_tol=1e-6, bond_max=p.bond_dim, seed=3)
    g.set_sop_problem(p)
    g.set_product_state(p.init_vecs)
    b0 = int(g.bonds().sum())
    for _ in range(2):
        g.step(p.dt)
        torch.cuda.synchronize()
        print(f"bond sum {int(g.bonds().sum())}, norm - 1 = {g.norm2() - 1:.2e}")
        assert abs(g.norm2() - 1.0) < 1e-10
    assert int(g.bonds().sum()) > b0
    g.close()
