"""GPU kernel checks against the oracle's definitions (through the C boundary)."""
import numpy as np
import pytest

from oracle import Oracle, householder_qr_lapack
from oracle.ttn_oracle import SNAP
from workloads import random_isometric_state, sbm_problem

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def T():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2503_15460_amd as mod
    return mod


def _cases():
    rng = np.random.default_rng(12)
    out = []
    for (m, n) in [(7, 4), (40, 16), (4096, 20), (8192, 8), (5120, 16), (300, 64), (20000, 33)]:
        M = rng.normal(size=(m, n)) + 1j * rng.normal(size=(m, n))
        out.append(("random", M))
    # product-state-like rank deficient: a single nonzero column, exact zeros elsewhere
    M = np.zeros((4096, 16), dtype=np.complex128)
    M[:, 0] = rng.normal(size=4096)
    M[5, 3] = 0.25 + 0.5j
    out.append(("rankdef", M))
    # rank deficient with rounding-size noise in the empty columns
    N = M + 1e-17 * (rng.normal(size=M.shape) + 1j * rng.normal(size=M.shape))
    out.append(("noisy_rankdef", N))
    return out


def _cholesky_route_cases():
    """Matrices for the Cholesky route: inside its range (random, graded
    columns with condition ~1e5) and outside it (rank-deficient, columns
    already triangular so that the Householder steps have nothing below the
    diagonal, square)."""
    rng = np.random.default_rng(13)
    inside, outside = [], []
    for (m, n) in [(65, 64), (1000, 48), (4096, 20), (20000, 33)]:
        inside.append(("random", rng.normal(size=(m, n)) + 1j * rng.normal(size=(m, n))))
    G = (rng.normal(size=(3000, 24)) + 1j * rng.normal(size=(3000, 24))) * np.logspace(0, -5, 24)
    inside.append(("graded", G))
    E = np.zeros((5000, 16), dtype=np.complex128)
    E[np.arange(16), np.arange(16)] = rng.uniform(0.5, 2.0, 16) * np.exp(1j * rng.uniform(0, 6.28, 16))
    outside.append(("triangular", E))
    # square: the last column has no entries below the diagonal
    outside.append(("square", rng.normal(size=(64, 64)) + 1j * rng.normal(size=(64, 64))))
    for name, M in _cases():
        if name != "random":
            outside.append((name, M))
    return inside, outside


@pytest.mark.parametrize("variant", [0, 1, 2, 3])
def test_qr_matches_oracle_householder(T, variant):
    cases = _cases()
    if variant == 3:  # matrices outside the Cholesky route go through the gate to the Householder kernels
        cases += _cholesky_route_cases()[1]
    for name, M in cases:
        if variant == 0 and M.size > 200_000:
            continue
        if variant == 2 and M.shape[1] > 48:  # the LDS-resident cooperative QR takes n <= 48
            continue
        Q, R = T.gpu_qr(M, variant)
        Qo, Ro = householder_qr_lapack(M, snap=SNAP)
        scale = max(1.0, np.abs(M).max())
        assert np.abs(Q - Qo).max() < 1e-12, (name, M.shape, np.abs(Q - Qo).max())
        assert np.abs(R - Ro).max() < 1e-12 * scale, (name, M.shape)
        assert np.abs(Q.conj().T @ Q - np.eye(M.shape[1])).max() < 1e-12


def test_cholesky_route_alone(T):
    """The Cholesky route by itself gives the oracle's Householder factors (the
    LAPACK signs) inside its range and declines the matrices a Householder step
    would snap or that have no full column rank; a 110592 x 64 block (the shape
    of the largest exciton nodes) is compared by sampled columns."""
    inside, outside = _cholesky_route_cases()
    for name, M in inside:
        Q, R = T.gpu_qr(M, 4)
        Qo, Ro = householder_qr_lapack(M, snap=SNAP)
        err = np.abs(Q - Qo).max()
        print(f"{name} {M.shape}: |Q - Q_householder| {err:.1e}")
        assert err < 1e-12 * max(1.0, np.linalg.cond(M) / 100), (name, M.shape, err)
        assert np.abs(R - Ro).max() < 1e-12 * np.abs(M).max() * max(1.0, np.linalg.cond(M) / 100)
        assert np.abs(Q.conj().T @ Q - np.eye(M.shape[1])).max() < 1e-13
    for name, M in outside:
        with pytest.raises(T.TTNError, match="NOCONV"):
            T.gpu_qr(M, 4)
    rng = np.random.default_rng(14)
    M = rng.normal(size=(110592, 64)) + 1j * rng.normal(size=(110592, 64))
    Q, R = T.gpu_qr(M, 4)
    Qh, Rh = T.gpu_qr(M, 1)
    assert np.abs(Q - Qh).max() < 1e-12 and np.abs(R - Rh).max() < 1e-12 * np.abs(M).max()
    assert np.abs(Q.conj().T @ Q - np.eye(64)).max() < 1e-13
    assert np.abs(Q @ R - M).max() < 1e-12 * np.abs(M).max()


def test_large_node_parity(T):
    """Spin-boson with bond 32: nodes of 32^3 elements use the many-work-group QR."""
    p = sbm_problem(n_modes=8, d=8, bond=32, alpha=0.3, dt=0.05)
    o0 = Oracle(p)
    assert max(int(np.prod(o0.shape(z))) for z in range(p.n_nodes)) >= 16384
    st = random_isometric_state(p.parent, p.local_dim, o0.bond, seed=6)
    g = T.TTN.from_problem(p)
    g.set_state(st)
    o0.set_state(st)
    for _ in range(3):
        g.step(p.dt)
        o0.step(p.dt)
        assert abs(g.expect(p.observables["sz"]) - o0.expect(p.observables["sz"])) < 1e-10


def test_launch_profiler_times_every_kernel(T):
    """The launch profiler reports positive times for every kernel of a sweep,
    including the cooperative QR (timed from the kernel's own clock), and the
    summed kernel time stays below the wall time of the profiled sweep."""
    import time
    import torch
    p = sbm_problem(n_modes=8, d=8, bond=32, alpha=0.3, dt=0.05)
    g = T.TTN.from_problem(p)
    g.set_state(random_isometric_state(p.parent, p.local_dim, Oracle(p).bond, seed=6))
    g.step(p.dt)
    torch.cuda.synchronize()
    T.profile_begin()
    t0 = time.perf_counter()
    g.step(p.dt)
    torch.cuda.synchronize()
    wall_ms = (time.perf_counter() - t0) * 1e3
    rows = T.profile_end()
    names = {r["name"] for r in rows}
    assert "k_qr_coop" in names
    for r in rows:
        assert r["calls"] > 0 and r["total_ms"] > 0.0, r
    assert sum(r["total_ms"] for r in rows) < wall_ms
    g.close()


def test_autotuned_tiles_give_the_same_results(T, tmp_path):
    """autotune = 1 times the register tiles of every tiled stage on the
    handle's own programs and fills the tile table; the tile changes no
    accumulation order, so the sweep is bit for bit the one of the fixed rule.
    The table survives a JSON round trip."""
    from workloads import vibronic_problem
    p = vibronic_problem(n_modes=12, dmin=4, dmax=8, leaf_bond=6, l_bond=12, m_bond=16)
    T.tile_table_clear()
    plain = T.TTN.from_problem(p)
    plain.set_product_state(p.init_vecs)
    plain.step(p.dt, 2)
    tuned = T.TTN(p.parent, p.local_dim, p.bond_dim, autotune=True)
    tuned.set_sop_problem(p)
    n = T.tile_table_size()
    print(f"tile table: {n} stage shapes tuned")
    assert n > 0
    tuned.set_product_state(p.init_vecs)
    tuned.step(p.dt, 2)
    for a, b in zip(plain.get_state(), tuned.get_state()):
        assert np.array_equal(a, b)
    path = str(tmp_path / "tiles.json")
    T.tile_table_save(path)
    T.tile_table_clear()
    assert T.tile_table_load(path) == n
    T.tile_table_clear()
