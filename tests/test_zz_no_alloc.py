"""The allocation-free QR entry point (ttn_qr_noalloc, for callers that cannot
allocate device memory) against the allocating one (ttn_debug_qr) through the
C boundary: same kernels, so the same Q and R to the last bit, on two calls in
a row with the second smaller (the shared static scratch keeps the first
call's contents)."""
import ctypes as C

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2503_15460_amd as T
    f = T.lib.ttn_qr_noalloc
    f.restype = C.c_int32
    f.argtypes = [C.c_int64, C.c_int32, C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p]
    T.lib.ttn_qr_noalloc_last_error.restype = C.c_char_p
    return T, torch


def _matrix(rows, cols, seed, rank_deficient=False):
    rng = np.random.default_rng(seed)
    M = rng.normal(size=(rows, cols)) + 1j * rng.normal(size=(rows, cols))
    if rank_deficient:  # a product-state-like factor: columns beyond the first two empty
        M[:, 2:] = 0.0
        M[0, 3] = 0.5
    return M


def _noalloc(T, torch, M, variant):
    rows, cols = M.shape
    dm = torch.from_numpy(np.ascontiguousarray(M).view(np.float64).copy()).to("cuda")
    dr = torch.full((2 * cols * cols,), float("nan"), dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    code = T.lib.ttn_qr_noalloc(rows, cols, dm.data_ptr(), dr.data_ptr(), variant, stream)
    assert code == 0, T.lib.ttn_qr_noalloc_last_error()
    torch.cuda.synchronize()
    Q = dm.cpu().numpy().view(np.complex128).reshape(rows, cols)
    R = dr.cpu().numpy().view(np.complex128).reshape(cols, cols)
    return Q, R


@pytest.mark.parametrize("variant", [1, 2])
def test_noalloc_qr_equals_allocating_entry_point(env, variant):
    T, torch = env
    cases = [(_matrix(8192, 20, 1), False), (_matrix(4096, 16, 2, rank_deficient=True), True)]
    for M, _ in cases:  # second call smaller than the first
        Qn, Rn = _noalloc(T, torch, M, variant)
        Qa, Ra = T.gpu_qr(M, variant)
        assert np.array_equal(Qn, Qa) and np.array_equal(Rn, Ra)
        assert np.abs(Qn @ Rn - M).max() < 1e-12 * np.abs(M).max()


def test_noalloc_qr_refuses_bad_sizes(env):
    T, torch = env
    buf = torch.zeros(2 * 100 * 65, dtype=torch.float64, device="cuda")
    r = torch.zeros(2 * 65 * 65, dtype=torch.float64, device="cuda")
    for rows, cols, var in ((100, 65, 1), (10, 20, 1), (100, 8, 3)):
        assert T.lib.ttn_qr_noalloc(rows, cols, buf.data_ptr(), r.data_ptr(), var, None) == -1
        assert T.lib.ttn_qr_noalloc_last_error()
    assert T.lib.ttn_qr_noalloc(100, 8, None, r.data_ptr(), 1, None) == -1
