"""GPU checks of the C boundary's options and error behaviour: a caller-owned
workspace (size query, too-small refusal, same results as library-owned
scratch), refused reserved options, the Hermiticity check on the device path,
and the handle state after a failed ttn_set_sop."""
import ctypes as C

import numpy as np
import pytest

from workloads import sbm_problem, vibronic_problem

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def T():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2503_15460_amd as mod
    return mod


def _run(T, p, n, **kw):
    g = T.TTN.from_problem(p, **kw)
    g.set_product_state(p.init_vecs)
    for _ in range(n):
        g.step(p.dt)
    return g


@pytest.mark.parametrize("make", [lambda: sbm_problem(n_modes=4, d=8, bond=4),
                                  lambda: vibronic_problem(n_modes=12, dmin=4, dmax=6, leaf_bond=4,
                                                           l_bond=8, m_bond=8)])
def test_caller_workspace(T, make):
    import torch
    p = make()
    ref = _run(T, p, 3)
    need = ref.workspace_size()
    assert need > 0
    small = torch.empty(need // 2, dtype=torch.uint8, device="cuda")
    g = T.TTN(p.parent, p.local_dim, p.bond_dim, hermitian=p.hermitian,
              workspace=(small.data_ptr(), small.numel()))
    with pytest.raises(T.TTNError) as e:
        g.set_sop_problem(p)
    assert e.value.code == -4 and str(need) in str(e.value)  # TTN_E_OOM names the size
    assert g.workspace_size() == need
    with pytest.raises(T.TTNError) as e:  # no operator after the failure
        g.set_product_state(p.init_vecs)
        g.step(p.dt)
    assert e.value.code == -7
    g.close()
    ws = torch.full((need,), 0xAB, dtype=torch.uint8, device="cuda")  # stale contents must not matter
    torch.cuda.synchronize()
    g2 = _run(T, p, 3, workspace=(ws.data_ptr(), ws.numel()))
    for a, b in zip(g2.get_state(), ref.get_state()):
        assert np.array_equal(a, b)  # same kernels, same scratch contents: bit-identical
    before = ref.counters()["device_bytes"]
    assert g2.counters()["device_bytes"] < before  # the scratch is not allocated by the library


def test_invalid_options_refused(T):
    """Flags outside 0/1, and step graphs together with subspace expansion
    (which changes the launch sequence from step to step), are refused."""
    p = sbm_problem(n_modes=2, d=4, bond=2)
    for fields in ({"use_graph": 2}, {"autotune": 2}, {"use_graph": 1, "spawn_tol": 1e-6}):
        opt = T._lib.Options()
        T.lib.ttn_default_options(C.byref(opt))
        for field, value in fields.items():
            setattr(opt, field, value)
        h = C.c_void_p()
        par = np.ascontiguousarray(p.parent, dtype=np.int32)
        ld = np.ascontiguousarray(p.local_dim, dtype=np.int32)
        bd = np.ascontiguousarray(p.bond_dim, dtype=np.int32)
        i32 = C.POINTER(C.c_int32)
        code = T.lib.ttn_create(len(par), par.ctypes.data_as(i32), ld.ctypes.data_as(i32),
                                bd.ctypes.data_as(i32), C.byref(opt), C.byref(h))
        assert code == -1 and not h.value


def test_numerically_hermitian_operator_runs(T):
    """A leaf operator Hermitian only up to rounding is accepted with
    hermitian = 1 and gives the same dynamics as the exact one."""
    p = sbm_problem(n_modes=3, d=6, bond=3)
    ref = _run(T, p, 4)
    q = sbm_problem(n_modes=3, d=6, bond=3)
    o = q.observables["sz"][0]
    m = np.array(q.op_mats[o], dtype=np.complex128)
    m[0, 1] += 1e-16
    m[1, 0] += 3e-17
    q.op_mats[o] = m
    g = _run(T, q, 4)
    assert abs(g.expect(q.observables["sz"]) - ref.expect(p.observables["sz"])) < 1e-12
    m2 = m.copy()
    m2[0, 1] += 1e-3
    q.op_mats[o] = m2
    with pytest.raises(T.TTNError) as e:
        T.TTN.from_problem(q)
    assert e.value.code == -1
