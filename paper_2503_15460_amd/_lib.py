"""ctypes binding of the HIP library ``libttn.so`` (argument marshalling only).

Every numerical step runs inside the library's HIP kernels.  Importing this
module does not need a GPU; calls that touch the device fail with a TTN error
when none is present.  If the library is missing the import fails loudly:
there is no fallback path.
"""
from __future__ import annotations

import atexit
import ctypes as C
import os
import weakref
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("TTN_LIBRARY", os.path.join(HERE, "libttn.so"))

TTN_OK = 0
ERRORS = {-1: "TTN_E_INVALID", -2: "TTN_E_TREE", -3: "TTN_E_DIMS", -4: "TTN_E_OOM", -5: "TTN_E_DEVICE",
          -6: "TTN_E_NOCONV", -7: "TTN_E_STATE"}
TTN_FP64, TTN_FP32, TTN_BF16X3 = 0, 1, 2
OBS_EXPECT, OBS_NORM, OBS_ENERGY, OBS_OVERLAP_T0, OBS_BILINEAR = 0, 1, 2, 3, 4

# every symbol declared in include/ttn.h and include/ttn_debug.h
EXPORTED = ["ttn_default_options", "ttn_create", "ttn_set_sop", "ttn_set_product_state", "ttn_step",
            "ttn_ground_sweeps", "ttn_set_coefficients",
            "ttn_observe", "ttn_apply_root_heff", "ttn_get_info", "ttn_state_size", "ttn_get_state",
            "ttn_set_state", "ttn_last_error", "ttn_destroy", "ttn_debug_dense_tree_operator",
            "ttn_debug_clamp_bonds", "ttn_debug_qr", "ttn_profile_begin", "ttn_profile_end",
            "ttn_batch_create", "ttn_batch_step", "ttn_batch_last_error", "ttn_batch_destroy",
            "ttn_workspace_size", "ttn_release_process_resources", "ttn_debug_hermiticity_defect",
            "ttn_debug_tree_operator_stats", "ttn_get_step_solves", "ttn_qr_noalloc", "ttn_qr_noalloc_last_error",
            "ttn_tile_table_save", "ttn_tile_table_load", "ttn_tile_table_size", "ttn_tile_table_clear",
            "ttn_debug_graph_captures", "ttn_batch_set_lockstep"]


class Options(C.Structure):
    _fields_ = [("precision", C.c_int32), ("krylov_tol", C.c_double), ("krylov_mmax", C.c_int32),
                ("hermitian", C.c_int32), ("hip_stream", C.c_void_p), ("workspace", C.c_void_p),
                ("workspace_bytes", C.c_size_t), ("use_graph", C.c_int32), ("autotune", C.c_int32),
                ("device", C.c_int32), ("seed", C.c_uint64), ("spawn_tol", C.c_double),
                ("bond_max", C.POINTER(C.c_int32))]


class KernelStat(C.Structure):
    _fields_ = [("name", C.c_char * 48), ("calls", C.c_int64), ("total_ms", C.c_double), ("flops", C.c_double),
                ("bytes", C.c_double)]


class TTNError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


def _runtime_file(handle, symbol: bytes) -> str:
    """Path of the shared object that provides ``symbol`` as seen from ``handle``."""
    class DlInfo(C.Structure):
        _fields_ = [("dli_fname", C.c_char_p), ("dli_fbase", C.c_void_p), ("dli_sname", C.c_char_p),
                    ("dli_saddr", C.c_void_p)]
    libdl = C.CDLL(None)
    libdl.dlsym.restype = C.c_void_p
    libdl.dlsym.argtypes = [C.c_void_p, C.c_char_p]
    libdl.dladdr.argtypes = [C.c_void_p, C.POINTER(DlInfo)]
    addr = libdl.dlsym(handle, symbol)
    info = DlInfo()
    if not addr or not libdl.dladdr(addr, C.byref(info)) or not info.dli_fname:
        return ""
    return os.path.realpath(info.dli_fname.decode())


def _check_one_hip_runtime(lib) -> None:
    """The library must use the HIP runtime torch has loaded: one runtime per
    process (two would each own the device and tear it down twice at exit)."""
    import torch
    mine = _runtime_file(lib._handle, b"hipMalloc")
    torch_lib = os.path.join(os.path.dirname(torch.__file__), "lib", "libamdhip64.so")
    theirs = ""
    if os.path.exists(torch_lib):
        theirs = _runtime_file(C.CDLL(torch_lib)._handle, b"hipMalloc")
    mapped = set()
    with open("/proc/self/maps") as f:
        for line in f:
            parts = line.split()
            if len(parts) >= 6 and "libamdhip64" in parts[-1]:
                mapped.add(os.path.realpath(parts[-1]))
    if not mine or (theirs and mine != theirs) or len(mapped) > 1:
        raise ImportError(f"libttn.so would use the HIP runtime {mine or '?'} while torch uses "
                          f"{theirs or '?'} (mapped: {sorted(mapped)}): one runtime per process is required")


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"HIP library not built: {LIB_PATH} (run __graft_entry__.build())")
    # One HIP runtime per process: PyTorch ships its own libamdhip64 (same
    # SONAME as the system one the library links), and stream handles cross the
    # boundary.  Loading torch first makes the dynamic loader bind the library
    # to torch's runtime; the check below makes that an enforced invariant.
    import torch  # noqa: F401
    lib = C.CDLL(LIB_PATH)
    _check_one_hip_runtime(lib)
    P = C.c_void_p
    i32p, i64p, dp = C.POINTER(C.c_int32), C.POINTER(C.c_int64), C.POINTER(C.c_double)
    sig = {
        "ttn_default_options": (None, [C.POINTER(Options)]),
        "ttn_create": (C.c_int32, [C.c_int32, i32p, i32p, i32p, C.POINTER(Options), C.POINTER(P)]),
        "ttn_set_sop": (C.c_int32, [P, C.c_int32, i32p, i64p, dp, C.c_int32, dp, i64p, i32p]),
        "ttn_set_product_state": (C.c_int32, [P, dp]),
        "ttn_step": (C.c_int32, [P, C.c_double, C.c_int32]),
        "ttn_ground_sweeps": (C.c_int32, [P, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_int32)]),
        "ttn_set_coefficients": (C.c_int32, [P, C.c_int32, dp, C.POINTER(C.c_int32)]),
        "ttn_observe": (C.c_int32, [P, C.c_int32, C.c_int32, i32p, dp, dp]),
        "ttn_apply_root_heff": (C.c_int32, [P, dp, dp]),
        "ttn_get_info": (C.c_int32, [P, i32p, i64p]),
        "ttn_state_size": (C.c_int32, [P, C.POINTER(C.c_size_t)]),
        "ttn_get_state": (C.c_int32, [P, dp, C.c_size_t]),
        "ttn_set_state": (C.c_int32, [P, dp, C.c_size_t]),
        "ttn_last_error": (C.c_char_p, [P]),
        "ttn_destroy": (None, [P]),
        "ttn_debug_dense_tree_operator": (C.c_int32, [C.c_int32, i32p, i32p, C.c_int32, i32p, i64p, dp,
                                                      C.c_int32, dp, i64p, i32p, C.c_int64, dp, i64p]),
        "ttn_debug_clamp_bonds": (C.c_int32, [C.c_int32, i32p, i32p, i32p, i32p]),
        "ttn_debug_qr": (C.c_int32, [C.c_int64, C.c_int32, dp, C.c_int32, dp, dp]),
        "ttn_profile_begin": (C.c_int32, []),
        "ttn_profile_end": (C.c_int32, [C.POINTER(KernelStat), C.c_int32, C.POINTER(C.c_int32)]),
        "ttn_batch_create": (C.c_int32, [C.c_int32, C.POINTER(P), C.c_int32, C.POINTER(P)]),
        "ttn_batch_step": (C.c_int32, [P, dp, C.c_int32]),
        "ttn_batch_last_error": (C.c_char_p, [P]),
        "ttn_batch_destroy": (None, [P]),
        "ttn_workspace_size": (C.c_int32, [P, C.POINTER(C.c_size_t)]),
        "ttn_get_step_solves": (C.c_int32, [P, C.c_int32, i32p, i32p, i32p, i32p]),
        "ttn_tile_table_save": (C.c_int32, [C.c_char_p]),
        "ttn_tile_table_load": (C.c_int32, [C.c_char_p, i32p]),
        "ttn_tile_table_size": (C.c_int32, [i64p]),
        "ttn_tile_table_clear": (None, []),
        "ttn_debug_graph_captures": (C.c_int32, [P, i64p]),
        "ttn_batch_set_lockstep": (C.c_int32, [P, C.c_int32]),
        "ttn_debug_tree_operator_stats": (C.c_int32, [C.c_int32, i32p, i32p, C.c_int32, i32p, i64p, dp, C.c_int32,
                                                      dp, i64p, i32p, i32p, i32p, i32p, i32p]),
        "ttn_debug_hermiticity_defect": (C.c_int32, [C.c_int32, i32p, i32p, C.c_int32, i32p, i64p, dp, C.c_int32,
                                                     dp, i64p, i32p, dp]),
        "ttn_release_process_resources": (None, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


lib = _load()

# Handles still open at interpreter exit are destroyed by an exit hook, before
# module teardown and before the HIP runtime and any profiler attached to it
# shut down, and the library's process-wide resources are released after them.
_LIVE: "weakref.WeakSet" = weakref.WeakSet()


@atexit.register
def _release_at_exit():
    for obj in [o for o in list(_LIVE) if isinstance(o, TTNBatch)]:
        obj.close()
    for obj in list(_LIVE):
        obj.close()
    lib.ttn_release_process_resources()


def _ptr(a: np.ndarray, ctype):
    return a.ctypes.data_as(C.POINTER(ctype))


def _check(code: int, handle=None):
    if code != TTN_OK:
        msg = lib.ttn_last_error(handle)
        raise TTNError(code, msg.decode() if msg else "")


def clamp_bonds(parent, local_dim, bond_dim) -> np.ndarray:
    parent = np.ascontiguousarray(parent, dtype=np.int32)
    ld = np.ascontiguousarray(local_dim, dtype=np.int32)
    bd = np.ascontiguousarray(bond_dim, dtype=np.int32)
    out = np.zeros(len(parent), dtype=np.int32)
    _check(lib.ttn_debug_clamp_bonds(len(parent), _ptr(parent, C.c_int32), _ptr(ld, C.c_int32),
                                     _ptr(bd, C.c_int32), _ptr(out, C.c_int32)))
    return out


def dense_tree_operator(problem, max_dim: int = 4096):
    """Dense matrix of the compiled sparse tree operator (host only)."""
    parent = np.ascontiguousarray(problem.parent, dtype=np.int32)
    ld = np.ascontiguousarray(problem.local_dim, dtype=np.int32)
    op_leaf, off, data, coeff, tptr, tops = problem.flat_sop()
    dim = int(np.prod([problem.local_dim[l] for l in problem.leaves()]))
    out = np.zeros(2 * dim * dim, dtype=np.float64)
    nent = np.zeros(1, dtype=np.int64)
    _check(lib.ttn_debug_dense_tree_operator(
        len(parent), _ptr(parent, C.c_int32), _ptr(ld, C.c_int32), len(op_leaf), _ptr(op_leaf, C.c_int32),
        _ptr(off, C.c_int64), _ptr(data, C.c_double), len(problem.term_ops), _ptr(coeff, C.c_double),
        _ptr(tptr, C.c_int64), _ptr(tops, C.c_int32), max_dim, _ptr(out, C.c_double), _ptr(nent, C.c_int64)))
    return out.view(np.complex128).reshape(dim, dim), int(nent[0])


def tree_operator_stats(problem) -> Dict[str, np.ndarray]:
    """Per node of the compiled tree operator (host only): channels on the bond
    above it, operator entries, products after the node-form compression, and
    the plain-SOP terms crossing the bond above it."""
    parent = np.ascontiguousarray(problem.parent, dtype=np.int32)
    ld = np.ascontiguousarray(problem.local_dim, dtype=np.int32)
    op_leaf, off, data, coeff, tptr, tops = problem.flat_sop()
    out = {k: np.zeros(len(parent), dtype=np.int32) for k in ("channels", "entries", "merged", "sop_terms")}
    _check(lib.ttn_debug_tree_operator_stats(
        len(parent), _ptr(parent, C.c_int32), _ptr(ld, C.c_int32), len(op_leaf), _ptr(op_leaf, C.c_int32),
        _ptr(off, C.c_int64), _ptr(data, C.c_double), len(problem.term_ops), _ptr(coeff, C.c_double),
        _ptr(tptr, C.c_int64), _ptr(tops, C.c_int32), _ptr(out["channels"], C.c_int32),
        _ptr(out["entries"], C.c_int32), _ptr(out["merged"], C.c_int32), _ptr(out["sop_terms"], C.c_int32)))
    return out


def tile_table_save(path: str) -> None:
    """Write the process-wide tile table (autotuner results) as JSON."""
    _check(lib.ttn_tile_table_save(os.fsencode(path)))


def tile_table_load(path: str) -> int:
    """Merge a saved tile table into the process-wide one; returns the entries read."""
    n = C.c_int32()
    _check(lib.ttn_tile_table_load(os.fsencode(path), C.byref(n)))
    return int(n.value)


def tile_table_size() -> int:
    n = C.c_int64()
    _check(lib.ttn_tile_table_size(C.byref(n)))
    return int(n.value)


def tile_table_clear() -> None:
    lib.ttn_tile_table_clear()


def hermiticity_defect(problem) -> float:
    """||G - G^dag||_F / ||G||_F as the library checks it (host only)."""
    parent = np.ascontiguousarray(problem.parent, dtype=np.int32)
    ld = np.ascontiguousarray(problem.local_dim, dtype=np.int32)
    op_leaf, off, data, coeff, tptr, tops = problem.flat_sop()
    out = np.zeros(1, dtype=np.float64)
    _check(lib.ttn_debug_hermiticity_defect(
        len(parent), _ptr(parent, C.c_int32), _ptr(ld, C.c_int32), len(op_leaf), _ptr(op_leaf, C.c_int32),
        _ptr(off, C.c_int64), _ptr(data, C.c_double), len(problem.term_ops), _ptr(coeff, C.c_double),
        _ptr(tptr, C.c_int64), _ptr(tops, C.c_int32), _ptr(out, C.c_double)))
    return float(out[0])


def gpu_qr(M: np.ndarray, variant: int):
    """Q, R of the library's QR kernels (variant 0: one work-group, 1: many, 2:
    cooperative, 3: Cholesky route with the variant-1 kernels behind it, 4:
    Cholesky route alone, TTN_E_NOCONV outside its range)."""
    A = np.ascontiguousarray(M, dtype=np.complex128)
    rows, cols = A.shape
    Q = np.zeros_like(A)
    R = np.zeros((cols, cols), dtype=np.complex128)
    _check(lib.ttn_debug_qr(rows, cols, _ptr(A.view(np.float64), C.c_double), variant,
                            _ptr(Q.view(np.float64), C.c_double), _ptr(R.view(np.float64), C.c_double)))
    return Q, R


def profile_begin():
    """Start event timing of every kernel launch (process wide)."""
    _check(lib.ttn_profile_begin())


def profile_end() -> List[Dict[str, float]]:
    """Stop timing; per kernel name: calls, total_ms, flops, bytes."""
    rows = (KernelStat * 64)()
    n = C.c_int32()
    _check(lib.ttn_profile_end(rows, 64, C.byref(n)))
    return [dict(name=rows[i].name.decode(), calls=int(rows[i].calls), total_ms=rows[i].total_ms,
                 flops=rows[i].flops, bytes=rows[i].bytes) for i in range(min(n.value, 64))]


def tree_operator_entries(problem) -> int:
    """Number of sparse tree-operator entries (hSOP channels over all nodes), host only."""
    parent = np.ascontiguousarray(problem.parent, dtype=np.int32)
    ld = np.ascontiguousarray(problem.local_dim, dtype=np.int32)
    op_leaf, off, data, coeff, tptr, tops = problem.flat_sop()
    out = np.zeros(2, dtype=np.float64)
    nent = np.zeros(1, dtype=np.int64)
    lib.ttn_debug_dense_tree_operator(
        len(parent), _ptr(parent, C.c_int32), _ptr(ld, C.c_int32), len(op_leaf), _ptr(op_leaf, C.c_int32),
        _ptr(off, C.c_int64), _ptr(data, C.c_double), len(problem.term_ops), _ptr(coeff, C.c_double),
        _ptr(tptr, C.c_int64), _ptr(tops, C.c_int32), 0, _ptr(out, C.c_double), _ptr(nent, C.c_int64))
    return int(nent[0])


def default_stream() -> Optional[int]:
    """HIP stream handle of torch's current stream (torch provides streams), if any."""
    try:
        import torch
        if torch.cuda.is_available():
            return int(torch.cuda.current_stream().cuda_stream)
    except Exception:
        pass
    return None


class TTN:
    """One tree tensor network on the GPU, driven through the C boundary."""

    def __init__(self, parent, local_dim, bond_dim, precision: int = TTN_FP64, krylov_tol: float = 0.0,
                 krylov_mmax: int = 40, hermitian: bool = True, stream: Optional[int] = None, device: int = 0,
                 workspace: Optional[Tuple[int, int]] = None, spawn_tol: float = 0.0, bond_max=None,
                 seed: int = 0, autotune: bool = False, use_graph: bool = False):
        self.parent = np.ascontiguousarray(parent, dtype=np.int32)
        self.local_dim = np.ascontiguousarray(local_dim, dtype=np.int32)
        bond = np.ascontiguousarray(bond_dim, dtype=np.int32)
        opt = Options()
        lib.ttn_default_options(C.byref(opt))
        opt.precision = precision
        opt.krylov_tol = krylov_tol
        opt.krylov_mmax = krylov_mmax
        opt.hermitian = 1 if hermitian else 0
        opt.hip_stream = stream if stream is not None else default_stream()
        opt.device = device
        if workspace is not None:  # (device pointer, bytes), caller-owned
            opt.workspace = int(workspace[0])
            opt.workspace_bytes = int(workspace[1])
        opt.spawn_tol = float(spawn_tol)
        opt.autotune = 1 if autotune else 0
        opt.use_graph = 1 if use_graph else 0
        opt.seed = int(seed)
        if bond_max is not None:  # subspace expansion: per-node largest bonds
            bm = np.ascontiguousarray(np.broadcast_to(np.asarray(bond_max, dtype=np.int32), self.parent.shape))
            opt.bond_max = _ptr(bm, C.c_int32)
        h = C.c_void_p()
        _check(lib.ttn_create(len(self.parent), _ptr(self.parent, C.c_int32), _ptr(self.local_dim, C.c_int32),
                              _ptr(bond, C.c_int32), C.byref(opt), C.byref(h)))
        self.h = h
        self.n = len(self.parent)
        _LIVE.add(self)

    @classmethod
    def from_problem(cls, p, bond_dim=None, **kw):
        t = cls(p.parent, p.local_dim, p.bond_dim if bond_dim is None else bond_dim,
                hermitian=kw.pop("hermitian", p.hermitian), **kw)
        t.set_sop_problem(p)
        return t

    def close(self):
        if getattr(self, "h", None):
            lib.ttn_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()

    def _c(self, code):
        _check(code, self.h)

    def set_sop_problem(self, p):
        self._op_leaf = list(p.op_leaf)
        op_leaf, off, data, coeff, tptr, tops = p.flat_sop()
        self._c(lib.ttn_set_sop(self.h, len(op_leaf), _ptr(op_leaf, C.c_int32), _ptr(off, C.c_int64),
                                _ptr(data, C.c_double), len(p.term_ops), _ptr(coeff, C.c_double),
                                _ptr(tptr, C.c_int64), _ptr(tops, C.c_int32)))

    def set_coefficients(self, coeff) -> bool:
        """New coefficients for the terms in place (one complex value per
        term, in term order); returns True if the operator was rebuilt."""
        c = np.ascontiguousarray(coeff, dtype=np.complex128)
        rebuilt = C.c_int32()
        self._c(lib.ttn_set_coefficients(self.h, len(c), _ptr(c.view(np.float64), C.c_double), C.byref(rebuilt)))
        return bool(rebuilt.value)

    def step_td(self, dt: float, coef_at, t: float, n_steps: int = 1) -> float:
        """n_steps steps of dt from time t of a generator whose coefficients
        depend on time: before every step the coefficients coef_at(t + dt/2)
        (the midpoint of that step) are set.  Returns the time reached."""
        for _ in range(int(n_steps)):
            self.set_coefficients(coef_at(t + 0.5 * dt))
            self.step(dt)
            t += dt
        return t

    def set_product_state(self, vecs: Dict[int, np.ndarray]):
        leaves = [z for z in range(self.n) if self.local_dim[z] > 0]
        flat = np.ascontiguousarray(np.concatenate([np.asarray(vecs[z], dtype=np.complex128) for z in leaves]))
        self._c(lib.ttn_set_product_state(self.h, _ptr(flat.view(np.float64), C.c_double)))

    def step(self, dt: float, n_steps: int = 1):
        self._c(lib.ttn_step(self.h, float(dt), int(n_steps)))

    def ground_sweeps(self, n_sweeps: int = 1, unconverged: bool = False):
        """n one-site ground-state sweeps (DMRG on trees); returns the energy
        <Psi|G|Psi> / <Psi|Psi> after them (and the number of fused local
        solves left above the tolerance when unconverged=True)."""
        e = C.c_double()
        bad = C.c_int32()
        self._c(lib.ttn_ground_sweeps(self.h, int(n_sweeps), C.byref(e), C.byref(bad)))
        return (e.value, bad.value) if unconverged else e.value

    def _obs(self, kind, ids=(), vecs=None) -> complex:
        arr = np.ascontiguousarray(ids, dtype=np.int32) if len(ids) else np.zeros(1, dtype=np.int32)
        out = np.zeros(2, dtype=np.float64)
        vp = _ptr(vecs, C.c_double) if vecs is not None else None
        self._c(lib.ttn_observe(self.h, kind, len(ids), _ptr(arr, C.c_int32), vp, _ptr(out, C.c_double)))
        return complex(out[0], out[1])

    def expect(self, op_ids: Sequence[int]) -> complex:
        return self._obs(OBS_EXPECT, list(op_ids))

    def norm2(self) -> float:
        return self._obs(OBS_NORM).real

    def energy(self) -> complex:
        return self._obs(OBS_ENERGY)

    def overlap_t0(self) -> complex:
        return self._obs(OBS_OVERLAP_T0)

    def bilinear(self, vecs: Dict[int, np.ndarray]) -> complex:
        leaves = [z for z in range(self.n) if self.local_dim[z] > 0]
        flat = np.ascontiguousarray(np.concatenate([np.asarray(vecs[z], dtype=np.complex128) for z in leaves]))
        return self._obs(OBS_BILINEAR, [], flat.view(np.float64))

    def apply_root_heff(self, x: np.ndarray) -> np.ndarray:
        xin = np.ascontiguousarray(x, dtype=np.complex128)
        y = np.zeros_like(xin)
        self._c(lib.ttn_apply_root_heff(self.h, _ptr(xin.view(np.float64), C.c_double),
                                        _ptr(y.view(np.float64), C.c_double)))
        return y

    def workspace_size(self) -> int:
        """Scratch bytes the current operator needs (a caller workspace's size)."""
        b = C.c_size_t()
        self._c(lib.ttn_workspace_size(self.h, C.byref(b)))
        return int(b.value)

    def step_solves(self):
        """(node, forward flag, matvecs) of every local exponential of the last step."""
        cap = 4 * self.n + 8
        node, fwd, mv = (np.zeros(cap, dtype=np.int32) for _ in range(3))
        n = C.c_int32()
        self._c(lib.ttn_get_step_solves(self.h, cap, _ptr(node, C.c_int32), _ptr(fwd, C.c_int32),
                                        _ptr(mv, C.c_int32), C.byref(n)))
        k = min(n.value, cap)
        return node[:k], fwd[:k], mv[:k]

    def graph_captures(self) -> int:
        """Step graphs captured so far (use_graph handles)."""
        n = C.c_int64()
        self._c(lib.ttn_debug_graph_captures(self.h, C.byref(n)))
        return int(n.value)

    def bonds(self) -> np.ndarray:
        b = np.zeros(self.n, dtype=np.int32)
        self._c(lib.ttn_get_info(self.h, _ptr(b, C.c_int32), None))
        return b

    def counters(self) -> Dict[str, int]:
        c = np.zeros(8, dtype=np.int64)
        self._c(lib.ttn_get_info(self.h, None, _ptr(c, C.c_int64)))
        keys = ["steps", "forward_solves", "backward_solves", "matvecs", "heff_flops", "device_bytes",
                "tree_op_entries", "redo"]
        return dict(zip(keys, (int(x) for x in c)))

    def shapes(self) -> List[List[int]]:
        b = self.bonds()
        kids = [[c for c in range(self.n) if self.parent[c] == z] for z in range(self.n)]
        out = []
        for z in range(self.n):
            dims = [int(self.local_dim[z])] if self.local_dim[z] > 0 else [int(b[c]) for c in kids[z]]
            out.append(dims + [int(b[z]) if self.parent[z] >= 0 else 1])
        return out

    def get_state(self) -> List[np.ndarray]:
        size = C.c_size_t()
        self._c(lib.ttn_state_size(self.h, C.byref(size)))
        buf = np.zeros(size.value // 8, dtype=np.float64)
        self._c(lib.ttn_get_state(self.h, _ptr(buf, C.c_double), size.value))
        flat = buf.view(np.complex128)
        out, off = [], 0
        for shp in self.shapes():
            n = int(np.prod(shp))
            out.append(flat[off:off + n].reshape(shp).copy())
            off += n
        return out

    def set_state(self, tensors: Sequence[np.ndarray]):
        flat = np.ascontiguousarray(np.concatenate([np.asarray(t, dtype=np.complex128).reshape(-1)
                                                    for t in tensors]))
        self._c(lib.ttn_set_state(self.h, _ptr(flat.view(np.float64), C.c_double), flat.nbytes))


class TTNBatch:
    """Instances advanced together (``ttn_batch_*``): their sweeps overlap on
    the device through the batch's HIP streams.  The TTN objects stay usable
    (observables, states) and must outlive the batch."""

    def __init__(self, insts: Sequence[TTN], n_streams: int = 0, lockstep: bool = False):
        self.insts = list(insts)
        arr = (C.c_void_p * len(self.insts))(*[t.h.value if isinstance(t.h, C.c_void_p) else t.h
                                               for t in self.insts])
        h = C.c_void_p()
        code = lib.ttn_batch_create(len(self.insts), arr, int(n_streams), C.byref(h))
        if code != TTN_OK:
            raise TTNError(code, lib.ttn_batch_last_error(None).decode())
        self.h = h
        _LIVE.add(self)
        if lockstep:
            code = lib.ttn_batch_set_lockstep(self.h, 1)
            if code != TTN_OK:
                raise TTNError(code, lib.ttn_batch_last_error(None).decode())

    def step(self, dt, n_steps: int = 1):
        dts = np.ascontiguousarray(np.broadcast_to(np.asarray(dt, dtype=np.float64), (len(self.insts),)))
        code = lib.ttn_batch_step(self.h, _ptr(dts, C.c_double), int(n_steps))
        if code != TTN_OK:
            raise TTNError(code, lib.ttn_batch_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            lib.ttn_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()
