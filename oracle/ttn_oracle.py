"""Plain CPU complex128 one-site TDVP (projector-splitting) sweep of a tree tensor network.

TEST INFRASTRUCTURE ONLY.  This is the reference the HIP library is checked
against; it is written for readability, not speed, and shares no code with the
library.  Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg
of ``bench.py`` may use it.

What it follows (paper: pyTTN, arXiv 2503.15460):

* Tree tensor network ansatz, Sec. II A (Eqs. for the wavefunction expansion,
  the SPF recursion and the SHF recursion).  Node ``z`` holds ``A^z`` with the
  children's indices first (node-id order) and the parent index last; a leaf
  holds ``(d, n)``; the root's parent index has dimension 1.
* SOP Hamiltonian, Sec. II B 1 (Eq. for the SOP form and the node-wise split
  into single-particle and mean-field operators).  This oracle keeps every
  term that crosses a node individually and aggregates only the terms lying
  entirely inside one child subtree and the terms lying entirely outside the
  node (the classical ML-MCTDH treatment).
* SPO and mean-field matrices, Sec. II C (the two projections of h_r^z and
  H_r^z onto the SPFs and SHFs) and the local equation of motion
  ``dA/dt = -i sum_r c_r h_r A H_r`` of Sec. II C, read with the transpose on
  the parent index: ``(H_eff A)_{I,i} = sum c_r h_{IJ} H_{ij} A_{J,j}``.
* The projector-splitting sweep (Sec. II C; details deferred by the paper to
  its TDVP references) read as the symmetric second-order sweep S(dt/2)
  followed by its mirror S*(dt/2), children in increasing id order in S and in
  decreasing order in S*, with the two root forward half steps merged into
  one full step.
* QR gauge shifts by Householder reflections in the LAPACK convention, with a
  relative zero-snap of 1e-12 for the rank-deficient factors of product states.
* Local exponentials: dense ``expm`` for local problems up to ``dense_max``
  unknowns, otherwise Lanczos (Hermitian) or Arnoldi (non-Hermitian) with full
  re-orthogonalisation and an a-posteriori error estimate.
* Time-dependent coefficients (Sec. II B; the interaction-picture chain form
  of Sec. II E 2): the paper does not state how a step treats them; read here
  as coefficients frozen at the midpoint of each step (``step_td``).

Readings of points the paper leaves open are listed in the repository's design
notes; in short: unoccupied SPFs of a product state are completed with unit
vectors (modified Gram-Schmidt at the leaves), bond dimensions are clamped to
what the tree can support, observables are returned raw (not renormalised).
"""
from __future__ import annotations

from typing import Callable, Dict, List, Optional, Sequence

import numpy as np
import scipy.linalg as sla

# --------------------------------------------------------------------- tree
def _children(parent: Sequence[int]) -> List[List[int]]:
    n = len(parent)
    kids: List[List[int]] = [[] for _ in range(n)]
    for c in range(n):
        if parent[c] >= 0:
            kids[parent[c]].append(c)
    return kids


def _leaf_sets(parent, local_dim) -> List[frozenset]:
    kids = _children(parent)
    n = len(parent)
    out: List[Optional[frozenset]] = [None] * n

    def rec(z):
        if local_dim[z] > 0:
            out[z] = frozenset([z])
        else:
            s = set()
            for c in kids[z]:
                rec(c)
                s |= out[c]
            out[z] = frozenset(s)
    root = [z for z in range(n) if parent[z] < 0][0]
    rec(root)
    return out  # type: ignore


def clamp_bonds(parent, local_dim, requested) -> np.ndarray:
    """Effective bond dimensions (reading of the paper's N_i = min(16, N_i)).

    First ``n_e = min(requested, prod dims inside, prod dims outside)``, then
    ``n_e <- min(n_e, prod of the other bonds at each end node)`` (a leaf's
    other "bond" is its physical index) until nothing changes, so that every
    matricisation used by the sweep has at least as many rows as columns.
    """
    parent = [int(p) for p in parent]
    local_dim = [int(d) for d in local_dim]
    n = len(parent)
    kids = _children(parent)
    sets = _leaf_sets(parent, local_dim)
    total = float(np.prod([float(local_dim[z]) for z in range(n) if local_dim[z] > 0]))
    b = [1] * n
    for c in range(n):
        if parent[c] < 0:
            continue
        inside = float(np.prod([float(local_dim[l]) for l in sets[c]]))
        b[c] = int(min(float(requested[c]), inside, total / inside))
    changed = True
    while changed:
        changed = False
        for z in range(n):
            inc = []  # (bond owner, dim) of every index of A^z
            if local_dim[z] > 0:
                inc.append((None, local_dim[z]))
            else:
                inc += [(c, b[c]) for c in kids[z]]
            if parent[z] >= 0:
                inc.append((z, b[z]))
            for i, (owner, dim) in enumerate(inc):
                if owner is None:
                    continue
                other = 1.0
                for j, (_, dj) in enumerate(inc):
                    if j != i:
                        other *= dj
                if dim > other:
                    b[owner] = int(other)
                    changed = True
    return np.asarray(b, dtype=np.int32)


# ---------------------------------------------------------------- helpers
def mode_product(A: np.ndarray, M: np.ndarray, axis: int) -> np.ndarray:
    """(A x_axis M)_{..i..} = sum_j M_{ij} A_{..j..}."""
    return np.moveaxis(np.tensordot(M, A, axes=([1], [axis])), 0, axis)


def contract_except(A: np.ndarray, B: np.ndarray, axis: int) -> np.ndarray:
    """M_{mn} = sum over every index but ``axis`` of conj(A)_{..m..} B_{..n..}."""
    a = np.moveaxis(A, axis, -1).reshape(-1, A.shape[axis])
    b = np.moveaxis(B, axis, -1).reshape(-1, B.shape[axis])
    return a.conj().T @ b


SNAP = 1e-12  # relative zero-snap of the QR (reading of the unstated QR convention)


def householder_qr_lapack(M: np.ndarray, snap: float = 0.0):
    """Thin QR by Householder reflections in the LAPACK zgeqr2/zung2r convention.

    Each reflector is ``H = I - tau v v^H`` with ``v_0 = 1``; for a column
    ``(alpha, x)``: if ``x == 0`` and ``Im alpha == 0`` then ``tau = 0``,
    otherwise ``beta = -sign(Re alpha) |(alpha, x)|``, ``tau = (beta -
    alpha)/beta``, ``v = (1, x/(alpha - beta))``.  The factorisation applies
    ``H^H`` to the trailing columns and ``Q = H_1 ... H_n`` restricted to the
    first ``n`` columns.  Plain loops.

    ``snap > 0``: a sub-column with ``|x| <= snap |M|_F`` is set to exactly zero
    (and so is ``Im alpha`` when ``|Im alpha| <= snap |M|_F``) before the
    reflector is formed, so that rounding noise in structurally empty columns
    cannot choose the completion of a rank-deficient factor.  ``snap = 0`` is
    plain LAPACK (pinned against numpy.linalg.qr).
    """
    A = np.array(M, dtype=np.complex128, copy=True)
    m, n = A.shape
    k = min(m, n)
    thr = snap * np.linalg.norm(A)
    taus = np.zeros(k, dtype=np.complex128)
    for i in range(k):
        x = A[i + 1:, i]
        xnorm = np.linalg.norm(x)
        if snap > 0.0 and xnorm <= thr:
            A[i + 1:, i] = 0.0
            xnorm = 0.0
            if abs(A[i, i].imag) <= thr:
                A[i, i] = A[i, i].real
        alpha = A[i, i]
        x = A[i + 1:, i]
        if xnorm == 0.0 and alpha.imag == 0.0:
            tau = 0.0
        else:
            beta = -np.copysign(np.sqrt(abs(alpha) ** 2 + xnorm ** 2), alpha.real)
            tau = complex((beta - alpha.real) / beta, -alpha.imag / beta)
            A[i + 1:, i] = x / (alpha - beta)
            A[i, i] = beta
        taus[i] = tau
        v = np.concatenate([[1.0], A[i + 1:, i]])
        if i + 1 < n:
            w = v.conj() @ A[i:, i + 1:]
            A[i:, i + 1:] -= np.conj(tau) * np.outer(v, w)
    R = np.triu(A[:k, :n])
    Q = np.zeros((m, k), dtype=np.complex128)
    Q[:k, :k] = np.eye(k)
    for i in range(k - 1, -1, -1):
        v = np.concatenate([[1.0], A[i + 1:, i]])
        w = v.conj() @ Q[i:, i:]
        Q[i:, i:] -= taus[i] * np.outer(v, w)
    return Q, R


def expm_krylov(apply: Callable[[np.ndarray], np.ndarray], v: np.ndarray, tau: float,
                hermitian: bool = True, tol: float = 1e-13, mmax: int = 40, dense_max: int = 512,
                counter: Optional[list] = None, _depth: int = 0) -> np.ndarray:
    """``exp(-i tau G) v`` for the linear map ``apply = G``.

    Dense ``scipy.linalg.expm`` for ``v.size <= dense_max``; otherwise Lanczos
    (Hermitian G: tridiagonal projection with full re-orthogonalisation) or
    Arnoldi.  Converged when the estimate ``|v| * h_{m+1,m} * |[exp(-i tau
    T_m) e_1]_m| <= tol * |v|``; otherwise the step is halved (up to 8 times).
    """
    shape = v.shape
    x = v.reshape(-1)
    n = x.size
    if n <= dense_max:
        G = np.empty((n, n), dtype=np.complex128)
        for j in range(n):
            e = np.zeros(n, dtype=np.complex128)
            e[j] = 1.0
            G[:, j] = apply(e.reshape(shape)).reshape(-1)
        if counter is not None:
            counter[0] += n
        return (sla.expm(-1j * tau * G) @ x).reshape(shape)
    beta0 = np.linalg.norm(x)
    if beta0 == 0.0:
        return v.copy()
    m_cap = min(mmax, n)
    V = np.zeros((m_cap + 1, n), dtype=np.complex128)
    Hm = np.zeros((m_cap + 1, m_cap), dtype=np.complex128)
    V[0] = x / beta0
    for j in range(m_cap):
        w = apply(V[j].reshape(shape)).reshape(-1).astype(np.complex128)
        if counter is not None:
            counter[0] += 1
        if hermitian:
            a = np.vdot(V[j], w)
            Hm[j, j] = a.real
            w = w - a.real * V[j]
            if j > 0:
                w = w - Hm[j - 1, j] * V[j - 1]
            for _ in range(2):  # full re-orthogonalisation (twice is enough)
                w = w - V[: j + 1].T @ (V[: j + 1].conj() @ w)
        else:
            for _ in range(2):
                h = V[: j + 1].conj() @ w
                Hm[: j + 1, j] += h
                w = w - V[: j + 1].T @ h
        b = np.linalg.norm(w)
        Hm[j + 1, j] = b
        if hermitian and j + 1 < m_cap:
            Hm[j, j + 1] = b
        T = Hm[: j + 1, : j + 1]
        y = sla.expm(-1j * tau * T)[:, 0]
        err = beta0 * b * abs(y[j])
        if b <= 1e-14 * beta0 or err <= tol * beta0:
            return (beta0 * (V[: j + 1].T @ y)).reshape(shape)
        V[j + 1] = w / b
    if _depth >= 8:
        raise RuntimeError("Krylov exponential did not converge")
    half = expm_krylov(apply, v, tau / 2, hermitian, tol, mmax, dense_max, counter, _depth + 1)
    return expm_krylov(apply, half, tau / 2, hermitian, tol, mmax, dense_max, counter, _depth + 1)


def dense_sop(problem) -> np.ndarray:
    """Dense generator ``sum_r c_r (x)_leaves h_{leaf,r}`` (leaves in depth-first order)."""
    leaves = leaf_order([int(x) for x in problem.parent], [int(x) for x in problem.local_dim])
    dims = [int(problem.local_dim[l]) for l in leaves]
    N = int(np.prod(dims))
    G = np.zeros((N, N), dtype=np.complex128)
    for c, ops in zip(problem.coeff, problem.term_ops):
        byleaf = {problem.op_leaf[o]: problem.op_mats[o] for o in ops}
        M = np.ones((1, 1), dtype=np.complex128)
        for l, d in zip(leaves, dims):
            M = np.kron(M, byleaf.get(l, np.eye(d)))
        G += c * M
    return G


def leaf_order(parent, local_dim) -> List[int]:
    """Leaves in depth-first order with children visited in id order."""
    kids = _children(parent)
    root = [z for z in range(len(parent)) if parent[z] < 0][0]
    out: List[int] = []

    def rec(z):
        if local_dim[z] > 0:
            out.append(z)
        for c in kids[z]:
            rec(c)
    rec(root)
    return out


def full_state(parent, local_dim, tensors) -> np.ndarray:
    """Contract a TTN into the dense state vector (leaves in depth-first order)."""
    kids = _children(parent)
    root = [z for z in range(len(parent)) if parent[z] < 0][0]

    def rec(z):
        # returns an array (leaf dims of the subtree..., n_z)
        if local_dim[z] > 0:
            return tensors[z]
        T = tensors[z]
        pos = 0
        for c in kids[z]:
            sub = rec(c)
            lead = sub.ndim - 1
            T = np.tensordot(sub, T, axes=([lead], [pos]))
            T = np.moveaxis(T, list(range(lead)), list(range(pos, pos + lead)))
            pos += lead
        return T
    return rec(root).reshape(-1)


# ------------------------------------------------------------------ oracle
class Oracle:
    """One-site TDVP sweep on a tree tensor network, complex128, CPU."""

    def __init__(self, problem, bond_dim=None, tol: float = 1e-13, mmax: int = 40,
                 dense_max: int = 0, hermitian: Optional[bool] = None):
        p = problem
        self.p = p
        self.parent = [int(x) for x in p.parent]
        self.local_dim = [int(x) for x in p.local_dim]
        self.n = len(self.parent)
        self.kids = _children(self.parent)
        self.root = [z for z in range(self.n) if self.parent[z] < 0][0]
        req = p.bond_dim if bond_dim is None else bond_dim
        self.bond = clamp_bonds(self.parent, self.local_dim, req)
        self.tol, self.mmax, self.dense_max = tol, mmax, dense_max
        self.hermitian = p.hermitian if hermitian is None else hermitian
        self.sets = _leaf_sets(self.parent, self.local_dim)
        # terms: coefficient and leaf -> operator matrix
        self.coef = np.asarray(p.coeff, dtype=np.complex128)
        self.terms: List[Dict[int, np.ndarray]] = []
        for ops in p.term_ops:
            if len(ops) == 0:
                raise ValueError("terms without operators are not supported")
            self.terms.append({p.op_leaf[o]: np.asarray(p.op_mats[o]) for o in ops})
        self.supp = [frozenset(t.keys()) for t in self.terms]
        self.A: List[Optional[np.ndarray]] = [None] * self.n
        self.A0: List[Optional[np.ndarray]] = [None] * self.n
        self.spo: List[Dict[object, np.ndarray]] = [dict() for _ in range(self.n)]
        self.mf: List[Dict[object, np.ndarray]] = [dict() for _ in range(self.n)]
        self.matvecs = [0]
        self.time = 0.0

    # ----------------------------------------------------- term geometry
    def touches(self, r: int, c: int) -> bool:
        return not self.supp[r].isdisjoint(self.sets[c])

    def inside(self, r: int, c: int) -> bool:
        return self.supp[r] <= self.sets[c]

    def crossing(self, r: int, c: int) -> bool:
        return self.touches(r, c) and not self.inside(r, c)

    def touches_outside(self, r: int, z: int) -> bool:
        return not self.supp[r] <= self.sets[z]

    # ------------------------------------------------------------ state
    def shape(self, z: int):
        dims = [self.local_dim[z]] if self.local_dim[z] > 0 else [int(self.bond[c]) for c in self.kids[z]]
        return dims + [int(self.bond[z]) if z != self.root else 1]

    def set_product_state(self, vecs: Dict[int, np.ndarray]) -> None:
        """Product state with unoccupied SPFs completed by unit vectors.

        Leaf: column 0 is the normalised vector, further columns are modified
        Gram-Schmidt of e_0, e_1, ... against the previous columns (vectors
        whose residual norm is below 1e-6 are skipped).  Interior node:
        matricised (children x parent) it is the first ``n`` columns of the
        identity.  The root is e_(0,...,0).
        """
        for z in range(self.n):
            shp = self.shape(z)
            if self.local_dim[z] > 0:
                d, nb = shp
                v = np.asarray(vecs[z], dtype=np.complex128)
                cols = [v / np.linalg.norm(v)]
                j = 0
                while len(cols) < nb:
                    e = np.zeros(d, dtype=np.complex128)
                    e[j] = 1.0
                    for q in cols:
                        e = e - np.vdot(q, e) * q
                    nr = np.linalg.norm(e)
                    if nr > 1e-6:
                        cols.append(e / nr)
                    j += 1
                self.A[z] = np.stack(cols, axis=1)
            else:
                rows = int(np.prod(shp[:-1]))
                self.A[z] = np.eye(rows, shp[-1], dtype=np.complex128).reshape(shp)
        self._after_state_set()

    def set_state(self, tensors: Sequence[np.ndarray]) -> None:
        """Arbitrary TTN; every non-root node must be an isometry toward its parent."""
        for z in range(self.n):
            t = np.asarray(tensors[z], dtype=np.complex128)
            if list(t.shape) != self.shape(z):
                raise ValueError(f"node {z}: shape {t.shape} != {self.shape(z)}")
            self.A[z] = t.copy()
        self._after_state_set()

    def _after_state_set(self):
        self.A0 = [a.copy() for a in self.A]
        self.time = 0.0
        self.build_all_spos()

    def state(self) -> List[np.ndarray]:
        return [a.copy() for a in self.A]

    def postorder(self) -> List[int]:
        out: List[int] = []

        def rec(z):
            for c in self.kids[z]:
                rec(c)
            out.append(z)
        rec(self.root)
        return out

    def build_all_spos(self):
        for z in self.postorder():
            if z != self.root:
                self.build_spo(z)

    # ----------------------------------------------------- environments
    def _apply_factors(self, X: np.ndarray, factors: Dict[int, np.ndarray]) -> np.ndarray:
        for axis, M in factors.items():
            X = mode_product(X, M, axis)
        return X

    def build_spo(self, c: int) -> None:
        """SPO matrices of node c (Sec. II C: h_r = <Phi|h_r|Phi> via the SPF recursion)."""
        A = self.A[c]
        pax = A.ndim - 1
        out: Dict[object, np.ndarray] = {}
        if self.local_dim[c] > 0:
            inside = [r for r in range(len(self.terms)) if self.inside(r, c)]
            if inside:
                h = sum(self.coef[r] * self.terms[r][c] for r in inside)
                out["in"] = contract_except(A, mode_product(A, h, 0), pax)
            for r in range(len(self.terms)):
                if self.crossing(r, c):
                    out[r] = contract_except(A, mode_product(A, self.terms[r][c], 0), pax)
        else:
            kids = self.kids[c]
            acc = None
            for k, ck in enumerate(kids):
                if "in" in self.spo[ck]:
                    t = mode_product(A, self.spo[ck]["in"], k)
                    acc = t if acc is None else acc + t
            for r in range(len(self.terms)):
                if self.inside(r, c) and not any(self.inside(r, ck) for ck in kids):
                    f = {k: self.spo[ck][r] for k, ck in enumerate(kids) if self.touches(r, ck)}
                    t = self.coef[r] * self._apply_factors(A, f)
                    acc = t if acc is None else acc + t
            if acc is not None:
                out["in"] = contract_except(A, acc, pax)
            for r in range(len(self.terms)):
                if self.crossing(r, c):
                    f = {k: self.spo[ck][r] for k, ck in enumerate(kids) if self.touches(r, ck)}
                    out[r] = contract_except(A, self._apply_factors(A, f), pax)
        self.spo[c] = out

    def build_mf(self, z: int, k: int) -> None:
        """Mean-field matrices of child k of z (Sec. II C, via the SHF recursion)."""
        A = self.A[z]
        kids = self.kids[z]
        c = kids[k]
        pax = A.ndim - 1
        is_root = z == self.root
        out: Dict[object, np.ndarray] = {}

        def factors(r):
            f = {}
            if not is_root and self.touches_outside(r, z):
                f[pax] = self.mf[z][r]
            for j, cj in enumerate(kids):
                if j != k and self.touches(r, cj):
                    f[j] = self.spo[cj][r]
            return f

        acc = None
        if not is_root and "out" in self.mf[z]:
            acc = mode_product(A, self.mf[z]["out"], pax)
        for j, cj in enumerate(kids):
            if j != k and "in" in self.spo[cj]:
                t = mode_product(A, self.spo[cj]["in"], j)
                acc = t if acc is None else acc + t
        for r in range(len(self.terms)):
            if self.touches(r, c):
                continue
            slots = sum(1 for j, cj in enumerate(kids) if j != k and self.touches(r, cj))
            slots += 1 if (not is_root and self.touches_outside(r, z)) else 0
            if slots >= 2:
                t = self.coef[r] * self._apply_factors(A, factors(r))
                acc = t if acc is None else acc + t
        if acc is not None:
            out["out"] = contract_except(A, acc, k)
        for r in range(len(self.terms)):
            if self.crossing(r, c):
                out[r] = contract_except(A, self._apply_factors(A, factors(r)), k)
        self.mf[c] = out

    # ------------------------------------------------- local operators
    def heff(self, z: int, X: np.ndarray) -> np.ndarray:
        """Effective generator at node z applied to X (local EOM of Sec. II C)."""
        pax = X.ndim - 1
        is_root = z == self.root
        Y = np.zeros_like(X)
        if self.local_dim[z] > 0:
            loc = [r for r in range(len(self.terms)) if self.inside(r, z)]
            if loc:
                h = sum(self.coef[r] * self.terms[r][z] for r in loc)
                Y += mode_product(X, h, 0)
            if "out" in self.mf[z]:
                Y += mode_product(X, self.mf[z]["out"], pax)
            for r in range(len(self.terms)):
                if self.crossing(r, z):
                    Y += self.coef[r] * mode_product(mode_product(X, self.terms[r][z], 0),
                                                     self.mf[z][r], pax)
            return Y
        kids = self.kids[z]
        for k, ck in enumerate(kids):
            if "in" in self.spo[ck]:
                Y += mode_product(X, self.spo[ck]["in"], k)
        if not is_root and "out" in self.mf[z]:
            Y += mode_product(X, self.mf[z]["out"], pax)
        for r in range(len(self.terms)):
            f = {k: self.spo[ck][r] for k, ck in enumerate(kids)
                 if self.touches(r, ck) and not self.inside(r, ck)}
            inside_one = any(self.inside(r, ck) for ck in kids)
            if inside_one:
                continue
            if not is_root and self.touches_outside(r, z):
                if not f:
                    continue  # entirely outside z: part of mf["out"]
                f[pax] = self.mf[z][r]
            if len(f) == 0:
                continue
            Y += self.coef[r] * self._apply_factors(X, f)
        return Y

    def keff(self, c: int, C: np.ndarray) -> np.ndarray:
        """Bond generator K(C) = sum_r c_r h_r C H_r^T on the bond above node c."""
        Y = np.zeros_like(C)
        if "in" in self.spo[c]:
            Y += self.spo[c]["in"] @ C
        if "out" in self.mf[c]:
            Y += C @ self.mf[c]["out"].T
        for r in range(len(self.terms)):
            if self.crossing(r, c):
                Y += self.coef[r] * (self.spo[c][r] @ C @ self.mf[c][r].T)
        return Y

    def _expm(self, apply, X, tau):
        return expm_krylov(apply, X, tau, hermitian=self.hermitian, tol=self.tol, mmax=self.mmax,
                           dense_max=self.dense_max, counter=self.matvecs)

    def forward(self, z: int, h: float) -> None:
        self.A[z] = self._expm(lambda X: self.heff(z, X), self.A[z], h)

    def backward(self, c: int, C: np.ndarray, h: float) -> np.ndarray:
        return self._expm(lambda X: self.keff(c, X), C, -h)

    # ---------------------------------------------------------- gauge
    @staticmethod
    def qr_along(A: np.ndarray, axis: int):
        """QR of A matricised with ``axis`` as the columns (rows: other indices in order).

        LAPACK-convention Householder with the relative zero-snap ``SNAP``.
        """
        M = np.moveaxis(A, axis, -1)
        shp = M.shape
        Q, R = householder_qr_lapack(M.reshape(-1, shp[-1]), snap=SNAP)
        return np.moveaxis(Q.reshape(shp[:-1] + (Q.shape[1],)), -1, axis), R

    # ---------------------------------------------------------- sweeps
    def _S(self, z: int, h: float) -> None:
        for k, c in enumerate(self.kids[z]):
            Q, R = self.qr_along(self.A[z], k)           # gauge down
            self.A[z] = Q
            self.A[c] = mode_product(self.A[c], R, self.A[c].ndim - 1)
            self.build_mf(z, k)
            if self.local_dim[c] > 0:
                self.forward(c, h)
            else:
                self._S(c, h)
            pax = self.A[c].ndim - 1                      # up: backward bond step
            Q, R = self.qr_along(self.A[c], pax)
            self.A[c] = Q
            self.build_spo(c)
            C = self.backward(c, R, h)
            self.A[z] = mode_product(self.A[z], C, k)
        if z != self.root:
            self.forward(z, h)

    def _Sstar(self, z: int, h: float) -> None:
        if z != self.root:
            self.forward(z, h)
        kids = self.kids[z]
        for k in range(len(kids) - 1, -1, -1):
            c = kids[k]
            Q, R = self.qr_along(self.A[z], k)           # down: backward bond step
            self.A[z] = Q
            self.build_mf(z, k)
            C = self.backward(c, R.T, h)
            self.A[c] = mode_product(self.A[c], C.T, self.A[c].ndim - 1)
            if self.local_dim[c] > 0:
                self.forward(c, h)
            else:
                self._Sstar(c, h)
            pax = self.A[c].ndim - 1                      # gauge up
            Q, R = self.qr_along(self.A[c], pax)
            self.A[c] = Q
            self.build_spo(c)
            self.A[z] = mode_product(self.A[z], R, k)

    def step(self, dt: float) -> None:
        """One symmetric sweep S(dt/2) S*(dt/2) with the root forward steps merged."""
        h = 0.5 * dt
        self._S(self.root, h)
        self.forward(self.root, dt)
        self._Sstar(self.root, h)
        self.time += dt

    def set_coefficients(self, coef) -> None:
        """New coefficients c_r for the same terms (Sec. II B: coefficients may
        depend on time).  The SPO matrices hold the inside aggregates, which
        carry coefficients, so they are rebuilt from the state; the mean fields
        are rebuilt by the sweep before every use."""
        coef = np.asarray(coef, dtype=np.complex128)
        if coef.shape != self.coef.shape:
            raise ValueError(f"expected {self.coef.shape[0]} coefficients, got {coef.shape}")
        self.coef = coef.copy()
        if self.A[self.root] is not None:
            self.build_all_spos()

    def step_td(self, dt: float, coef_at: Callable[[float], np.ndarray]) -> None:
        """One step of a generator with time-dependent coefficients: the
        coefficients are frozen at the midpoint of the step, c_r(t + dt/2),
        and the sweep of ``step`` propagates over dt (second order in dt, like
        the symmetric sweep itself)."""
        self.set_coefficients(coef_at(self.time + 0.5 * dt))
        self.step(dt)

    # ------------------------------------------------------ observables
    def _contract(self, bra, ket, leaf_ops: Dict[int, np.ndarray]) -> complex:
        def rec(z):
            if self.local_dim[z] > 0:
                K = ket[z]
                if z in leaf_ops:
                    K = mode_product(K, leaf_ops[z], 0)
                return bra[z].conj().T @ K
            K = ket[z]
            for k, c in enumerate(self.kids[z]):
                K = mode_product(K, rec(c), k)
            return contract_except(bra[z], K, K.ndim - 1)
        return complex(rec(self.root)[0, 0])

    def expect(self, op_ids: Sequence[int]) -> complex:
        """<Psi| prod_ops |Psi> (raw, not divided by the norm)."""
        ops = {self.p.op_leaf[o]: np.asarray(self.p.op_mats[o]) for o in op_ids}
        return self._contract(self.A, self.A, ops)

    def norm2(self) -> float:
        return self._contract(self.A, self.A, {}).real

    def energy(self) -> complex:
        return sum(self.coef[r] * self._contract(self.A, self.A, self.terms[r])
                   for r in range(len(self.terms)))

    def overlap_t0(self) -> complex:
        """a(t) = <Psi(0)|Psi(t)> (Sec. IV A)."""
        return self._contract(self.A0, self.A, {})

    def overlap(self, other: Sequence[np.ndarray]) -> complex:
        return self._contract(other, self.A, {})

    def bilinear(self, leaf_vecs: Dict[int, np.ndarray]) -> complex:
        """(b|Psi) = sum b_x Psi_x for a product vector b (no complex conjugation).

        Used for the HEOM reduced density matrix, rho_S = <0_aux|rho) (SI, end of
        the free-pole HEOM / pseudomode section).
        """
        # children are contracted one at a time from the front
        def rec2(z):
            if self.local_dim[z] > 0:
                return np.asarray(leaf_vecs[z], dtype=np.complex128) @ self.A[z]
            K = self.A[z]
            for c in self.kids[z]:
                K = np.tensordot(rec2(c), K, axes=([0], [0]))
            return K.reshape(-1)
        return complex(rec2(self.root)[0])

    def dense_state(self) -> np.ndarray:
        return full_state(self.parent, self.local_dim, self.A)
