"""Plain CPU one-site TDVP sweep of the multi-set tree tensor network, complex128.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may use it; it shares no code with
the HIP library.

What it follows (paper: pyTTN, arXiv 2503.15460):

* The multi-set ansatz of Sec. II A: |Psi> = sum_alpha |alpha> |Psi^alpha>,
  every |Psi^alpha> a tree tensor network of one common tree shape with its
  own coefficient tensors (and bonds).
* A generator of block form G = sum_{alpha beta} |alpha><beta| (x) G_{alpha beta},
  every block a sum of products of leaf operators (Sec. II B 1); a term
  without operators is a constant of its block.
* The one-site projector-splitting sweep of Sec. II C, which the paper applies
  to both the single- and the multi-set forms and whose multi-set details it
  defers to its references.  Reading taken here: the tangent space of the
  multi-set manifold is the direct sum of the sets' tangent spaces, so the
  sweep visits the nodes in the single-set order (S(dt/2), the root over dt,
  S*(dt/2)) and at every node evolves the tensors of all sets together; the
  gauge moves (QR) are made set by set, and the bond steps evolve the bond
  matrices of all sets together.  The local equation couples the sets through
  the environments <Phi^alpha| h_r |Phi^beta> of every term r of block
  (alpha, beta), which between different sets are not identities even where
  the term has no operator (they are overlaps of the two sets' bases), so
  every term keeps its own environment matrix at every node (no inside or
  outside aggregates as in the single-set oracle).

Local exponentials, the QR convention and the zero-snap are those of the
single-set oracle.
"""
from __future__ import annotations

from typing import Dict, List, Sequence

import numpy as np

from .ttn_oracle import (SNAP, _children, clamp_bonds, contract_except, expm_krylov, full_state,
                         householder_qr_lapack, leaf_order, mode_product)


class MultiSetOracle:
    """One-site TDVP sweep of a multi-set tree tensor network (CPU, complex128)."""

    def __init__(self, problem, bond_dim=None, tol: float = 1e-13, mmax: int = 40, dense_max: int = 0,
                 hermitian=None):
        p = problem
        self.p = p
        self.parent = [int(x) for x in p.parent]
        self.local_dim = [int(x) for x in p.local_dim]
        self.n = len(self.parent)
        self.kids = _children(self.parent)
        self.root = [z for z in range(self.n) if self.parent[z] < 0][0]
        self.S = int(p.meta["n_sets"])
        req = np.asarray(p.bond_dim if bond_dim is None else bond_dim)
        if req.ndim == 1:
            req = np.tile(req, (self.S, 1))
        self.bond = [clamp_bonds(self.parent, self.local_dim, req[a]) for a in range(self.S)]
        self.tol, self.mmax, self.dense_max = tol, mmax, dense_max
        self.hermitian = p.hermitian if hermitian is None else hermitian
        # term r: block (alpha, beta), coefficient, leaf -> operator
        self.pair = [tuple(int(x) for x in ab) for ab in p.meta["set_pair"]]
        self.coef = np.asarray(p.coeff, dtype=np.complex128)
        self.ops: List[Dict[int, np.ndarray]] = [{p.op_leaf[o]: np.asarray(p.op_mats[o]) for o in t}
                                                 for t in p.term_ops]
        if len(self.pair) != len(self.ops):
            raise ValueError("one set pair per term is needed")
        self.A: List[List[np.ndarray]] = [[None] * self.n for _ in range(self.S)]
        self.E: List[Dict[int, np.ndarray]] = [dict() for _ in range(self.n)]  # node -> term -> n_a x n_b
        self.M: List[Dict[int, np.ndarray]] = [dict() for _ in range(self.n)]
        self.matvecs = [0]
        self.time = 0.0

    # ------------------------------------------------------------ state
    def shape(self, a: int, z: int):
        b = self.bond[a]
        dims = [self.local_dim[z]] if self.local_dim[z] > 0 else [int(b[c]) for c in self.kids[z]]
        return dims + [int(b[z]) if z != self.root else 1]

    def set_product_state(self, vecs: Dict[int, np.ndarray], weights: Sequence[complex]) -> None:
        """Set alpha: the product state of ``vecs`` (unoccupied functions as in
        the single-set oracle: unit vectors after modified Gram-Schmidt at the
        leaves, identity columns above) with root amplitude weights[alpha]."""
        for a in range(self.S):
            for z in range(self.n):
                shp = self.shape(a, z)
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
                    self.A[a][z] = np.stack(cols, axis=1)
                else:
                    rows = int(np.prod(shp[:-1]))
                    self.A[a][z] = np.eye(rows, shp[-1], dtype=np.complex128).reshape(shp)
            self.A[a][self.root] = self.A[a][self.root] * weights[a]
        self.build_all_E()

    def set_state(self, tensors: Sequence[Sequence[np.ndarray]]) -> None:
        """tensors[alpha][z]; every non-root node an isometry toward its parent."""
        for a in range(self.S):
            for z in range(self.n):
                t = np.asarray(tensors[a][z], dtype=np.complex128)
                if list(t.shape) != self.shape(a, z):
                    raise ValueError(f"set {a} node {z}: shape {t.shape} != {self.shape(a, z)}")
                self.A[a][z] = t.copy()
        self.build_all_E()

    def state(self) -> List[List[np.ndarray]]:
        return [[t.copy() for t in As] for As in self.A]

    def dense_state(self) -> np.ndarray:
        """sum_alpha e_alpha (x) Psi^alpha as one vector (set index first)."""
        return np.concatenate([full_state(self.parent, self.local_dim, self.A[a]) for a in range(self.S)])

    # ----------------------------------------------------- environments
    def _postorder(self) -> List[int]:
        out: List[int] = []

        def rec(z):
            for c in self.kids[z]:
                rec(c)
            out.append(z)
        rec(self.root)
        return out

    def build_all_E(self) -> None:
        for z in self._postorder():
            if z != self.root:
                self.build_E(z)

    def build_E(self, c: int) -> None:
        """<Phi^alpha_c| h_r |Phi^beta_c> for every term r of block (alpha, beta):
        the SPF recursion of Sec. II A / II C taken between two sets' bases
        (identity where the term has no operator on a leaf)."""
        out = {}
        for r, (a, b) in enumerate(self.pair):
            X = self.A[b][c]
            if self.local_dim[c] > 0:
                O = self.ops[r].get(c)
                if O is not None:
                    X = mode_product(X, O, 0)
            else:
                for k, ck in enumerate(self.kids[c]):
                    X = mode_product(X, self.E[ck][r], k)
            out[r] = contract_except(self.A[a][c], X, X.ndim - 1)
        self.E[c] = out

    def build_M(self, z: int, k: int) -> None:
        """Mean-field matrices of child k of z between the sets' SHF bases (the
        SHF recursion of Sec. II A / II C)."""
        c = self.kids[z][k]
        out = {}
        for r, (a, b) in enumerate(self.pair):
            X = self.A[b][z]
            for j, cj in enumerate(self.kids[z]):
                if j != k:
                    X = mode_product(X, self.E[cj][r], j)
            if z != self.root:
                X = mode_product(X, self.M[z][r], X.ndim - 1)
            out[r] = contract_except(self.A[a][z], X, k)
        self.M[c] = out

    # ------------------------------------------------- local operators
    def heff(self, z: int, Xs: List[np.ndarray]) -> List[np.ndarray]:
        """Local equation of motion of Sec. II C for the tensors of all sets at
        node z: (H_eff X)_alpha = sum_beta sum_{r in (alpha, beta)} c_r
        (x)_children E_r (x)_parent M_r X_beta."""
        Ys = [np.zeros(self.shape(a, z), dtype=np.complex128) for a in range(self.S)]
        for r, (a, b) in enumerate(self.pair):
            X = Xs[b]
            if self.local_dim[z] > 0:
                O = self.ops[r].get(z)
                if O is not None:
                    X = mode_product(X, O, 0)
            else:
                for k, ck in enumerate(self.kids[z]):
                    X = mode_product(X, self.E[ck][r], k)
            if z != self.root:
                X = mode_product(X, self.M[z][r], X.ndim - 1)
            Ys[a] = Ys[a] + self.coef[r] * X
        return Ys

    def keff(self, c: int, Cs: List[np.ndarray]) -> List[np.ndarray]:
        """Bond generator on the bond above c: (K C)_alpha = sum_beta sum_r c_r
        E_r C_beta M_r^T."""
        Ys = [np.zeros((int(self.bond[a][c]), int(self.bond[a][c])), dtype=np.complex128)
              for a in range(self.S)]
        for r, (a, b) in enumerate(self.pair):
            Ys[a] = Ys[a] + self.coef[r] * (self.E[c][r] @ Cs[b] @ self.M[c][r].T)
        return Ys

    def _expm_sets(self, apply, Xs: List[np.ndarray], tau: float) -> List[np.ndarray]:
        """exp(-i tau L) on the tensors of all sets stacked into one vector."""
        shapes = [x.shape for x in Xs]
        sizes = [x.size for x in Xs]
        cuts = np.cumsum([0] + sizes)

        def split(v):
            return [v[cuts[a]:cuts[a + 1]].reshape(shapes[a]) for a in range(self.S)]

        def f(v):
            return np.concatenate([y.reshape(-1) for y in apply(split(v))])
        v = np.concatenate([x.reshape(-1) for x in Xs])
        out = expm_krylov(f, v, tau, hermitian=self.hermitian, tol=self.tol, mmax=self.mmax,
                          dense_max=self.dense_max, counter=self.matvecs)
        return split(out)

    def forward(self, z: int, h: float) -> None:
        new = self._expm_sets(lambda Xs: self.heff(z, Xs), [self.A[a][z] for a in range(self.S)], h)
        for a in range(self.S):
            self.A[a][z] = new[a]

    def backward(self, c: int, Cs: List[np.ndarray], h: float) -> List[np.ndarray]:
        return self._expm_sets(lambda Xs: self.keff(c, Xs), Cs, -h)

    # ---------------------------------------------------------- gauge
    @staticmethod
    def qr_along(A: np.ndarray, axis: int):
        M = np.moveaxis(A, axis, -1)
        shp = M.shape
        Q, R = householder_qr_lapack(M.reshape(-1, shp[-1]), snap=SNAP)
        return np.moveaxis(Q.reshape(shp[:-1] + (Q.shape[1],)), -1, axis), R

    # ---------------------------------------------------------- sweeps
    def _S(self, z: int, h: float) -> None:
        for k, c in enumerate(self.kids[z]):
            for a in range(self.S):                      # gauge down, set by set
                Q, R = self.qr_along(self.A[a][z], k)
                self.A[a][z] = Q
                self.A[a][c] = mode_product(self.A[a][c], R, self.A[a][c].ndim - 1)
            self.build_M(z, k)
            if self.local_dim[c] > 0:
                self.forward(c, h)
            else:
                self._S(c, h)
            Rs = []
            for a in range(self.S):                      # gauge up, set by set
                Q, R = self.qr_along(self.A[a][c], self.A[a][c].ndim - 1)
                self.A[a][c] = Q
                Rs.append(R)
            self.build_E(c)
            Cs = self.backward(c, Rs, h)                 # all sets' bond matrices together
            for a in range(self.S):
                self.A[a][z] = mode_product(self.A[a][z], Cs[a], k)
        if z != self.root:
            self.forward(z, h)

    def _Sstar(self, z: int, h: float) -> None:
        if z != self.root:
            self.forward(z, h)
        kids = self.kids[z]
        for k in range(len(kids) - 1, -1, -1):
            c = kids[k]
            Rs = []
            for a in range(self.S):
                Q, R = self.qr_along(self.A[a][z], k)
                self.A[a][z] = Q
                Rs.append(R.T)
            self.build_M(z, k)
            Cs = self.backward(c, Rs, h)
            for a in range(self.S):
                self.A[a][c] = mode_product(self.A[a][c], Cs[a].T, self.A[a][c].ndim - 1)
            if self.local_dim[c] > 0:
                self.forward(c, h)
            else:
                self._Sstar(c, h)
            for a in range(self.S):
                Q, R = self.qr_along(self.A[a][c], self.A[a][c].ndim - 1)
                self.A[a][c] = Q
                self.A[a][z] = mode_product(self.A[a][z], R, k)
            self.build_E(c)

    def step(self, dt: float) -> None:
        """S(dt/2), the root over dt, S*(dt/2) for all sets together."""
        h = 0.5 * dt
        self._S(self.root, h)
        self.forward(self.root, dt)
        self._Sstar(self.root, h)
        self.time += dt

    # ------------------------------------------------------ observables
    def populations(self) -> np.ndarray:
        """<Psi^alpha|Psi^alpha> for every set (the state populations)."""
        return np.array([np.vdot(full_state(self.parent, self.local_dim, self.A[a]),
                                 full_state(self.parent, self.local_dim, self.A[a])).real
                         for a in range(self.S)])


def dense_multiset(problem) -> np.ndarray:
    """The block generator sum_{alpha beta} |alpha><beta| (x) G_{alpha beta} as
    one dense matrix (set index first, leaves in depth-first order)."""
    leaves = leaf_order([int(x) for x in problem.parent], [int(x) for x in problem.local_dim])
    dims = [int(problem.local_dim[l]) for l in leaves]
    N = int(np.prod(dims))
    S = int(problem.meta["n_sets"])
    G = np.zeros((S * N, S * N), dtype=np.complex128)
    for (a, b), c, ops in zip(problem.meta["set_pair"], problem.coeff, problem.term_ops):
        byleaf = {problem.op_leaf[o]: problem.op_mats[o] for o in ops}
        M = np.ones((1, 1), dtype=np.complex128)
        for l, d in zip(leaves, dims):
            M = np.kron(M, byleaf.get(l, np.eye(d)))
        G[a * N:(a + 1) * N, b * N:(b + 1) * N] += c * M
    return G
