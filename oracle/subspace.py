"""Subspace expansion by the two-site energy variance (bond-dimension adaptation).

TEST INFRASTRUCTURE ONLY (same rules as the rest of ``oracle/``).  There is no
HIP counterpart of this module.  It holds three things, each pinned against
the one before: the dense definition of what a bond expansion computes (small
trees), the one-site-cost form of the same residual with a Krylov iteration
for its dominant singular pairs, and the projector-splitting sweep with the
expansions at the bond crossings.

What it follows (paper: pyTTN, arXiv 2503.15460, Sec. II D):

* The bond between node z and its k-th child c is widened by new single
  particle functions of c that are orthogonal to the current ones, with zero
  coefficients, so the state does not change.
* The gain in the squared error of the time derivative is the expectation of
  the operator Delta^(z,k) = (1 - P^(z,k)) W (1 - P^(z,k)) in the new
  functions, where W collects the overlaps of the error Psi_e' - Psi_M' with
  the orthonormal functions Theta_{i I} of everything outside c (centre at z).
* Functions are spawned along the eigenvectors of Delta with the largest
  eigenvalues lambda_s, while dt sqrt(lambda_s) >= eps_S (TDVP: c = dt), up to
  a maximum bond dimension.  By the symmetry of the mixed-canonical gauge the
  same construction spawns single hole functions of c (new functions of
  everything outside c); each bond is tried once per direction of the sweep.
* Only the dominant eigenpairs are needed, and the operator can act on
  single-site objects at about single-site cost, so they come from a Krylov
  iteration rather than a dense two-site decomposition.

Reading (the paper defers the details to its reference on MCTDH spawning):
with X the two-site projection of G Psi, matricised as (indices below c) x
(indices outside c), the error restricted to the two-site space and
orthogonal to the one-site tangent space is R = (1 - P_c) X (1 - P_o^T),
where P_c projects onto the column space of A^c (c's current functions, or
the centre's columns) and P_o onto the column space of A^z matricised along
bond k (the outside functions the bond reaches); the transpose appears
because X's rows are coordinate vectors on the outside.  Delta = R R^dag, so
new functions below the bond are the dominant left singular vectors of R
(lambda_s = sigma_s^2) and new functions outside it the conjugated dominant
right singular vectors.  The formula holds with the centre at z or at c.

The dense definition uses vectors of the whole state: X = V2^dag G Psi with
V2 the orthonormal two-site embedding, SVDs from numpy; it is exact up to
rounding and meant for a few hundred to a few thousand basis states.  Where
the sweep widens which side of a bond is a further reading, stated in
``AdaptiveOracle``.
"""
from __future__ import annotations

from typing import List, Tuple

import numpy as np

from .ttn_oracle import Oracle, full_state, mode_product

RANK_TOL = 1e-12  # relative singular-value cut for the span projectors


def move_centre_down(o: Oracle, path: List[int]) -> None:
    """Gauge-shift the orthogonality centre from the root along ``path`` (QR, Sec. II C)."""
    z = o.root
    for c in path:
        k = o.kids[z].index(c)
        Q, R = o.qr_along(o.A[z], k)
        o.A[z] = Q
        o.A[c] = mode_product(o.A[c], R, o.A[c].ndim - 1)
        z = c


def _span_projector(M: np.ndarray) -> np.ndarray:
    """Orthogonal projector onto the column space of M (numerical rank by RANK_TOL)."""
    U, s, _ = np.linalg.svd(M, full_matrices=False)
    if s.size == 0 or s[0] == 0.0:
        return np.zeros((M.shape[0], M.shape[0]), dtype=np.complex128)
    r = int(np.sum(s > RANK_TOL * s[0]))
    return U[:, :r] @ U[:, :r].conj().T


def two_site_embedding(o: Oracle, z: int, k: int) -> Tuple[np.ndarray, Tuple[int, ...], Tuple[int, ...]]:
    """Dense V2 with Psi = V2 vec(T) for two-site coefficients T of (z, c = k-th child).

    T is indexed (indices of A^c except its parent index) + (indices of A^z
    except index k); all nodes other than z and c keep their current tensors.
    With the orthogonality centre at z or at c, V2 has orthonormal columns.
    Returns V2, the shape of the c side and the shape of the outside.
    """
    c = o.kids[z][k]
    below = o.A[c].shape[:-1]
    outside = o.A[z].shape[:k] + o.A[z].shape[k + 1:]
    nb, no = int(np.prod(below)), int(np.prod(outside))
    saved_c, saved_z = o.A[c], o.A[z]
    ident = np.eye(nb, dtype=np.complex128).reshape(below + (nb,))
    cols = []
    try:
        o.A[c] = ident
        for j in range(nb * no):
            e = np.zeros(nb * no, dtype=np.complex128)
            e[j] = 1.0
            T = np.moveaxis(e.reshape((nb,) + outside), 0, k)  # A^z with a bond of size nb
            o.A[z] = T
            cols.append(full_state(o.parent, o.local_dim, o.A))
    finally:
        o.A[c], o.A[z] = saved_c, saved_z
    return np.stack(cols, axis=1), below, outside


def residual(o: Oracle, z: int, k: int, G: np.ndarray, centre: str) -> np.ndarray:
    """R = (1 - P_c) X (1 - P_o^T) for the bond (z, k-th child), matricised (below c) x (outside c).

    ``centre`` names where the orthogonality centre is, "z" or "c"; the node
    on the other side of the bond must be an isometry toward it (checked), so
    that the two-site embedding is orthonormal.
    """
    c = o.kids[z][k]
    V2, below, outside = two_site_embedding(o, z, k)
    psi = full_state(o.parent, o.local_dim, o.A)
    nb, no = int(np.prod(below)), int(np.prod(outside))
    X = (V2.conj().T @ (G @ psi)).reshape(nb, no)
    Ac = o.A[c].reshape(nb, -1)                          # (below c) x bond
    Az = np.moveaxis(o.A[z], k, -1).reshape(no, -1)      # (outside c) x bond
    Pc = _span_projector(Ac)
    Po = _span_projector(Az)
    if centre == "z":
        assert np.allclose(Ac.conj().T @ Ac, np.eye(Ac.shape[1]), atol=1e-12), "A^c must be an isometry"
    elif centre == "c":
        assert np.allclose(Az.conj().T @ Az, np.eye(Az.shape[1]), atol=1e-12), "A^z must be an isometry"
    else:
        raise ValueError(centre)
    I_b = np.eye(nb, dtype=np.complex128)
    I_o = np.eye(no, dtype=np.complex128)
    # the rows of X are coordinate vectors on the outside: projecting a row x
    # onto the span of the columns of Az is x Po^T
    return (I_b - Pc) @ X @ (I_o - Po.T)


def _room(o: Oracle, z: int, k: int, chi_max: int) -> int:
    """How many functions the bond (z, k-th child) may still gain: up to chi_max
    and up to what both sides can hold as orthonormal columns (the rows of A^c
    below the bond and of A^z along it), so every matricisation keeps rows >=
    columns."""
    c = o.kids[z][k]
    nb = int(np.prod(o.A[c].shape[:-1]))
    no = int(np.prod(o.A[z].shape[:k] + o.A[z].shape[k + 1:]))
    return max(0, min(chi_max, nb, no) - o.A[c].shape[-1])


def _take(s: np.ndarray, dt: float, eps_s: float, room: int) -> int:
    take = 0
    while take < min(room, s.size) and abs(dt) * s[take] >= eps_s:
        take += 1
    return take


def spawn(o: Oracle, z: int, k: int, G: np.ndarray, dt: float, eps_s: float, chi_max: int,
          centre: str, side: str) -> Tuple[np.ndarray, np.ndarray]:
    """Singular values of R and the functions to add (columns), by the spawning rule.

    Functions are taken in decreasing sigma while |dt| sigma >= eps_s and the
    bond stays within chi_max and within what both sides can hold.  side
    "below": left singular vectors (new functions of c, basis below c);
    "outside": conjugated right singular vectors (new single hole functions,
    basis outside c).
    """
    R = residual(o, z, k, G, centre)
    U, s, Vh = np.linalg.svd(R, full_matrices=False)
    take = _take(s, dt, eps_s, _room(o, z, k, chi_max))
    if side == "below":
        return s, U[:, :take]
    if side == "outside":
        return s, Vh[:take].T
    raise ValueError(side)


def expand(o: Oracle, z: int, k: int, vecs: np.ndarray, side: str) -> None:
    """Widen the bond (z, k-th child) by the given orthonormal functions, zero coefficients.

    side "below": A^c gains ``vecs`` as new columns (basis below c) and A^z
    zero slices along k; side "outside": A^z gains ``vecs`` as new slices
    along k (basis outside c) and A^c zero columns.  Either way the state is
    unchanged; which tensor is the centre does not matter.
    """
    c = o.kids[z][k]
    s = vecs.shape[1]
    if s == 0:
        return
    below = o.A[c].shape[:-1]
    outside = o.A[z].shape[:k] + o.A[z].shape[k + 1:]
    if side == "below":
        o.A[c] = np.concatenate([o.A[c], vecs.reshape(below + (s,))], axis=-1)
        pad = np.zeros(o.A[z].shape[:k] + (s,) + o.A[z].shape[k + 1:], dtype=np.complex128)
        o.A[z] = np.concatenate([o.A[z], pad], axis=k)
    elif side == "outside":
        new = np.moveaxis(vecs.reshape(outside + (s,)), -1, k)
        o.A[z] = np.concatenate([o.A[z], new], axis=k)
        pad = np.zeros(below + (s,), dtype=np.complex128)
        o.A[c] = np.concatenate([o.A[c], pad], axis=-1)
    else:
        raise ValueError(side)
    o.bond[c] += s


# ------------------------------------------------------ one-site-cost form
# The same residual without forming X: the two-site generator is kept as a
# list of (coefficient, factors below c, factors outside c) built from the
# environments the sweep maintains, and X acts on a vector through the two
# node tensors one after the other, A^z then A^c (or back), which costs about
# one single-site matvec; the dominant singular pairs then come from a
# Krylov (Golub-Kahan-Lanczos) iteration, the iterative route Sec. II D takes.

def two_site_terms(o: Oracle, z: int, k: int):
    """The two-site generator at (z, c = k-th child) as (coef, below factors, outside factors).

    Factor dictionaries map an axis of the two-site tensor (indices below c,
    then A^z's indices without k) to a matrix; SPOs of c's children (or c's
    own leaf operators) act below, SPOs of z's other children and z's mean
    field act outside.  Terms confined to one of these pieces enter through
    the aggregated "in" / "out" environments, every other term individually.
    """
    c = o.kids[z][k]
    nbel = o.A[c].ndim - 1
    ckids = o.kids[c]
    zother = [cj for j, cj in enumerate(o.kids[z]) if j != k]
    ax = {cj: nbel + i for i, cj in enumerate(zother)}
    pax = nbel + len(zother)
    has_out = z != o.root
    out = []
    # aggregates
    if o.local_dim[c] > 0:
        loc = [r for r in range(len(o.terms)) if o.inside(r, c)]
        if loc:
            out.append((1.0, {0: sum(o.coef[r] * o.terms[r][c] for r in loc)}, {}))
    else:
        for j, cj in enumerate(ckids):
            if "in" in o.spo[cj]:
                out.append((1.0, {j: o.spo[cj]["in"]}, {}))
    for cj in zother:
        if "in" in o.spo[cj]:
            out.append((1.0, {}, {ax[cj]: o.spo[cj]["in"]}))
    if has_out and "out" in o.mf[z]:
        out.append((1.0, {}, {pax: o.mf[z]["out"]}))
    # terms spanning two or more pieces
    for r in range(len(o.terms)):
        below_hit = ([0] if o.touches(r, c) else []) if o.local_dim[c] > 0 else \
            [j for j, cj in enumerate(ckids) if o.touches(r, cj)]
        other_hit = [cj for cj in zother if o.touches(r, cj)]
        outside_hit = has_out and o.touches_outside(r, z)
        if len(below_hit) + len(other_hit) + int(outside_hit) < 2:
            continue  # confined to one piece: part of an aggregate above
        # spanning several pieces, the term crosses each of them: own SPOs / mean field
        if o.local_dim[c] > 0:
            fb = {0: o.terms[r][c]} if below_hit else {}
        else:
            fb = {j: o.spo[ckids[j]][r] for j in below_hit}
        fo = {ax[cj]: o.spo[cj][r] for cj in other_hit}
        if outside_hit:
            fo[pax] = o.mf[z][r]
        out.append((o.coef[r], fb, fo))
    return out


def _apply(X: np.ndarray, factors, conj: bool = False, transpose: bool = False, shift: int = 0) -> np.ndarray:
    for axis, M in factors.items():
        M2 = M.T if transpose else M
        X = mode_product(X, M2.conj() if conj else M2, axis - shift)
    return X


def heff2(o: Oracle, z: int, k: int, T: np.ndarray) -> np.ndarray:
    """Two-site generator applied to a two-site tensor T (below c, then outside c)."""
    Y = np.zeros_like(T)
    for coef, fb, fo in two_site_terms(o, z, k):
        Y += coef * _apply(_apply(T, fb), fo)
    return Y


class ResidualOperator:
    """R = (1 - P_c) X (1 - P_o^T) applied to vectors at one-site cost.

    X w = sum_t c_t F_t,below A^c (A^z^T (F_t,outside^T w)): per term the
    outside factors act on w, the result is contracted with A^z down to the
    bond, expanded through A^c and the factors below c act last.  X^dag runs
    the same chain backwards with conjugated factors.
    """

    def __init__(self, o: Oracle, z: int, k: int):
        c = o.kids[z][k]
        self.below = o.A[c].shape[:-1]
        self.outside = o.A[z].shape[:k] + o.A[z].shape[k + 1:]
        self.nbel = len(self.below)
        self.nb, self.no = int(np.prod(self.below)), int(np.prod(self.outside))
        self.Ac = o.A[c].reshape(self.nb, -1)
        self.Az = np.moveaxis(o.A[z], k, -1).reshape(self.no, -1)
        self.Pc = _span_projector(self.Ac)
        self.Po = _span_projector(self.Az)
        self.terms = two_site_terms(o, z, k)

    def X(self, w: np.ndarray) -> np.ndarray:
        W = w.reshape(self.outside)
        y = np.zeros(self.nb, dtype=np.complex128)
        for coef, fb, fo in self.terms:
            u = _apply(W, fo, transpose=True, shift=self.nbel).reshape(-1)
            t = self.Ac @ (self.Az.T @ u)
            y += coef * _apply(t.reshape(self.below), fb).reshape(-1)
        return y

    def XH(self, y: np.ndarray) -> np.ndarray:
        Y = y.reshape(self.below)
        w = np.zeros(self.no, dtype=np.complex128)
        for coef, fb, fo in self.terms:
            u = _apply(Y, fb, conj=True, transpose=True).reshape(-1)
            t = self.Az.conj() @ (self.Ac.conj().T @ u)
            w += np.conj(coef) * _apply(t.reshape(self.outside), fo, conj=True, shift=self.nbel).reshape(-1)
        return w

    def R(self, w: np.ndarray) -> np.ndarray:
        w = w - self.Po.T @ w
        y = self.X(w)
        return y - self.Pc @ y

    def RH(self, y: np.ndarray) -> np.ndarray:
        y = y - self.Pc @ y
        w = self.XH(y)
        return w - self.Po.conj() @ w


def krylov_singular(op: ResidualOperator, m: int, start: np.ndarray):
    """Golub-Kahan-Lanczos bidiagonalisation of R with full re-orthogonalisation.

    ``start`` is a (seeded) vector below c; the iteration starts from
    R^dag start, so it stays in the row space of R (at most nb dimensional)
    and m = nb steps reproduce the dense singular values.  Returns the
    singular values of the bidiagonal and the corresponding approximate left
    (below c) and right (outside c) singular vectors of R, largest first.
    """
    q = op.RH(start)
    if np.linalg.norm(q) == 0.0:
        return np.zeros(0), np.zeros((op.nb, 0), dtype=np.complex128), np.zeros((op.no, 0), dtype=np.complex128)
    q = q / np.linalg.norm(q)
    Q, P, alpha, beta = [q], [], [], []
    for j in range(m):
        p = op.R(Q[-1])
        if P:
            p -= beta[-1] * P[-1]
            for v in P:  # full re-orthogonalisation
                p -= np.vdot(v, p) * v
        a = np.linalg.norm(p)
        if a <= 1e-14:
            break
        P.append(p / a)
        alpha.append(a)
        qn = op.RH(P[-1]) - a * Q[-1]
        for v in Q:
            qn -= np.vdot(v, qn) * v
        b = np.linalg.norm(qn)
        if b <= 1e-14 or j == m - 1:
            break
        Q.append(qn / b)
        beta.append(b)
    n = len(alpha)
    if n == 0:  # R vanishes on the start vector's Krylov space
        return np.zeros(0), np.zeros((op.nb, 0), dtype=np.complex128), np.zeros((op.no, 0), dtype=np.complex128)
    B = np.diag(np.asarray(alpha, dtype=np.complex128))
    for i in range(n - 1):
        B[i, i + 1] = beta[i]
    Ub, s, Vbh = np.linalg.svd(B)
    left = np.stack(P[:n], axis=1) @ Ub
    right = np.stack(Q[:n], axis=1) @ Vbh.conj().T
    return s, left, right


# ------------------------------------------------------ the adaptive sweep
def spawn_krylov(o: Oracle, z: int, k: int, dt: float, eps_s: float, chi_max: int, side: str,
                 rng: np.random.Generator) -> np.ndarray:
    """New functions for the bond (z, k-th child) by the one-site-cost route.

    Golub-Kahan-Lanczos on R with as many steps as R has rows below c (exact
    on the trees this oracle handles), then the spawning rule of ``spawn``.
    Columns are orthonormal and orthogonal to the current functions on that
    side of the bond.
    """
    op = ResidualOperator(o, z, k)
    start = rng.normal(size=op.nb) + 1j * rng.normal(size=op.nb)
    s, left, right = krylov_singular(op, op.nb, start)
    take = _take(s, dt, eps_s, _room(o, z, k, chi_max))
    return left[:, :take] if side == "below" else right[:, :take].conj()


class AdaptiveOracle(Oracle):
    """The projector-splitting sweep with subspace expansion at the bond crossings.

    Sec. II D widens a bond with zero coefficients (the state is unchanged)
    when the orthogonality centre crosses it.  Reading: in the splitting, the
    evolution of the bond space is counted by the forward steps on both sides
    and subtracted once by the backward bond step, so the widening must come
    after the forward step of the side that does not see the new directions
    and before the bond step and the forward step of the side that does.  Per
    bond (z above c):

    * S (going up, forward steps after the children): with the centre at c,
      after c's forward step and before the QR, backward bond step and z's
      forward step, new functions below the bond (new SPFs of c);
    * S* (going down, forward steps before the children): with the centre at
      z, after z's forward step and before the QR, backward bond step and c's
      forward step, new single hole functions of c.

    Widening elsewhere (e.g. with the centre at z before S's gauge-only move
    down) either loses the new directions in the next QR or counts them twice.
    ``chi_max`` caps every bond, ``eps_s`` is the spawning tolerance
    (criterion |h| sigma >= eps_s with h the substep), ``seed`` seeds the
    Krylov start vectors.
    """

    def __init__(self, problem, eps_s: float, chi_max: int, seed: int = 0, **kw):
        super().__init__(problem, **kw)
        self.eps_s, self.chi_max = eps_s, chi_max
        self.rng = np.random.default_rng(seed)
        self.spawned = 0

    def _grow(self, z: int, k: int, h: float, side: str) -> bool:
        vecs = spawn_krylov(self, z, k, h, self.eps_s, self.chi_max, side, self.rng)
        if vecs.shape[1] == 0:
            return False
        expand(self, z, k, vecs, side)
        self.spawned += vecs.shape[1]
        return True

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
            if self._grow(z, k, h, "below"):             # centre at c: new functions of c
                self.build_mf(z, k)
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
            if self._grow(z, k, h, "outside"):           # centre at z: new hole functions of c
                self.build_spo(c)
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
