"""Subspace expansion by the two-site energy variance, written out densely.

TEST INFRASTRUCTURE ONLY (same rules as the rest of ``oracle/``).  There is no
HIP counterpart of this module: it fixes what a bond expansion must compute,
on trees small enough for dense vectors.

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
  same construction with the centre at c spawns single hole functions of c
  (new functions of everything outside c) when the sweep moves up.

Reading (the paper defers the details to its reference on MCTDH spawning):
with X the two-site projection of G Psi, matricised as (indices below c) x
(indices outside c), the error restricted to the two-site space and
orthogonal to the one-site tangent space is R = (1 - P_c) X (1 - P_o), where
P_c projects onto the span of c's current functions (the columns of A^c) and
P_o onto the span the current coefficients reach on the outside (the row
space of A^z along bond k).  Delta = R R^dag, so the spawned functions are
the dominant left singular vectors of R and lambda_s = sigma_s^2; moving up,
the roles swap: P_o becomes the projector onto the current single hole
functions and P_c the column space of the centre A^c, and the new single hole
functions are the dominant right singular vectors.

Everything here uses dense vectors of the whole state: X = V2^dag G Psi with
V2 the orthonormal two-site embedding, SVDs from numpy.  It is exact up to
rounding and meant for a few hundred to a few thousand basis states.
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
    """R = (1 - P_c) X (1 - P_o) for the bond (z, k-th child), matricised (below c) x (outside c).

    ``centre`` is "z" (spawning functions of c: P_c from the isometry A^c,
    P_o from the row space of A^z along k) or "c" (spawning single hole
    functions: P_o from the isometry A^z, P_c from the column space of A^c).
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


def spawn(o: Oracle, z: int, k: int, G: np.ndarray, dt: float, eps_s: float, chi_max: int,
          centre: str) -> Tuple[np.ndarray, np.ndarray]:
    """Singular values of R and the functions to add (columns), by the spawning rule.

    Functions are taken in decreasing sigma while |dt| sigma >= eps_s and the
    bond stays within chi_max.  centre "z": left singular vectors (new
    functions of c, in the basis below c); centre "c": right singular vectors
    conjugated (new single hole functions, in the basis outside c).
    """
    R = residual(o, z, k, G, centre)
    U, s, Vh = np.linalg.svd(R, full_matrices=False)
    n_now = o.A[o.kids[z][k]].shape[-1]
    room = max(0, chi_max - n_now)
    take = 0
    while take < min(room, s.size) and abs(dt) * s[take] >= eps_s:
        take += 1
    vecs = U[:, :take] if centre == "z" else Vh[:take].T  # outside: conjugated right singular vectors
    return s, vecs


def expand(o: Oracle, z: int, k: int, vecs: np.ndarray, centre: str) -> None:
    """Widen the bond (z, k-th child) by the given orthonormal functions, zero coefficients.

    centre "z": the columns of A^c gain ``vecs`` (basis below c) and A^z gains
    zero slices along k; centre "c": A^z gains ``vecs`` as new columns along k
    (basis outside c) and A^c gains zero slices along its parent index.
    """
    c = o.kids[z][k]
    s = vecs.shape[1]
    if s == 0:
        return
    below = o.A[c].shape[:-1]
    outside = o.A[z].shape[:k] + o.A[z].shape[k + 1:]
    if centre == "z":
        o.A[c] = np.concatenate([o.A[c], vecs.reshape(below + (s,))], axis=-1)
        pad = np.zeros(o.A[z].shape[:k] + (s,) + o.A[z].shape[k + 1:], dtype=np.complex128)
        o.A[z] = np.concatenate([o.A[z], pad], axis=k)
    else:
        new = np.moveaxis(vecs.reshape(outside + (s,)), -1, k)
        o.A[z] = np.concatenate([o.A[z], new], axis=k)
        pad = np.zeros(below + (s,), dtype=np.complex128)
        o.A[c] = np.concatenate([o.A[c], pad], axis=-1)
    o.bond[c] += s
