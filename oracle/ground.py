"""Plain CPU one-site ground-state sweep (DMRG on trees), complex128.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may use it; it shares no code with
the HIP library.

What it follows (paper: pyTTN, arXiv 2503.15460, Sec. II C, "Variational
Updating Schemes"): besides the one-site projector-splitting integrator, the
same single-site machinery serves ground-state optimisation (one-site
alternating least squares, DMRG on trees); the paper defers the details to
its references.  Reading taken here: the sweep visits the nodes in the order
of the time-evolution sweep S followed by its mirror S*; at every node the
site tensor is replaced by the eigenvector of the lowest eigenvalue of the
same local effective generator as the local equation of motion of Sec. II C;
there is no backward bond step, the R factor of every gauge move is absorbed
into the next node as it is.  Each local eigenproblem is solved by a dense
Hermitian eigendecomposition of the explicit local matrix (small trees only).
"""
from __future__ import annotations

import numpy as np

from .ttn_oracle import Oracle


class GroundOracle(Oracle):
    """One-site DMRG sweeps on the tree of an Oracle (Hermitian generators)."""

    def __init__(self, problem, bond_dim=None, max_local: int = 4096):
        super().__init__(problem, bond_dim=bond_dim, hermitian=True)
        self.max_local = max_local
        self.local_values = []  # lowest local eigenvalue of every node update, in order

    def local_matrix(self, z: int) -> np.ndarray:
        """The local effective generator at node z as an explicit matrix (its
        columns are the generator applied to the unit tensors)."""
        shape = self.A[z].shape
        n = int(np.prod(shape))
        if n > self.max_local:
            raise ValueError(f"local problem of {n} unknowns exceeds the dense limit {self.max_local}")
        H = np.empty((n, n), dtype=np.complex128)
        for j in range(n):
            e = np.zeros(n, dtype=np.complex128)
            e[j] = 1.0
            H[:, j] = self.heff(z, e.reshape(shape)).reshape(-1)
        return H

    def forward(self, z: int, h: float) -> None:
        """Node update: the lowest eigenvector of the local generator (h unused)."""
        H = self.local_matrix(z)
        defect = np.linalg.norm(H - H.conj().T) / max(1.0, np.linalg.norm(H))
        if defect > 1e-10:
            raise ValueError(f"local generator at node {z} is not Hermitian ({defect:.1e})")
        w, V = np.linalg.eigh(H)
        self.local_values.append(float(w[0]))
        self.A[z] = V[:, 0].reshape(self.A[z].shape)

    def backward(self, c: int, C: np.ndarray, h: float) -> np.ndarray:
        """No backward bond step: the bond factor is absorbed unchanged."""
        return C

    def sweep(self) -> float:
        """One sweep S, root update, S*; returns <Psi|H|Psi> / <Psi|Psi> after it."""
        self._S(self.root, 0.0)
        self.forward(self.root, 0.0)
        self._Sstar(self.root, 0.0)
        return float((self.energy() / self.norm2()).real)
