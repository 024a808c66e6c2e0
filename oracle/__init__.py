"""CPU oracle for the one-site TDVP sweep (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It shares no code with the HIP library.
``oracle.subspace`` holds the dense definition of the bond expansion by the
two-site energy variance (small trees only); ``oracle.ground`` the one-site
ground-state sweep (DMRG on trees, dense local eigensolves); ``oracle.multiset``
the sweep of the multi-set ansatz (all sets evolved together at every node).
"""
from .ttn_oracle import (Oracle, clamp_bonds, dense_sop, full_state, expm_krylov,
                         householder_qr_lapack)

__all__ = ["Oracle", "clamp_bonds", "dense_sop", "full_state", "expm_krylov",
           "householder_qr_lapack"]
