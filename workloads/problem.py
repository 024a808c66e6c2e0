"""Problem description shared by the CPU oracle and the HIP library.

A problem is the input of the paper's problem statement (Sec. II A, Eqs. for the
wavefunction expansion and Sec. II B, Eq. for the SOP Hamiltonian):

* a tree given as a parent array (root has parent -1); node ids are assigned in
  pre-order so the children of every node are ordered by node id;
* ``local_dim[z] > 0`` iff ``z`` is a leaf (a physical degree of freedom);
* ``bond_dim[z]``: requested number of single-particle functions on the bond
  from ``z`` to its parent (1 for the root);
* SOP operator ``H = sum_r c_r prod_alpha h_{alpha,r}``: a table of dense
  single-leaf operators and a list of terms, each a coefficient and at most one
  operator id per leaf;
* an initial product state (one vector per leaf), a time step and a step count.

Time evolution is ``d/dt psi = -i G psi`` with ``G`` the SOP operator (for the
unitary models ``G = H / hbar``).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Dict, List, Optional

import numpy as np


@dataclass
class Problem:
    name: str
    parent: np.ndarray
    local_dim: np.ndarray
    bond_dim: np.ndarray
    op_leaf: List[int]
    op_mats: List[np.ndarray]
    coeff: np.ndarray
    term_ops: List[List[int]]
    init_vecs: Dict[int, np.ndarray]
    dt: float = 0.05
    n_steps: int = 100
    hermitian: bool = True
    leaf_names: Dict[str, int] = field(default_factory=dict)
    observables: Dict[str, List[int]] = field(default_factory=dict)
    meta: Dict[str, object] = field(default_factory=dict)

    # ----------------------------------------------------------------- views
    @property
    def n_nodes(self) -> int:
        return int(len(self.parent))

    @property
    def n_terms(self) -> int:
        return int(len(self.term_ops))

    def leaves(self) -> List[int]:
        return [z for z in range(self.n_nodes) if self.local_dim[z] > 0]

    def children(self, z: int) -> List[int]:
        return [c for c in range(self.n_nodes) if self.parent[c] == z]

    def add_op(self, leaf: int, mat: np.ndarray) -> int:
        mat = np.asarray(mat, dtype=np.complex128)
        d = int(self.local_dim[leaf])
        if mat.shape != (d, d):
            raise ValueError(f"operator on leaf {leaf} must be {d}x{d}, got {mat.shape}")
        self.op_leaf.append(int(leaf))
        self.op_mats.append(mat)
        return len(self.op_mats) - 1

    # ------------------------------------------------------ flat ABI arrays
    def flat_sop(self):
        """Flattened SOP arrays in the layout of the C boundary.

        Returns ``(op_leaf int32[n_ops], op_offset int64[n_ops+1],
        op_data float64[2*sum d^2] complex-interleaved row-major, coeff
        float64[2*n_terms], term_ptr int64[n_terms+1], term_ops int32[...])``.
        """
        op_leaf = np.asarray(self.op_leaf, dtype=np.int32)
        sizes = [m.size for m in self.op_mats]
        op_offset = np.zeros(len(sizes) + 1, dtype=np.int64)
        op_offset[1:] = np.cumsum(sizes)
        if self.op_mats:
            data = np.concatenate([np.ascontiguousarray(m).reshape(-1) for m in self.op_mats])
        else:
            data = np.zeros(0, dtype=np.complex128)
        op_data = np.ascontiguousarray(data.astype(np.complex128)).view(np.float64)
        coeff = np.ascontiguousarray(np.asarray(self.coeff, dtype=np.complex128)).view(np.float64)
        term_ptr = np.zeros(self.n_terms + 1, dtype=np.int64)
        term_ptr[1:] = np.cumsum([len(t) for t in self.term_ops])
        flat = [o for t in self.term_ops for o in t]
        term_ops = np.asarray(flat, dtype=np.int32)
        return op_leaf, op_offset, op_data, coeff, term_ptr, term_ops

    def flat_init(self) -> np.ndarray:
        """Initial leaf vectors concatenated in leaf-id order (complex interleaved)."""
        vecs = [np.asarray(self.init_vecs[z], dtype=np.complex128) for z in self.leaves()]
        return np.ascontiguousarray(np.concatenate(vecs)).view(np.float64)

    def copy(self) -> "Problem":
        return Problem(self.name, self.parent.copy(), self.local_dim.copy(), self.bond_dim.copy(),
                       list(self.op_leaf), [m.copy() for m in self.op_mats], self.coeff.copy(),
                       [list(t) for t in self.term_ops],
                       {k: v.copy() for k, v in self.init_vecs.items()}, self.dt, self.n_steps,
                       self.hermitian, dict(self.leaf_names), dict(self.observables), dict(self.meta))


class TreeBuilder:
    """Builds a pre-order numbered tree from a nested specification.

    A spec is either ``("leaf", bond, d, name)`` or ``("node", bond, [children])``.
    The root's bond is forced to 1.
    """

    def __init__(self, spec):
        self.parent: List[int] = []
        self.local_dim: List[int] = []
        self.bond_dim: List[int] = []
        self.names: Dict[str, int] = {}
        self._add(spec, -1)
        self.bond_dim[0] = 1

    def _add(self, spec, par: int) -> int:
        z = len(self.parent)
        self.parent.append(par)
        if spec[0] == "leaf":
            _, bond, d, name = spec
            self.local_dim.append(int(d))
            self.bond_dim.append(int(bond))
            if name is not None:
                self.names[name] = z
        elif spec[0] == "node":
            _, bond, kids = spec
            self.local_dim.append(0)
            self.bond_dim.append(int(bond))
            if not kids:
                raise ValueError("interior node without children")
            for k in kids:
                self._add(k, z)
        else:
            raise ValueError(f"bad tree spec {spec!r}")
        return z

    def arrays(self):
        return (np.asarray(self.parent, dtype=np.int32), np.asarray(self.local_dim, dtype=np.int32),
                np.asarray(self.bond_dim, dtype=np.int32))


def empty_problem(name: str, spec, **kw) -> Problem:
    tb = TreeBuilder(spec)
    parent, local_dim, bond_dim = tb.arrays()
    return Problem(name=name, parent=parent, local_dim=local_dim, bond_dim=bond_dim,
                   op_leaf=[], op_mats=[], coeff=np.zeros(0, dtype=np.complex128), term_ops=[],
                   init_vecs={}, leaf_names=dict(tb.names), **kw)


def balanced_spec(items: List[object], bond_of_level, arity: int = 2, level: int = 0):
    """Nested spec of a balanced ``arity``-ary tree over ``items`` (leaf specs).

    ``bond_of_level(level)`` gives the requested bond of an interior node at the
    given height above the leaves' parents (0 = parent of leaves).
    """
    if len(items) == 1:
        return items[0]
    groups = np.array_split(np.arange(len(items)), min(arity, len(items)))
    kids = [balanced_spec([items[i] for i in g], bond_of_level, arity) for g in groups]
    height = _height(kids)
    return ("node", bond_of_level(height), kids)


def _height(kids) -> int:
    def h(s):
        if s[0] == "leaf":
            return -1
        return 1 + max(h(k) for k in s[2])
    return 1 + max(h(k) for k in kids)


def add_term(p: Problem, coef: complex, ops: List[int]) -> None:
    leaves = [p.op_leaf[o] for o in ops]
    if len(set(leaves)) != len(leaves):
        raise ValueError("a term may hold at most one operator per leaf")
    p.term_ops.append(list(ops))
    p.coeff = np.append(p.coeff, np.complex128(coef))
