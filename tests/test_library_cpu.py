"""Host-side checks of the HIP library (no GPU needed): exported symbols, tree
validation, bond clamping and the sparse tree operator (hSOP) compiler."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2503_15460_amd as T
from oracle import clamp_bonds as oracle_clamp
from oracle import dense_sop
from workloads import heom_sbm_problem, sbm_problem, vibronic_problem
from workloads.models import boson_ops

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    names = set()
    for h in ("ttn.h", "ttn_debug.h"):
        src = open(os.path.join(ROOT, "include", h)).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        names |= set(re.findall(r"\b(ttn_[a-z_0-9]+)\s*\(", src))
    return names


def test_every_declared_symbol_is_exported():
    names = declared_symbols()
    assert len(names) >= 15
    for n in names:
        assert hasattr(T.lib, n), n
    assert names == set(T._lib.EXPORTED)


def test_clamp_matches_oracle():
    for p in (sbm_problem(), vibronic_problem(), heom_sbm_problem(),
              sbm_problem(n_modes=5, d=3, bond=100)):
        assert np.array_equal(T.clamp_bonds(p.parent, p.local_dim, p.bond_dim),
                              oracle_clamp(p.parent, p.local_dim, p.bond_dim))


def test_tree_errors():
    with pytest.raises(T.TTNError) as e:
        T.clamp_bonds([-1, 0, 1, 2], [0, 0, 2, 2], [1, 2, 2, 2])  # node 2 has a child but d > 0
    assert "E_DIMS" in str(e.value)
    with pytest.raises(T.TTNError) as e:
        T.clamp_bonds([-1, -1, 0], [0, 2, 2], [1, 1, 1])
    assert "E_TREE" in str(e.value)
    with pytest.raises(T.TTNError) as e:
        T.clamp_bonds([1, 2, 0], [2, 0, 0], [1, 1, 1])  # cycle, no root
    assert "E_TREE" in str(e.value)


def _small_vibronic():
    return vibronic_problem(n_modes=8, dmin=2, dmax=2, leaf_bond=2, l_bond=3, m_bond=3)


@pytest.mark.parametrize("make", [
    lambda: sbm_problem(n_modes=4, d=3, bond=4),
    lambda: sbm_problem(n_modes=5, d=2, bond=4, alpha=0.7),
    _small_vibronic,
    lambda: heom_sbm_problem(K=2, levels=3),
])
def test_tree_operator_equals_sop(make):
    """The compiled hierarchical SOP represents exactly the SOP generator (Sec. II B 2)."""
    p = make()
    G = dense_sop(p)
    D, n_ent = T.dense_tree_operator(p, max_dim=5000)
    assert np.abs(G - D).max() <= 1e-12 * max(1.0, np.abs(G).max())
    assert n_ent > 0


def test_tree_operator_compresses_star_coupling():
    """Star-coupled bath: O(1) channels per node (the hSOP form), not O(N) per node."""
    per_node = []
    for n in (8, 16, 32, 64):
        p = sbm_problem(n_modes=n, d=2, bond=4)
        per_node.append(T.tree_operator_entries(p) / p.n_nodes)
    assert max(per_node) < 4.0
    assert per_node[-1] - per_node[0] < 0.2


def test_invalid_sop_rejected():
    p = sbm_problem(n_modes=2, d=2, bond=2)
    p.term_ops.append([p.observables["sz"][0], p.observables["sz"][0]])  # two ops on one leaf
    p.coeff = np.append(p.coeff, 1.0)
    with pytest.raises(T.TTNError) as e:
        T.dense_tree_operator(p)
    assert "E_INVALID" in str(e.value)


@pytest.mark.parametrize("where", ["coefficient", "operator"])
def test_non_finite_sop_rejected(where):
    """A NaN coefficient or an infinite operator entry is refused on the host."""
    p = sbm_problem(n_modes=2, d=2, bond=2)
    if where == "coefficient":
        p.coeff = np.array(p.coeff, dtype=np.complex128)
        p.coeff[1] = complex(np.nan, 0.0)
    else:
        p.op_mats[p.observables["sz"][0]] = np.array([[np.inf, 0], [0, -1]], dtype=np.complex128)
    with pytest.raises(T.TTNError) as e:
        T.dense_tree_operator(p)
    assert "E_INVALID" in str(e.value)
