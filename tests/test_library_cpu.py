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
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if not h.endswith(".h"):
            continue
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


def test_node_with_too_many_children_is_refused():
    """Node tensors carry at most 8 indices: a root with 8 leaf children is a
    legal tree shape the library does not take (TTN_E_TREE, not a crash)."""
    ok = T.clamp_bonds([-1] + [0] * 7, [0] + [2] * 7, [1] + [2] * 7)  # 7 children: accepted
    assert ok.tolist() == [1] + [2] * 7
    with pytest.raises(T.TTNError) as e:
        T.clamp_bonds([-1] + [0] * 8, [0] + [2] * 8, [1] + [2] * 8)
    assert "E_TREE" in str(e.value)


def _dense_defect(p):
    G = dense_sop(p)
    return np.linalg.norm(G - G.conj().T) / np.linalg.norm(G)


def test_hermiticity_defect_is_the_dense_norm():
    """The host check of hermitian = 1 evaluates ||G - G^dag||_F / ||G||_F from
    the leaf operators; it equals the norm of the dense matrices."""
    p = sbm_problem(n_modes=3, d=3, bond=3)
    assert T.hermiticity_defect(p) < 1e-14
    h = heom_sbm_problem(K=1, levels=3)  # non-Hermitian generator
    d_dense, d_lib = _dense_defect(h), T.hermiticity_defect(h)
    assert d_dense > 1e-2 and abs(d_lib - d_dense) < 1e-10 * d_dense
    # Hermitian only as a sum: sigma_+ and sigma_- written as separate terms
    q = sbm_problem(n_modes=2, d=3, bond=3)
    sp = np.array([[0, 1], [0, 0]], dtype=np.complex128)
    spin = q.op_leaf[q.observables["sz"][0]]
    q.op_leaf = list(q.op_leaf) + [spin, spin]
    q.op_mats = list(q.op_mats) + [sp, sp.conj().T]
    n = len(q.op_leaf)
    q.term_ops = list(q.term_ops) + [[n - 2], [n - 1]]
    q.coeff = np.append(np.asarray(q.coeff, dtype=np.complex128), [0.3 + 0.2j, 0.3 - 0.2j])
    assert T.hermiticity_defect(q) < 1e-12 and _dense_defect(q) < 1e-14
    q.coeff[-1] = 0.3 + 0.2j  # now not Hermitian
    d_dense, d_lib = _dense_defect(q), T.hermiticity_defect(q)
    assert d_dense > 1e-2 and abs(d_lib - d_dense) < 1e-10 * d_dense


def test_numerically_hermitian_operator_is_accepted():
    """A leaf operator that is Hermitian up to rounding (not bit-symmetric)
    passes the check; a perturbation above the tolerance does not."""
    p = sbm_problem(n_modes=2, d=4, bond=3)
    o = p.observables["sz"][0]
    m = np.array(p.op_mats[o], dtype=np.complex128)
    m[0, 1] += 1e-15
    p.op_mats[o] = m
    assert T.hermiticity_defect(p) < 1e-12
    m = m.copy()
    m[0, 1] += 1e-3
    p.op_mats[o] = m
    assert T.hermiticity_defect(p) > 1e-7


def test_tile_table_round_trip(tmp_path):
    """The autotuner's table is persisted as JSON: a saved table loads back
    with the same entries; entries naming tiles this build lacks are skipped."""
    T.tile_table_clear()
    src = tmp_path / "tiles.json"
    src.write_text('{"ttn_tile_table": 1, "entries": [\n'
                   ' ["f64|nmax=16|nmin=16|N=65536|ents=12|R1=1", 1, 16, 12.5],\n'
                   ' ["f32|nmax=48|nmin=48|N=7077888|ents=71|R1=1", 3, 16, 300.25],\n'
                   ' ["f64|nmax=8|nmin=8|N=4096|ents=3|R1=0", 5, 7, 1.0]\n'
                   ']}\n')
    assert T.tile_table_load(str(src)) == 2
    assert T.tile_table_size() == 2
    out = tmp_path / "saved.json"
    T.tile_table_save(str(out))
    import json
    rec = json.loads(out.read_text())
    assert sorted(e[0] for e in rec["entries"]) == sorted([
        "f64|nmax=16|nmin=16|N=65536|ents=12|R1=1", "f32|nmax=48|nmin=48|N=7077888|ents=71|R1=1"])
    T.tile_table_clear()
    assert T.tile_table_size() == 0
    assert T.tile_table_load(str(out)) == 2
    T.tile_table_clear()
    with pytest.raises(T.TTNError):
        T.tile_table_load(str(tmp_path / "missing.json"))
