"""The C-ABI library loads and exports every function the header declares
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ambddc.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(ambddc_[a-z0-9_]+)\s*\(", txt)))


def test_header_declares_the_binding_surface():
    from paper_1301_0191_amd._lib import EXPORTED
    assert sorted(EXPORTED) == _declared()


def test_library_exports_every_declared_symbol():
    from paper_1301_0191_amd._lib import LIB_PATH
    if not os.path.exists(LIB_PATH):
        pytest.skip("libambddc.so not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(LIB_PATH)
    for name in _declared():
        assert hasattr(lib, name), name


def test_binding_refuses_missing_library(tmp_path):
    from paper_1301_0191_amd import _lib
    saved = _lib._lib
    _lib._lib = None
    try:
        with pytest.raises(RuntimeError, match="not built"):
            _lib.load(str(tmp_path / "missing.so"))
    finally:
        _lib._lib = saved


def test_default_options_without_gpu():
    from paper_1301_0191_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libambddc.so not built")
    lib = _lib.load()
    opt = _lib.Options()
    lib.ambddc_default_options(ctypes.byref(opt))
    assert opt.tau == 10.0 and opt.nev_max == 10 and opt.lobpcg_block == 16
    assert opt.precision == 0


def _oracle_structure(prob, initial="c+e"):
    """Level-1 structure counts from the oracle's own classification."""
    import numpy as np
    from oracle.substructure import classify, level1_input
    inp = level1_input(prob, Ke=False)
    node_sets, globs = classify(inp)
    dof_iface = np.zeros(inp.n_dof, dtype=bool)
    for g in globs:
        dof_iface[g["dofs"]] = True
    sub_dofs = [set() for _ in range(inp.n_sub)]
    for e, dd in enumerate(inp.elem_dofs):
        sub_dofs[int(inp.elem_sub[e])].update(int(x) for x in dd[dd >= 0])
    sizes = np.array([[sum(1 for j in d if not dof_iface[j]), sum(1 for j in d if dof_iface[j])]
                      for d in sub_dofs])
    types = [g["type"] for g in globs]
    n_coarse = 0
    for g in globs:
        if g["type"] == "corner":
            n_coarse += len(g["dofs"])
        elif (g["type"] == "edge" and initial != "c") or (g["type"] == "face" and
                                                           initial == "c+e+f"):
            n_coarse += len(np.unique(inp.dof_comp[g["dofs"]]))
    return dict(n_free=inp.n_dof, n_sub=inp.n_sub, n_interface=int(dof_iface.sum()),
                n_faces=types.count("face"), n_edges=types.count("edge"),
                n_corners=types.count("corner"), n_coarse_initial=n_coarse,
                n_pairs=types.count("face"), sub_sizes=sizes)


@pytest.mark.parametrize("case", ["c1", "c2", "ragged", "elasticity", "c3_boxes"])
def test_host_analysis_matches_oracle_classification(case):
    """ambddc_analyze (host integer logic of the library: DOF numbering,
    glob classification, initial constraints, pairs) against the oracle."""
    import numpy as np
    from paper_1301_0191_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libambddc.so not built")
    import workloads as W
    from paper_1301_0191_amd import analyze
    if case in ("c1", "c2"):
        prob = W.CONFIGS[case](0)
    elif case == "ragged":
        prob = W.make_problem((9, 7, 6), None, coeff="lognormal", seed=3,
                              cuts=[[0, 1, 5, 9], [0, 3, 7], [0, 4, 6]])
    elif case == "elasticity":
        prob = W.tiny_elasticity(shape=(6, 6, 6), subs=(3, 2, 2), seed=2)
    else:
        # uneven boxes with elasticity DOFs, like the elasticity workload's cuts
        prob = W.make_problem((20, 18, 16), None, dof_per_node=3, seed=4,
                              cuts=[[0, 5, 11, 20], [0, 7, 18], [0, 6, 10, 16]])
    for fa in ("c+e", "c+e+f", "c"):
        got = analyze(prob.coords, prob.elem_nodes, prob.dirichlet, prob.dof_per_node,
                      prob.elem_to_sub, initial=fa)
        want = _oracle_structure(prob, initial=fa)
        for k in ("n_free", "n_sub", "n_interface", "n_faces", "n_edges", "n_corners",
                  "n_coarse_initial", "n_pairs"):
            assert got[k] == want[k], (case, fa, k, got[k], want[k])
        np.testing.assert_array_equal(got["sub_sizes"], want["sub_sizes"])
