"""Host logic of libdefmm against the oracle, on the CPU (no device use).

The plan builder in the library is written independently of the oracle; both
follow the paper's definitions (Morton/Ncrit tree of Sec. 4.2.1, Alg. 1 with
the MAC of eq. macdirref, best direction of Alg. 2), so the trees and the
M2L/P2P lists must agree exactly (integer data, compared after sorting).
"""
import ctypes

import numpy as np
import pytest

import oracle
from paper_2202_04894_amd import defmm
from paper_2202_04894_amd import workloads as W


def test_library_exports_every_declared_symbol():
    """Every entry point declared in include/defmm.h is exported by libdefmm.so."""
    import os
    import re
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    hdr = open(os.path.join(root, "include", "defmm.h")).read()
    declared = set(re.findall(r"^\s*(?:defmm_status|const char\*|size_t)\s+(defmm_\w+)\s*\(", hdr, re.M))
    assert len(declared) >= 20
    L = ctypes.CDLL(defmm.LIB_PATH)
    for name in sorted(declared):
        assert hasattr(L, name), name
    assert set(defmm.EXPORTS) == declared


def test_library_directions_match_the_closed_form():
    """The library derives its direction set by splitting father patches
    (Sec. 2.1); the goldens enumerate the closed form of Sec. 4.1.2 (E = 0, 1 as
    FP64 values, E = 2 as exact integer vectors).  Same vectors bit for bit,
    same fathers, and at E = 3..6 the same set as the oracle's own derivation."""
    import os
    golden = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
    rows = np.loadtxt(os.path.join(golden, "directions_E0_E1.txt"))
    for E in (0, 1):
        d, f = defmm.directions(E)
        g = rows[rows[:, 0] == E]
        np.testing.assert_allclose(d, g[:, 2:5], atol=1e-15)
        np.testing.assert_array_equal(f, g[:, 5].astype(np.int64))
    r2 = np.loadtxt(os.path.join(golden, "directions_E2.txt"), dtype=np.int64)
    d, f = defmm.directions(2)
    np.testing.assert_array_equal(d, r2[:, 1:4] / np.sqrt(r2[:, 4].astype(np.float64))[:, None])
    np.testing.assert_array_equal(f, r2[:, 5])
    for E in range(3, 7):
        d, f = defmm.directions(E)
        do, fo = oracle.directions(E)
        np.testing.assert_array_equal(d, do)
        np.testing.assert_array_equal(f, fo)
    with pytest.raises(defmm.DefmmError):
        defmm.directions(-1)


def _sorted_rows(*cols):
    a = np.column_stack([np.asarray(c).astype(np.int64).reshape(len(c), -1) for c in cols])
    return a[np.lexsort(a.T[::-1])] if len(a) else a


CASES = [
    ("sphere", 3000, 40.0, dict(L=4, ncrit=16)),
    ("ellipsoid", 4000, 64.0, dict(L=5, ncrit=24, hf_threshold=1.0, dir_refine=1, eta=0.5)),
    ("cube_surface", 3000, 0.0, dict(L=3, ncrit=10)),
    ("cube_volume", 2000, 25.0, dict(L=6, ncrit=20, eta=0.7)),
    # screened kernel at a screening that would make Helmholtz levels high-frequency
    ("sphere", 3000, 40.0, dict(L=4, ncrit=16, kernel=oracle.YUKAWA)),
]


@pytest.mark.parametrize("geom,n,kappa,kw", CASES)
def test_lists_match_oracle(geom, n, kappa, kw):
    X = W.GENERATORS[geom](n, 77)
    o = oracle.FMM(X, None, kappa, oracle.Params(**kw))
    screened = kw.get("kernel", oracle.HELMHOLTZ) == oracle.YUKAWA
    prm = defmm.Params(order_L=kw["L"], ncrit=kw["ncrit"], eta=kw.get("eta", 1.0),
                       hf_threshold=kw.get("hf_threshold", 2.0), dir_refine=kw.get("dir_refine", 0),
                       flags=defmm.YUKAWA if screened else 0)
    p = defmm.Plan.inspect(X, None, kappa, prm)
    D, org = p.geometry()
    Do, oo = o.geometry()
    assert D == Do and np.array_equal(org, oo)
    ct, co = p.tree(0), o.cells(0)
    np.testing.assert_array_equal(ct["perm"], o.perm(0))
    for k in ("level", "ijk", "first", "count", "is_leaf"):
        np.testing.assert_array_equal(ct[k], co[k])
    mp, mo = p.m2l(), o.m2l()
    assert len(mp["t"]) == len(mo["t"]) > 0 or kappa == 0
    np.testing.assert_array_equal(_sorted_rows(mp["level"], mp["t"], mp["s"], mp["delta"], mp["dir"]),
                                  _sorted_rows(mo["level"], mo["t"], mo["s"], mo["delta"], mo["dir"]))
    pp, po = p.p2p(), o.p2p()
    np.testing.assert_array_equal(_sorted_rows(pp["t"], pp["s"]), _sorted_rows(po["t"], po["s"]))
    st, info = p.stats(), o.info()
    assert st["m2l_pairs"] == info["m2l_pairs"]
    assert st["p2p_point_pairs"] == info["p2p_point_pairs"]
    assert st["eff_expansions"] == info["exp_x"]
    assert st["unique_offsets"] == info["unique_offsets"]
    assert st["levels"] == info["levels_x"]
    if screened:
        assert st["hf_levels"] == 0 and info["lstar"] == -1


def test_lists_match_oracle_distinct_sets():
    X = W.sphere(2500, 3)
    Y = W.cube_volume(1800, 4) * 0.6
    kw = dict(L=4, ncrit=12, hf_threshold=1.0)
    o = oracle.FMM(X, Y, 30.0, oracle.Params(**kw))
    p = defmm.Plan.inspect(X, Y, 30.0, defmm.Params(order_L=4, ncrit=12, hf_threshold=1.0))
    for which in (0, 1):
        ct, co = p.tree(which), o.cells(which)
        for k in ("level", "ijk", "first", "count", "is_leaf"):
            np.testing.assert_array_equal(ct[k], co[k])
    mp, mo = p.m2l(), o.m2l()
    np.testing.assert_array_equal(_sorted_rows(mp["level"], mp["t"], mp["s"], mp["delta"], mp["dir"]),
                                  _sorted_rows(mo["level"], mo["t"], mo["s"], mo["delta"], mo["dir"]))
    pp, po = p.p2p(), o.p2p()
    np.testing.assert_array_equal(_sorted_rows(pp["t"], pp["s"]), _sorted_rows(po["t"], po["s"]))
    st, info = p.stats(), o.info()
    assert st["eff_expansions"] == info["exp_x"] + info["exp_y"]


def test_invalid_arguments_are_rejected():
    X = W.sphere(100, 1)
    bad = [(dict(order_L=1), 0.0), (dict(order_L=9), 0.0), (dict(ncrit=0), 0.0), (dict(eta=0.0), 0.0),
           (dict(), -1.0), (dict(), float("nan")), (dict(precision=7), 0.0), (dict(m2l_mode=5), 0.0),
           (dict(flags=8), 0.0), (dict(flags=defmm.YUKAWA), -2.0)]
    for kw, kappa in bad:
        with pytest.raises(defmm.DefmmError, match="invalid argument"):
            defmm.Plan.inspect(X, None, kappa, defmm.Params(**kw))
    Xn = X.copy()
    Xn[5, 1] = np.inf
    with pytest.raises(defmm.DefmmError, match="non-finite"):
        defmm.Plan.inspect(Xn, None, 1.0, defmm.Params())
    # the dense M2L needs device matrices: an inspection plan accepts the mode
    for mode in (defmm.M2L_AUTO, defmm.M2L_DENSE):
        assert defmm.Plan.inspect(X, None, 1.0, defmm.Params(m2l_mode=mode)).stats()["m2l_pairs"] >= 0


def test_degenerate_geometries_build():
    p = defmm.Plan.inspect(np.zeros((0, 3)), None, 2.0, defmm.Params())
    assert p.stats()["m2l_pairs"] == 0
    Xc = np.tile([[0.1, 0.2, 0.3]], (500, 1))
    p = defmm.Plan.inspect(Xc, None, 2.0, defmm.Params(ncrit=16))
    st = p.stats()
    assert st["m2l_pairs"] == 0 and st["levels"] == 22
