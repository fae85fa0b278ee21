"""The device builder (HIP kernels: bounding cube, Morton sort, Ncrit tree,
level-synchronous dual tree traversal, best directions, marks) against the
host builder of the inspection plan, which the CPU tests pin to the oracle:
trees, M2L and P2P lists (in list order), marks and geometry are identical.
"""
import numpy as np
import pytest

from paper_2202_04894_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _defmm():
    from paper_2202_04894_amd import defmm
    return defmm


CASES = [
    ("sphere", 3000, None, 24.0, dict(order_L=5, ncrit=24, eta=0.5, hf_threshold=2.0, dir_refine=1)),
    ("ellipsoid", 5000, None, 48.0, dict(order_L=4, ncrit=20, hf_threshold=1.0)),
    ("cube_surface", 4000, None, 30.0, dict(order_L=3, ncrit=40, eta=0.7, dir_refine=2)),
    ("cube_volume", 3000, None, 12.0, dict(order_L=6, ncrit=50)),
    ("cube_volume", 6000, None, 6.0, dict(order_L=3, ncrit=3)),
    ("sphere", 4000, None, 0.0, dict(order_L=4, ncrit=32)),
    ("sphere", 2500, "cube_volume", 30.0, dict(order_L=4, ncrit=12, hf_threshold=1.0)),
    ("ellipsoid", 60000, None, 120.0, dict(order_L=5, ncrit=64, dir_refine=1)),
]


def _compare(X, Y, kappa, kw):
    defmm = _defmm()
    prm = defmm.Params(precision=defmm.C64, **kw)
    dev = defmm.Plan(X, Y, kappa, prm)
    host = defmm.Plan.inspect(X, Y, kappa, prm)
    D1, o1 = dev.geometry()
    D2, o2 = host.geometry()
    assert D1 == D2 and np.array_equal(o1, o2)
    for which in ((0,) if Y is None else (0, 1)):
        a, b = dev.tree(which), host.tree(which)
        for k in ("level", "ijk", "first", "count", "is_leaf", "perm"):
            np.testing.assert_array_equal(a[k], b[k], err_msg=f"tree {which} {k}")
        ma, mb = dev.marks(which), host.marks(which)
        for k in ("cell", "dir"):
            np.testing.assert_array_equal(ma[k], mb[k], err_msg=f"marks {which} {k}")
    ma, mb = dev.m2l(), host.m2l()
    for k in ("level", "t", "s", "delta", "dir"):
        np.testing.assert_array_equal(ma[k], mb[k], err_msg=f"m2l {k}")
    pa, pb = dev.p2p(), host.p2p()
    for k in ("t", "s"):
        np.testing.assert_array_equal(pa[k], pb[k], err_msg=f"p2p {k}")
    sa, sb = dev.stats(), host.stats()
    assert sa == sb
    return sa


@pytest.mark.parametrize("geom,n,ygeom,kappa,kw", CASES)
def test_device_builder_equals_host_builder(geom, n, ygeom, kappa, kw):
    X = W.GENERATORS[geom](n, 201)
    Y = None if ygeom is None else W.GENERATORS[ygeom](n // 2, 202) * 0.6
    st = _compare(X, Y, kappa, kw)
    assert st["m2l_pairs"] > 0


def test_device_builder_degenerate_inputs():
    # coincident points (the tree runs to the deepest level), one point, two points
    _compare(np.tile([[0.3, -0.2, 0.1]], (300, 1)), None, 5.0, dict(ncrit=16))
    _compare(np.array([[0.1, 0.2, 0.3]]), None, 5.0, dict())
    _compare(np.array([[0.1, 0.2, 0.3], [0.4, -0.5, 0.6]]), None, 5.0, dict(ncrit=1))


def test_device_builder_rejects_non_finite():
    defmm = _defmm()
    X = W.sphere(500, 3)
    X[7, 2] = np.nan
    with pytest.raises(defmm.DefmmError, match="non-finite"):
        defmm.Plan(X, None, 4.0, defmm.Params())
