"""The full-size downward-pass check, run on the CPU against the oracle's own
matvec: it accepts the oracle's expansions and potentials to rounding, and it
rejects a local expansion or a potential with one element changed."""
import numpy as np
import pytest

import oracle
from downward_check import downward_check
from paper_2202_04894_amd import workloads as W


@pytest.mark.parametrize("geom,n,kappa,kw", [
    ("sphere", 4000, 48.0, dict(L=4, ncrit=16, eta=0.5, hf_threshold=0.75, dir_refine=1)),
    ("ellipsoid", 3000, 0.0, dict(L=3, ncrit=12)),
])
def test_downward_check_accepts_the_oracle_and_rejects_a_change(geom, n, kappa, kw):
    X = W.GENERATORS[geom](n, 41)
    q = W.charges(n, 42)
    prm = oracle.Params(**kw)
    F = oracle.FMM(X, None, kappa, prm)
    p = F.apply(q)
    D, org = F.geometry()
    cells = F.cells(0)
    tree = dict(cells, perm=F.perm(0))
    ex = F.expansions(0)
    args = dict(kappa=kappa, L=prm.L, kernel=oracle.HELMHOLTZ, hf_threshold=prm.hf_threshold,
                dir_refine=prm.dir_refine, D=D, origin=org, tree=tree, m2l=F.m2l(), p2p=F.p2p(),
                mult=(ex["cell"], ex["dir"], ex["M"]), X=X, q=q, n_local=400, n_leaf=40, tol=1e-12, seed=1)
    n_loc, n_leaf = downward_check(loc=(ex["cell"], ex["dir"], ex["L"]), p=p, **args)
    assert n_loc > 50 and n_leaf == 40
    # one element of every local expansion changed by 1e-9 of its scale
    bad = ex["L"].copy()
    bad[:, 7] += 1e-9 * np.abs(bad).max(axis=1)
    with pytest.raises(AssertionError):
        downward_check(loc=(ex["cell"], ex["dir"], bad), p=p, **args)
    # one potential per leaf changed
    pb = p.copy()
    perm = tree["perm"]
    for c in np.nonzero(cells["is_leaf"])[0]:
        pb[perm[cells["first"][c]]] *= 1 + 1e-9
    with pytest.raises(AssertionError):
        downward_check(loc=(ex["cell"], ex["dir"], ex["L"]), p=pb, **args)
