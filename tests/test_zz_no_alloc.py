"""The allocation-free matvec (defmm_matvec_noalloc), whose workspace is the
library's static device array, against the workspace matvec (defmm_matvec) on
the same plan and charges: the same kernels in the same order, so the same
bits.  Two calls in a row, the second on a smaller input, so a call that
depended on what the previous call left in the shared array would show."""
import numpy as np
import pytest

from paper_2202_04894_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def test_noalloc_matches_workspace_matvec_on_two_calls():
    from paper_2202_04894_amd import defmm
    cases = [
        ("sphere", 8192, 16.0, dict(order_L=4, ncrit=32, precision=defmm.C128)),
        ("ellipsoid", 3000, 30.0, dict(order_L=5, ncrit=24, eta=0.5, hf_threshold=1.0, dir_refine=1,
                                       precision=defmm.C64)),
    ]
    cap = defmm.noalloc_capacity()
    assert cap == 64 << 20
    for geom, n, kappa, kw in cases:
        X = W.GENERATORS[geom](n, 61)
        plan = defmm.Plan(X, None, kappa, defmm.Params(**kw))
        assert plan.stats()["m2l_pairs"] > 0
        q = torch.as_tensor(W.charges(n, 62), device="cuda").to(plan.cdtype)
        ref = defmm.Workspace(plan).matvec(q).cpu().numpy()
        p = torch.full((plan.nx,), float("nan"), dtype=plan.cdtype, device="cuda")
        defmm.matvec_noalloc(plan, q, p)
        got = p.cpu().numpy()
        print(f"noalloc {geom} n={n}: max |diff| = {np.abs(got - ref).max():.3e}", flush=True)
        np.testing.assert_array_equal(got, ref)


def test_noalloc_rejects_a_plan_beyond_its_capacity():
    from paper_2202_04894_amd import defmm
    X = W.sphere(300_000, 63)
    plan = defmm.Plan(X, None, 40.0, defmm.Params(order_L=5, ncrit=64, precision=defmm.C64))
    q = torch.zeros(plan.ny, dtype=plan.cdtype, device="cuda")
    p = torch.zeros(plan.nx, dtype=plan.cdtype, device="cuda")
    with pytest.raises(defmm.DefmmError, match="allocation-free"):
        defmm.matvec_noalloc(plan, q, p)
