"""defmm_matvec_graph: the matvec captured once into a HIP graph and replayed.
Every replay is checked bit for bit against the eager matvec on the same
charges, with the program's own eager work and synchronisations between the
replays; changes of q/p buffers or of the execution choices recapture."""
import numpy as np
import pytest

from paper_2202_04894_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec_name", ["C64", "C128"])
def test_graph_replays_equal_eager(prec_name):
    from paper_2202_04894_amd import defmm
    prec = getattr(defmm, prec_name)
    X = W.ellipsoid(20000, 41)
    plan = defmm.Plan(X, None, 60.0, defmm.Params(order_L=5, ncrit=32, precision=prec))
    wg, we = defmm.Workspace(plan), defmm.Workspace(plan)
    s = torch.cuda.Stream()
    q = torch.empty(plan.ny, dtype=plan.cdtype, device="cuda")
    p = torch.empty(plan.nx, dtype=plan.cdtype, device="cuda")
    p2 = torch.empty_like(p)
    for k in range(6):
        qk = torch.as_tensor(W.charges(plan.ny, 50 + k), device="cuda").to(plan.cdtype)
        with torch.cuda.stream(s):
            q.copy_(qk)
            out = p2 if k == 3 else p           # a new output buffer recaptures
            if k == 2:
                wg.set_overlap(False)           # a new execution choice recaptures
            if k == 4:
                wg.set_overlap(True)            # near field forked after the gather
            if k == 5:                          # ... and after M2F
                wg.set_tuning(overlap=2, p2p_waves_per_cu=3, m2l_variant=2, dense_levels=0)
            wg.matvec(q, out, stream=s, graph=True)
        s.synchronize()
        ref = we.matvec(qk)
        torch.cuda.synchronize()
        # eager work of the program between replays
        junk = torch.randn(1 << 16, device="cuda").sum()
        torch.cuda.synchronize()
        assert torch.equal(out, ref), (prec_name, k)
        assert float(junk) == float(junk)


def test_graph_needs_a_created_stream():
    from paper_2202_04894_amd import defmm
    X = W.sphere(2000, 3)
    plan = defmm.Plan(X, None, 10.0, defmm.Params(ncrit=32))
    ws = defmm.Workspace(plan)
    q = torch.zeros(plan.ny, dtype=plan.cdtype, device="cuda")

    class Null:
        cuda_stream = 0
    with pytest.raises(defmm.DefmmError, match="null stream"):
        ws.matvec(q, stream=Null(), graph=True)
