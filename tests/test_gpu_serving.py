"""Serving on the GPU: requests of different sizes, geometries and kappa run
concurrently (own workspace and stream each, shared cached plans) and give
the same potentials as each request alone, bit for bit: every kernel owns
its outputs and sums in a fixed order, and no state is shared between
workspaces.  Also checked against a direct plan/workspace matvec, and with
a memory budget that forces queueing."""
import numpy as np
import pytest

from paper_2202_04894_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _requests(n_matvecs=3):
    from paper_2202_04894_amd.serving import Request
    specs = [("sphere", 20000, 40.0, 5), ("ellipsoid", 35000, 90.0, 4), ("sphere", 20000, 40.0, 5),
             ("cube_surface", 12000, 25.0, 4), ("ellipsoid", 50000, 120.0, 5), ("sphere", 8000, 8.0, 4)]
    out = []
    for i, (kind, n, kD, L) in enumerate(specs):
        gseed = 700 + n

        def mk(kind=kind, n=n, gseed=gseed):
            return W.GENERATORS[kind](n, gseed)

        def ch(k, n=n, i=i):
            return W.charges(n, 4000 + 100 * i + k, np.complex64)

        out.append(Request(rid=i, geometry=f"{kind}-{n}-{kD}-{L}", make_points=mk, n_points=n, kappa=kD / 2,
                           order_L=L, ncrit=64, n_matvecs=n_matvecs, charges=ch, arrival=0.0))
    return out


def _run(reqs, slots, budget=64 << 30):
    from paper_2202_04894_amd.serving import DeviceExecutor, Scheduler
    ex = DeviceExecutor(keep_results=True)
    sch = Scheduler(ex, budget_bytes=budget, max_slots=slots, keep_results=True)
    out = sch.run(reqs)
    torch.cuda.synchronize()
    return out, sch.stats


def test_mix_equals_alone_bitwise():
    reqs = _requests()
    mix, st = _run(reqs, slots=6)
    assert all(o.ok for o in mix), [o.error for o in mix]
    assert st["max_running"] >= 3 and st["builds"] == 5 and st["cache_hits"] == 1
    for r in reqs:
        alone, _ = _run([r], slots=1)
        for a, b in zip(alone[0].results, mix[r.rid].results):
            assert np.array_equal(a, b), r.rid
    for o in mix:
        assert len(o.matvec_ms) == 3 and min(o.matvec_ms) > 0 and o.done >= o.admitted >= 0


def test_serving_matches_direct_matvec():
    from paper_2202_04894_amd import defmm
    r = _requests()[1]
    out, _ = _run([r], slots=1)
    X = torch.as_tensor(r.make_points(), device="cuda")
    plan = defmm.Plan(X, None, r.kappa, defmm.Params(order_L=r.order_L, ncrit=r.ncrit, precision=defmm.C64))
    ws = defmm.Workspace(plan)
    for k in range(r.n_matvecs):
        p = ws.matvec(torch.as_tensor(r.charges(k), device="cuda")).cpu().numpy()
        assert np.array_equal(p, out[0].results[k])


def test_budget_forces_queueing_on_device():
    from paper_2202_04894_amd.serving import DeviceExecutor
    reqs = _requests(n_matvecs=2)
    ex = DeviceExecutor()
    fps = []
    for r in reqs:
        plan, pb, wb = ex.build(r)
        fps.append(pb + wb)
        ex.release_plan(plan)
    # room for the largest request and a little more: requests queue, plans
    # are built, used and evicted in turn, and the budget is never exceeded
    budget = int(1.2 * max(fps))
    out, st = _run(reqs, slots=6, budget=budget)
    assert all(o.ok for o in out), [o.error for o in out]
    assert st["peak_bytes"] <= budget and st["evictions"] > 0 and st["max_running"] < len(reqs)
    print("footprints (MB):", [round(f / 2 ** 20, 1) for f in fps], "stats:", st)


def test_solve_requests_in_the_mix():
    """GMRES solves as serving requests (alpha x + G (w x) = b, a data-dependent
    number of matvecs each), admitted and run concurrently with matvec requests:
    every solve converges in the FMM's own residual, and its solution meets the
    system built from the oracle's FP64 direct sum up to the method error of the
    paper-literal knobs."""
    import oracle
    from paper_2202_04894_amd.serving import Request, SURFACE_AREA
    reqs = _requests(n_matvecs=2)[:3]
    specs = [("sphere", 4000, 20.0, 5), ("ellipsoid", 6000, 30.0, 4), ("sphere", 3000, 12.0, 5)]
    for i, (kind, n, kD, L) in enumerate(specs):
        gseed = 900 + n

        def mk(kind=kind, n=n, gseed=gseed):
            return W.GENERATORS[kind](n, gseed)

        reqs.append(Request(rid=10 + i, geometry=f"{kind}-{n}-{kD}-{L}", make_points=mk, n_points=n,
                            kappa=kD / 2, order_L=L, ncrit=64, n_matvecs=0, arrival=0.0,
                            solve=dict(alpha=0.5, weight=SURFACE_AREA[kind] / n, tol=1e-5, restart=30,
                                       maxiter=150, seed=77 + i)))
    out, st = _run(reqs, slots=6)
    assert all(o.ok for o in out), [o.error for o in out]
    assert st["max_running"] >= 4
    for r, o in zip(reqs, out):
        if r.solve is None:
            assert len(o.results) == 2
            continue
        assert o.info["converged"] and o.info["matvecs"] > o.info["iterations"] > 1, o.info
        x, b = (v.astype(np.complex128) for v in o.results)
        X = r.make_points()
        D = float((X.max(0) - X.min(0)).max())
        w = np.full(r.n_points, r.solve["weight"])
        Gx = oracle.direct_sum(X, X, w * x, r.kappa, 1e-12 * D)
        true_res = np.linalg.norm(0.5 * x + Gx - b) / np.linalg.norm(b)
        print(f"solve {r.rid}: {o.info['iterations']} iterations, {o.info['matvecs']} matvecs, "
              f"direct-sum residual {true_res:.2e}")
        assert true_res < 5e-2, true_res
