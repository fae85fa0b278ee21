"""GMRES driver on top of the matvec.

CPU: the GMRES routine against numpy.linalg.solve on small dense systems
(operators given as torch matrix products on the CPU), including a
nonsymmetric complex system and a restart.  GPU: a second-kind system
alpha x + G (w x) = b on sphere points solved through libdefmm; the solution
is checked with an independent residual, alpha x + G (w x) - b computed by
the oracle's FP64 direct sum, which differs from the FMM only by the
method's approximation error.
"""
import numpy as np
import pytest

from paper_2202_04894_amd import solve

torch = pytest.importorskip("torch")


def _dense_case(n, seed, shift):
    rng = np.random.default_rng(seed)
    A = (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(n) + shift * np.eye(n)
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    return A, b


@pytest.mark.parametrize("n,restart,shift", [(40, 50, 3.0), (60, 8, 2.5), (25, 25, 1.5 + 1.0j)])
def test_gmres_matches_dense_solve(n, restart, shift):
    A, b = _dense_case(n, n, shift)
    At = torch.as_tensor(A)
    bt = torch.as_tensor(b)
    r = solve.gmres(lambda x: At @ x, bt, tol=1e-12, restart=restart, maxiter=400)
    assert r.converged
    ref = np.linalg.solve(A, b)
    assert np.linalg.norm(r.x.numpy() - ref) <= 1e-9 * np.linalg.norm(ref)
    # the residual estimates decrease within a cycle
    assert r.residuals[-1] <= 1e-12


def test_gmres_exact_in_few_steps_on_low_rank_update():
    """alpha I + rank-3: the Krylov space holds the solution after 4 steps."""
    rng = np.random.default_rng(3)
    n = 30
    U = rng.standard_normal((n, 3)) + 1j * rng.standard_normal((n, 3))
    Vt = rng.standard_normal((3, n))
    A = 2.0 * np.eye(n) + U @ Vt / n
    b = rng.standard_normal(n).astype(np.complex128)
    At = torch.as_tensor(A)
    r = solve.gmres(lambda x: At @ x, torch.as_tensor(b), tol=1e-12, restart=20)
    assert r.converged and r.iterations <= 4


def test_gmres_zero_rhs():
    r = solve.gmres(lambda x: 2 * x, torch.zeros(5, dtype=torch.complex128))
    assert r.converged and r.iterations == 0 and float(torch.abs(r.x).max()) == 0.0


@pytest.mark.gpu
@pytest.mark.parametrize("prec_name", ["C128", "C64"])
def test_second_kind_solve_on_the_gpu(prec_name):
    import oracle
    from paper_2202_04894_amd import defmm
    from paper_2202_04894_amd import workloads as W
    prec = getattr(defmm, prec_name)
    n, kappa, alpha = 3000, 12.0, 0.5
    X = W.sphere(n, 41)
    w = np.full(n, 4 * np.pi / n)  # equal-area point quadrature on the unit sphere
    b = W.charges(n, 42)
    prm = defmm.Params(order_L=5, ncrit=24, eta=0.5, dir_refine=1, precision=prec)
    plan = defmm.Plan(X, None, kappa, prm)
    ws = defmm.Workspace(plan)
    op = solve.SecondKindOperator(ws, alpha, w)
    bt = torch.as_tensor(b, device="cuda").to(plan.cdtype)
    tol = 1e-10 if prec == defmm.C128 else 1e-5
    r = solve.gmres(op, bt, tol=tol, restart=40, maxiter=200)
    assert r.converged, r.residuals[-5:]
    x = r.x.cpu().numpy().astype(np.complex128)
    D, _ = plan.geometry()
    Gx = oracle.direct_sum(X, X, w * x, kappa, 1e-12 * D)
    true_res = np.linalg.norm(alpha * x + Gx - b) / np.linalg.norm(b)
    # FMM method error of these settings plus the solve tolerance
    assert true_res < 5e-3, true_res
    assert op.matvecs >= r.iterations
