"""Iterative solves on top of the FMM matvec: restarted GMRES on the device.

The paper names boundary-integral solves as the use the fast matvec is for
(its conclusion); this module runs them without leaving the GPU.  Every
product with the kernel matrix is one defmm matvec (libdefmm's HIP kernels);
the Krylov basis, the Arnoldi inner products and the small least-squares
problem stay in torch tensors on the same device and stream.

`SecondKindOperator` is the discretised operator of a second-kind integral
equation with point quadrature, x -> alpha x + G (w * x), where G is the
Helmholtz kernel matrix the plan evaluates (self-pairs excluded) and w the
quadrature weights.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


class SecondKindOperator:
    """x -> alpha * x + G (w * x) on the plan's points (X = Y)."""

    def __init__(self, workspace, alpha: complex, weights=None, stream=None):
        import torch
        plan = workspace.plan
        if plan.nx != plan.ny:
            raise ValueError("a second-kind operator needs the same target and source points")
        self.ws, self.alpha, self.stream = workspace, alpha, stream
        self.n, self.dtype = plan.nx, plan.cdtype
        w = np.ones(self.n) if weights is None else np.asarray(weights, dtype=np.float64)
        real = torch.float32 if self.dtype == torch.complex64 else torch.float64
        self.w = torch.as_tensor(w, device="cuda").to(real)
        self._q = torch.empty(self.n, dtype=self.dtype, device="cuda")
        self._p = torch.empty(self.n, dtype=self.dtype, device="cuda")
        self.matvecs = 0

    def __call__(self, x):
        import torch
        torch.mul(x, self.w, out=self._q)
        self.ws.matvec(self._q, self._p, stream=self.stream)
        self.matvecs += 1
        return self.alpha * x + self._p


@dataclass
class GmresResult:
    x: object
    converged: bool
    iterations: int
    residuals: list = field(default_factory=list)  # relative residual estimate after each iteration


def gmres(op, b, tol: float = 1e-6, restart: int = 30, maxiter: int = 300, x0=None) -> GmresResult:
    """Restarted GMRES(restart) for op(x) = b, op a callable on 1-D complex
    device tensors (Saad and Schultz; modified Gram-Schmidt Arnoldi, Givens
    rotations on the Hessenberg matrix).  Stops when the residual estimate
    |r| / |b| <= tol or after maxiter inner iterations; the true residual is
    recomputed at each restart."""
    import torch
    dev, dt = b.device, b.dtype
    n = b.shape[0]
    bnorm = float(torch.linalg.vector_norm(b))
    x = torch.zeros_like(b) if x0 is None else x0.clone()
    res = []
    if bnorm == 0.0:
        return GmresResult(x, True, 0, [0.0])
    it = 0
    while it < maxiter:
        r = b - op(x)
        beta = float(torch.linalg.vector_norm(r))
        if beta / bnorm <= tol:
            res.append(beta / bnorm)
            return GmresResult(x, True, it, res)
        m = min(restart, maxiter - it)
        V = torch.empty((m + 1, n), dtype=dt, device=dev)
        V[0] = r / beta
        H = np.zeros((m + 1, m), dtype=np.complex128)
        cs = np.zeros(m, dtype=np.complex128)
        sn = np.zeros(m, dtype=np.complex128)
        g = np.zeros(m + 1, dtype=np.complex128)
        g[0] = beta
        k_done = 0
        for k in range(m):
            w = op(V[k])
            for j in range(k + 1):  # modified Gram-Schmidt
                h = torch.vdot(V[j], w)
                H[j, k] = complex(h)
                w = w - h * V[j]
            H[k + 1, k] = float(torch.linalg.vector_norm(w))
            if H[k + 1, k] != 0.0:
                V[k + 1] = w / H[k + 1, k]
            for j in range(k):  # earlier rotations
                t = cs[j] * H[j, k] + sn[j] * H[j + 1, k]
                H[j + 1, k] = -np.conj(sn[j]) * H[j, k] + np.conj(cs[j]) * H[j + 1, k]
                H[j, k] = t
            # rotation [[cs, sn], [-conj(sn), conj(cs)]] taking (a, c) to (rho, 0)
            a, c = H[k, k], H[k + 1, k]
            rho = np.hypot(abs(a), abs(c))
            cs[k], sn[k] = (1.0, 0.0) if rho == 0.0 else (np.conj(a) / rho, np.conj(c) / rho)
            H[k, k] = cs[k] * a + sn[k] * c
            H[k + 1, k] = 0.0
            g[k + 1] = -np.conj(sn[k]) * g[k]
            g[k] = cs[k] * g[k]
            it += 1
            k_done = k + 1
            res.append(abs(g[k + 1]) / bnorm)
            if res[-1] <= tol or H[k, k] == 0.0:
                break
        y = np.linalg.solve(np.triu(H[:k_done, :k_done]), g[:k_done])
        x = x + torch.as_tensor(y, device=dev).to(dt) @ V[:k_done]
        if res[-1] <= tol:
            r = b - op(x)
            true = float(torch.linalg.vector_norm(r)) / bnorm
            res[-1] = true
            if true <= tol:
                return GmresResult(x, True, it, res)
    return GmresResult(x, False, it, res)
