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


class GmresStepper:
    """Restarted GMRES(restart) for op(x) = b as a resumable state machine
    (Saad and Schultz; modified Gram-Schmidt Arnoldi, complex Givens rotations
    on the Hessenberg matrix).

    `advance()` enqueues the next piece of device work without waiting for it:
    a residual b - op(x) (at the start and at every restart) or one Arnoldi
    step (one operator application, its orthogonalisation and normalisation).
    The few scalars the host needs (residual norm, Hessenberg column) are
    copied back asynchronously behind an event; `ready()` says whether that
    work has finished, and the next `advance()` consumes it on the host (the
    rotations, the convergence test, the small triangular solve at a restart)
    before enqueuing more.  A solve thus issues a data-dependent number of
    operator applications, and a serving loop can interleave many solves on
    one device.  `advance()` returns True once the solve has finished:
    converged when the residual estimate |r| / |b| <= tol, confirmed by a true
    residual, or stopped after maxiter inner iterations.

    With CPU tensors (stream None) every step completes at once."""

    def __init__(self, op, b, tol: float = 1e-6, restart: int = 30, maxiter: int = 300, x0=None, stream=None,
                 timed: bool = False):
        import torch
        self.torch = torch
        self.timed = timed  # events that can time the solve (the last one marks its end)
        self.op, self.b, self.tol = op, b, float(tol)
        self.restart, self.maxiter = int(restart), int(maxiter)
        self.stream = stream
        self.cuda = b.is_cuda
        self.x = torch.zeros_like(b) if x0 is None else x0.clone()
        self.residuals, self.iterations = [], 0
        self.converged, self.finished = False, False
        self.event = None
        self.state = "start"
        self.host = torch.zeros(self.restart + 2, dtype=torch.complex128, pin_memory=self.cuda)
        self._enqueue_residual(first=True)

    # -- device side
    def _ctx(self):
        import contextlib
        return self.torch.cuda.stream(self.stream) if (self.cuda and self.stream is not None) \
            else contextlib.nullcontext()

    def _publish(self, vals):
        """Copy a few device scalars to pinned host memory behind an event."""
        torch = self.torch
        v = torch.stack([t.to(torch.complex128).reshape(()) for t in vals])
        self.host[:v.shape[0]].copy_(v, non_blocking=True)
        if self.cuda:
            self.event = torch.cuda.Event(enable_timing=self.timed)
            self.event.record(self.stream if self.stream is not None else torch.cuda.current_stream())

    def _enqueue_residual(self, first=False):
        torch = self.torch
        with self._ctx():
            self.r = self.b - self.op(self.x)
            norms = [torch.linalg.vector_norm(self.r)]
            if first:
                norms.append(torch.linalg.vector_norm(self.b))
            self._publish(norms)
        self.state = "residual0" if first else "residual"

    def _enqueue_arnoldi(self):
        torch = self.torch
        k = self.k
        with self._ctx():
            w = self.op(self.V[k])
            hs = []
            for j in range(k + 1):  # modified Gram-Schmidt
                h = torch.vdot(self.V[j], w)
                hs.append(h)
                w = w - h * self.V[j]
            hn = torch.linalg.vector_norm(w)
            self.V[k + 1] = w / hn
            self._publish(hs + [hn])
        self.state = "arnoldi"

    # -- host side
    def ready(self) -> bool:
        return self.finished or self.event is None or self.event.query()

    def advance(self) -> bool:
        if self.finished:
            return True
        if self.cuda and self.event is not None:
            self.event.synchronize()
        torch = self.torch
        h = self.host.numpy()
        if self.state == "residual0":
            self.bnorm = float(h[1].real)
            if self.bnorm == 0.0:
                self.x = torch.zeros_like(self.b)
                self.residuals.append(0.0)
                return self._finish(True)
        if self.state in ("residual0", "residual"):
            beta = float(h[0].real)
            if beta / self.bnorm <= self.tol:
                if self.state == "residual" and self.residuals:
                    self.residuals[-1] = beta / self.bnorm
                else:
                    self.residuals.append(beta / self.bnorm)
                return self._finish(True)
            if self.state == "residual" and self.residuals and self.residuals[-1] <= self.tol:
                self.residuals[-1] = beta / self.bnorm  # the estimate was optimistic: restart
            if self.iterations >= self.maxiter:
                return self._finish(False)
            m = min(self.restart, self.maxiter - self.iterations)
            self.m = m
            with self._ctx():
                self.V = torch.empty((m + 1, self.b.shape[0]), dtype=self.b.dtype, device=self.b.device)
                self.V[0] = self.r / beta
            self.H = np.zeros((m + 1, m), dtype=np.complex128)
            self.cs = np.zeros(m, dtype=np.complex128)
            self.sn = np.zeros(m, dtype=np.complex128)
            self.g = np.zeros(m + 1, dtype=np.complex128)
            self.g[0] = beta
            self.k = 0
            self._enqueue_arnoldi()
            return False
        # an Arnoldi step has finished: Hessenberg column k
        k, H, cs, sn, g = self.k, self.H, self.cs, self.sn, self.g
        H[:k + 1, k] = h[:k + 1]
        H[k + 1, k] = h[k + 1].real
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
        self.iterations += 1
        self.residuals.append(abs(g[k + 1]) / self.bnorm)
        done_cycle = self.residuals[-1] <= self.tol or H[k, k] == 0.0 or k + 1 == self.m
        if not done_cycle:
            self.k = k + 1
            self._enqueue_arnoldi()
            return False
        kd = k + 1
        y = np.linalg.solve(np.triu(H[:kd, :kd]), g[:kd])
        with self._ctx():
            self.x = self.x + torch.as_tensor(y).to(device=self.b.device, dtype=self.b.dtype) @ self.V[:kd]
        # the true residual decides (at convergence) or starts the next cycle
        self._enqueue_residual()
        return False

    def _finish(self, converged):
        self.converged, self.finished = converged, True
        return True

    def result(self) -> "GmresResult":
        return GmresResult(self.x, self.converged, self.iterations, list(self.residuals))


def gmres(op, b, tol: float = 1e-6, restart: int = 30, maxiter: int = 300, x0=None, stream=None) -> GmresResult:
    """Restarted GMRES(restart) for op(x) = b, op a callable on 1-D complex
    device tensors, run to the end (GmresStepper driven until it finishes)."""
    st = GmresStepper(op, b, tol=tol, restart=restart, maxiter=maxiter, x0=x0, stream=stream)
    while not st.advance():
        pass
    return st.result()
