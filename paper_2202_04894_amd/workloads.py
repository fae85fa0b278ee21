"""Seeded synthetic inputs (point clouds and charges).

This module holds no FMM arithmetic: it only draws points and charges with
numpy's PCG64 generator, so both the GPU path and the oracle can be fed the
same inputs.  The shapes mirror the distributions of the paper's numerical
section (surface of a sphere, an elongated ellipsoid concentrated at a pole,
the surface of a cube, the volume of a cube).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


def sphere(n: int, seed: int) -> np.ndarray:
    """Uniform on the unit sphere: g ~ N(0, I3), x = g / |g|."""
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((n, 3))
    return g / np.linalg.norm(g, axis=1, keepdims=True)


def _ellipsoid_by_area(rng, n, axes, cap_x=None):
    a, b, c = axes
    out = np.empty((0, 3))
    while out.shape[0] < n:
        m = max(2 * (n - out.shape[0]), 1024)
        g = rng.standard_normal((m, 3))
        u = g / np.linalg.norm(g, axis=1, keepdims=True)
        # area element of the map u -> (a ux, b uy, c uz), up to a constant:
        w = c * np.sqrt(u[:, 0] ** 2 / a ** 2 + u[:, 1] ** 2 / b ** 2 + u[:, 2] ** 2 / c ** 2)
        w = w / (c / min(a, b, c))  # max of the density is 1
        keep = rng.random(m) < w
        pts = u[keep] * np.array([a, b, c])
        if cap_x is not None:
            pts = pts[pts[:, 0] > cap_x]
        out = np.concatenate([out, pts], axis=0)
    return out[:n]


def ellipsoid(n: int, seed: int, axes=(1.0, 0.5, 0.25), cap_fraction=0.7, cap_x=0.8) -> np.ndarray:
    """Ellipsoid surface, uniform by area; cap_fraction of the points restricted to x > cap_x."""
    rng = np.random.default_rng(seed)
    n_cap = int(round(cap_fraction * n))
    cap = _ellipsoid_by_area(rng, n_cap, axes, cap_x)
    rest = _ellipsoid_by_area(rng, n - n_cap, axes, None)
    pts = np.concatenate([cap, rest], axis=0)
    return pts[rng.permutation(n)]


def cube_surface(n: int, seed: int) -> np.ndarray:
    """Surface of [-1,1]^3: face uniform in 6, two free coordinates uniform in [-1,1]."""
    rng = np.random.default_rng(seed)
    face = rng.integers(0, 6, n)
    uv = rng.uniform(-1.0, 1.0, (n, 2))
    pts = np.empty((n, 3))
    axis = face // 2
    sign = np.where(face % 2 == 0, 1.0, -1.0)
    for a in range(3):
        sel = axis == a
        others = [d for d in range(3) if d != a]
        pts[sel, a] = sign[sel]
        pts[sel, others[0]] = uv[sel, 0]
        pts[sel, others[1]] = uv[sel, 1]
    return pts


def cube_volume(n: int, seed: int) -> np.ndarray:
    """Uniform in the volume of [-1,1]^3."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-1.0, 1.0, (n, 3))


def charges(n: int, seed: int, dtype=np.complex128) -> np.ndarray:
    """Complex charges, real and imaginary parts i.i.d. N(0,1)."""
    rng = np.random.default_rng(seed)
    z = rng.standard_normal((n, 2))
    return (z[:, 0] + 1j * z[:, 1]).astype(dtype)


def sample_targets(n: int, k: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    k = min(k, n)
    return np.sort(rng.choice(n, size=k, replace=False)).astype(np.int64)


GENERATORS = {"sphere": sphere, "ellipsoid": ellipsoid, "cube_surface": cube_surface,
              "cube_volume": cube_volume}


@dataclass
class Workload:
    """One synthetic workload: geometry, size, wavenumber and method knobs."""
    name: str
    geometry: str
    n: int
    kappa_d: float          # kappa times the side D of the bounding cube (D = 2 here)
    L: int
    ncrit: int
    precision: str          # "c128" or "c64"
    seed: int
    eta: float = 1.0
    hf_threshold: float = 2.0
    dir_refine: int = 0
    check_targets: int = 0  # 0: all targets against the direct sum
    extra: dict = field(default_factory=dict)
    kernel: str = "helmholtz"  # or "yukawa": exp(-kappa r)/(4 pi r), kappa the screening constant

    @property
    def kappa(self) -> float:
        return self.kappa_d / 2.0

    def points(self) -> np.ndarray:
        return GENERATORS[self.geometry](self.n, 1000 + self.seed)

    def charges(self, index: int = 0, dtype=np.complex128) -> np.ndarray:
        return charges(self.n, 2000 + 100 * self.seed + index, dtype)

    def targets(self) -> np.ndarray:
        if self.check_targets <= 0:
            return np.arange(self.n, dtype=np.int64)
        return sample_targets(self.n, self.check_targets, 3000 + self.seed)


# The paper's method on the paper's kinds of inputs, at the sizes the build
# measures (sphere, pole-concentrated ellipsoid, cube surface).
WORKLOADS = {
    "sphere8k": Workload("sphere8k", "sphere", 8192, 32.0, 4, 32, "c128", 1),
    "sphere1m": Workload("sphere1m", "sphere", 1048576, 256.0, 5, 64, "c64", 2, check_targets=2048),
    "ellipsoid2m": Workload("ellipsoid2m", "ellipsoid", 2097152, 512.0, 5, 64, "c64", 3,
                            check_targets=2048),
    "cube8m": Workload("cube8m", "cube_surface", 8388608, 1024.0, 6, 64, "c64", 5,
                       check_targets=2048),
    # the screened kernel on the sphere1m points: low-frequency expansions only
    "sphere1m_yukawa": Workload("sphere1m_yukawa", "sphere", 1048576, 16.0, 5, 64, "c64", 2,
                                check_targets=2048, kernel="yukawa"),
}
