"""Seeded synthetic inputs and the named workloads.

This module holds input generation only: grid coordinates, Gaussian lumps,
noise, random dipole axes and the parameter sets of the workloads.  It contains
none of the DDI method's arithmetic, so both the HIP path (through the tests
and the benchmark) and the CPU oracle can take their inputs from it.

The densities follow the paper's test problems: smooth, rapidly decaying
Gaussian-type densities in a box (Sec. 2.2, Exs. 2.1-2.3) and condensate-like
wave functions (Sec. 3.2).  Workloads:

``c1_32``    3D, 32^3 on [-8,8)^3, rho = exp(-(x^2+y^2) - z^2/4)/(2 pi^(3/2)), n = m = z,
             quadrature 32 x 16 x 32, FP64.
``c2_128``   3D, 128^3 on [-12,12)^3, psi = seeded mixture of 1-4 anisotropic
             Gaussian lumps, random unit n, quadrature 96 x 48 x 96, tol 1e-13, FP64.
``c3_512``   quasi-2D, 512^2 on [-16,16)^2, mixture of 1-6 lumps plus 10% random-phase
             noise, n tilted 45 degrees from z, polar 128 x 256, FP64.
``c4_256``   3D, 256^3 on [-16,16)^3, same mixture recipe, quadrature 128 x 64 x 128, mixed precision.
``c5_gf``    ground-state gradient flow at 128^3 on [-8,8)^3, V = (x^2+y^2+25 z^2)/2,
             beta = 200, lambda = 150, n = z, dt = 0.01, 200 steps.
"""
from __future__ import annotations

import math

import numpy as np

WORKLOADS = {
    "c1_32": dict(dim=3, n=(32, 32, 32), L=(8.0, 8.0, 8.0), quad=(32, 16, 32),
                  tol=1e-13, prec="fp64", kind="c1"),
    "c2_128": dict(dim=3, n=(128, 128, 128), L=(12.0, 12.0, 12.0), quad=(96, 48, 96),
                   tol=1e-13, prec="fp64", kind="mixture", lumps=(1, 4)),
    "c3_512": dict(dim=2, n=(512, 512), L=(16.0, 16.0), quad=(128, 1, 256),
                   tol=1e-13, prec="fp64", kind="mixture2d", lumps=(1, 6), noise=0.1),
    "c4_256": dict(dim=3, n=(256, 256, 256), L=(16.0, 16.0, 16.0), quad=(128, 64, 128),
                   tol=1e-7, prec="mixed", kind="mixture", lumps=(1, 4)),
    "c5_gf": dict(dim=3, n=(128, 128, 128), L=(8.0, 8.0, 8.0), quad=(96, 48, 96),
                  tol=1e-13, prec="fp64", kind="gf", beta=200.0, lam=150.0,
                  gamma=(1.0, 1.0, 5.0), dt=0.01, steps=200),
}


def grid_axes(n, L):
    """x_l = -L + l h with h = 2L/N, l = 0..N-1, per axis (half-open box [-L, L))."""
    return [-Li + (2.0 * Li / ni) * np.arange(ni, dtype=np.float64) for ni, Li in zip(n, L)]


def c1_density(n=(32, 32, 32), L=(8.0, 8.0, 8.0)):
    """rho = exp(-(x^2+y^2)/1 - z^2/4) / (2 pi^(3/2)) (unit mass)."""
    x, y, z = np.meshgrid(*grid_axes(n, L), indexing="ij")
    return np.exp(-(x * x + y * y) - z * z / 4.0) / (2.0 * math.pi ** 1.5)


def gaussian_density(n, L, sigma):
    """rho = exp(-|x|^2/sigma^2) on the grid (the densities of Exs. 2.1 and 2.2)."""
    grids = np.meshgrid(*grid_axes(n, L), indexing="ij")
    return np.exp(-sum(g * g for g in grids) / sigma ** 2)


def mixture_lumps(seed, dim, lumps=(1, 4), centre=3.0, widths=(0.5, 2.5)):
    """Seeded lump parameters: K in [lumps[0], lumps[1]] lumps, each with a centre
    uniform in [-centre, centre]^d, per-axis widths uniform in ``widths`` and a
    constant phase uniform in [0, 2 pi).  Returns (lumps, rng) where lumps is a
    list of (coef, centre, widths) and rng continues the same stream."""
    rng = np.random.default_rng(seed)
    K = int(rng.integers(lumps[0], lumps[1] + 1))
    out = []
    for _ in range(K):
        c = rng.uniform(-centre, centre, size=dim)
        w = rng.uniform(widths[0], widths[1], size=dim)
        th = rng.uniform(0.0, 2.0 * math.pi)
        out.append((complex(math.cos(th), math.sin(th)), c, w))
    return out, rng


def lumps_on_grid(lumps, n, L):
    """psi(x) = sum_a coef_a exp(-sum_i (x_i - c_i)^2 / (2 w_i^2))."""
    axes = grid_axes(n, L)
    psi = np.zeros(tuple(n), dtype=np.complex128)
    for coef, c, w in lumps:
        f = None
        for i, ax in enumerate(axes):
            g = np.exp(-(ax - c[i]) ** 2 / (2.0 * w[i] ** 2))
            shape = [1] * len(n)
            shape[i] = n[i]
            g = g.reshape(shape)
            f = g if f is None else f * g
        psi += coef * f
    return psi


def normalise(psi, n, L):
    """Scale so that prod(h) sum |psi|^2 = 1 (Eq. norm on the grid). Returns (psi, scale)."""
    cell = float(np.prod([2.0 * Li / ni for ni, Li in zip(n, L)]))
    s = 1.0 / math.sqrt(cell * float(np.sum(np.abs(psi) ** 2)))
    return psi * s, s


def random_axis(rng):
    """A unit vector from a normalised standard-normal draw."""
    v = rng.standard_normal(3)
    return v / np.linalg.norm(v)


def mixture_workload(name, seed=0):
    """psi, rho, dipole axis and lump description for a mixture workload.

    3D (c2/c4): psi = sum of lumps, normalised; n = random unit vector drawn after
    the lumps.  2D (c3): lumps, then i.i.d. noise 0.1 max|psi| xi e^{i eta} per
    grid point (xi ~ U[0,1], eta ~ U[0, 2 pi)), renormalised; n tilted 45 degrees
    from z in the x-z plane.
    """
    wl = WORKLOADS[name]
    dim, n, L = wl["dim"], wl["n"], wl["L"]
    lumps, rng = mixture_lumps(seed, dim, wl.get("lumps", (1, 4)))
    psi = lumps_on_grid(lumps, n, L)
    noise = wl.get("noise", 0.0)
    if noise:
        xi = rng.uniform(0.0, 1.0, size=n)
        eta = rng.uniform(0.0, 2.0 * math.pi, size=n)
        psi = psi + noise * np.max(np.abs(psi)) * xi * np.exp(1j * eta)
    psi, scale = normalise(psi, n, L)
    if dim == 3:
        dip = random_axis(rng)
    else:
        dip = np.array([math.sin(math.pi / 4), 0.0, math.cos(math.pi / 4)])
    rho = psi.real ** 2 + psi.imag ** 2
    return dict(psi=psi, rho=rho, dip_n=dip, lumps=lumps, scale=scale,
                exact_mixture=(noise == 0.0))


def gf_initial(n, L, gamma):
    """Normalised harmonic-oscillator Gaussian exp(-sum gamma_i x_i^2 / 2) (a positive initial guess)."""
    grids = np.meshgrid(*grid_axes(n, L), indexing="ij")
    psi = np.exp(-0.5 * sum(gamma[i] * grids[i] ** 2 for i in range(len(n)))).astype(np.complex128)
    return normalise(psi, n, L)[0]


def random_field(seed, shape, complex_=False):
    """Standard-normal test field (for adjoint and finite-difference checks)."""
    rng = np.random.default_rng(seed)
    if complex_:
        return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    return rng.standard_normal(shape)


def dip_rot(t):
    """The rotating dipole orientation of the dynamics example: n(t) = (sin(t/5), 0, cos(t/5))."""
    return np.array([math.sin(t / 5.0), 0.0, math.cos(t / 5.0)])
