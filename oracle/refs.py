"""Analytic references for the dipole-dipole interaction (test infrastructure only).

These are the "exact" potentials the paper uses to measure its errors
(Sec. 2.2).  They pin the oracle: a dropped prefactor, a wrong sign of the
symbol or a transposed axis in the quadrature shows up as an O(1) error here.

* ``phi_gaussian_3d``: Ex. 2.1, rho = exp(-|x|^2/sigma^2), Phi = -(n.m) rho - 3 n^T G m
  with the Hessian G of Eq. Hessian_Ex1.
* ``phi_gaussian_2d``: Ex. 2.2, rho = exp(-|x|^2/sigma^2) in 2D, the I0/I1 form.
* ``phi_gaussian_2d_radial``: the same Phi by its Fourier integral in polar coordinates (J0, J2),
  optionally with a radial weight: with the partition q of Eq. 3.9 it gives I_2 of the split.
* ``phi_gaussian_product``: Ex. 2.3.  For rho = prod_i G_{a_i}(x_i - c_i) with the
  heat kernel G_b(y) = (4 pi b)^(-1/2) exp(-y^2/(4b)), the Poisson potential is
  u = int_0^inf prod_i G_{a_i+s} ds (3D, as in Eqs. Coulomb:3D:aniso:z/xy) and the
  fractional one u = (2/sqrt(pi)) int_0^inf prod_i G_{a_i+t^2} dt (2D, as in
  Eq. Coulomb:2D:aniso); Phi follows by differentiating under the integral
  (Eq. DDI-Eqv and Eq. DDI:2D:aniso).  Each integral is split at 1, the infinite
  piece mapped to a finite interval, and both integrated by adaptive
  Gauss-Kronrod quadrature (scipy.integrate.quad), as the paper describes.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import integrate, special


def _series_hessian_coeffs(t, sigma, terms=30):
    """2 f'(t) and 4 f''(t) for f(t) = (sigma^3 sqrt(pi)/4) erf(sqrt(t)/sigma)/sqrt(t).

    Uses erf(s)/s = (2/sqrt(pi)) sum_k (-1)^k s^(2k) / (k! (2k+1)), so
    f(t) = (sigma^2/2) sum_k (-1)^k (t/sigma^2)^k / (k! (2k+1)); the Hessian of the
    radial function u(x) = f(|x|^2) is 2 f'(t) I + 4 f''(t) x x^T.
    """
    a = np.zeros_like(t)
    b = np.zeros_like(t)
    s2 = sigma * sigma
    for k in range(1, terms):
        ck = (-1) ** k / (math.factorial(k) * (2 * k + 1)) * (s2 / 2) / s2 ** k
        a += 2 * ck * k * t ** (k - 1)
        if k >= 2:
            b += 4 * ck * k * (k - 1) * t ** (k - 2)
    return a, b


def phi_gaussian_3d(x, y, z, sigma, dip_n, dip_m=None):
    """Ex. 2.1: Phi for rho = exp(-|x|^2/sigma^2) (Eqs. extDensGausDipolar, Hessian_Ex1).

    For r/sigma >= 0.5 the printed closed form of g_jl is used; closer to the
    origin (where that form cancels catastrophically) the Taylor series of the
    same Poisson potential is used.  The two agree at the switch (tested).
    """
    n = np.asarray(dip_n, float)
    m = n if dip_m is None else np.asarray(dip_m, float)
    X = np.stack(np.broadcast_arrays(np.asarray(x, float), np.asarray(y, float),
                                     np.asarray(z, float)), axis=-1)
    r2 = np.sum(X * X, axis=-1)
    r = np.sqrt(r2)
    rho = np.exp(-r2 / sigma ** 2)
    s = r / sigma
    diag = np.empty_like(r)
    off = np.empty_like(r)
    far = s >= 0.5
    rf = r[far]
    e = np.exp(-rf ** 2 / sigma ** 2)
    erf = special.erf(rf / sigma)
    sp = math.sqrt(math.pi)
    diag[far] = sigma ** 2 / (2 * rf ** 2) * e - sigma ** 3 * sp / (4 * rf ** 3) * erf
    off[far] = (-3 * sigma ** 2 / (2 * rf ** 4) * e - e / rf ** 2
                + 3 * sigma ** 3 * sp / (4 * rf ** 5) * erf)
    near = ~far
    diag[near], off[near] = _series_hessian_coeffs(r2[near], sigma)
    nm = float(n @ m)
    xn = X @ n
    xm = X @ m
    nGm = diag * nm + off * xn * xm
    return -nm * rho - 3.0 * nGm


def phi_gaussian_2d(x, y, sigma, dip_n, dip_m=None):
    """Ex. 2.2: Phi for rho = exp(-|x|^2/sigma^2) in the quasi-2D model.

    With r = |x|^2/(2 sigma^2) and exponentially scaled Bessel functions
    (e^{-r} I_nu(r) = special.ive(nu, r)).
    """
    n = np.asarray(dip_n, float)
    m = n if dip_m is None else np.asarray(dip_m, float)
    x = np.asarray(x, float)
    y = np.asarray(y, float)
    x, y = np.broadcast_arrays(x, y)
    r = (x * x + y * y) / (2 * sigma ** 2)
    i0 = special.i0e(r)
    i1 = special.i1e(r)
    with np.errstate(divide="ignore", invalid="ignore"):
        i1_over_2r = np.where(r > 1e-12, i1 / (2 * np.where(r > 1e-12, r, 1.0)), 0.25)
    # (1 + 2r)/(2r) I1 = I1/(2r) + I1
    bracket2 = i0 - (i1_over_2r + i1)
    npm = n[0] * m[0] + n[1] * m[1]
    xn = x * n[0] + y * n[1]
    xm = x * m[0] + y * m[1]
    sp = math.sqrt(math.pi)
    t1 = 3 * sp / (4 * sigma) * (npm * (i0 - i1) - 2 * xn * xm / sigma ** 2 * bracket2)
    t2 = 3 * sp * n[2] * m[2] / sigma * (r * i0 - r * i1 - 0.5 * i0)
    return t1 + t2


def heat_kernel(b, y):
    """G_b(y) = (4 pi b)^(-1/2) exp(-y^2/(4 b))."""
    return np.exp(-y * y / (4 * b)) / np.sqrt(4 * math.pi * b)


def _integrand_3d(s, a, y, nm_mat):
    b = a + s
    G = np.prod(heat_kernel(b, y))
    D = np.outer(y / (2 * b), y / (2 * b))
    D[np.diag_indices(3)] -= 1.0 / (2 * b)
    return G * np.sum(nm_mat * D)


def _integrand_2d(t, a, y, nm_mat, n3m3):
    b = a + t * t
    G = np.prod(heat_kernel(b, y))
    D = np.outer(y / (2 * b), y / (2 * b))
    D[np.diag_indices(2)] -= 1.0 / (2 * b)
    lap = np.trace(D)
    return G * (np.sum(nm_mat * D) - n3m3 * lap)


def _semi_infinite(f, epsrel=1e-13):
    """int_0^inf f(s) ds = int_0^1 f(s) ds + int_0^1 f(1/tau)/tau^2 dtau."""
    kw = dict(epsabs=0.0, epsrel=epsrel, limit=400)
    p1, _ = integrate.quad(f, 0.0, 1.0, **kw)
    p2, _ = integrate.quad(lambda tau: f(1.0 / tau) / (tau * tau) if tau > 0 else 0.0,
                           0.0, 1.0, **kw)
    return p1 + p2


def phi_gaussian_product(point, a, c, dip_n, dip_m=None, epsrel=1e-13):
    """Phi at one point for rho = prod_i G_{a_i}(x_i - c_i) (d = len(a)).

    3D: Phi = -(n.m) rho - 3 sum_ij n_i m_j d_ij u,   u = int_0^inf prod G_{a+s} ds.
    2D: Phi = -3/2 (sum_ij n_i m_j d_ij u - n3 m3 Lap u),  u = 2/sqrt(pi) int_0^inf prod G_{a+t^2} dt.
    d_ij prod G_b(y) = prod G_b(y) * D_ij with D_ii = y_i^2/(4b_i^2) - 1/(2b_i),
    D_ij = y_i y_j / (4 b_i b_j).
    """
    a = np.asarray(a, float)
    c = np.asarray(c, float)
    y = np.asarray(point, float) - c
    n = np.asarray(dip_n, float)
    m = n if dip_m is None else np.asarray(dip_m, float)
    d = a.size
    if d == 3:
        nm_mat = np.outer(n, m)
        rho = np.prod(heat_kernel(a, y))
        hess = _semi_infinite(lambda s: _integrand_3d(s, a, y, nm_mat), epsrel)
        return -float(n @ m) * rho - 3.0 * hess
    nm_mat = np.outer(n[:2], m[:2])
    val = _semi_infinite(lambda t: _integrand_2d(t, a, y, nm_mat, n[2] * m[2]), epsrel)
    return -1.5 * (2.0 / math.sqrt(math.pi)) * val


def gaussian_lumps_to_products(lumps, scale=1.0):
    """Expand rho = |sum_a c_a g_a|^2 into sum of weighted heat-kernel products.

    ``lumps``: list of (coef complex, centre (d,), widths (d,)) with
    g_a(x) = exp(-sum_i (x_i - mu_i)^2 / (2 s_i^2)).  The product g_a g_b is an
    axis-aligned Gaussian, so rho = sum_ab w_ab prod_i G_{b_i}(x_i - mu_i) with
    b = s^2/2, 1/s^2 = 1/s_a^2 + 1/s_b^2, mu = s^2 (mu_a/s_a^2 + mu_b/s_b^2).
    Returns a list of (weight, a (d,), centre (d,)).
    """
    out = []
    for ca, mua, sa in lumps:
        for cb, mub, sb in lumps:
            mua_, mub_ = np.asarray(mua, float), np.asarray(mub, float)
            sa_, sb_ = np.asarray(sa, float), np.asarray(sb, float)
            s2 = 1.0 / (1.0 / sa_ ** 2 + 1.0 / sb_ ** 2)
            mu = s2 * (mua_ / sa_ ** 2 + mub_ / sb_ ** 2)
            K = np.exp(-(mua_ - mub_) ** 2 / (2 * (sa_ ** 2 + sb_ ** 2)))
            weight = (scale ** 2) * float(np.real(ca * np.conj(cb))) * float(
                np.prod(K * np.sqrt(2 * math.pi * s2)))
            out.append((weight, s2 / 2.0, mu))
    return out


def phi_mixture(point, products, dip_n, dip_m=None, epsrel=1e-12):
    """Sum of phi_gaussian_product over the expansion of gaussian_lumps_to_products."""
    return sum(w * phi_gaussian_product(point, a, c, dip_n, dip_m, epsrel) for w, a, c in products)


def phi_gaussian_2d_radial(x, y, sigma, dip_n, dip_m=None, weight=None, epsabs=1e-17):
    """Ex. 2.2 by its Fourier integral in polar coordinates, optionally with a radial weight w(|k|):
    for rho = exp(-|x|^2/sigma^2), rhohat(k) = pi sigma^2 exp(-sigma^2 |k|^2/4), and with
    k = |k| (cos t, sin t) the 2D symbol is 3/2 |k| [A0 - n3 m3 + Ac cos 2t + As sin 2t],
    A0 = (n1 m1 + n2 m2)/2, Ac = (n1 m1 - n2 m2)/2, As = (n1 m2 + n2 m1)/2.  The angular integral
    of exp(i k.x) against 1, cos 2t, sin 2t gives 2 pi J0(|k| r) and -2 pi J2(|k| r) (cos 2p, sin 2p)
    at x = r (cos p, sin p), so
        Phi(x) = 3/(4 pi) int_0^inf k^2 w(k) rhohat(k) [(A0 - n3 m3) J0(kr) - J2(kr)(Ac cos 2p + As sin 2p)] dk.
    With w = 1 this is Phi of Ex. 2.2 (an independent form of phi_gaussian_2d); with w = q it is
    I_2 of Eq. 3.9 for that density.  Evaluated point by point with adaptive Gauss-Kronrod.
    """
    n = np.asarray(dip_n, float)
    m = n if dip_m is None else np.asarray(dip_m, float)
    A0 = 0.5 * (n[0] * m[0] + n[1] * m[1]) - n[2] * m[2]
    Ac = 0.5 * (n[0] * m[0] - n[1] * m[1])
    As = 0.5 * (n[0] * m[1] + n[1] * m[0])
    x, y = np.broadcast_arrays(np.asarray(x, float), np.asarray(y, float))
    out = np.empty(x.shape)
    kcut = 2.0 * math.sqrt(math.log(1e300)) / sigma          # rhohat below 1e-300 beyond
    for idx in np.ndindex(x.shape):
        r = math.hypot(x[idx], y[idx])
        ph = math.atan2(y[idx], x[idx])
        ang = Ac * math.cos(2 * ph) + As * math.sin(2 * ph)

        def f(k):
            w = 1.0 if weight is None else weight(k)
            rh = math.pi * sigma * sigma * math.exp(-sigma * sigma * k * k / 4)
            return k * k * w * rh * (A0 * special.j0(k * r) - special.jv(2, k * r) * ang)

        val, _ = integrate.quad(f, 0.0, kcut, epsabs=epsabs, epsrel=1e-13, limit=500)
        out[idx] = 3.0 / (4.0 * math.pi) * val
    return out
