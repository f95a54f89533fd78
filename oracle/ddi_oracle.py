"""Plain FP64 CPU oracle for the dipole-dipole interaction (DDI) quadrature.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``): the product path never
imports this module.

What is computed (Bao, Tang & Zhang, Sec. 2.1):

* the DDI potential is the inverse Fourier integral of the dipolar symbol times
  the density transform (Eq. DDI-Con);
* the integral is truncated to a ball of radius Kmax and written in spherical
  (3D) or polar (2D) coordinates so that the Jacobian |k|^(d-1) cancels the
  singularity of the symbol at k = 0 (Eq. DDI-Trun1);
* the resulting smooth integral is discretised by a tensor quadrature in
  (|k|, cos(theta), phi) / (|k|, phi).

The NUFFT in the GPU path approximates exactly this discrete sum to its
tolerance; here the sum is evaluated directly:

    rhohat_q = prod(h) * sum_l rho_l exp(-i k_q . x_l)        (trapezoid rule for the transform)
    Phi_l    = sum_q c_q Re[rhohat_q exp(+i k_q . x_l)]
    c_q      = chi_q W_q Uhat(k_q) / (2 pi)^d

Readings where the paper is silent (each is listed, with its reason, in the
design notes of the repository):

* quadrature: Gauss-Legendre in |k| on [0, Kmax], Gauss-Legendre in
  u = cos(theta) on [-1, 1], uniform azimuths phi_c = 2 pi c / N_phi;
* Kmax defaults to pi * sqrt(sum_i 1/h_i^2) (circumradius of the Nyquist box);
* nodes with |k_i| > pi/h_i on some axis are dropped (chi_q = 0), so the result
  is the exact DDI of the band-limited interpolant of rho;
* grid x_l = -L + l h on the half-open box [-L, L), N points per axis;
* Phi is the real part of the sum.

Sums over the grid are taken axis by axis for one block of nodes at a time;
each per-node sum is the definition above, and a BLAS matrix product serves as
the step that sums over the last axis.  No FFT, NUFFT, interpolation or kernel
approximation appears anywhere in the DDI part.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
from scipy import special

TWO_PI = 2.0 * math.pi


# --------------------------------------------------------------------------
# Problem description (mirrors the quantities of Sec. 1 and Sec. 2.1)
# --------------------------------------------------------------------------
@dataclass
class DDIProblem:
    """Grid, dipole axes and quadrature sizes of one DDI evaluation.

    dim     : 2 or 3 (Eq. DipGPE0 holds in d = 2, 3).
    n       : grid points per axis (length ``dim``), box [-L_i, L_i).
    L       : half box lengths.
    dip_n   : dipole axis n (3 components; in 2D n_perp = (n1, n2), n3 = n[2]).
    dip_m   : second dipole axis m (Eq. dipmn); ``None`` means m = n.
    n_rad, n_pol, n_azi : quadrature sizes (n_pol unused in 2D).
    kmax    : radius of the Fourier ball; <= 0 selects pi*sqrt(sum 1/h^2).
    mask    : drop nodes outside the Nyquist box.
    stretch : per-axis factors S_i of the quadrature (k = S k' with k' on the spherical/polar
              rule, weights times det S); (1, 1, 1) is the rule of Eq. DDI-Trun1 itself.
    """

    dim: int
    n: tuple
    L: tuple
    dip_n: tuple = (0.0, 0.0, 1.0)
    dip_m: tuple | None = None
    n_rad: int = 32
    n_pol: int = 16
    n_azi: int = 32
    kmax: float = 0.0
    mask: bool = True
    stretch: tuple = (1.0, 1.0, 1.0)
    _cache: dict = field(default_factory=dict, repr=False, compare=False)

    @property
    def h(self):
        return tuple(2.0 * Li / ni for Li, ni in zip(self.L, self.n))

    @property
    def cell(self):
        """prod(h): the trapezoid weight of one grid point."""
        return float(np.prod(self.h))

    def axes(self):
        """Grid coordinates x_l = -L + l h, l = 0..N-1, per axis."""
        return [-Li + hi * np.arange(ni, dtype=np.float64)
                for Li, hi, ni in zip(self.L, self.h, self.n)]

    def kmax_value(self):
        """Radius of the ball in k' (= k without stretch): the circumradius of the Nyquist box
        seen through the stretch, pi sqrt(sum 1/(h_i S_i)^2), unless given."""
        if self.kmax > 0:
            return float(self.kmax)
        return math.pi * math.sqrt(sum(1.0 / (hi * si) ** 2 for hi, si in zip(self.h, self.stretch)))


# --------------------------------------------------------------------------
# 1D Gauss-Legendre rule, written out (Newton iteration on P_n)
# --------------------------------------------------------------------------
def gauss_legendre(n: int):
    """Nodes and weights of the n-point Gauss-Legendre rule on [-1, 1].

    The nodes are the zeros of the Legendre polynomial P_n, found by Newton's
    method on the three-term recurrence
        (j+1) P_{j+1}(x) = (2j+1) x P_j(x) - j P_{j-1}(x),
    and the weights are w = 2 / ((1 - x^2) P_n'(x)^2) with
    P_n'(x) = n (x P_n(x) - P_{n-1}(x)) / (x^2 - 1).
    Pinned against numpy.polynomial.legendre.leggauss in the tests.
    """
    if n < 1:
        raise ValueError("n must be positive")
    x = np.cos(np.pi * (np.arange(1, n + 1) - 0.25) / (n + 0.5))
    for _ in range(100):
        p0 = np.ones_like(x)
        p1 = x.copy()
        for j in range(1, n):
            p0, p1 = p1, ((2 * j + 1) * x * p1 - j * p0) / (j + 1)
        dp = n * (x * p1 - p0) / (x * x - 1.0)
        dx = p1 / dp
        x = x - dx
        if np.max(np.abs(dx)) < 1e-16:
            break
    # final evaluation at the converged nodes
    p0 = np.ones_like(x)
    p1 = x.copy()
    for j in range(1, n):
        p0, p1 = p1, ((2 * j + 1) * x * p1 - j * p0) / (j + 1)
    dp = n * (x * p1 - p0) / (x * x - 1.0)
    w = 2.0 / ((1.0 - x * x) * dp * dp)
    order = np.argsort(x)
    return x[order], w[order]


# --------------------------------------------------------------------------
# Quadrature of Eq. DDI-Trun1
# --------------------------------------------------------------------------
@dataclass
class Quadrature:
    k: np.ndarray        # (M, d) node coordinates
    W: np.ndarray        # (M,) quadrature weights including the Jacobian |k|^(d-1)
    index: np.ndarray    # (M, 3) (radial, polar, azimuthal) indices; polar = 0 in 2D
    kmax: float
    n_nominal: int


def quadrature(prob: DDIProblem, apply_mask: bool | None = None) -> Quadrature:
    """Spherical (3D) / polar (2D) tensor quadrature of Eq. DDI-Trun1.

    Radial: r_a = Kmax (1 + t_a)/2, weight Kmax w_a / 2 (GL on [0, Kmax]).
    3D: u_b = cos(theta_b) GL on [-1, 1] (sin(theta) d theta = du),
        k = r (sqrt(1-u^2) cos phi, sqrt(1-u^2) sin phi, u),
        W = w^r_a r_a^2 w^u_b (2 pi / N_phi).
    2D: k = r (cos phi, sin phi), W = w^r_a r_a (2 pi / N_phi).
    Nodes with |k_i| > pi / h_i on some axis are removed when masking.
    With a stretch S (a reading for anisotropic boxes): k = S k', W = W' det S.
    """
    if apply_mask is None:
        apply_mask = prob.mask
    kmax = prob.kmax_value()
    t, wt = gauss_legendre(prob.n_rad)
    r = 0.5 * kmax * (1.0 + t)
    wr = 0.5 * kmax * wt
    phi = TWO_PI * np.arange(prob.n_azi, dtype=np.float64) / prob.n_azi
    wphi = TWO_PI / prob.n_azi
    if prob.dim == 3:
        u, wu = gauss_legendre(prob.n_pol)
        a, b, c = np.meshgrid(np.arange(prob.n_rad), np.arange(prob.n_pol),
                              np.arange(prob.n_azi), indexing="ij")
        a, b, c = a.ravel(), b.ravel(), c.ravel()
        s = np.sqrt(1.0 - u[b] ** 2)
        k = np.stack([r[a] * s * np.cos(phi[c]), r[a] * s * np.sin(phi[c]), r[a] * u[b]], axis=1)
        W = wr[a] * r[a] ** 2 * wu[b] * wphi
        index = np.stack([a, b, c], axis=1)
    elif prob.dim == 2:
        a, c = np.meshgrid(np.arange(prob.n_rad), np.arange(prob.n_azi), indexing="ij")
        a, c = a.ravel(), c.ravel()
        k = np.stack([r[a] * np.cos(phi[c]), r[a] * np.sin(phi[c])], axis=1)
        W = wr[a] * r[a] * wphi
        index = np.stack([a, np.zeros_like(a), c], axis=1)
    else:
        raise ValueError("dim must be 2 or 3")
    S = np.asarray(prob.stretch[:prob.dim], dtype=np.float64)
    k = k * S[None, :]
    W = W * float(np.prod(S))
    n_nom = k.shape[0]
    if apply_mask:
        lim = np.array([math.pi / hi for hi in prob.h])
        keep = np.all(np.abs(k) <= lim[None, :], axis=1)
        k, W, index = k[keep], W[keep], index[keep]
    return Quadrature(k=k, W=W, index=index, kmax=kmax, n_nominal=n_nom)


def dipolar_symbol(k: np.ndarray, dim: int, dip_n, dip_m=None) -> np.ndarray:
    """Fourier symbol of U_dip (Eq. DipKer; two axes: Eq. dipmn).

    3D: Uhat = 3 (n.k)(m.k)/|k|^2 - n.m
    2D: Uhat = 3 [(n_perp.k)(m_perp.k) - n3 m3 |k|^2] / (2 |k|)
    """
    n = np.asarray(dip_n, dtype=np.float64)
    m = n if dip_m is None else np.asarray(dip_m, dtype=np.float64)
    if dim == 3:
        kk = np.sum(k * k, axis=1)
        return 3.0 * (k @ n) * (k @ m) / kk - float(n @ m)
    kk = np.sum(k * k, axis=1)
    kn = k @ n[:2]
    km = k @ m[:2]
    return 3.0 * (kn * km - n[2] * m[2] * kk) / (2.0 * np.sqrt(kk))


def node_coefficients(prob: DDIProblem, quad: Quadrature | None = None) -> np.ndarray:
    """c_q = W_q Uhat(k_q) / (2 pi)^d  (Eq. DDI-Con prefactor, Eq. DDI-Trun1 weights)."""
    if quad is None:
        quad = quadrature(prob)
    U = dipolar_symbol(quad.k, prob.dim, prob.dip_n, prob.dip_m)
    return quad.W * U / TWO_PI ** prob.dim


# --------------------------------------------------------------------------
# Direct nonuniform DFTs
# --------------------------------------------------------------------------
def _phases(x: np.ndarray, kcol: np.ndarray, sign: float) -> np.ndarray:
    """exp(sign * i * k x) for all grid coordinates x (rows) and nodes k (cols)."""
    arg = np.outer(x, kcol)
    return np.cos(arg) + (1j * sign) * np.sin(arg)


def rhohat(rho: np.ndarray, prob: DDIProblem, k: np.ndarray, sign: float = -1.0,
           block: int = 2048) -> np.ndarray:
    """rhohat_q = prod(h) sum_l f_l exp(sign i k_q . x_l) for a real or complex grid f.

    With sign = -1 this is the trapezoid rule for the Fourier transform of
    Eq. DipKer's convention fhat(k) = int f(x) exp(-i k.x) dx.
    Evaluated node block by node block; the sum over the last grid axis is a
    BLAS matrix product, the remaining axes are summed with einsum.
    """
    xs = prob.axes()
    out = np.empty(k.shape[0], dtype=np.complex128)
    f = np.asarray(rho)
    cell = prob.cell
    for s in range(0, k.shape[0], block):
        kb = k[s:s + block]
        Elast = _phases(xs[-1], kb[:, -1], sign)                     # (N_last, B)
        inner = f.reshape(-1, f.shape[-1]) @ Elast                    # (prod other, B)
        if prob.dim == 3:
            inner = inner.reshape(f.shape[0], f.shape[1], -1)
            Ey = _phases(xs[1], kb[:, 1], sign)
            Ex = _phases(xs[0], kb[:, 0], sign)
            t = np.einsum("xyq,yq->xq", inner, Ey)
            out[s:s + block] = cell * np.einsum("xq,xq->q", t, Ex)
        else:
            Ex = _phases(xs[0], kb[:, 0], sign)
            out[s:s + block] = cell * np.einsum("xq,xq->q", inner, Ex)
    return out


def nodes_to_grid(g: np.ndarray, prob: DDIProblem, k: np.ndarray, sign: float = +1.0,
                  block: int = 2048, real: bool = True) -> np.ndarray:
    """Phi_l = sum_q g_q exp(sign i k_q . x_l) (real part if ``real``).

    Summed over node blocks in order; within a block the sum over nodes is a
    BLAS matrix product.
    """
    xs = prob.axes()
    shape = tuple(prob.n)
    acc = np.zeros(shape, dtype=np.float64 if real else np.complex128)
    for s in range(0, k.shape[0], block):
        kb = k[s:s + block]
        gb = g[s:s + block]
        Elast = _phases(xs[-1], kb[:, -1], sign)                      # (N_last, B)
        if prob.dim == 3:
            Ex = _phases(xs[0], kb[:, 0], sign)
            Ey = _phases(xs[1], kb[:, 1], sign)
            T = (Ex[:, None, :] * Ey[None, :, :]) * gb[None, None, :]   # (Nx, Ny, B)
            T = T.reshape(-1, kb.shape[0])
        else:
            Ex = _phases(xs[0], kb[:, 0], sign)
            T = Ex * gb[None, :]
        Et = np.ascontiguousarray(Elast.T)                            # (B, N_last)
        if real:
            part = (np.ascontiguousarray(T.real) @ np.ascontiguousarray(Et.real)
                    - np.ascontiguousarray(T.imag) @ np.ascontiguousarray(Et.imag))
        else:
            part = T @ Et
        acc += part.reshape(shape)
    return acc


# --------------------------------------------------------------------------
# The DDI operator A: rho -> Phi, its adjoint, and the pieces
# --------------------------------------------------------------------------
def ddi_nodes(prob: DDIProblem):
    """(k, c) of the masked quadrature, in natural (radial, polar, azimuthal) order."""
    key = "nodes"
    if key not in prob._cache:
        quad = quadrature(prob)
        prob._cache[key] = (quad, node_coefficients(prob, quad))
    return prob._cache[key]


def ddi_apply(rho: np.ndarray, prob: DDIProblem, return_rhohat: bool = False):
    """Phi = U_dip * rho by the quadrature of Eq. DDI-Trun1 (Eq. DDI-Con).

    rho: real grid of shape prob.n.  Returns Phi (same shape, float64).
    """
    quad, c = ddi_nodes(prob)
    rh = rhohat(np.asarray(rho, dtype=np.float64), prob, quad.k, sign=-1.0)
    phi = nodes_to_grid(c * rh, prob, quad.k, sign=+1.0, real=True)
    return (phi, rh) if return_rhohat else phi


def ddi_apply_adjoint(sigma: np.ndarray, prob: DDIProblem) -> np.ndarray:
    """Literal transpose of ddi_apply with respect to the plain dot product on the grid.

    A_{jl} = prod(h) sum_q c_q Re[exp(-i k_q.x_l) exp(i k_q.x_j)], so
    (A^T s)_l = sum_j A_{jl} s_j = prod(h) sum_q c_q Re[exp(-i k_q.x_l) sum_j s_j exp(i k_q.x_j)]:
    a sign-(+) transform to the nodes, the weights, and a sign-(-) sum back.
    """
    quad, c = ddi_nodes(prob)
    sh = rhohat(np.asarray(sigma, dtype=np.float64), prob, quad.k, sign=+1.0)
    return nodes_to_grid(c * sh, prob, quad.k, sign=-1.0, real=True)


# --------------------------------------------------------------------------
# The split of Eq. 3.9: Phi ~ I_1 + I_2 with a partition of unity in k
# --------------------------------------------------------------------------
def split_q(k: np.ndarray, s: float) -> np.ndarray:
    """The partition q of Eq. 3.9 at nodes k of shape (M, d) (a reading; the paper asks for a C^inf q
    that decays exponentially with p = (1 - q) Uhat smooth):

    3D: q = exp(-|k|^2 / s^2).  Uhat is homogeneous of degree 0, P(k)/|k|^2 with P quadratic, and
        (1 - q)/|k|^2 is an entire function of |k|^2, so p is smooth (entire).
    2D: q = erfc(|k| / s).  The 2D symbol is homogeneous of degree 1, P(k)/|k|, so p is smooth only
        if (1 - q)/|k| is; a q that is smooth in |k|^2 leaves an odd power of |k| in p.  With
        1 - q = erf(|k|/s), erf(z)/z is an even entire function and p is entire.  q is C^inf as a
        function of |k| (all the polar rule of I_2 integrates) and decays like exp(-|k|^2/s^2).

    In both dimensions the kernel of I_1 then decays like exp(-s^2 r^2 / 4)."""
    k = np.asarray(k)
    kk = np.sum(k * k, axis=-1)
    if k.shape[-1] == 3:
        return np.exp(-kk / (s * s))
    return special.erfc(np.sqrt(kk) / s)


def split_one_minus_q(u: np.ndarray, s: float, dim: int) -> np.ndarray:
    """1 - q at |k|^2 = u, evaluated without cancellation: -expm1(-u/s^2) (3D), erf(|k|/s) (2D)."""
    if dim == 3:
        return -np.expm1(-u / (s * s))
    return special.erf(np.sqrt(u) / s)


def split_defaults(L, tol: float):
    """(s, R_2) for a box of half lengths L and a target relative accuracy tol (reading).

    I_1 is a circular convolution with period 4 L_i (zero-padded box); its kernel, the inverse
    transform of (1 - q) Uhat, decays like exp(-s^2 r^2 / 4), and the nearest image of the
    density lies 2 L_min away, so s^2 L_min^2 = ln(1/tol).  The integrand of I_2 carries
    exp(-|k|^2/s^2), so the ball radius R_2 = s sqrt(ln(1/tol)) = ln(1/tol) / L_min.
    """
    lt = math.log(1.0 / tol)
    s = math.sqrt(lt) / min(L)
    return s, s * math.sqrt(lt)


def split_short_range(rho: np.ndarray, prob: DDIProblem, s: float) -> np.ndarray:
    """I_1 of Eq. 3.9: (2 pi)^-d int_Omega exp(i k.x) p(k) rhohat(k) dk, p = (1 - q) Uhat,
    over the Nyquist box Omega = {|k_i| <= pi/h_i}, by the regular FFT (3D and 2D).

    The trapezoid rule in k on the grid of the box zero-padded to [-L, 3L) per axis
    (2 N_i points, k_m = 2 pi m / (2 N_i h_i), m in (-N_i, N_i): the Nyquist planes
    m_i = -N_i are left out, so the set is symmetric and the sum real), with rhohat(k_m) the
    trapezoid rule of the transform.  With F = fftn of rho padded with zeros at the end,
    rhohat(k_m) = prod(h) exp(-i k_m L) F_m and (2 pi)^-d prod(dk) prod(h) = 1/prod(2N), so
    I_1 = ifftn(p F) on the first N_i points of each axis.  (The FFT is the library step
    that evaluates these trapezoid sums; nothing else is reordered.)
    """
    d = prob.dim
    rho = np.asarray(rho, dtype=np.float64)
    pad = tuple(2 * n for n in prob.n)
    F = np.fft.fftn(rho, s=pad, axes=tuple(range(d)))
    ks = [TWO_PI * np.fft.fftfreq(2 * n, d=h) for n, h in zip(prob.n, prob.h)]
    K = np.stack(np.meshgrid(*ks, indexing="ij"), axis=-1)
    u = np.sum(K * K, axis=-1)
    n = np.asarray(prob.dip_n, dtype=np.float64)
    m = n if prob.dip_m is None else np.asarray(prob.dip_m, dtype=np.float64)
    with np.errstate(invalid="ignore", divide="ignore"):
        if d == 3:
            U = 3.0 * (K @ n) * (K @ m) / u - float(n @ m)
        else:
            U = 3.0 * ((K @ n[:2]) * (K @ m[:2]) - n[2] * m[2] * u) / (2.0 * np.sqrt(u))
    p = split_one_minus_q(u, s, d) * U
    p[u == 0.0] = 0.0                                    # (1 - q) Uhat vanishes at k = 0
    for ax, na in enumerate(prob.n):                     # Nyquist planes m_i = -N_i
        idx = [slice(None)] * d
        idx[ax] = na
        p[tuple(idx)] = 0.0
    out = np.fft.ifftn(p * F)
    return out.real[tuple(slice(0, na) for na in prob.n)].copy()


def split_long_range_nodes(prob: DDIProblem, s: float):
    """(k_q, c_q q(k_q)) for I_2 of Eq. 3.9: the spherical (3D) or polar (2D) quadrature of
    Eq. DDI-Trun1 on the ball of radius prob.kmax, weights times q."""
    quad = quadrature(prob)
    return quad.k, node_coefficients(prob, quad) * split_q(quad.k, s)


def split_long_range(rho: np.ndarray, prob: DDIProblem, s: float) -> np.ndarray:
    """I_2 of Eq. 3.9 by the same direct sums as ddi_apply over the weighted nodes."""
    k, c = split_long_range_nodes(prob, s)
    rh = rhohat(np.asarray(rho, dtype=np.float64), prob, k, sign=-1.0)
    return nodes_to_grid(c * rh, prob, k, sign=+1.0, real=True)


def split_apply(rho: np.ndarray, prob: DDIProblem, s: float) -> np.ndarray:
    """Phi ~ I_1 + I_2 (Eq. 3.9); prob's quadrature is that of the I_2 ball."""
    return split_short_range(rho, prob, s) + split_long_range(rho, prob, s)


# --------------------------------------------------------------------------
# GPE energy (Eq. energy, split as in Sec. 3.2) and its gradient
# --------------------------------------------------------------------------
@dataclass
class GPEParams:
    beta: float = 0.0
    lam: float = 0.0
    gamma: tuple = (1.0, 1.0, 1.0)
    V: np.ndarray | None = None      # optional real grid overriding the harmonic trap


def trap_potential(prob: DDIProblem, gp: GPEParams) -> np.ndarray:
    """V(x) = 1/2 sum_i gamma_i^2 x_i^2 (Eq. Vpoten) unless gp.V is given."""
    if gp.V is not None:
        return np.asarray(gp.V, dtype=np.float64)
    xs = prob.axes()
    grids = np.meshgrid(*xs, indexing="ij")
    return 0.5 * sum((gp.gamma[i] ** 2) * grids[i] ** 2 for i in range(prob.dim))


def fourier_mu2(prob: DDIProblem) -> np.ndarray:
    """|mu_p|^2 with mu_p = 2 pi p / (2 L) for p in [-N/2, N/2) in numpy FFT order (Sec. 4.1 sets)."""
    mus = [TWO_PI * np.fft.fftfreq(ni, d=2.0 * Li / ni) for ni, Li in zip(prob.n, prob.L)]
    grids = np.meshgrid(*mus, indexing="ij")
    return sum(g * g for g in grids)


def gpe_energy_grad(psi: np.ndarray, prob: DDIProblem, gp: GPEParams, grad: bool = True, ops=None):
    """Energy parts (Sec. 3.2) and G = dE_h / d conj(psi) on the grid.

    E_kin = 1/2 prod(h)/prod(N) sum_p |mu_p|^2 |psihat_p|^2      (psihat: DFT of psi)
    E_pot = prod(h) sum V |psi|^2
    E_int = beta/2 prod(h) sum |psi|^4
    E_dip = lam/2 prod(h) sum Phi |psi|^2, Phi = A |psi|^2
    G     = prod(h) [ -1/2 Lap psi + V psi + beta |psi|^2 psi + lam/2 (A rho + A^T rho) psi ]
    Returns (E, G) with E = [kin, pot, int, dip, total]; G is None if not grad.
    The DFT over the grid is numpy's FFT (a library step).  ops: optional (A, A^T) as callables
    on real grids (e.g. the split of Eq. 3.9); ddi_apply and ddi_apply_adjoint otherwise.
    """
    apply_A, apply_At = ops if ops is not None else (lambda r: ddi_apply(r, prob),
                                                     lambda r: ddi_apply_adjoint(r, prob))
    psi = np.asarray(psi, dtype=np.complex128)
    cell = prob.cell
    rho = (psi.real ** 2 + psi.imag ** 2)
    V = trap_potential(prob, gp)
    phi = apply_A(rho)
    psih = np.fft.fftn(psi)
    mu2 = fourier_mu2(prob)
    ntot = float(np.prod(prob.n))
    e_kin = 0.5 * cell / ntot * float(np.sum(mu2 * (psih.real ** 2 + psih.imag ** 2)))
    e_pot = cell * float(np.sum(V * rho))
    e_int = 0.5 * gp.beta * cell * float(np.sum(rho * rho))
    e_dip = 0.5 * gp.lam * cell * float(np.sum(phi * rho))
    E = np.array([e_kin, e_pot, e_int, e_dip, e_kin + e_pot + e_int + e_dip])
    if not grad:
        return E, None
    lap_term = np.fft.ifftn(0.5 * mu2 * psih)          # -1/2 Lap psi
    phit = apply_At(rho)
    G = cell * (lap_term + V * psi + gp.beta * rho * psi + 0.5 * gp.lam * (phi + phit) * psi)
    return E, G


def chemical_potential(E: np.ndarray) -> float:
    """mu = E + E_int + E_dip (Sec. 3.2)."""
    return float(E[4] + E[2] + E[3])


def virial(E: np.ndarray) -> float:
    """I = 2 E_kin - 2 E_pot + 3 E_int + 3 E_dip (Eq. vir_iden, 3D)."""
    return float(2 * E[0] - 2 * E[1] + 3 * E[2] + 3 * E[3])


def gf_step(phi_n: np.ndarray, prob: DDIProblem, gp: GPEParams, dt: float, n_inner: int = 1):
    """One step of the gradient flow with discrete normalisation (Eqs. gf-eq2, gf-colb2, gffg33).

    The DDI Phi^n = A |phi^n|^2 is evaluated once per step (Eq. gf-colb2).  The
    linear system of Eq. gf-eq2, (1/dt - 1/2 Lap + B) phi1 = phi^n/dt with the
    frozen coefficient B = V + beta|phi^n|^2 + lam Phi^n, is solved by the
    stabilised Fourier iteration
        (1/dt + alpha - 1/2 Lap) phi1_{j+1} = phi^n/dt + (alpha - B) phi1_j,
        phi1_0 = phi^n, alpha = (max B + min B)/2,
    taken ``n_inner`` times, each step diagonal in Fourier space; then phi1 is
    normalised so that prod(h) sum |phi|^2 = 1 (Eq. gffg33).
    """
    phi_n = np.asarray(phi_n, dtype=np.complex128)
    rho = phi_n.real ** 2 + phi_n.imag ** 2
    B = trap_potential(prob, gp) + gp.beta * rho + gp.lam * ddi_apply(rho, prob)
    alpha = 0.5 * (float(B.max()) + float(B.min()))
    mu2 = fourier_mu2(prob)
    denom = 1.0 / dt + alpha + 0.5 * mu2
    rhs0 = np.fft.fftn(phi_n) / dt
    phi1 = phi_n
    for _ in range(n_inner):
        phi1 = np.fft.ifftn((rhs0 + np.fft.fftn((alpha - B) * phi1)) / denom)
    norm = math.sqrt(prob.cell * float(np.sum(phi1.real ** 2 + phi1.imag ** 2)))
    return phi1 / norm


def ts_step(psi_n: np.ndarray, prob: DDIProblem, gp: GPEParams, dt: float, delta: float = 0.0, q: float = 0.0):
    """One step of the second-order time splitting of Eq. tssp2 for the dipolar GPE of
    Eq. DipGPE1 with the cubic nonlinearity (sigma = 1), a time-independent dipole axis and the
    damping f = delta >= 0 (Case I: delta = 0; Case II: linear damping delta > 0):

        psi1      = IDFT[ exp(-i dt |mu_p|^2 / 4) DFT(psi_n) ]
        psi2      = psi1 exp(-i [dt V + H + G]) exp(-F),   rho1 = |psi1|^2,
                    H = beta s rho1,  G = lam s (A rho1),  F = delta dt,
                    s = dt (delta = 0) or (1 - exp(-2 delta dt)) / (2 delta)
        psi^{n+1} = IDFT[ exp(-i dt |mu_p|^2 / 4) DFT(psi2) ]

    (H, G, F are the Case I / Case II closed forms of Eqs. fun1-fun2 with h(phi, s) =
    phi exp(-2 delta s).)  The DFT is numpy's FFT (a library step); A is ddi_apply.

    q > 0 (with delta > 0): Case III, the loss f(rho) = delta rho^q, whose closed forms for
    sigma = 1 share one function of rho1,
        w = [(1 + 2 q delta dt rho1^q)^(1 - 1/q) - 1] / (2 delta (q - 1) rho1^(q-1))   (q != 1)
        w = ln(1 + 2 delta dt rho1) / (2 delta)                                          (q = 1)
    with H = beta w, G = lam (A w), F = ln(1 + 2 q delta dt rho1^q) / (2 q).
    """
    psi = np.asarray(psi_n, dtype=np.complex128)
    kin = np.exp(-0.25j * dt * fourier_mu2(prob))
    psi1 = np.fft.ifftn(kin * np.fft.fftn(psi))
    rho1 = psi1.real ** 2 + psi1.imag ** 2
    if q > 0.0:
        if not delta > 0.0:
            raise ValueError("Case III needs delta > 0")
        x = 2.0 * q * delta * dt * rho1 ** q
        if q == 1.0:
            w = np.log1p(x) / (2.0 * delta)
        else:
            with np.errstate(divide="ignore", invalid="ignore"):
                w = np.expm1((1.0 - 1.0 / q) * np.log1p(x)) / (2.0 * delta * (q - 1.0) * rho1 ** (q - 1.0))
            w = np.where(rho1 > 0.0, w, 0.0)
        theta = dt * trap_potential(prob, gp) + gp.beta * w
        if gp.lam != 0.0:
            theta = theta + gp.lam * ddi_apply(w, prob)
        psi2 = psi1 * np.exp(-1j * theta) * np.exp(-np.log1p(x) / (2.0 * q))
        return np.fft.ifftn(kin * np.fft.fftn(psi2))
    s = dt if delta == 0.0 else -math.expm1(-2.0 * delta * dt) / (2.0 * delta)
    theta = dt * trap_potential(prob, gp) + gp.beta * s * rho1
    if gp.lam != 0.0:
        theta = theta + gp.lam * s * ddi_apply(rho1, prob)
    psi2 = psi1 * np.exp(-1j * theta) * math.exp(-delta * dt)
    return np.fft.ifftn(kin * np.fft.fftn(psi2))


def ts_steps_rotating(psi0: np.ndarray, prob: DDIProblem, gp: GPEParams, t0: float, dt: float, steps: int,
                      axis) -> np.ndarray:
    """Eq. tssp2 (Case I, delta = 0) with a time-dependent dipole axis n(t) = m(t) = axis(t), as
    in Eq. dip_rot.  G of Eq. fun2 is lam int_{t_n}^{t_{n+1}} U_dip(., tau) * rho dtau; it is taken
    by the midpoint rule, lam dt U_dip(., t_n + dt/2) * rho (a reading: second order, like the
    splitting).  Each step sets the problem's axis and then takes ts_step."""
    psi = np.asarray(psi0, dtype=np.complex128)
    for j in range(steps):
        prob.dip_n = tuple(float(v) for v in axis(t0 + (j + 0.5) * dt))
        prob.dip_m = None
        prob._cache.clear()                  # the node coefficients depend on the axis
        psi = ts_step(psi, prob, gp, dt)
    return psi


# --------------------------------------------------------------------------
# Error metrics (Eq. error_l2 and the relative max-norm)
# --------------------------------------------------------------------------
def rel_l2(approx, exact) -> float:
    """e_h = ||Phi - Phi_h||_2 / ||Phi||_2 (Eq. error_l2)."""
    exact = np.asarray(exact)
    return float(np.linalg.norm((np.asarray(approx) - exact).ravel()) / np.linalg.norm(exact.ravel()))


def rel_linf(approx, exact) -> float:
    """max |Phi - Phi_h| / max |Phi|."""
    exact = np.asarray(exact)
    return float(np.max(np.abs(np.asarray(approx) - exact)) / np.max(np.abs(exact)))


def nodes_to_points(g: np.ndarray, prob: DDIProblem, k: np.ndarray, points: np.ndarray,
                    block: int = 65536) -> np.ndarray:
    """Phi at selected grid points: Phi_l = Re sum_q g_q exp(+i k_q . x_l) for each index row of
    ``points`` (shape (P, d)); the same sum as nodes_to_grid, one point at a time."""
    xs = prob.axes()
    X = np.stack([xs[a][points[:, a]] for a in range(prob.dim)], axis=1)      # (P, d)
    out = np.zeros(points.shape[0])
    for s in range(0, k.shape[0], block):
        arg = X @ k[s:s + block].T                                              # (P, B)
        gb = g[s:s + block]
        out += np.cos(arg) @ gb.real - np.sin(arg) @ gb.imag
    return out
