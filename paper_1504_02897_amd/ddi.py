"""ctypes binding of libddi (include/ddi.h) and the autograd functions.

Argument marshalling only: every step of the DDI path runs in the HIP library.
Tensors are torch device tensors (C-contiguous, on the plan's device); work is
enqueued on ``torch.cuda.current_stream()``.  If the library is missing the
import of this module raises: there is no fallback.
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libddi.so")

DDI_FP64 = 0
DDI_MIXED = 1
_STATUS = {0: "DDI_OK", 1: "DDI_EINVAL", 2: "DDI_ENOMEM", 3: "DDI_EDEVICE", 4: "DDI_ENOTSUP", 5: "DDI_EINTERNAL"}


class DDIError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{_STATUS.get(status, status)}: {message}")
        self.status = status


class DDIParams(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("n", ctypes.c_int64 * 3), ("L", ctypes.c_double * 3),
                ("dip_n", ctypes.c_double * 3), ("dip_m", ctypes.c_double * 3),
                ("n_rad", ctypes.c_int64), ("n_pol", ctypes.c_int64), ("n_azi", ctypes.c_int64),
                ("kmax", ctypes.c_double), ("nyquist_mask", ctypes.c_int32), ("tol", ctypes.c_double),
                ("prec", ctypes.c_int32), ("kernel_width", ctypes.c_int32),
                ("split", ctypes.c_int32), ("split_s", ctypes.c_double), ("stretch", ctypes.c_double * 3)]


class GPEParamsC(ctypes.Structure):
    _fields_ = [("beta", ctypes.c_double), ("lam", ctypes.c_double), ("gamma", ctypes.c_double * 3),
                ("V_dev", ctypes.c_void_p)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("m_eff", ctypes.c_int64), ("m_nominal", ctypes.c_int64), ("m_half", ctypes.c_int64),
                ("apply_window", ctypes.c_int64),
                ("n_fine", ctypes.c_int64 * 3),
                ("width", ctypes.c_int32), ("es_beta", ctypes.c_double), ("kmax", ctypes.c_double),
                ("spread_items", ctypes.c_int64), ("spread_entries", ctypes.c_int64),
                ("workspace_bytes", ctypes.c_int64),
                ("split", ctypes.c_int32), ("split_s", ctypes.c_double)]


EXPORTED = ["ddi_plan", "ddi_apply", "ddi_apply_adjoint", "ddi_type2", "ddi_type1", "gpe_energy_grad",
            "gpe_energy_grad_noalloc",
            "gpe_gf_step", "gpe_ts_step", "gpe_ts_step_loss", "ddi_set_dipole", "ddi_profile_apply", "ddi_plan_info", "ddi_plan_nodes", "ddi_destroy", "ddi_last_error"]
STAGES = ["fft_last_pad", "fft_axis1_t2", "fft_axis0_t2", "interp", "spread", "spread_reduce", "fft_axis0_t1",
          "fft_axis1_t1", "fft_last_trunc"]


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    if not os.path.exists(path):
        raise ImportError(f"libddi.so not found at {path}; build it with `python -m paper_1504_02897_amd.build`")
    lib = ctypes.CDLL(path)
    vp, i32, f64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double
    lib.ddi_plan.argtypes = [ctypes.POINTER(DDIParams), vp, ctypes.POINTER(vp)]
    for name in ("ddi_apply", "ddi_apply_adjoint", "ddi_type2", "ddi_type1"):
        getattr(lib, name).argtypes = [vp, vp, vp, vp]
    lib.gpe_energy_grad.argtypes = [vp, ctypes.POINTER(GPEParamsC), vp, ctypes.POINTER(f64), vp, vp]
    lib.gpe_energy_grad_noalloc.argtypes = [vp, ctypes.POINTER(GPEParamsC), vp, vp, vp, vp]
    lib.gpe_gf_step.argtypes = [vp, ctypes.POINTER(GPEParamsC), f64, i32, vp, vp, vp, vp]
    lib.gpe_ts_step.argtypes = [vp, ctypes.POINTER(GPEParamsC), f64, f64, vp, vp, vp]
    lib.ddi_set_dipole.argtypes = [vp, ctypes.POINTER(f64), ctypes.POINTER(f64), vp]
    lib.gpe_ts_step_loss.argtypes = [vp, ctypes.POINTER(GPEParamsC), f64, f64, f64, vp, vp, vp]
    lib.ddi_profile_apply.argtypes = [vp, vp, vp, i32, i32, ctypes.POINTER(f64), vp]
    lib.ddi_plan_info.argtypes = [vp, ctypes.POINTER(PlanInfo)]
    lib.ddi_plan_nodes.argtypes = [vp, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(f64), ctypes.POINTER(f64)]
    lib.ddi_destroy.argtypes = [vp]
    lib.ddi_destroy.restype = None
    lib.ddi_last_error.argtypes = []
    lib.ddi_last_error.restype = ctypes.c_char_p
    for name in EXPORTED:
        if name not in ("ddi_destroy", "ddi_last_error"):
            getattr(lib, name).restype = ctypes.c_int
    return lib


_lib = load_library()


def _check(status):
    if status != 0:
        raise DDIError(status, _lib.ddi_last_error().decode())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def make_params(dim, n, L, dip_n=(0.0, 0.0, 1.0), dip_m=None, quad=(32, 16, 32), kmax=0.0,
                nyquist_mask=True, tol=1e-13, prec="fp64", kernel_width=0, split=False, split_s=0.0,
                stretch=(1.0, 1.0, 1.0)) -> DDIParams:
    """The ddi_params struct of a plan; the arguments are those of DDIPlan."""
    if prec not in ("fp64", "mixed"):
        raise ValueError("prec must be 'fp64' or 'mixed'")
    p = DDIParams()
    p.dim = int(dim)
    nn = list(n) + [1] * (3 - len(n))
    LL = list(L) + [1.0] * (3 - len(L))
    for i in range(3):
        p.n[i] = int(nn[i])
        p.L[i] = float(LL[i])
        p.dip_n[i] = float(dip_n[i])
        p.dip_m[i] = 0.0 if dip_m is None else float(dip_m[i])
    p.n_rad, p.n_pol, p.n_azi = (int(quad[0]), int(quad[1]), int(quad[2]))
    p.kmax = float(kmax)
    p.nyquist_mask = 1 if nyquist_mask else 0
    p.tol = float(tol)
    p.prec = DDI_MIXED if prec == "mixed" else DDI_FP64
    p.kernel_width = int(kernel_width)
    p.split = 1 if split else 0
    p.split_s = float(split_s)
    st = list(stretch) + [1.0] * (3 - len(stretch))
    for i in range(3):
        p.stretch[i] = float(st[i])
    return p


class DDIPlan:
    """A DDI plan: quadrature, kernel tables, spread schedule and workspace on one GPU.

    dim, n, L        grid (n points per axis on [-L, L)).
    dip_n, dip_m     dipole axes (dip_m None means m = n).
    quad             (n_rad, n_pol, n_azi); n_pol ignored in 2D.
    prec             "fp64" or "mixed".
    split, split_s   the split of Eq. 3.9 (3D and 2D): Phi = I_1 + I_2, I_1 by the zero-padded FFT,
                     I_2 over the ball of radius kmax (quad and kmax are then I_2's;
                     kmax = 0 and split_s = 0 select the defaults from tol and the box).
    stretch          per-axis factors of the quadrature (k = S k', weights times det S) for
                     anisotropic boxes; (1, 1, 1) is the plain rule.
    """

    def __init__(self, dim, n, L, dip_n=(0.0, 0.0, 1.0), dip_m=None, quad=(32, 16, 32), kmax=0.0,
                 nyquist_mask=True, tol=1e-13, prec="fp64", kernel_width=0, split=False, split_s=0.0,
                 stretch=(1.0, 1.0, 1.0)):
        p = make_params(dim, n, L, dip_n, dip_m, quad, kmax, nyquist_mask, tol, prec, kernel_width,
                        split, split_s, stretch)
        self.dim = int(dim)
        self.shape = tuple(int(v) for v in n[:dim])
        self.L = tuple(float(v) for v in L[:dim])
        self.prec = prec
        self.real_dtype = torch.float32 if prec == "mixed" else torch.float64
        self.complex_dtype = torch.complex64 if prec == "mixed" else torch.complex128
        self.device = torch.device("cuda", torch.cuda.current_device())
        self._h = ctypes.c_void_p()
        _check(_lib.ddi_plan(ctypes.byref(p), _stream(), ctypes.byref(self._h)))
        info = PlanInfo()
        _check(_lib.ddi_plan_info(self._h, ctypes.byref(info)))
        self.info = {"m_eff": info.m_eff, "m_nominal": info.m_nominal, "m_half": info.m_half, "apply_window": info.apply_window,
                     "n_fine": tuple(info.n_fine),
                     "width": info.width, "es_beta": info.es_beta, "kmax": info.kmax,
                     "spread_items": info.spread_items, "spread_entries": info.spread_entries,
                     "workspace_bytes": info.workspace_bytes,
                     "split": bool(info.split), "split_s": info.split_s}
        self.m_eff = int(info.m_eff)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                torch.cuda.synchronize(self.device)
            except Exception:
                pass
            _lib.ddi_destroy(h)
            self._h = None

    @property
    def cell(self):
        return float(np.prod([2.0 * Li / ni for Li, ni in zip(self.L, self.shape)]))

    # ---------------------------------------------------------------- checks
    def _grid(self, t, complex_=False, name="input"):
        want = self.complex_dtype if complex_ else self.real_dtype
        if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
            raise TypeError(f"{name} must be a CUDA tensor")
        if t.dtype != want:
            raise TypeError(f"{name} must have dtype {want}, got {t.dtype}")
        if tuple(t.shape) != self.shape:
            raise ValueError(f"{name} must have shape {self.shape}, got {tuple(t.shape)}")
        return t.contiguous()

    def _nodes(self, t, name="g"):
        if not isinstance(t, torch.Tensor) or t.device.type != "cuda" or t.dtype != self.complex_dtype:
            raise TypeError(f"{name} must be a CUDA tensor of dtype {self.complex_dtype}")
        if tuple(t.shape) != (self.m_eff,):
            raise ValueError(f"{name} must have shape ({self.m_eff},)")
        return t.contiguous()

    # ---------------------------------------------------------------- operators
    def apply(self, rho, out=None):
        rho = self._grid(rho, name="rho")
        out = torch.empty_like(rho) if out is None else self._grid(out, name="out")
        _check(_lib.ddi_apply(self._h, _ptr(rho), _ptr(out), _stream()))
        return out

    def apply_adjoint(self, phibar, out=None):
        phibar = self._grid(phibar, name="phibar")
        out = torch.empty_like(phibar) if out is None else self._grid(out, name="out")
        _check(_lib.ddi_apply_adjoint(self._h, _ptr(phibar), _ptr(out), _stream()))
        return out

    def profile(self, x, sign=1, reps=10, out=None):
        """Mean per-stage milliseconds of `reps` applies (sign +1) or adjoints (sign -1), keyed by STAGES."""
        x = self._grid(x, name="input")
        out = torch.empty_like(x) if out is None else self._grid(out, name="out")
        ms = (ctypes.c_double * len(STAGES))()
        _check(_lib.ddi_profile_apply(self._h, _ptr(x), _ptr(out), int(sign), int(reps), ms, _stream()))
        return dict(zip(STAGES, list(ms)))

    def type2(self, rho, out=None):
        rho = self._grid(rho, name="rho")
        if out is None:
            out = torch.empty(self.m_eff, dtype=self.complex_dtype, device=rho.device)
        _check(_lib.ddi_type2(self._h, _ptr(rho), _ptr(out), _stream()))
        return out

    def type1(self, g, out=None):
        g = self._nodes(g)
        if out is None:
            out = torch.empty(self.shape, dtype=self.real_dtype, device=g.device)
        _check(_lib.ddi_type1(self._h, _ptr(g), _ptr(out), _stream()))
        return out

    def _gp(self, beta, lam, gamma, V):
        gp = GPEParamsC()
        gp.beta, gp.lam = float(beta), float(lam)
        g = list(gamma) + [1.0] * (3 - len(gamma))
        for i in range(3):
            gp.gamma[i] = float(g[i])
        if V is not None:
            V = self._grid(V, name="V")
            gp.V_dev = V.data_ptr()
        else:
            gp.V_dev = None
        return gp, V

    def energy_grad(self, psi, beta, lam, gamma=(1.0, 1.0, 1.0), V=None, grad=True):
        """(E[5] numpy: kin, pot, int, dip, total; G = dE/dconj(psi) or None)."""
        psi = self._grid(psi, complex_=True, name="psi")
        gp, V = self._gp(beta, lam, gamma, V)
        E = (ctypes.c_double * 5)()
        G = torch.empty_like(psi) if grad else None
        _check(_lib.gpe_energy_grad(self._h, ctypes.byref(gp), _ptr(psi), E,
                                    _ptr(G) if grad else None, _stream()))
        return np.array(list(E)), G

    def energy_grad_noalloc(self, psi, beta, lam, gamma=(1.0, 1.0, 1.0), V=None, E_out=None, grad_out=None,
                            grad=True):
        """The same energies and gradient through gpe_energy_grad_noalloc, which allocates nothing and
        does not synchronise: E_out (float64 CUDA tensor of 5) and grad_out (or new tensors) receive
        them on the current stream.  Returns (E_out, G or None)."""
        psi = self._grid(psi, complex_=True, name="psi")
        gp, V = self._gp(beta, lam, gamma, V)
        if E_out is None:
            E_out = torch.empty(5, dtype=torch.float64, device=psi.device)
        elif E_out.device.type != "cuda" or E_out.dtype != torch.float64 or E_out.numel() != 5 or not E_out.is_contiguous():
            raise TypeError("E_out must be a contiguous float64 CUDA tensor of 5 elements")
        G = None
        if grad:
            G = torch.empty_like(psi) if grad_out is None else self._grid(grad_out, complex_=True, name="grad_out")
        _check(_lib.gpe_energy_grad_noalloc(self._h, ctypes.byref(gp), _ptr(psi), _ptr(E_out),
                                            _ptr(G) if grad else None, _stream()))
        return E_out, G

    def gf_step(self, psi, beta, lam, gamma=(1.0, 1.0, 1.0), dt=0.01, n_inner=1, V=None, out=None,
                residual=None):
        """One gradient-flow step (gpe_gf_step); out may be psi.  residual: optional float64 CUDA
        tensor of one element that receives max|out - psi| / dt (the stopping quantity)."""
        psi = self._grid(psi, complex_=True, name="psi")
        gp, V = self._gp(beta, lam, gamma, V)
        out = torch.empty_like(psi) if out is None else self._grid(out, complex_=True, name="out")
        if residual is not None and (not isinstance(residual, torch.Tensor) or residual.device.type != "cuda"
                                     or residual.dtype != torch.float64 or residual.numel() != 1):
            raise TypeError("residual must be a float64 CUDA tensor of one element")
        _check(_lib.gpe_gf_step(self._h, ctypes.byref(gp), float(dt), int(n_inner), _ptr(psi), _ptr(out),
                                None if residual is None else _ptr(residual), _stream()))
        return out

    def ts_step(self, psi, beta, lam, gamma=(1.0, 1.0, 1.0), dt=0.001, delta=0.0, V=None, out=None):
        """One time-splitting step of the dynamics (gpe_ts_step); out may be psi (in place)."""
        psi = self._grid(psi, complex_=True, name="psi")
        gp, V = self._gp(beta, lam, gamma, V)
        out = torch.empty_like(psi) if out is None else self._grid(out, complex_=True, name="out")
        _check(_lib.gpe_ts_step(self._h, ctypes.byref(gp), float(dt), float(delta), _ptr(psi), _ptr(out),
                                _stream()))
        return out

    def ts_step_loss(self, psi, beta, lam, gamma=(1.0, 1.0, 1.0), dt=0.001, delta=1.0, q=2.0, V=None, out=None):
        """One time-splitting step with the loss f(rho) = delta rho^q (gpe_ts_step_loss)."""
        psi = self._grid(psi, complex_=True, name="psi")
        gp, V = self._gp(beta, lam, gamma, V)
        out = torch.empty_like(psi) if out is None else self._grid(out, complex_=True, name="out")
        _check(_lib.gpe_ts_step_loss(self._h, ctypes.byref(gp), float(dt), float(delta), float(q), _ptr(psi),
                                     _ptr(out), _stream()))
        return out

    def set_dipole(self, dip_n, dip_m=None):
        """New dipole axes (ddi_set_dipole): the node coefficients are re-evaluated on the device."""
        n = (ctypes.c_double * 3)(*[float(v) for v in dip_n])
        m = None if dip_m is None else (ctypes.c_double * 3)(*[float(v) for v in dip_m])
        _check(_lib.ddi_set_dipole(self._h, n, m, _stream()))

    def nodes(self):
        """(index [M,3] int32, k [M,3] float64, c [M] float64) in plan order."""
        M = self.m_eff
        idx = np.zeros((M, 3), dtype=np.int32)
        k = np.zeros((M, 3), dtype=np.float64)
        c = np.zeros(M, dtype=np.float64)
        _check(_lib.ddi_plan_nodes(self._h, idx.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                   k.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                   c.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return idx, k, c


class DDIFunction(torch.autograd.Function):
    """Phi = A rho with backward rhobar = A^T Phibar (the hand-written adjoint)."""

    @staticmethod
    def forward(ctx, rho, plan):
        ctx.plan = plan
        return plan.apply(rho)

    @staticmethod
    def backward(ctx, grad_out):
        return ctx.plan.apply_adjoint(grad_out.contiguous()), None


def ddi_apply(rho, plan):
    return DDIFunction.apply(rho, plan)


class GPEEnergy(torch.autograd.Function):
    """E(psi) (Sec. 3.2) with backward dE/dpsi in torch's complex convention (2 dE/dconj(psi))."""

    @staticmethod
    def forward(ctx, psi, plan, beta, lam, gamma=(1.0, 1.0, 1.0)):
        E, G = plan.energy_grad(psi, beta, lam, gamma, grad=True)
        ctx.save_for_backward(G)
        return torch.tensor(E[4], dtype=torch.float64, device=psi.device)

    @staticmethod
    def backward(ctx, grad_out):
        (G,) = ctx.saved_tensors
        return 2.0 * G * grad_out.to(G.real.dtype), None, None, None, None
