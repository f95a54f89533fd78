"""New dipole axes on an existing plan (ddi_set_dipole) and the time splitting with a rotating
axis (Eq. dip_rot), through the C ABI.

A plan whose axes were changed must give what a plan built for the new axes gives (FP64: rel
Linf <= 1e-14, the coefficients are re-evaluated on the device in another rounding order;
mixed: <= 1e-6).  The rotating-axis steps are checked element by element against the oracle's
(FP64 bar 1e-12).
"""
import math

import numpy as np
import pytest

from oracle import ddi_oracle as O
from paper_1504_02897_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1504_02897_amd.ddi import DDIError, DDIPlan  # noqa: E402

DEV = "cuda:0"


def say(msg):
    print(msg, flush=True)


def relinf(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / np.max(np.abs(np.asarray(b))))


def to_dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV, dtype)


N1, M1 = (0.0, 0.0, 1.0), None
N2, M2 = (0.48, -0.6, 0.64), (0.0, 0.6, 0.8)
VARIANTS = [
    # (name, dim, n, L, quad, prec, split, tol)
    ("full_fp64_3d", 3, (32, 32, 32), (8.0,) * 3, (16, 8, 16), "fp64", False, 1e-14),
    ("split_fp64_3d", 3, (32, 32, 32), (8.0,) * 3, (16, 16, 32), "fp64", True, 1e-14),
    ("full_mixed_3d", 3, (32, 32, 32), (8.0,) * 3, (16, 8, 16), "mixed", False, 1e-6),
    ("full_fp64_2d", 2, (64, 64), (8.0, 8.0), (24, 1, 48), "fp64", False, 1e-14),
]


@pytest.mark.parametrize("v", VARIANTS, ids=lambda v: v[0])
def test_set_dipole_matches_a_fresh_plan(v):
    name, dim, n, L, quad, prec, split, tol = v
    say(f"case: set_dipole {name}")
    kw = dict(quad=quad, prec=prec, tol=1e-13 if prec == "fp64" else 1e-7, split=split)
    a = DDIPlan(dim, n, L, dip_n=N1, dip_m=M1, **kw)
    b = DDIPlan(dim, n, L, dip_n=N2, dip_m=M2, **kw)
    a.set_dipole(N2, M2)
    rho = I.random_field(21, n) ** 2
    dt = torch.float64 if prec == "fp64" else torch.float32
    pa = a.apply(to_dev(rho, dt)).double().cpu().numpy()
    pb = b.apply(to_dev(rho, dt)).double().cpu().numpy()
    err = relinf(pa, pb)
    say(f"  rel Linf vs a plan built for the new axes {err:.3e}")
    assert err <= tol
    _, _, ca = a.nodes()
    _, _, cb = b.nodes()
    assert np.max(np.abs(ca - cb)) <= 1e-14 * np.max(np.abs(cb))
    # and back: the first axes again
    a.set_dipole(N1, M1)
    c0 = DDIPlan(dim, n, L, dip_n=N1, dip_m=M1, **kw)
    assert relinf(a.apply(to_dev(rho, dt)).double().cpu().numpy(),
                  c0.apply(to_dev(rho, dt)).double().cpu().numpy()) <= tol


def test_set_dipole_rejects_bad_axes():
    p = DDIPlan(3, (16, 16, 16), (6.0,) * 3, quad=(8, 4, 8))
    for bad in [(0.0, 0.0, 0.0), (float("nan"), 0.0, 1.0), (float("inf"), 0.0, 0.0)]:
        with pytest.raises(DDIError):
            p.set_dipole(bad)
    with pytest.raises(DDIError):
        p.set_dipole((0.0, 0.0, 1.0), (float("nan"), 0.0, 0.0))


def test_ts_rotating_axis_matches_oracle():
    """Six steps of Eq. tssp2 with n(t) = (sin 5t, 0, cos 5t): before each step the plan's axis is
    set to n(t_n + dt/2) (the midpoint reading of Eq. fun2), as the oracle does."""
    say("case: ts rotating axis 16^3 fp64, 6 steps")
    n, L = (16, 16, 16), (6.0,) * 3
    quad = (16, 8, 16)
    plan = DDIPlan(3, n, L, dip_n=(0.0, 0.0, 1.0), quad=quad, tol=1e-13)
    prob = O.DDIProblem(dim=3, n=n, L=L, dip_n=(0.0, 0.0, 1.0), n_rad=quad[0], n_pol=quad[1], n_azi=quad[2])
    gp = O.GPEParams(beta=30.0, lam=20.0, gamma=(1.0, 1.0, 2.0))
    lumps, _ = I.mixture_lumps(0, 3, (2, 2), centre=1.0, widths=(0.8, 1.5))
    psi, _ = I.normalise(I.lumps_on_grid(lumps, n, L), n, L)

    def axis(t):
        return np.array([math.sin(5.0 * t), 0.0, math.cos(5.0 * t)])

    dt, steps = 0.01, 6
    x = to_dev(psi, torch.complex128)
    for j in range(steps):
        plan.set_dipole(axis((j + 0.5) * dt))
        plan.ts_step(x, gp.beta, gp.lam, gp.gamma, dt=dt, out=x)
    ref = O.ts_steps_rotating(psi, prob, gp, 0.0, dt, steps, axis)
    err = relinf(x.cpu().numpy(), ref)
    say(f"  rel Linf = {err:.3e}")
    assert err < 1e-12
    # not the fixed-axis evolution
    fixed = psi
    prob0 = O.DDIProblem(dim=3, n=n, L=L, dip_n=(0.0, 0.0, 1.0), n_rad=quad[0], n_pol=quad[1], n_azi=quad[2])
    for _ in range(steps):
        fixed = O.ts_step(fixed, prob0, gp, dt)
    assert relinf(fixed, ref) > 1e-6
