"""Ground states by the gradient flow with discrete normalisation (Sec. 3.1).

Each step calls ``gpe_gf_step`` of the HIP library: one DDI evaluation (Eq. gf-colb2), the
stabilised backward-Euler Fourier solve of Eq. gf-eq2 and the normalisation of
Eq. gffg33.  The energies of Sec. 3.2 are evaluated by ``gpe_energy_grad`` every
``energy_every`` steps.  The paper stops when max|phi^{n+1} - phi^n| / dt <= eps0; that residual
is computed by ``gpe_gf_step`` itself (a reduction in the library, on the steps that report), is
reported with the energies and, if ``eps0`` is given, ends the flow.  Apart from the checkpoint
copies, this driver launches no device work of its own.
State can be checkpointed to an ``.npz`` file and resumed.

Eq. gf-eq2 is a linear system; each step solves it with ``n_inner`` stabilised Fourier
iterations.  The flow's fixed point is the ground state only when those iterations have
converged (their contraction factor is about (max B - min B) / (2 (1/dt + alpha))): at 128^3 on
[-12,12)^3, 30 iterations at dt = 0.02 reproduce the energies of the paper's Table 7, while a
single iteration leaves errors of about 1e-3 in the energy parts.
"""
from __future__ import annotations

import os

import numpy as np
import torch

from .ddi import DDIPlan


def ground_state(plan: DDIPlan, psi0: torch.Tensor, beta: float, lam: float, gamma=(1.0, 1.0, 1.0),
                 dt: float = 0.01, steps: int = 200, n_inner: int = 1, energy_every: int = 10,
                 eps0: float | None = None, checkpoint: str | None = None, checkpoint_every: int = 50,
                 resume: bool = False):
    """Run the flow from psi0; returns (psi, history) with history rows
    (step, E_kin, E_pot, E_int, E_dip, E, mu, residual)."""
    psi = psi0.contiguous()
    start = 0
    history = []
    if resume and checkpoint and os.path.exists(checkpoint):
        with np.load(checkpoint, allow_pickle=False) as z:
            psi = torch.from_numpy(z["psi"]).to(psi0.device, psi0.dtype).contiguous()
            start = int(z["step"])
            history = [tuple(r) for r in z["history"].tolist()]
    nxt = torch.empty_like(psi)
    res_dev = torch.zeros(1, dtype=torch.float64, device=psi.device)   # written by gpe_gf_step
    for step in range(start + 1, steps + 1):
        report = step % energy_every == 0 or step == steps
        plan.gf_step(psi, beta, lam, gamma, dt=dt, n_inner=n_inner, out=nxt, residual=res_dev if report else None)
        done = False
        if report:
            E, _ = plan.energy_grad(nxt, beta, lam, gamma, grad=False)    # synchronises the stream
            res = float(res_dev.cpu()[0])
            mu = float(E[4] + E[2] + E[3])
            history.append((step, *[float(v) for v in E], mu, res))
            done = eps0 is not None and res <= eps0
        psi, nxt = nxt, psi
        if checkpoint and (step % checkpoint_every == 0 or step == steps or done):
            np.savez(checkpoint, psi=psi.cpu().numpy(), step=step, history=np.array(history, dtype=np.float64))
        if done:
            break
    return psi, history
