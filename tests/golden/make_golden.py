"""Write the stored oracle values used by the full-size GPU parity tests.

Calls only ``oracle/`` (and the input generators).  Run from the repository root:

    python tests/golden/make_golden.py            # all workloads (several minutes on 8 cores)
    python tests/golden/make_golden.py c3_512     # one workload

For each workload it stores, for the seeded input of ``paper_1504_02897_amd.inputs``:
  * rhohat at a seeded sample of quadrature nodes, keyed by (radial, polar, azimuthal) index;
  * Phi at a seeded sample of grid points plus the max and l2 norm of Phi over the grid
    (only where the full oracle Phi is affordable: c2_128 and c3_512).
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import ddi_oracle as O  # noqa: E402
from paper_1504_02897_amd import inputs as I  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def problem(name, dip):
    wl = I.WORKLOADS[name]
    return O.DDIProblem(dim=wl["dim"], n=wl["n"], L=wl["L"], dip_n=tuple(float(v) for v in dip),
                        n_rad=wl["quad"][0], n_pol=wl["quad"][1], n_azi=wl["quad"][2])


def make(name, full_phi, n_nodes=256, n_points=96, seed=0):
    t0 = time.time()
    wl = I.WORKLOADS[name]
    data = I.mixture_workload(name, seed=seed)
    rho = data["rho"]
    if wl["prec"] == "mixed":
        rho = rho.astype(np.float32).astype(np.float64)   # the mixed path sees the FP32-rounded density
    prob = problem(name, data["dip_n"])
    quad, c = O.ddi_nodes(prob)
    rng = np.random.default_rng(1000 + seed)
    sel = np.sort(rng.choice(quad.k.shape[0], size=n_nodes, replace=False))
    rh_sel = O.rhohat(rho, prob, quad.k[sel])
    out = {
        "_source": "written by tests/golden/make_golden.py from oracle/ddi_oracle.py (direct FP64 sums)",
        "workload": name, "seed": seed, "dip_n": [float(v) for v in data["dip_n"]],
        "rho_precision": "float32-rounded" if wl["prec"] == "mixed" else "float64",
        "m_eff": int(quad.k.shape[0]),
        "node_index": quad.index[sel].tolist(),
        "rhohat": [[float(z.real), float(z.imag)] for z in rh_sel],
        "rhohat_absmax_sample": float(np.max(np.abs(rh_sel))),
        "rhohat0": float(np.real(O.rhohat(rho, prob, np.zeros((1, wl["dim"])))[0])),
    }
    if full_phi:
        phi, _ = O.ddi_apply(rho, prob, return_rhohat=True)
        pts = np.stack([rng.integers(0, n, size=n_points) for n in wl["n"]], axis=1)
        imax = np.unravel_index(np.argmax(np.abs(phi)), phi.shape)
        pts = np.concatenate([pts, np.array(imax)[None, :]], axis=0)
        out.update({
            "points": pts.tolist(),
            "phi": [float(phi[tuple(p)]) for p in pts],
            "phi_absmax": float(np.max(np.abs(phi))),
            "phi_l2": float(np.linalg.norm(phi.ravel())),
        })
    path = os.path.join(HERE, f"{name}_seed{seed}.json")
    with open(path, "w") as f:
        json.dump(out, f)
    print(f"{path}: {time.time() - t0:.1f} s", flush=True)


if __name__ == "__main__":
    which = sys.argv[1:] or ["c3_512", "c4_256", "c2_128"]
    for w in which:
        make(w, full_phi=(w in ("c2_128", "c3_512")))
