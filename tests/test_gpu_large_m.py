"""Parity of the VALU tile kernels against the oracle.

The matrix-core interpolation and spread address each node's kernel-weight rows (3 axes x 16
values) with 32-bit byte offsets, so a 3D plan uses them only while (M + 1) * 384 bytes stay
below 2^31, M < 5,592,405 nodes.  Beyond that the plan falls back to the VALU forms of the same
tile schedule: the FP64 interpolation with the tile broadcast from LDS to lanes holding one
entry's weights each, and the staged spread (FP32 with Kahan compensation).  A 16^3 grid with a
6.1M-node spherical rule (192 x 160 x 320, Sec. 2.1) runs both; type-2 at every node and type-1
on the whole grid are compared with the oracle's direct sums.

FP64 bar: rel Linf <= 1e-12.  Mixed bar (type-1, the Kahan spread): rel Linf <= 1e-6 against the
FP64 oracle on the FP32-rounded node values.
"""
import numpy as np
import pytest

from oracle import ddi_oracle as O

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1504_02897_amd.ddi import DDIPlan  # noqa: E402

DEV = "cuda:0"
M_ROWS_LIMIT = 5_592_405          # first M with (M + 1) * 384 >= 2^31
QUAD = (192, 160, 320)
N = (16, 16, 16)
L = (3.0, 3.0, 3.0)
DIP = (0.6, 0.0, 0.8)


def say(msg):
    print(msg, flush=True)


def relinf(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / np.max(np.abs(np.asarray(b))))


def rows_by_index(plan, prob):
    """Oracle rows of the plan's nodes, matched by (radial, polar, azimuthal) index only."""
    idx, _, _ = plan.nodes()
    quad, _ = O.ddi_nodes(prob)
    npol, nazi = prob.n_pol, prob.n_azi

    def lin(t):
        t = t.astype(np.int64)
        return (t[:, 0] * npol + t[:, 1]) * nazi + t[:, 2]

    qk = lin(quad.index)
    order = np.argsort(qk, kind="stable")
    want = lin(idx)
    pos = np.searchsorted(qk[order], want)
    assert np.all(pos < qk.size) and np.all(qk[order][np.minimum(pos, qk.size - 1)] == want)
    return order[pos], quad


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_valu_tile_kernels_beyond_row_limit(prec):
    say(f"case: 16^3, quadrature {QUAD}, {prec} (VALU tile kernels)")
    tol = 1e-13 if prec == "fp64" else 1e-7
    plan = DDIPlan(3, N, L, dip_n=DIP, quad=QUAD, prec=prec, tol=tol)
    prob = O.DDIProblem(dim=3, n=N, L=L, dip_n=DIP, n_rad=QUAD[0], n_pol=QUAD[1], n_azi=QUAD[2])
    assert plan.m_eff >= M_ROWS_LIMIT
    rows, quad = rows_by_index(plan, prob)
    k = quad.k[rows]
    rng = np.random.default_rng(21)
    if prec == "fp64":
        rho = np.abs(rng.standard_normal(N)) + 0.1
        rh = plan.type2(torch.from_numpy(rho).to(DEV)).cpu().numpy()
        err2 = relinf(rh, O.rhohat(rho, prob, k))
        say(f"  type2 rel Linf = {err2:.3e}")
        assert err2 < 1e-12
    g = rng.standard_normal(plan.m_eff) + 1j * rng.standard_normal(plan.m_eff)
    if prec == "fp64":
        gd = torch.from_numpy(g).to(DEV)
    else:
        g = g.astype(np.complex64).astype(np.complex128)
        gd = torch.from_numpy(g.astype(np.complex64)).to(DEV)
    phi = plan.type1(gd).cpu().numpy().astype(np.float64)
    err1 = relinf(phi, O.nodes_to_grid(g, prob, k))
    say(f"  type1 rel Linf = {err1:.3e}")
    assert err1 < (1e-12 if prec == "fp64" else 1e-6)
