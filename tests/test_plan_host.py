"""The plan builder's host tables on the CPU (no device): the library's plan.cpp is compiled
with g++ into a small driver (tests/host/plan_tables.cpp) that writes every table a plan uploads.

Checked against what fixes them independently of the library:
- nodes and coefficients: the oracle's quadrature of Eq. DDI-Trun1 (and its stretched form and
  the I_2 weights of Eq. 3.9);
- the +-k pairs of the tensor rule: k_partner = -k with equal coefficients, one member kept;
- kernel rows and deconvolution together: for every node, axis and grid mode m, the deconvolved
  kernel row reproduces the exact phase exp(-i t m) of the type-2 sum (Sec. 2.1 via the NUFFT),
  to the accuracy the plan's width was chosen for;
- schedules: every (tile, node) pair of the spread exactly once, the chunking and reduce slots,
  the packed weight-row offsets, the per-node gather lists, the interpolation groups, and the
  last-axis and axis-1 windows containing every support.
"""
import ctypes
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import ddi_oracle as O
from paper_1504_02897_amd.ddi import DDIParams, make_params

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HARNESS = os.path.join(ROOT, "tests", "host", "plan_tables.cpp")
PLAN_CPP = os.path.join(ROOT, "paper_1504_02897_amd", "csrc", "plan.cpp")
ROCM_INC = "/opt/rocm/include"
K_OFF_BIAS = 8      # entry offsets are stored biased by this
K_ENT_PAD = 32      # zero entries after the last one


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None or not os.path.isdir(ROCM_INC):
        pytest.skip("g++ or the ROCm headers are not available")
    exe = str(tmp_path_factory.mktemp("plan_host") / "plan_tables")
    cmd = [gxx, "-std=c++17", "-O2", "-D__HIP_PLATFORM_AMD__", "-I" + ROCM_INC, HARNESS, PLAN_CPP, "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return exe


def run_tables(driver, tmp_path, **kw):
    p = make_params(**kw)
    assert ctypes.sizeof(p) == ctypes.sizeof(DDIParams)
    pin, pout = tmp_path / "params.bin", tmp_path / "tables.bin"
    pin.write_bytes(bytes(p))
    r = subprocess.run([driver, str(pin), str(pout)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    raw = pout.read_bytes()
    out, off = {}, 0
    while off < len(raw):
        n = int(np.frombuffer(raw, np.uint32, 1, off)[0]); off += 4
        name = raw[off:off + n].decode(); off += n
        typ = chr(raw[off]); off += 1
        cnt = int(np.frombuffer(raw, np.int64, 1, off)[0]); off += 8
        dt = np.int32 if typ == "i" else np.float64
        out[name] = np.frombuffer(raw, dt, cnt, off).copy()
        off += cnt * np.dtype(dt).itemsize
    if "message_chars" in out:
        out["message"] = "".join(chr(c) for c in out["message_chars"])
    return out


CASES = {
    # name: (plan arguments, oracle problem arguments)
    "3d_fp64": (dict(dim=3, n=(32, 32, 32), L=(8.0,) * 3, dip_n=(0.6, 0.0, 0.8), quad=(32, 16, 32), tol=1e-13),
                dict(dim=3, n=(32, 32, 32), L=(8.0,) * 3, dip_n=(0.6, 0.0, 0.8), n_rad=32, n_pol=16, n_azi=32)),
    "3d_mixed": (dict(dim=3, n=(32, 32, 32), L=(8.0,) * 3, quad=(24, 12, 24), tol=1e-6, prec="mixed"),
                 dict(dim=3, n=(32, 32, 32), L=(8.0,) * 3, n_rad=24, n_pol=12, n_azi=24)),
    "2d_fp64": (dict(dim=2, n=(64, 64), L=(8.0, 8.0), dip_n=(0.6, 0.0, 0.8), quad=(32, 1, 64), tol=1e-13),
                dict(dim=2, n=(64, 64), L=(8.0, 8.0), dip_n=(0.6, 0.0, 0.8), n_rad=32, n_pol=1, n_azi=64)),
    "3d_aniso": (dict(dim=3, n=(32, 32, 32), L=(8.0, 8.0, 2.0), quad=(32, 16, 32), tol=1e-13, stretch=(1.0, 1.0, 4.0)),
                 dict(dim=3, n=(32, 32, 32), L=(8.0, 8.0, 2.0), n_rad=32, n_pol=16, n_azi=32, stretch=(1.0, 1.0, 4.0))),
    "3d_split": (dict(dim=3, n=(32, 32, 32), L=(8.0,) * 3, dip_n=(0.0, 0.6, 0.8), quad=(16, 16, 32), tol=1e-13,
                      split=True),
                 dict(dim=3, n=(32, 32, 32), L=(8.0,) * 3, dip_n=(0.0, 0.6, 0.8), n_rad=16, n_pol=16, n_azi=32)),
    # a small ball whose supports end on the last position of a tile: the axis-1 window is tight
    "3d_split_64": (dict(dim=3, n=(64, 64, 64), L=(8.0,) * 3, quad=(12, 12, 24), tol=1e-13, split=True, split_s=1.5),
                    dict(dim=3, n=(64, 64, 64), L=(8.0,) * 3, n_rad=12, n_pol=12, n_azi=24)),
    # grid sizes 3 * 2^a (radix 3 in the FFT passes): fine axes 192, 96, 48
    "3d_radix3": (dict(dim=3, n=(96, 48, 24), L=(12.0, 8.0, 6.0), dip_n=(0.6, 0.0, 0.8), quad=(24, 12, 24), tol=1e-13),
                  dict(dim=3, n=(96, 48, 24), L=(12.0, 8.0, 6.0), dip_n=(0.6, 0.0, 0.8), n_rad=24, n_pol=12, n_azi=24)),
    "2d_radix3": (dict(dim=2, n=(96, 192), L=(8.0, 16.0), dip_n=(0.7071067811865476, 0.0, 0.7071067811865476),
                       quad=(32, 1, 64), tol=1e-13),
                  dict(dim=2, n=(96, 192), L=(8.0, 16.0), dip_n=(0.7071067811865476, 0.0, 0.7071067811865476),
                       n_rad=32, n_pol=1, n_azi=64)),
    # the 2D split: I_2 weights times erfc(|k|/s) on the small polar ball
    "2d_split": (dict(dim=2, n=(128, 128), L=(16.0, 16.0), dip_n=(0.0, -0.896, 0.44404),
                      dip_m=(0.0, -0.52476, 0.85125), quad=(32, 1, 64), tol=1e-13, split=True),
                 dict(dim=2, n=(128, 128), L=(16.0, 16.0), dip_n=(0.0, -0.896, 0.44404),
                      dip_m=(0.0, -0.52476, 0.85125), n_rad=32, n_pol=1, n_azi=64)),
}


@pytest.fixture(scope="module")
def tables(driver, tmp_path_factory):
    got = {}
    for name, (kw, _) in CASES.items():
        t = run_tables(driver, tmp_path_factory.mktemp(name), **kw)
        assert int(t["status"][0]) == 0, t.get("message")
        got[name] = t
    return got


def geometry(t):
    dim, w, zalign, rows, wmax, split = (int(v) for v in t["dim_w_zalign_rows_wmax_split"])
    M = t["c"].size
    return dict(dim=dim, w=w, zalign=zalign, rows=bool(rows), wmax=wmax, split=bool(split), M=M,
                N=t["N"], nf=t["nf"], W=t["W"], tile=t["tile"], ntiles=t["ntiles"], ib=t["ib"], h=t["h"],
                kmax=t["cell_beta_kmax_mnom_splits"][2], split_s=t["cell_beta_kmax_mnom_splits"][4],
                index=t["index"].reshape(M, 3), k=t["k"].reshape(M, 3), l0=t["l0"].reshape(M, 3),
                wts=t["wts"].reshape(M, 3, wmax))


@pytest.mark.parametrize("name", list(CASES))
def test_nodes_and_coefficients_match_the_oracle_quadrature(tables, name):
    g = geometry(tables[name])
    prob = O.DDIProblem(**CASES[name][1], kmax=g["kmax"] if g["split"] else 0.0)
    if g["split"]:
        kq, c_or = O.split_long_range_nodes(prob, g["split_s"])
        quad = O.quadrature(prob)
    else:
        quad, c_or = O.ddi_nodes(prob)
        kq = quad.k
        assert abs(g["kmax"] - quad.kmax) <= 1e-14 * quad.kmax
    M = g["M"]
    assert M == kq.shape[0]
    key = {tuple(v): i for i, v in enumerate(quad.index.tolist())}
    rows = np.array([key[tuple(v)] for v in g["index"].tolist()])
    assert np.unique(rows).size == M
    d = g["dim"]
    k_lib = g["k"][:, :d]
    assert np.max(np.abs(k_lib - kq[rows])) <= 1e-13 * np.max(np.abs(kq))
    c = tables[name]["c"]
    assert np.max(np.abs(c - c_or[rows])) <= 1e-13 * np.max(np.abs(c_or))


@pytest.mark.parametrize("name", list(CASES))
def test_half_set_keeps_one_member_of_each_pair(tables, name):
    t, g = tables[name], geometry(tables[name])
    idx, k, c, hf = g["index"], g["k"], t["c"], t["half_factor"]
    nrad, npol, nazi = CASES[name][0]["quad"]
    if g["dim"] == 2:
        npol = 1
    pos = {tuple(v): i for i, v in enumerate(idx.tolist())}
    kscale = np.max(np.abs(k))
    pairs = 0
    for q in range(g["M"]):
        a, b, cc = idx[q]
        partner = (a, npol - 1 - b if g["dim"] == 3 else 0, (cc + nazi // 2) % nazi)
        p = pos.get(partner)
        if p is None:
            assert hf[q] == 1.0
            continue
        pairs += 1
        assert np.max(np.abs(k[p] + k[q])) <= 1e-15 * kscale
        assert abs(c[p] - c[q]) <= 1e-14 * np.max(np.abs(c))
        assert sorted((hf[q], hf[p])) == [0.0, 2.0]
    assert pairs > 0.9 * g["M"]
    # the sum of the factors counts every node once
    assert np.sum(hf) == g["M"]


@pytest.mark.parametrize("name", list(CASES))
def test_deconvolved_kernel_rows_reproduce_each_mode(tables, name):
    """deconv[m] * sum_i wts[i] exp(-2 pi i (l0 + i) m / n_f) = exp(-i t m) for t = k_a h_a and every
    mode m in [-N/2, N/2): the type-2 sum of one mode, as the NUFFT evaluates it."""
    t, g = tables[name], geometry(tables[name])
    off = 3 - g["dim"]
    tol = CASES[name][0]["tol"]
    worst = 0.0
    for a in range(off, 3):
        N, nf, W = int(g["N"][a]), int(g["nf"][a]), int(g["W"][a])
        assert W == g["w"]
        m = np.arange(N) - N // 2
        tq = g["k"][:, a - off] * g["h"][a]
        assert np.all(np.abs(tq) <= np.pi * (1 + 1e-14))
        wts = g["wts"][:, a, :]
        assert np.all(wts[:, W:] == 0.0)
        pos = g["l0"][:, a, None] + np.arange(W)[None, :]
        assert np.all((g["l0"][:, a] >= 0) & (g["l0"][:, a] < nf))
        ph = np.exp(-2j * np.pi * (pos[:, :, None] * m[None, None, :] % nf) / nf)
        approx = t[f"deconv{a}"][None, :] * np.einsum("qi,qim->qm", wts[:, :W], ph)
        exact = np.exp(-1j * tq[:, None] * m[None, :])
        worst = max(worst, float(np.max(np.abs(approx - exact))))
    # the extreme modes |m| = N/2 carry the largest 1/phihat: measured 4.5e-13 (3D) and 9.4e-13
    # (2D) at tol 1e-13 (w = 14), 2.7e-6 at tol 1e-6 (mixed, w = 7)
    assert worst <= 20 * tol, worst


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("which", [0, 1])
def test_schedules_cover_every_support_once(tables, name, which):
    t, g = tables[name], geometry(tables[name])
    pre = f"s{which}_"
    M, nf, tile, ntiles = g["M"], g["nf"], g["tile"], g["ntiles"]
    used = np.ones(M, bool) if which == 0 else t["half_factor"] > 0
    nslots, z0, nz, ny = (int(v) for v in t[pre + "nslots_z0_nz_ny"])
    lst = t[pre + "list"]
    # (tile, node) pairs from the supports
    want = []
    for q in np.nonzero(used)[0]:
        per_axis = []
        for a in range(3):
            cells = (g["l0"][q, a] + np.arange(g["W"][a])) % nf[a]
            per_axis.append(np.unique(cells // tile[a]))
        tid = (per_axis[0][:, None, None] * ntiles[1] + per_axis[1][None, :, None]) * ntiles[2] + per_axis[2][None, None, :]
        want.append(np.stack([tid.ravel(), np.full(tid.size, q)], 1))
    want = np.concatenate(want)
    # (tile, node) pairs from the work items; padding items (tile -1, no entries) only fill the
    # per-XCD regions to equal length
    items = t[pre + "items"].reshape(-1, 4)
    pad = items[:, 0] < 0
    assert np.all(items[pad, 2] == 0) and np.all(items[pad, 3] == -1)
    items = items[~pad]
    got = np.concatenate([np.stack([np.full(cnt, tl), lst[st:st + cnt]], 1) for tl, st, cnt, _ in items] + [np.zeros((0, 2), np.int64)])
    assert got.shape[0] == lst.size == want.shape[0]
    ordw = np.lexsort((want[:, 1], want[:, 0]))
    ordg = np.lexsort((got[:, 1], got[:, 0]))
    assert np.array_equal(want[ordw], got[ordg])
    # the items' ranges partition the list
    cover = np.zeros(lst.size, np.int64)
    for _, st, cnt, _ in items:
        cover[st:st + cnt] += 1
    assert np.all(cover == 1)
    # last-axis window: a multiple of the alignment holding every support; its tiles (and only
    # those) have items, empty ones included
    za = g["zalign"]
    assert z0 % za == 0 and nz % za == 0 and 0 < nz <= nf[2]
    zc = (g["l0"][used, 2, None] + np.arange(g["W"][2])[None, :]) % nf[2]
    assert np.all((zc - z0) % nf[2] < nz)
    tz_in = ((np.arange(ntiles[2]) * tile[2] - z0) % nf[2]) < nz
    tiles_with_items = np.unique(items[:, 0])
    all_in = [tid for tid in range(int(np.prod(ntiles))) if tz_in[tid % ntiles[2]]]
    assert np.array_equal(tiles_with_items, np.array(all_in))
    if which == 1 and g["dim"] == 3 and not g["split"] and nf[2] >= 8 * za:
        assert nz < nf[2]          # the kept member of each pair lies on one side
    # axis-1 window (3D): centred, whole tiles, every support inside
    if g["dim"] == 3:
        assert ny % 2 == 0 and (ny == nf[1] or (ny // 2) % tile[1] == 0)
        yc = (g["l0"][used, 1, None] + np.arange(g["W"][1])[None, :]) % nf[1]
        signed = np.where(yc < nf[1] // 2, yc, yc - nf[1])
        assert np.all((signed >= -(ny // 2)) & (signed < ny // 2))
    else:
        assert ny == nf[1]
    # chunks: split tiles have reduce items whose slots partition [0, nslots)
    chunk_max = 512 if g["rows"] else 256
    assert np.all(items[:, 2] <= chunk_max)
    red = t[pre + "reduces"].reshape(-1, 3)
    slots = items[items[:, 3] >= 0]
    assert slots.shape[0] == nslots == (int(red[:, 2].sum()) if red.size else 0)
    seen = np.zeros(nslots, np.int64)
    for tl, first, ns in red:
        mine = slots[slots[:, 0] == tl]
        assert np.array_equal(np.sort(mine[:, 3]), np.arange(first, first + ns))
        seen[first:first + ns] += 1
        lens = mine[np.argsort(mine[:, 3]), 2]
        assert np.all(lens[:-1] == lens[0]) and 0 < lens[-1] <= lens[0]
    assert np.all(seen == 1)
    if red.size:
        # a tile is either written whole by one item or summed from its slots
        assert not np.any(np.isin(items[items[:, 3] < 0, 0], red[:, 0]))
    # per node, the list positions of its entries in increasing order
    gptr, gpos = t[pre + "gptr"], t[pre + "gpos"]
    assert gptr[0] == 0 and gptr[-1] == lst.size
    for q in range(0, M, max(1, M // 500)):
        assert np.array_equal(gpos[gptr[q]:gptr[q + 1]], np.nonzero(lst == q)[0])
    # packed weight-row offsets: the tile origin minus the support origin, per axis
    ent = t[pre + "ent"]
    if g["rows"]:
        assert ent.size == 2 * (lst.size + K_ENT_PAD)
        assert np.all(ent[2 * lst.size:] == 0)
        node, packed = ent[0:2 * lst.size:2], ent[1:2 * lst.size:2]
        assert np.array_equal(node, lst)
        tile_of = np.empty(lst.size, np.int64)
        for tl, st, cnt, _ in items:
            tile_of[st:st + cnt] = tl
        org = np.stack([tile_of // (ntiles[1] * ntiles[2]) * tile[0], (tile_of // ntiles[2]) % ntiles[1] * tile[1],
                        tile_of % ntiles[2] * tile[2]], 1)
        for a in range(3):
            d = ((packed >> (8 * a)) & 255) - K_OFF_BIAS
            assert np.all((d >= -(tile[a] - 1)) & (d <= g["W"][a] - 1))
            assert np.all((g["l0"][node, a] + d - org[:, a]) % nf[a] == 0)
    else:
        assert ent.size == 0
    # interpolation: LDS groups and direct nodes cover the selected nodes once; a group's
    # supports start in its block
    ii = t[pre + "interp_items"].reshape(-1, 5)
    cov = np.zeros(M, np.int64)
    for st, cnt, ox, oy, oz in ii:
        cov[st:st + cnt] += 1
        blk = g["l0"][st:st + cnt] // g["ib"] * g["ib"]
        assert np.all(blk == np.array([ox, oy, oz]))
    np.add.at(cov, t[pre + "interp_direct"], 1)
    assert np.array_equal(cov, used.astype(np.int64))


def test_twiddle_tables_are_the_roots_of_unity(tables):
    """twiddle_table(n)[k] = exp(-2 pi i k / n) within one ulp (reference: 40-digit mpmath); the
    exact zeros come out of the long-double angle within 2e-19."""
    mp = pytest.importorskip("mpmath")
    mp.mp.dps = 40
    t = tables["3d_fp64"]
    for n in (4, 64, 256, 1024, 12, 96, 192, 768):
        tw = t[f"twiddle{n}"]
        assert tw.size == 2 * n
        ang = [2 * mp.pi * k / n for k in range(n)]
        re = np.array([float(mp.cos(x)) for x in ang])
        im = np.array([float(-mp.sin(x)) for x in ang])
        ulp = lambda v: np.maximum(np.spacing(np.abs(v)), 2.5e-19)
        assert np.all(np.abs(tw[0::2] - re) <= ulp(re))
        assert np.all(np.abs(tw[1::2] - im) <= ulp(im))


def test_rejected_parameters_report_an_error(driver, tmp_path):
    t = run_tables(driver, tmp_path, dim=3, n=(40, 32, 32), L=(8.0,) * 3)
    assert int(t["status"][0]) != 0
    assert "power" in t["message"]
    # 3 * 2^a is taken, but a 2D first axis below 96 points does not fill whole 64-point tiles
    t = run_tables(driver, tmp_path, dim=2, n=(48, 64), L=(8.0, 8.0))
    assert int(t["status"][0]) != 0 and "tile" in t["message"]


def test_in_register_dfts_match_the_direct_sum(tmp_path):
    """The in-register DFTs of the FFT passes (csrc/fft_regs.h), every radix the plans use
    (2, 4, 8, 16 and the radix-3 forms 12 and 24), both signs, against the direct sum in long
    double (tests/host/fft_regs_check.cpp, built with g++)."""
    gxx = shutil.which("g++")
    if gxx is None or not os.path.isdir(ROCM_INC):
        pytest.skip("g++ or the ROCm headers are not available")
    exe = str(tmp_path / "fft_regs_check")
    src = os.path.join(ROOT, "tests", "host", "fft_regs_check.cpp")
    r = subprocess.run([gxx, "-std=c++17", "-O2", "-D__HIP_PLATFORM_AMD__", "-I" + ROCM_INC, src, "-o", exe],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
