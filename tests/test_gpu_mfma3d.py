"""Matrix-core DFT stages of the 3D column passes (y forward, z convolution
with K^, y inverse; BF16 / FP16 split precision) against the FP64 oracle.

* Reduced grids that run the same kernel instances as the 256 x 256 x 64
  grains (padded y 512, z 128: the x axis is short, the x passes stay FP32),
  and grids with the other padded lengths (64 ... 1024), with vacuum, four
  regions and non-cubic cells: B_demag over every cell within 1e-4 of the
  oracle (the FP32 path within 1e-5 beside it).
* The full 256 x 256 x 64 grain geometry: sparse sources (the oracle's field
  is a short sum at any cell) and a uniformly magnetised box (Aharoni's
  factors), within 1e-4.
* A short Dormand-Prince run on the matrix-core path follows the FP32 one.
"""
import numpy as np
import pytest

from oracle import demag as odemag
from oracle import fields as ofields
from oracle.constants import MU0
from paper_1406_7635_amd import synth
from tests.aharoni import prism_factors
from tests.gpu_helpers import log, make_ctx, make_pair, rel_inf, to_np

pytestmark = pytest.mark.gpu

PRECS = ("bf16", "fp16")
GRIDS = [
    ((8, 131, 33), (3e-9, 3e-9, 3e-9)),     # py 512, pz 128: the grain instances
    ((12, 70, 40), (2e-9, 3e-9, 2.5e-9)),   # py 256, pz 128
    ((10, 300, 17), (3e-9, 2e-9, 3e-9)),    # py 1024, pz 64
    ((6, 20, 20), (2e-9, 2e-9, 4e-9)),      # py 64, pz 64
    ((5, 1, 60), (2e-9, 2e-9, 2e-9)),       # no y pass, pz 128
]


@pytest.mark.parametrize("grid,cell", GRIDS, ids=[str(g[0]) for g in GRIDS])
def test_demag_error_reduced_grids(gpu, grid, cell):
    case = synth.random_problem(grid, cell, seed=sum(grid) + 5, nregions=4, vacuum=True)
    log("mfma3d demag", grid)
    ctx, prob, m = make_pair(case)
    prob.workers = -1
    ref = prob.demag_field(case["m0"].astype(np.float64))
    _, bd32 = ctx.beff(m, want_demag=True)
    errs = {"fp32": rel_inf(to_np(bd32), ref)}
    for prec in PRECS:
        ctx.set_conv_precision(prec)
        _, bd = ctx.beff(m, want_demag=True)
        errs[prec] = rel_inf(to_np(bd), ref)
    ctx.set_conv_precision("fp32")
    log("  rel errors", {k: "%.2e" % v for k, v in errs.items()})
    assert errs["fp32"] < 1e-5
    for prec in PRECS:
        assert errs[prec] < 1e-4, prec
    ctx.close()


def _sparse_grains(nsrc=6, seed=44):
    grid, cell = (256, 256, 64), (3e-9, 3e-9, 3e-9)
    nx, ny, nz = grid
    rng = np.random.Generator(np.random.PCG64(seed))
    region = np.zeros((nz, ny, nx), dtype=np.uint8)
    src = np.stack([rng.integers(0, nz, nsrc), rng.integers(0, ny, nsrc), rng.integers(0, nx, nsrc)], axis=1)
    src[0] = (0, 0, 0)
    src[1] = (nz - 1, ny - 1, nx - 1)
    for z, y, x in src:
        region[z, y, x] = 1
    p = synth.material(8e5, 1.5e-11, alpha=0.01, region=1)
    return {"grid": grid, "cell": cell, "region": region, "params": p,
            "m0": synth.random_sphere(grid, seed + 1)}, src


@pytest.mark.parametrize("prec", ("fp32",) + PRECS)
def test_grains_sparse_sources_full_size(gpu, prec):
    case, src = _sparse_grains()
    nx, ny, nz = case["grid"]
    cell = case["cell"]
    log("mfma3d grains sparse sources", prec)
    ctx, m = make_ctx(case)
    ctx.set_conv_precision(prec)
    _, bd = ctx.beff(m, want_demag=True)
    bd = to_np(bd)
    rng = np.random.Generator(np.random.PCG64(7))
    tgt = [tuple(s) for s in src]
    for z, y, x in src:
        for d in ((0, 0, 1), (0, 1, 0), (1, 0, 0), (0, -3, 0), (2, 5, -7)):
            tgt.append((min(max(z + d[0], 0), nz - 1), min(max(y + d[1], 0), ny - 1),
                        min(max(x + d[2], 0), nx - 1)))
    tgt += [tuple(v) for v in np.stack([rng.integers(0, nz, 80), rng.integers(0, ny, 80),
                                        rng.integers(0, nx, 80)], axis=1)]
    tgt = np.array(tgt)
    M = np.array([8e5 * case["m0"][:, z, y, x].astype(np.float64) for z, y, x in src])
    ref = np.zeros((len(tgt), 3))
    for j, (z, y, x) in enumerate(src):
        N = odemag.tensor_at((tgt[:, 2] - x) * cell[0], (tgt[:, 1] - y) * cell[1], (tgt[:, 0] - z) * cell[2], cell)
        ref[:, 0] += N["xx"] * M[j, 0] + N["xy"] * M[j, 1] + N["xz"] * M[j, 2]
        ref[:, 1] += N["xy"] * M[j, 0] + N["yy"] * M[j, 1] + N["yz"] * M[j, 2]
        ref[:, 2] += N["xz"] * M[j, 0] + N["yz"] * M[j, 1] + N["zz"] * M[j, 2]
    ref *= -MU0
    got = np.stack([bd[:, z, y, x] for z, y, x in tgt])
    err = rel_inf(got, ref)
    log("  rel error %.2e" % err)
    assert err < (1e-5 if prec == "fp32" else 1e-4)
    ctx.close()


@pytest.mark.parametrize("prec", ("fp32",) + PRECS)
def test_grains_uniform_box_full_size(gpu, prec):
    grid, cell = (256, 256, 64), (3e-9, 3e-9, 3e-9)
    p = synth.material(8e5, 1.5e-11, alpha=0.01)
    d = np.array([0.36, -0.48, 0.8])
    case = {"grid": grid, "cell": cell, "region": np.zeros(grid[::-1], dtype=np.uint8), "params": p,
            "m0": synth.uniform_m(grid, d)}
    log("mfma3d grains uniform box", prec)
    ctx, m = make_ctx(case)
    ctx.set_conv_precision(prec)
    _, bd = ctx.beff(m, want_demag=True)
    mean = to_np(bd).reshape(3, -1).mean(axis=1)
    nxx, nyy, nzz = prism_factors(grid[0] * cell[0], grid[1] * cell[1], grid[2] * cell[2])
    mv = to_np(m)[:, 0, 0, 0]
    ref = -MU0 * 8e5 * np.array([nxx, nyy, nzz]) * mv
    err = np.max(np.abs(mean - ref)) / (MU0 * 8e5)
    log("  box factor error %.2e" % err)
    assert err < (1e-5 if prec == "fp32" else 1e-4)
    ctx.close()


def test_dp45_run_follows_fp32(gpu):
    """Dormand-Prince (MaxErr 1e-5) to 0.2 ps on a 3D grid, matrix-core BF16
    path against the FP32 path from the same state (m within 1e-4)."""
    import torch

    case = synth.random_problem((10, 70, 40), (3e-9, 3e-9, 3e-9), seed=12, nregions=3)
    log("mfma3d DP45 run")
    ms = []
    for prec in ("fp32", "bf16"):
        ctx, m = make_ctx(case)
        ctx.set_conv_precision(prec)
        t, dt, st = ctx.run(m, 2e-13, dt=1e-14, max_attempts=1000, opts=None)
        assert t == pytest.approx(2e-13, rel=1e-12)
        ms.append(to_np(m))
        ctx.close()
    d = float(np.max(np.abs(ms[0] - ms[1])))
    log("  |m_bf16 - m_fp32| %.2e" % d)
    assert d < 1e-4
