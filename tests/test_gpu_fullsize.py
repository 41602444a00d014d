"""GPU parity at the full benchmark sizes, in the launch configuration the
benchmark times (same padded sizes, same kernel instances).

* 1024 x 1024 x 1 vortex film (2 nm, the throughput workload): B_demag,
  B_eff and the torque against the FP64 oracle over every cell, and a short
  adaptive Dormand-Prince trajectory against the oracle's (m within 1e-3).
* 256 x 256 x 64 Voronoi grains (3 nm, 256 regions): the oracle cannot
  convolve this grid in a test's time, so the demag path is checked on
  sparse sources (a handful of magnetised cells, vacuum elsewhere) where the
  oracle's field at any cell is a short sum over the sources; the local terms
  (exchange over the 256-region pair table, anisotropy, Zeeman) are checked
  over every cell with the magnetostatic term off; and a uniformly magnetised
  box must reproduce the exact box-averaged demagnetising factors.
* 512 x 256 x 2 film (the one-pass thin-grid convolution): B_demag, B_eff and
  the torque against the oracle over every cell.
"""
import numpy as np
import pytest

from oracle import demag as odemag
from oracle import integrate as ointegrate
from oracle.constants import MU0
from paper_1406_7635_amd import synth
from tests.aharoni import prism_factors
from tests.gpu_helpers import log, make_ctx, make_pair, rel_inf, to_np

pytestmark = pytest.mark.gpu


def test_film_1024_fields_full(gpu):
    case = synth.vortex_film(seed=2, n=1024)
    log("film 1024: full-grid B_eff / torque parity")
    ctx, prob, m = make_pair(case)
    b, bd = ctx.beff(m, want_demag=True)
    tau = ctx.torque(m)
    m64 = case["m0"].astype(np.float64)
    prob.workers = -1
    t = prob.terms(m64)
    assert rel_inf(to_np(bd), t["demag"]) < 1e-5
    ref_b = sum(t[k] for k in ("demag", "exch", "anis1", "anis2", "zeeman")) * prob.magnetic
    assert rel_inf(to_np(b), ref_b) < 1e-5
    assert rel_inf(to_np(tau), prob.torque(m64)) < 1e-5
    ctx.close()


def test_film_1024_rk45_trajectory(gpu):
    """Adaptive RK45 (MaxErr 1e-5) from the vortex to t = 2e-13 s on both sides."""
    case = synth.vortex_film(seed=2, n=1024)
    t_end = 2e-13
    log("film 1024: RK45 to", t_end)
    ctx, prob, m = make_pair(case)
    prob.workers = -1
    t, dt, st = ctx.run(m, t_end, dt=1e-14, max_attempts=1000, opts=None)
    assert t == pytest.approx(t_end, rel=1e-12)
    it = ointegrate.Integrator(prob.torque, case["m0"], "rk45", dt=1e-14, max_err=1e-5)
    it.run(t_end)
    got = to_np(m)
    assert np.max(np.abs(got - it.m)) < 1e-3
    assert np.allclose(np.sum(got * got, axis=0), 1.0, atol=1e-5)
    ctx.close()


def _sparse_grains(nsrc=6, seed=44):
    """The 256 x 256 x 64 grain geometry with vacuum everywhere except nsrc
    magnetised cells (region 1, Msat 8e5) at random positions with random m."""
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


def test_grains_demag_sparse_sources_full_size(gpu):
    """B_demag(r) = -mu0 sum_j N(r - r_j) M_j over the sources, at sampled
    cells (near the sources, corners, random), on the 512 x 512 x 128 padded grid."""
    case, src = _sparse_grains()
    nx, ny, nz = case["grid"]
    cell = case["cell"]
    log("grains 256x256x64: sparse-source demag")
    ctx, m = make_ctx(case)
    _, bd = ctx.beff(m, want_demag=True)
    bd = to_np(bd)
    rng = np.random.Generator(np.random.PCG64(7))
    tgt = [tuple(s) for s in src]
    for z, y, x in src:  # neighbours of every source
        for d in ((0, 0, 1), (0, 1, 0), (1, 0, 0), (0, 0, -1), (0, -3, 0), (2, 5, -7)):
            tgt.append((min(max(z + d[0], 0), nz - 1), min(max(y + d[1], 0), ny - 1),
                        min(max(x + d[2], 0), nx - 1)))
    tgt += [(0, 0, nx - 1), (nz - 1, 0, 0), (0, ny - 1, 0), (nz // 2, ny // 2, nx // 2)]
    tgt += [tuple(v) for v in np.stack([rng.integers(0, nz, 100), rng.integers(0, ny, 100),
                                        rng.integers(0, nx, 100)], axis=1)]
    tgt = np.array(tgt)
    M = np.array([8e5 * case["m0"][:, z, y, x].astype(np.float64) for z, y, x in src])  # [nsrc, 3]
    ref = np.zeros((len(tgt), 3))
    for j, (z, y, x) in enumerate(src):
        X = (tgt[:, 2] - x) * cell[0]
        Y = (tgt[:, 1] - y) * cell[1]
        Z = (tgt[:, 0] - z) * cell[2]
        N = odemag.tensor_at(X, Y, Z, cell)
        ref[:, 0] += N["xx"] * M[j, 0] + N["xy"] * M[j, 1] + N["xz"] * M[j, 2]
        ref[:, 1] += N["xy"] * M[j, 0] + N["yy"] * M[j, 1] + N["yz"] * M[j, 2]
        ref[:, 2] += N["xz"] * M[j, 0] + N["yz"] * M[j, 1] + N["zz"] * M[j, 2]
    ref *= -MU0
    got = np.stack([bd[:, z, y, x] for z, y, x in tgt])
    assert rel_inf(got, ref) < 1e-5
    ctx.close()


def test_grains_local_terms_full_size(gpu):
    """Exchange over the 256-region pair table (S = 0.9 between grains),
    anisotropy with per-grain axes and Zeeman: every cell, demag off."""
    case = synth.grains(seed=3)
    rng = np.random.Generator(np.random.PCG64(33))
    case["params"]["bext"][:] = rng.uniform(-0.05, 0.05, case["params"]["bext"].shape)
    log("grains 256x256x64: local terms")
    ctx, prob, m = make_pair(case, demag=False)
    b = ctx.beff(m)
    m64 = case["m0"].astype(np.float64)
    assert rel_inf(to_np(b), prob.beff(m64)) < 1e-5
    ctx.close()


def test_grains_uniform_box_factors(gpu):
    """A uniformly magnetised 256 x 256 x 64 box of 3 nm cells: the cell average
    of B_demag is -mu0 Msat N_box m with Aharoni's prism factors (closed form)."""
    grid, cell = (256, 256, 64), (3e-9, 3e-9, 3e-9)
    p = synth.material(8e5, 1.5e-11, alpha=0.01)
    d = np.array([0.36, -0.48, 0.8])
    case = {"grid": grid, "cell": cell, "region": np.zeros(grid[::-1], dtype=np.uint8), "params": p,
            "m0": synth.uniform_m(grid, d)}
    log("grains 256x256x64: uniform box")
    ctx, m = make_ctx(case)
    _, bd = ctx.beff(m, want_demag=True)
    mean = to_np(bd).reshape(3, -1).mean(axis=1)
    nxx, nyy, nzz = prism_factors(grid[0] * cell[0], grid[1] * cell[1], grid[2] * cell[2])
    mv = to_np(m)[:, 0, 0, 0]
    ref = -MU0 * 8e5 * np.array([nxx, nyy, nzz]) * mv
    assert np.max(np.abs(mean - ref)) < 1e-5 * MU0 * 8e5
    ctx.close()


def test_thin_film_512x256x2_fields_full(gpu):
    """Two-layer film at an ensemble member's largest size and beyond: the
    one-pass y/z convolution (kernel in z space) against the FP64 oracle over
    every cell."""
    case = synth.random_problem((512, 256, 2), (3e-9, 3e-9, 2e-9), seed=8, nregions=4, vacuum=True)
    log("thin film 512x256x2: full-grid B_eff / torque parity")
    ctx, prob, m = make_pair(case)
    prob.workers = -1
    b, bd = ctx.beff(m, want_demag=True)
    m64 = case["m0"].astype(np.float64)
    t = prob.terms(m64)
    assert rel_inf(to_np(bd), t["demag"]) < 1e-5
    ref_b = sum(t[k] for k in ("demag", "exch", "anis1", "anis2", "zeeman")) * prob.magnetic
    assert rel_inf(to_np(b), ref_b) < 1e-5
    assert rel_inf(to_np(ctx.torque(m)), prob.torque(m64)) < 1e-5
    ctx.close()
