"""Periodic boundary conditions on the GPU against the oracle (FP32 GPU vs
FP64 CPU), paper section "Magnetostatic field", paragraph "Periodic boundary
conditions".

The images enter the FP64 kernel only; the field passes are those of the open
grid.  Checked: the image sums of the tensor (the GPU folds the window octant
with the tensor's parities, the oracle evaluates every signed displacement),
B_eff and the torque on 2D, thin-3D and 3D grids with images along one, two or
three axes, the wrapped exchange coefficients bit for bit, the paper's film
and rod tables through the library, a short Dormand-Prince run, and the
refusals (negative counts, oversized windows, the surrogate).
"""
import numpy as np
import pytest

from oracle import demag as odemag
from oracle import fields as ofields
from oracle import integrate as ointegrate
from oracle.constants import MU0
from paper_1406_7635_amd import mm, synth
from tests.gpu_helpers import log, rel_inf, to_np

pytestmark = pytest.mark.gpu

CASES = [
    ((16, 12, 1), (2e-9, 3e-9, 2.5e-9), (2, 3, 0)),     # film, images in-plane
    ((24, 20, 1), (3e-9, 3e-9, 2e-9), (1, 0, 4)),       # film, stacked images along z
    ((33, 17, 2), (2e-9, 2e-9, 3e-9), (3, 0, 2)),       # thin 3D (pz = 4), ragged
    ((20, 16, 3), (2e-9, 3e-9, 2e-9), (1, 1, 0)),       # thin 3D (pz = 8)
    ((12, 10, 6), (3e-9, 2e-9, 1.5e-9), (0, 2, 1)),     # 3D
    ((8, 8, 8), (2e-9, 2e-9, 2e-9), (2, 2, 2)),         # every axis periodic
    ((100, 70, 1), (3e-9, 3e-9, 3e-9), (4, 4, 0)),      # several tiles
    # periodic power-of-two axes transformed at their own length (no padding)
    ((128, 64, 1), (2e-9, 2e-9, 2e-9), (2, 2, 0)),      # x and y unpadded
    ((64, 256, 1), (3e-9, 2e-9, 2e-9), (0, 3, 0)),      # y unpadded, x open
    ((256, 100, 1), (2e-9, 3e-9, 2e-9), (1, 0, 0)),     # x unpadded, y open
    ((32, 20, 5), (2e-9, 2e-9, 2e-9), (2, 0, 1)),       # 3D, x unpadded
]


def pair(case, pbc, demag=True):
    import torch

    ctx = mm.Context(case["grid"], case["cell"], case["region"], case["params"], demag=demag, pbc=pbc)
    prob = ofields.Problem(case["grid"], case["cell"], case["region"], case["params"], demag=demag, pbc=pbc)
    m = torch.from_numpy(np.ascontiguousarray(case["m0"])).to("cuda:0")
    return ctx, prob, m


def oracle_image_sums(grid, cell, pbc):
    """[6, nz, ny, nx]: sum of N over the window displacements congruent to each
    box displacement (i, j, k) >= 0 (periodic axes) or equal to it."""
    w = odemag.tensor_window(grid, cell, pbc)
    rx, ry, rz = odemag.window_radius(grid, pbc)
    nx, ny, nz = grid
    out = np.zeros((6, nz, ny, nx))
    dk, dj, di = np.meshgrid(np.arange(-rz, rz + 1), np.arange(-ry, ry + 1), np.arange(-rx, rx + 1), indexing="ij")
    for c in range(6):
        keep = np.ones(dk.shape, bool)
        idx = []
        for d, n, p in ((dk, nz, pbc[2]), (dj, ny, pbc[1]), (di, nx, pbc[0])):
            if p > 0:
                idx.append(d % n)
            else:
                keep &= d >= 0
                idx.append(d)
        np.add.at(out[c], tuple(a[keep] for a in idx), w[c][keep])
    return out


@pytest.mark.parametrize("grid,cell,pbc", CASES[:5], ids=[str(c[0]) + str(c[2]) for c in CASES[:5]])
def test_tensor_image_sums(gpu, grid, cell, pbc):
    case = synth.random_problem(grid, cell, seed=3)
    ctx, _, _ = pair(case, pbc, demag=False)
    got = to_np(ctx.tensor_dump())
    ref = oracle_image_sums(grid, cell, pbc)
    log("tensor image sums", grid, pbc)
    for c in range(6):
        scale = np.max(np.abs(ref[c])) + 1e-300
        assert np.max(np.abs(got[c] - ref[c])) <= 1e-10 * scale + 1e-12 * np.max(np.abs(ref)), c
    ctx.close()


@pytest.mark.parametrize("grid,cell,pbc", CASES, ids=[str(c[0]) + str(c[2]) for c in CASES])
def test_beff_and_torque_parity(gpu, grid, cell, pbc):
    case = synth.random_problem(grid, cell, seed=sum(grid) + sum(pbc), nregions=4, vacuum=True)
    log("pbc beff parity", grid, pbc)
    ctx, prob, m = pair(case, pbc)
    b, bd = ctx.beff(m, want_demag=True)
    m64 = case["m0"].astype(np.float64)
    assert rel_inf(to_np(bd), prob.terms(m64)["demag"]) < 1e-5
    assert rel_inf(to_np(b), prob.beff(m64)) < 1e-5
    assert rel_inf(to_np(ctx.torque(m)), prob.torque(m64)) < 1e-5
    e = ctx.energy(m)
    ref = prob.energy(m64)
    for k in ("demag", "exch", "total"):
        assert e[k] == pytest.approx(ref[k], rel=2e-5, abs=1e-6 * abs(ref["total"]) + 1e-30), k
    ctx.close()


def test_exchange_coefficients_wrap_bit_exact(gpu):
    case = synth.random_problem((9, 7, 4), (2e-9, 3e-9, 4e-9), seed=12, nregions=6, vacuum=True)
    ctx, _, _ = pair(case, (1, 0, 2), demag=False)
    got = to_np(ctx.exchange_dump()).astype(np.float32)
    reg = case["region"]
    cell = case["cell"]
    periodic = {2: True, 1: False, 0: True}  # array axis -> periodic (x: 2, y: 1, z: 0)
    for f, (axis, sgn) in enumerate([(2, -1), (2, 1), (1, -1), (1, 1), (0, -1), (0, 1)]):
        d = cell[2 - axis]
        idx = np.indices(reg.shape)
        nb = idx.copy()
        nb[axis] += sgn
        n = reg.shape[axis]
        if periodic[axis]:
            nb[axis] %= n
            ok = np.ones(reg.shape, bool)
        else:
            ok = (nb[axis] >= 0) & (nb[axis] < n)
        rn = reg[tuple(np.clip(nb[a], 0, reg.shape[a] - 1) for a in range(3))]
        c = ofields.exchange_coefficient(case["params"], reg, rn).astype(np.float32)
        exp = np.zeros(reg.shape, dtype=np.float32)
        exp[ok] = (c * np.float32(1.0 / (d * d)))[ok]
        np.testing.assert_array_equal(got[f], exp)
    ctx.close()


def _uniform_average(grid, pbc, comp):
    import torch

    params = synth.material(1.0 / MU0, 0.0)
    nx, ny, nz = grid
    ctx = mm.Context(grid, (1e-9, 1e-9, 1e-9), np.zeros((nz, ny, nx), np.uint8), params, pbc=pbc)
    m = torch.zeros((3, nz, ny, nx), dtype=torch.float32, device="cuda:0")
    m[comp] = 1.0
    _, bd = ctx.beff(m, want_demag=True)
    v = float(bd[comp].double().mean())
    ctx.close()
    return v


@pytest.mark.parametrize("P", [1, 4, 16, 64])
def test_paper_pbc_tables(gpu, P):
    """tabPBC1 (film 2 x 2 x 1, images along x and y) and tabPBC2 (rod 2 x 2 x 1,
    images along z) through the library, against the oracle's exact sums
    (FP32 rounding) and the paper's printed values (its kernel's accuracy)."""
    import os

    golden = os.path.join(os.path.dirname(__file__), "golden")
    for name, pbc, comp in (("tab_pbc_film.txt", (P, P, 0), 2), ("tab_pbc_rod.txt", (0, 0, P), 0)):
        rows = {int(r.split()[0]): float(r.split()[1]) for r in open(os.path.join(golden, name))
                if r.strip() and not r.startswith("#")}
        got = _uniform_average((2, 2, 1), pbc, comp)
        M = np.zeros((3, 1, 2, 2))
        M[comp] = 1.0 / MU0
        ref = odemag.demag_field_fft_pbc(M, odemag.tensor_window((2, 2, 1), (1e-9,) * 3, pbc), pbc)[comp].mean()
        log("table", name, P, got, ref, rows[P])
        assert abs(got - ref) < 2e-6
        assert abs(got - rows[P]) < 1.5e-3


def test_adaptive_run_matches_oracle(gpu):
    case = synth.vortex_film(seed=2, n=32)
    case["params"]["alpha"][0] = 0.1
    pbc = (2, 2, 0)
    ctx, prob, m = pair(case, pbc)
    t_end = 5e-12
    t, dt, st = ctx.run(m, t_end, dt=1e-14, solver=45, opts=mm.solver_opts(max_err=1e-5))
    assert t == pytest.approx(t_end, rel=1e-12)
    it = ointegrate.Integrator(prob.torque, case["m0"], "rk45", dt=1e-14, max_err=1e-5)
    it.run(t_end)
    err = np.max(np.abs(to_np(m) - it.m))
    log("pbc DP45 steps", st["steps"], "oracle steps", it.nsteps, "max |dm|", err)
    assert err < 1e-3
    ctx.close()


def test_unpadded_periodic_lengths_and_run(gpu):
    """A periodic axis whose length is a power of two is transformed at that
    length (the paper's remark that periodic directions need no padding):
    the padded lengths the library reports, and a Dormand-Prince run of a
    64 x 64 film periodic in x and y against the oracle."""
    for grid, pbc, want in (((128, 64, 1), (2, 2, 0), (128, 64, 1)), ((64, 256, 1), (0, 3, 0), (128, 256, 1)),
                            ((256, 100, 1), (1, 0, 0), (256, 256, 1)), ((32, 20, 5), (2, 0, 1), (32, 64, 16)),
                            ((48, 64, 1), (1, 1, 0), (128, 64, 1))):
        case = synth.random_problem(grid, (2e-9, 2e-9, 2e-9), seed=4)
        ctx = mm.Context(case["grid"], case["cell"], case["region"], case["params"], pbc=pbc, demag=False)
        info = ctx.info()
        assert (info["px"], info["py"], info["pz"]) == want, (grid, pbc)
        ctx.close()
    case = synth.vortex_film(seed=2, n=64)
    case["params"]["alpha"][0] = 0.1
    pbc = (1, 1, 0)
    ctx, prob, m = pair(case, pbc)
    t_end = 5e-12
    t, dt, st = ctx.run(m, t_end, dt=1e-14, solver=45, opts=mm.solver_opts(max_err=1e-5))
    assert t == pytest.approx(t_end, rel=1e-12)
    it = ointegrate.Integrator(prob.torque, case["m0"], "rk45", dt=1e-14, max_err=1e-5)
    it.run(t_end)
    err = np.max(np.abs(to_np(m) - it.m))
    log("unpadded pbc DP45 steps", st["steps"], "oracle steps", it.nsteps, "max |dm|", err)
    assert err < 1e-3
    ctx.close()


FUSED_CASES = [
    ((64, 32, 1), (1, 1, 0), False),    # x and y unpadded
    ((128, 40, 1), (2, 0, 0), False),   # x unpadded, y open, ragged
    ((32, 20, 5), (1, 0, 1), False),    # 3D, x unpadded
    ((64, 24, 1), (1, 0, 0), True),     # x unpadded, with DMI
    ((128, 40, 1), (0, 0, 0), False),   # open x (padded fused pass): the same bars
]


@pytest.mark.parametrize("grid,pbc,dmi", FUSED_CASES, ids=[str(c[0]) + str(c[1]) + str(c[2]) for c in FUSED_CASES])
def test_fused_stage_pass_unpadded_x(gpu, grid, pbc, dmi):
    """Dormand-Prince attempts on grids whose x axis is periodic and unpadded,
    where the x-inverse of each inner stage and the x-forward of the next run
    as one pass that hands the torque over in place of the cell's own
    x-inverse result: three accepted attempts at a fixed step against the
    oracle's embedded steps (m within 2e-6, error estimate within 5 %)."""
    case = synth.random_problem(grid, (2e-9, 2e-9, 2e-9), seed=sum(grid) + 11, nregions=4)
    if dmi:
        rng = np.random.Generator(np.random.PCG64(5))
        case["params"]["dind"] = np.zeros(256)
        case["params"]["dind"][:4] = rng.uniform(-3e-3, 3e-3, 4)
    ctx, prob, m = pair(case, pbc)
    info = ctx.info()
    assert info["px"] == (grid[0] if pbc[0] else 2 * grid[0])
    f = prob.torque
    m_ref = case["m0"].astype(np.float64)
    k1 = f(m_ref)
    dt = 2e-14
    opts = mm.solver_opts(max_err=1.0)  # every attempt accepted, dt grows at most 2x
    t = 0.0
    for _ in range(3):
        acc, t1, dtn, err = ctx.rk45_step(m, t, dt, opts)
        assert acc
        ms, k1, eps = ointegrate.embedded_step(f, m_ref, k1, dt, ointegrate.DP45)
        m_ref = ointegrate.normalize(ms)  # k1 of the next attempt: the last stage's (first same as last)
        d = float(np.max(np.abs(to_np(m) - m_ref)))
        log("fused unpadded-x DP45", grid, pbc, "dmi" if dmi else "", "|dm| %.2e err %.3e / %.3e" % (d, err, eps))
        assert d < 2e-6
        # the estimate is a small difference of stage torques: FP32 leaves it a
        # few per cent off the FP64 value (it only scales the next step)
        assert abs(err - eps) <= 5e-2 * eps
        t = t1
    ctx.close()


def test_bad_images_and_surrogate_rejected(gpu):
    """Negative image counts and oversized windows are refused; the surrogate
    (trained for open boundaries) refuses a periodic grid."""
    case = synth.random_problem((32, 32, 1), (2e-9, 2e-9, 2e-9), seed=1)
    with pytest.raises(mm.MMError):
        ctx = mm.Context(case["grid"], case["cell"], case["region"], case["params"], pbc=(-1, 0, 0))
    with pytest.raises(mm.MMError):
        mm.Context(case["grid"], case["cell"], case["region"], case["params"], pbc=(4096, 4096, 0))
    ctx = mm.Context(case["grid"], case["cell"], case["region"], case["params"], pbc=(1, 1, 0))
    sur = mm.Surrogate(32, 32, synth.sno_random_weights(seed=1), 1.0)
    with pytest.raises(mm.MMError):
        ctx.set_surrogate(sur, 1e-4)
    sur.close()
    ctx.close()
