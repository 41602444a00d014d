"""Induced DMI on the GPU against the FP64 oracle (section
"Dzyaloshinskii-Moriya interaction"): B_eff, torque and energies with the
boundary rule at open edges, at vacuum cells and at uncoupled region
interfaces, on 2D and 3D grids (the DMI x passes) and without demag (the
local pass), with periodic axes, the periodic cycloid's closed form through
the library, and a short Dormand-Prince run."""
import math

import numpy as np
import pytest

from oracle import fields as ofields
from oracle import integrate as ointegrate
from paper_1406_7635_amd import mm, synth
from tests.gpu_helpers import log, rel_inf, to_np

pytestmark = pytest.mark.gpu


def pair(case, pbc=(0, 0, 0), demag=True):
    import torch

    ctx = mm.Context(case["grid"], case["cell"], case["region"], case["params"], demag=demag, pbc=pbc)
    prob = ofields.Problem(case["grid"], case["cell"], case["region"], case["params"], demag=demag, pbc=pbc)
    return ctx, prob, torch.from_numpy(np.ascontiguousarray(case["m0"])).to("cuda:0")


def with_dmi(case, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    case["params"]["dind"] = np.zeros(256)
    case["params"]["dind"][:4] = rng.uniform(-3e-3, 3e-3, 4)
    # a zero interface scale between regions 0 and 1: a DMI boundary inside
    case["params"]["exch_scale"][1] = 0.0  # pair (1, 0) at index 1 * (1 + 1) / 2 + 0
    return case


CASES = [((100, 70, 1), (2e-9, 2e-9, 1e-9), (0, 0, 0), True),
         ((33, 20, 3), (2e-9, 3e-9, 1e-9), (0, 0, 0), True),
         ((40, 24, 2), (2e-9, 2e-9, 1e-9), (1, 0, 0), True),
         ((37, 21, 1), (1e-9, 1.5e-9, 1e-9), (0, 0, 0), False),
         ((64, 1, 1), (1e-9, 1e-9, 1e-9), (0, 0, 0), False)]


@pytest.mark.parametrize("grid,cell,pbc,demag", CASES, ids=[str(c[0]) + str(c[2]) + str(c[3]) for c in CASES])
def test_dmi_fields_and_energy(gpu, grid, cell, pbc, demag):
    case = with_dmi(synth.random_problem(grid, cell, seed=sum(grid) + 3, nregions=4, vacuum=True), seed=grid[0])
    ctx, prob, m = pair(case, pbc, demag)
    m64 = case["m0"].astype(np.float64)
    log("dmi parity", grid, pbc, demag)
    assert rel_inf(to_np(ctx.beff(m)), prob.beff(m64)) < 1e-5
    assert rel_inf(to_np(ctx.torque(m)), prob.torque(m64)) < 1e-5
    e, ref = ctx.energy(m), prob.energy(m64)
    for k in ("exch", "total"):
        assert e[k] == pytest.approx(ref[k], rel=2e-5, abs=1e-6 * abs(ref["total"]) + 1e-30), k
    ctx.close()


def test_periodic_cycloid_through_library(gpu):
    import torch

    n, delta, turns, d, aex = 128, 1e-9, 3, 2e-3, 1e-11
    k = 2 * math.pi * turns / (n * delta)
    params = synth.material(8e5, aex, alpha=0.1)
    params["dind"] = np.zeros(256)
    params["dind"][0] = d
    ctx = mm.Context((n, 1, 1), (delta,) * 3, np.zeros((1, 1, n), np.uint8), params, demag=False, pbc=(1, 1, 0))
    x = np.arange(n) * delta
    m = torch.from_numpy(np.stack([np.sin(k * x), 0 * x, np.cos(k * x)])[:, None, None, :].astype(np.float32)).cuda()
    b = to_np(ctx.beff(m))
    # exchange (2A/Msat)(2 cos k Delta - 2)/Delta^2 m plus DMI -(2D/Msat) sin(k Delta)/Delta m
    ref = (2 * aex / 8e5 * (2 * math.cos(k * delta) - 2) / delta ** 2
           - 2 * d / 8e5 * math.sin(k * delta) / delta) * to_np(m)
    assert rel_inf(b, ref) < 1e-5
    ctx.close()


def test_dmi_dp45_run(gpu):
    case = synth.vortex_film(seed=2, n=32)
    case["params"]["alpha"][0] = 0.1
    case["params"]["dind"] = np.zeros(256)
    case["params"]["dind"][0] = 2e-3
    ctx, prob, m = pair(case)
    t_end = 5e-12
    t, dt, st = ctx.run(m, t_end, dt=1e-14, solver=45, opts=mm.solver_opts(max_err=1e-5))
    it = ointegrate.Integrator(prob.torque, case["m0"], "rk45", dt=1e-14, max_err=1e-5)
    it.run(t_end)
    err = np.max(np.abs(to_np(m) - it.m))
    log("dmi DP45: steps", st["steps"], "oracle", it.nsteps, "max |dm|", err)
    assert err < 1e-3
    ctx.close()
