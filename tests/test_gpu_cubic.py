"""Cubic anisotropy on the GPU against the FP64 oracle (section
"Magneto-crystalline anisotropy", paragraph "Cubic"): B_eff, torque and
energies on 2D and 3D grids with a random cubic frame and constants per
region, rebuilt tables after new parameters, removal, and a short
Dormand-Prince run (the fused field passes carry the term too)."""
import numpy as np
import pytest

from oracle import fields as ofields
from oracle import integrate as ointegrate
from paper_1406_7635_amd import mm, synth
from tests.gpu_helpers import log, make_pair, rel_inf, to_np

pytestmark = pytest.mark.gpu


def add_cubic(params, nregions, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    params["kc"] = np.zeros((256, 3))
    params["anis_c1"] = np.zeros((256, 3))
    params["anis_c2"] = np.zeros((256, 3))
    for r in range(nregions):
        q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
        params["anis_c1"][r] = q[:, 0]
        params["anis_c2"][r] = q[:, 1]
        params["kc"][r] = rng.normal(size=3) * np.array([3e5, 3e5, 3e5])
    return params


def _set(ctx, params):
    ctx.set_cubic_anisotropy(params["kc"], params["anis_c1"], params["anis_c2"])


@pytest.mark.parametrize("grid,cell", [((100, 70, 1), (3e-9, 3e-9, 3e-9)), ((33, 20, 3), (2e-9, 3e-9, 2.5e-9)),
                                       ((17, 1, 1), (1e-9, 2e-9, 2e-9))])
def test_cubic_fields_and_energy(gpu, grid, cell):
    case = synth.random_problem(grid, cell, seed=sum(grid), nregions=3, vacuum=True)
    add_cubic(case["params"], 3, seed=grid[0])
    ctx, prob, m = make_pair(case)
    _set(ctx, case["params"])
    m64 = case["m0"].astype(np.float64)
    log("cubic parity", grid)
    b = ctx.beff(m)
    assert rel_inf(to_np(b), prob.beff(m64)) < 1e-5
    assert rel_inf(to_np(ctx.torque(m)), prob.torque(m64)) < 1e-5
    e, ref = ctx.energy(m), prob.energy(m64)
    for k in ("anis", "total"):
        assert e[k] == pytest.approx(ref[k], rel=2e-5, abs=1e-6 * abs(ref["total"]) + 1e-30), k
    # new parameters (Msat) rebuild the cubic table
    p2 = dict(case["params"])
    p2["msat"] = np.asarray(case["params"]["msat"]) * 1.5
    ctx.set_params(p2)
    prob2 = ofields.Problem(case["grid"], case["cell"], case["region"], p2)
    assert rel_inf(to_np(ctx.beff(m)), prob2.beff(m64)) < 1e-5
    # removal
    ctx.set_cubic_anisotropy(None, None, None)
    p3 = {k: v for k, v in p2.items() if k not in ("kc", "anis_c1", "anis_c2")}
    prob3 = ofields.Problem(case["grid"], case["cell"], case["region"], p3)
    assert rel_inf(to_np(ctx.beff(m)), prob3.beff(m64)) < 1e-5
    ctx.close()


def test_cubic_dp45_run(gpu):
    case = synth.vortex_film(seed=2, n=32)
    case["params"]["alpha"][0] = 0.1
    add_cubic(case["params"], 1, seed=9)
    ctx, prob, m = make_pair(case)
    _set(ctx, case["params"])
    t_end = 5e-12
    t, dt, st = ctx.run(m, t_end, dt=1e-14, solver=45, opts=mm.solver_opts(max_err=1e-5))
    it = ointegrate.Integrator(prob.torque, case["m0"], "rk45", dt=1e-14, max_err=1e-5)
    it.run(t_end)
    err = np.max(np.abs(to_np(m) - it.m))
    log("cubic DP45: steps", st["steps"], "oracle", it.nsteps, "max |dm|", err)
    assert err < 1e-3
    ctx.close()
