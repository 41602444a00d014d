"""GPU parity of the integrators against the oracle and closed forms.

Trajectory tolerance 1e-3 on m (max over cells of |m - m_ref| per component);
closed forms at FP32-limited accuracy.
"""
import math

import numpy as np
import pytest

from oracle import fields as ofields
from oracle import integrate as ointegrate
from oracle.constants import GAMMA_LL, MU0
from paper_1406_7635_amd import mm, synth
from tests.gpu_helpers import log, make_pair, rel_inf, to_np

pytestmark = pytest.mark.gpu


def test_rk4_film_200_steps(gpu):
    """32x32x4 film, random m, 200 fixed RK4 steps of 1e-13 s: B_eff at step 0
    and m every 50 steps against the oracle."""
    case = synth.parity_cube(seed=1)
    ctx, prob, m = make_pair(case)
    m_ref = case["m0"].astype(np.float64)
    assert rel_inf(to_np(ctx.beff(m)), prob.beff(m_ref)) < 1e-5
    f = prob.torque
    for step in range(1, 201):
        ctx.rk4_step(m, case["dt"])
        m_ref = ointegrate.rk4_step(f, m_ref, case["dt"])
        if step % 50 == 0:
            err = np.max(np.abs(to_np(m) - m_ref))
            log("rk4 step", step, "max |dm|", err)
            assert err < 1e-3
    assert rel_inf(to_np(ctx.beff(m)), prob.beff(m_ref)) < 1e-3


@pytest.mark.parametrize("solver", [45, 23])
def test_adaptive_run_matches_oracle(gpu, solver):
    case = synth.vortex_film(seed=2, n=48)
    case["params"]["alpha"][0] = 0.1
    ctx, prob, m = make_pair(case)
    t_end = 10e-12
    t, dt, st = ctx.run(m, t_end, dt=1e-14, solver=solver, opts=mm.solver_opts(max_err=1e-5))
    assert t == pytest.approx(t_end, rel=1e-12)
    assert st["evals"] == (6 if solver == 45 else 3) * (st["steps"] + st["rejects"]) + 1
    it = ointegrate.Integrator(prob.torque, case["m0"], "rk45" if solver == 45 else "rk23",
                               dt=1e-14, max_err=1e-5)
    it.run(t_end)
    err = np.max(np.abs(to_np(m) - it.m))
    log("solver", solver, "steps", st["steps"], "oracle steps", it.nsteps, "max |dm|", err)
    assert err < 1e-3
    assert np.allclose(np.linalg.norm(to_np(m), axis=0), 1.0, atol=1e-6)


def test_single_steps_match_run(gpu):
    case = synth.vortex_film(seed=3, n=32)
    ctx, _, m = make_pair(case)
    m2 = m.clone()
    t, dt = 0.0, 1e-14
    for _ in range(20):
        acc, t, dt, err = ctx.rk45_step(m, t, dt)
    ctx.reset_solver()
    t2, dt2, st = ctx.run(m2, 1.0, dt=1e-14, max_attempts=20)
    assert t2 == pytest.approx(t, rel=1e-12)
    assert np.max(np.abs(to_np(m) - to_np(m2))) == 0.0


@pytest.mark.parametrize("grid", [(32, 32, 8), (64, 48, 6), (20, 64, 5)])
def test_dp45_attempts_multilayer_tile_order(gpu, grid):
    """Grids of several layers whose x tiles never straddle two planes, where
    the x-inverse and fused passes take their tiles y block by y block over
    all planes: B_eff at the start, three accepted Dormand-Prince attempts at
    a fixed step against the oracle's embedded steps (m within 2e-6), and the
    torque of the result."""
    case = synth.random_problem(grid, (2e-9, 2.5e-9, 3e-9), seed=sum(grid) + 7, nregions=3)
    ctx, prob, m = make_pair(case)
    f = prob.torque
    m_ref = case["m0"].astype(np.float64)
    assert rel_inf(to_np(ctx.beff(m)), prob.beff(m_ref)) < 1e-5
    k1 = f(m_ref)
    t, dt = 0.0, 2e-14
    opts = mm.solver_opts(max_err=1.0)
    for _ in range(3):
        acc, t, _, err = ctx.rk45_step(m, t, dt, opts)
        assert acc
        ms, k1, eps = ointegrate.embedded_step(f, m_ref, k1, dt, ointegrate.DP45)
        m_ref = ointegrate.normalize(ms)
        d = float(np.max(np.abs(to_np(m) - m_ref)))
        log("multilayer DP45", grid, "|dm| %.2e err %.3e / %.3e" % (d, err, eps))
        assert d < 2e-6
    assert rel_inf(to_np(ctx.torque(m)), prob.torque(to_np(m).astype(np.float64))) < 1e-5
    ctx.close()


def _macrospin(alpha, b, msat=1.0 / MU0):
    p = synth.material(msat, 1e-11, alpha=alpha, bext=b)
    return {"grid": (1, 1, 1), "cell": (1e-9, 1e-9, 1e-9), "region": np.zeros((1, 1, 1), np.uint8),
            "params": p}


def test_undamped_precession(gpu):
    """Figure figtqLL: m_x = cos(gamma 0.1 T t)."""
    case = _macrospin(0.0, (0, 0, 0.1))
    case["m0"] = synth.uniform_m((1, 1, 1), (1, 0, 0))
    ctx, _, m = make_pair(case, demag=False)
    t, dt = 0.0, 1e-14
    for t_end in (0.1e-9, 0.37e-9, 1e-9):
        t, dt, _ = ctx.run(m, t_end, t=t, dt=dt, opts=mm.solver_opts(max_err=1e-7))
        assert to_np(m)[0, 0, 0, 0] == pytest.approx(math.cos(0.1 * GAMMA_LL * t_end), abs=2e-5)


def test_damped_macrospin(gpu):
    alpha, B, th0 = 0.3, 0.5, 2.5
    case = _macrospin(alpha, (0, 0, B))
    case["m0"] = synth.uniform_m((1, 1, 1), (math.sin(th0), 0, math.cos(th0)))
    ctx, _, m = make_pair(case, demag=False)
    t = 0.2e-9
    ctx.run(m, t, opts=mm.solver_opts(max_err=1e-7))
    a = GAMMA_LL * B / (1 + alpha ** 2)
    th = 2 * math.atan(math.tan(th0 / 2) * math.exp(-alpha * a * t))
    ref = [math.sin(th) * math.cos(a * t), math.sin(th) * math.sin(a * t), math.cos(th)]
    np.testing.assert_allclose(to_np(m)[:, 0, 0, 0], ref, atol=5e-5)


def test_relax_macrospin_and_film(gpu):
    case = _macrospin(0.5, (0.05, 0.02, 0.1))
    case["m0"] = synth.uniform_m((1, 1, 1), (-1, 0.3, -0.2))
    ctx, _, m = make_pair(case, demag=False)
    r = ctx.relax(m)
    b = np.array([0.05, 0.02, 0.1])
    np.testing.assert_allclose(to_np(m)[:, 0, 0, 0], b / np.linalg.norm(b), atol=1e-4)
    assert r["converged"]
    film = synth.random_problem((16, 12, 2), (3e-9, 3e-9, 3e-9), seed=4, nregions=2)
    ctx, prob, m = make_pair(film)
    e0 = ctx.energy(m)["total"]
    r = ctx.relax(m, max_steps=20000)
    log("film relax: steps", r["steps"], "converged", r["converged"], "max torque / gamma",
        r["max_torque"] / GAMMA_LL, "T")
    assert r["converged"]
    assert r["energy"] < e0
    ref = prob.energy(to_np(m))["total"]
    assert r["energy"] == pytest.approx(ref, rel=1e-4)
    # section "Energy minimization": residual torques of 1e-4 ... 1e-7 gamma_LL T
    assert r["max_torque"] / GAMMA_LL < 1e-4
