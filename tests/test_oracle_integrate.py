"""Pins of the oracle's integrators and relax (CPU).

Paper sections "Landau-Lifshitz torque" (figure figtqLL: undamped precession,
m_x = cos(gamma B t)), "Dynamics" (figure figConvergence: solver orders),
"Adaptive time step" (figure figMaxErr: error proportional to MaxErr),
"Energy minimization" (relax), plus the exact damped macrospin and the
Kittel frequency of a single cell.
"""
import math

import numpy as np
import pytest

from oracle import fields, integrate
from oracle.constants import GAMMA_LL, MU0
from paper_1406_7635_amd import synth


def _macrospin(alpha=0.0, b=(0, 0, 0.1), cell=(1e-9, 1e-9, 1e-9), msat=1.0 / MU0, ku1=0.0,
               u=(1, 0, 0), demag=False):
    p = synth.material(msat, 1e-11, alpha=alpha, bext=b, ku1=ku1, anis_u=u)
    return fields.Problem((1, 1, 1), cell, np.zeros((1, 1, 1), np.uint8), p, demag=demag)


def _m(v):
    v = np.asarray(v, float)
    return (v / np.linalg.norm(v)).reshape(3, 1, 1, 1)


def test_undamped_precession():
    """Appendix script for figure figtqLL: 0.1 T along z, m0 = x."""
    prob = _macrospin()
    it = integrate.Integrator(prob.torque, _m((1, 0, 0)), "rk45", max_err=1e-9)
    for t_end in (0.1e-9, 0.37e-9, 1e-9):
        it.run(t_end)
        mx = it.m[0, 0, 0, 0]
        assert mx == pytest.approx(math.cos(0.1 * GAMMA_LL * t_end), abs=2e-7)


@pytest.mark.parametrize("alpha", [0.05, 0.3])
def test_damped_macrospin_closed_form(alpha):
    """tan(theta/2) = tan(theta0/2) exp(-alpha gamma B t/(1+alpha^2)),
    phi = phi0 + gamma B t/(1+alpha^2), the exact solution of the LL equation."""
    B = 0.5
    prob = _macrospin(alpha=alpha, b=(0, 0, B))
    th0 = 2.5
    it = integrate.Integrator(prob.torque, _m((math.sin(th0), 0, math.cos(th0))), "rk45",
                              max_err=1e-9)
    t = 0.2e-9
    it.run(t)
    a = GAMMA_LL * B / (1 + alpha ** 2)
    th = 2 * math.atan(math.tan(th0 / 2) * math.exp(-alpha * a * t))
    ph = a * t
    ref = np.array([math.sin(th) * math.cos(ph), math.sin(th) * math.sin(ph), math.cos(th)])
    np.testing.assert_allclose(it.m[:, 0, 0, 0], ref, atol=1e-6)


def _period_error(solver, dt):
    """Fixed-step error after one precession period (script for figConvergence)."""
    prob = _macrospin()
    period = 2 * math.pi / (0.1 * GAMMA_LL)
    n = int(round(period / dt))
    dt = period / n
    m = _m((1, 0, 1))
    if solver == "rk4":
        for _ in range(n):
            m = integrate.rk4_step(prob.torque, m, dt)
    else:
        tab = integrate.SOLVERS[solver]
        k1 = prob.torque(m)
        for _ in range(n):
            ms, k1, _ = integrate.embedded_step(prob.torque, m, k1, dt, tab)
            m = integrate.normalize(ms)
    return float(np.linalg.norm(m[:, 0, 0, 0] - _m((1, 0, 1))[:, 0, 0, 0]))


@pytest.mark.parametrize("solver,order", [("rk4", 4), ("rk45", 5), ("rk23", 3)])
def test_convergence_order(solver, order):
    period = 2 * math.pi / (0.1 * GAMMA_LL)
    dts = [period / n for n in (24, 48, 96)] if order < 5 else [period / n for n in (12, 24, 48)]
    errs = [_period_error(solver, dt) for dt in dts]
    slopes = [math.log(errs[i] / errs[i + 1]) / math.log(dts[i] / dts[i + 1]) for i in range(2)]
    assert all(abs(s - order) < 0.3 for s in slopes), slopes


def test_error_proportional_to_maxerr():
    """Figure figMaxErr: the error after one period scales linearly with MaxErr."""
    prob = _macrospin()
    period = 2 * math.pi / (0.1 * GAMMA_LL)
    errs = []
    tols = [1e-4, 1e-5, 1e-6]
    for tol in tols:
        it = integrate.Integrator(prob.torque, _m((1, 0, 1)), "rk45", max_err=tol)
        it.run(period)
        errs.append(float(np.linalg.norm(it.m[:, 0, 0, 0] - _m((1, 0, 1))[:, 0, 0, 0])))
    slope = math.log(errs[0] / errs[-1]) / math.log(tols[0] / tols[-1])
    assert 0.6 < slope < 1.4, (errs, slope)


def test_kittel_frequency():
    """Single 4x4x2 nm cell, Msat 8e5, B = 1.5 T along z, tiny tilt, no damping:
    f = gamma/2pi sqrt((B + mu0 Ms (Nx - Nz)) (B + mu0 Ms (Ny - Nz)))."""
    cell = (4e-9, 4e-9, 2e-9)
    Ms, B = 8e5, 1.5
    prob = _macrospin(b=(0, 0, B), cell=cell, msat=Ms, demag=True)
    N = prob.octant[:, 0, 0, 0]
    f = GAMMA_LL / (2 * math.pi) * math.sqrt((B + MU0 * Ms * (N[0] - N[2])) *
                                             (B + MU0 * Ms * (N[1] - N[2])))
    tilt = math.radians(0.1)
    it = integrate.Integrator(prob.torque, _m((math.sin(tilt), 0, math.cos(tilt))), "rk45",
                              max_err=1e-10)
    ts, xs = [0.0], [float(it.m[0, 0, 0, 0])]
    t_end = 20.0 / f
    while it.t < t_end:
        it.step(t_end)
        ts.append(it.t)
        xs.append(float(it.m[0, 0, 0, 0]))
    ts, xs = np.array(ts), np.array(xs)
    idx = np.nonzero((xs[:-1] > 0) & (xs[1:] <= 0))[0]
    tz = ts[idx] - xs[idx] * (ts[idx + 1] - ts[idx]) / (xs[idx + 1] - xs[idx])
    f_sim = (len(tz) - 1) / (tz[-1] - tz[0])
    assert f_sim == pytest.approx(f, rel=1e-5)


def test_relax_macrospin_and_uniaxial():
    prob = _macrospin(alpha=0.5, b=(0.05, 0.02, 0.1))
    m, e, tq, _ = integrate.relax(prob, _m((-1, 0.3, -0.2)))
    b = np.array([0.05, 0.02, 0.1])
    np.testing.assert_allclose(m[:, 0, 0, 0], b / np.linalg.norm(b), atol=1e-4)
    prob2 = _macrospin(alpha=0.5, b=(0, 0, 0), ku1=5e5, u=(0, 0.6, 0.8), msat=8e5)
    m2, _, tq2, _ = integrate.relax(prob2, _m((0.5, 0.2, 0.3)))
    assert abs(float(np.dot(m2[:, 0, 0, 0], [0, 0.6, 0.8]))) == pytest.approx(1.0, abs=1e-7)
    assert tq2 / GAMMA_LL < 1e-4


def test_relax_lowers_energy_of_small_film():
    case = synth.random_problem((8, 6, 2), (3e-9, 3e-9, 3e-9), 4, nregions=2)
    prob = fields.Problem(case["grid"], case["cell"], case["region"], case["params"])
    m0 = case["m0"].astype(np.float64)
    e0 = prob.energy(m0)["total"]
    m, e, tq, steps = integrate.relax(prob, m0, max_steps=3000)
    assert e < e0
    assert np.allclose(np.linalg.norm(m, axis=0), 1.0, atol=1e-12)


@pytest.mark.parametrize("solver", ["rk45", "rk23"])
def test_error_estimate_order(solver):
    """The per-step error estimate eps = dt max|sum (b - b*) k| of an embedded
    pair of orders (q+1, q) scales as dt^(q+1) for small dt."""
    prob = _macrospin(alpha=0.1)
    tab = integrate.SOLVERS[solver]
    m = _m((1, 0.2, 0.4))
    k1 = prob.torque(m)
    dts = [2e-12, 1e-12, 0.5e-12]
    eps = [integrate.embedded_step(prob.torque, m, k1, dt, tab)[2] for dt in dts]
    slopes = [math.log(eps[i] / eps[i + 1]) / math.log(2.0) for i in range(2)]
    q = tab["order_low"]
    assert all(abs(s - (q + 1)) < 0.3 for s in slopes), slopes


def _dt_for_eps(prob, m, tab, target):
    """The step whose error estimate is `target`, from eps = C dt^(q+1)
    (pinned by test_error_estimate_order), refined twice."""
    q = tab["order_low"]
    k1 = prob.torque(m)
    dt = 1e-12
    for _ in range(3):
        eps = integrate.embedded_step(prob.torque, m, k1, dt, tab)[2]
        dt *= (target / eps) ** (1.0 / (q + 1))
    return dt


@pytest.mark.parametrize("solver", ["rk45", "rk23"])
@pytest.mark.parametrize("ratio", [4.0, 30.0])
def test_rejected_step_retries_at_headroom_target(solver, ratio):
    """Section "Adaptive time step": the controller keeps the error per step
    close to MaxErr, with headroom 0.8.  Since eps = C dt^(q+1) for an
    embedded pair of orders (q+1, q), a step rejected with eps = r MaxErr must
    be retried at the step that brings eps to 0.8^(q+1) MaxErr whatever r
    (r = 4, 30; both below the 0.1 clamp).  An exponent other than 1/(q+1)
    misses this target by r^(1 - (q+1)/p) for exponent 1/p (about 30 % at
    r = 4 for p = q), and a headroom applied to eps instead of dt misses it by
    0.8^q."""
    prob = _macrospin(alpha=0.1)
    tab = integrate.SOLVERS[solver]
    q = tab["order_low"]
    m = _m((1, 0.2, 0.4))
    max_err = 1e-6
    dt = _dt_for_eps(prob, m, tab, ratio * max_err)
    it = integrate.Integrator(prob.torque, m, solver, dt=dt, max_err=max_err)
    acc, eps1 = it.step()
    assert not acc and eps1 == pytest.approx(ratio * max_err, rel=1e-3)
    acc, eps2 = it.step()
    assert acc
    assert eps2 / max_err == pytest.approx(0.8 ** (q + 1), rel=0.03), eps2 / max_err


@pytest.mark.parametrize("solver", ["rk45", "rk23"])
def test_accepted_step_grows_to_headroom_target(solver):
    """An accepted step with eps well below MaxErr grows dt so that the next
    attempt's eps lands near 0.8^(q+1) MaxErr (the state moves a little
    between the two attempts, hence the looser bound)."""
    prob = _macrospin(alpha=0.1)
    tab = integrate.SOLVERS[solver]
    q = tab["order_low"]
    m = _m((1, 0.2, 0.4))
    max_err = 1e-6
    # eps = r MaxErr with 0.8 (1/r)^(1/(q+1)) = 1.6 keeps the growth below the clamp
    r = (0.8 / 1.6) ** (q + 1)
    dt = _dt_for_eps(prob, m, tab, r * max_err)
    it = integrate.Integrator(prob.torque, m, solver, dt=dt, max_err=max_err)
    acc, eps1 = it.step()
    assert acc
    assert it.dt / dt == pytest.approx(0.8 * (max_err / eps1) ** (1.0 / (q + 1)), rel=1e-12)
    acc, eps2 = it.step()
    assert eps2 / max_err == pytest.approx(0.8 ** (q + 1), rel=0.08), eps2 / max_err


@pytest.mark.parametrize("solver", ["rk45", "rk23"])
def test_step_factor_clamps(solver):
    """Readings of the step law at its extremes: eps = 0 (m along B, no
    torque) doubles dt; an error far above MaxErr shrinks dt tenfold."""
    prob = _macrospin(alpha=0.1)
    it = integrate.Integrator(prob.torque, _m((0, 0, 1)), solver, dt=1e-13, max_err=1e-6)
    acc, eps = it.step()
    assert acc and eps == 0.0 and it.dt == 2e-13
    m = _m((1, 0.2, 0.4))
    tab = integrate.SOLVERS[solver]
    dt = _dt_for_eps(prob, m, tab, 1e-5) * 1e3 ** (1.0 / (tab["order_low"] + 1))
    it = integrate.Integrator(prob.torque, m, solver, dt=dt, max_err=1e-9)
    acc, eps = it.step()
    assert not acc and eps > 1e6 * 1e-9
    assert it.dt == pytest.approx(0.1 * dt, rel=1e-15)
