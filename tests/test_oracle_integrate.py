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
