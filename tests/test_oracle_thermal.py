"""Pins of the oracle's thermal field and Heun's method (CPU only).

Paper section "Thermal fluctuations" (Brown's random field, Heun with a fixed
step) and section "Dynamics" (RK12).  The generator is pinned by the published
known-answer vectors of Philox4x32-10; the field's statistics by the
Boltzmann equilibrium of free macrospins in a field (mean projection = the
Langevin function coth x - 1/x, x = Msat V B / kB T), which holds only if the
variance prefactor and the Heun (Stratonovich) discretisation are right; the
solver by its convergence order.
"""
import math

import numpy as np
import pytest

from oracle import fields, integrate, thermal
from oracle.constants import GAMMA_LL, KB
from paper_1406_7635_amd import synth

# Philox4x32-10 known-answer vectors (counter, key, output) published with the
# generator (Random123 distribution, kat_vectors)
KAT = [
    ((0, 0, 0, 0), (0, 0), (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
    ((0xFFFFFFFF,) * 4, (0xFFFFFFFF, 0xFFFFFFFF), (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
    ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0),
     (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1)),
]


@pytest.mark.parametrize("ctr,key,out", KAT)
def test_philox_known_answers(ctr, key, out):
    got = thermal.philox4x32_10([[v] for v in ctr], key)[:, 0]
    assert [int(v) for v in got] == list(out)


def test_uniforms_open_interval():
    x = np.array([0, 255, 256, 0xFFFFFFFF], dtype=np.uint64)
    u = thermal.uniforms(x)
    assert u[0] == u[1] == 0.5 / 2 ** 24 and u[2] == 1.5 / 2 ** 24
    assert u[3] == 1.0 - 0.5 / 2 ** 24


def test_normal_moments_and_independence():
    eta = np.concatenate([thermal.normals(1 << 17, s, seed=12345) for s in range(4)], axis=1)
    n = eta.shape[1]
    assert np.all(np.abs(eta.mean(axis=1)) < 5 / math.sqrt(n))
    assert np.all(np.abs(eta.var(axis=1) - 1.0) < 8 / math.sqrt(n))
    assert np.all(np.abs((eta ** 4).mean(axis=1) - 3.0) < 40 / math.sqrt(n))
    c = np.corrcoef(eta)
    assert np.all(np.abs(c[np.triu_indices(3, 1)]) < 5 / math.sqrt(n))
    # consecutive steps and cells are uncorrelated
    a, b = thermal.normals(1 << 16, 7, seed=1), thermal.normals(1 << 16, 8, seed=1)
    assert abs(np.corrcoef(a[0], b[0])[0, 1]) < 5 / math.sqrt(1 << 16)
    assert abs(np.corrcoef(a[0, :-1], a[0, 1:])[0, 1]) < 5 / math.sqrt(1 << 16)
    # the seed selects another stream
    assert not np.allclose(thermal.normals(64, 0, seed=1), thermal.normals(64, 0, seed=2))


def test_thermal_field_zero_without_temperature_or_magnetisation():
    p = synth.material(8e5, 1e-11, alpha=0.1)
    p = synth.material(0.0, 0.0, alpha=0.1, region=1, params=p)
    temp = np.zeros(256)
    temp[0] = 300.0
    temp[2] = 300.0
    region = np.array([[[0, 1, 2, 0]]], dtype=np.uint8)
    b = thermal.thermal_field(region, p, temp, (2e-9,) * 3, 1e-13, 0, 7)
    assert np.all(b[:, 0, 0, 1] == 0)  # Msat = 0
    assert np.all(b[:, 0, 0, 2] == 0)  # region 2 unset: Msat = 0
    assert np.all(b[:, 0, 0, 0] != 0)


class _FreeSpins:
    """n x n uncoupled macrospins in a uniform field B along z: the torque is
    the oracle's Landau-Lifshitz torque of B + the extra (thermal) field."""

    def __init__(self, n, msat, b, alpha, cell):
        self.params = synth.material(msat, 0.0, alpha=alpha)
        self.region = np.zeros((1, n, n), np.uint8)
        self.cell = (cell,) * 3
        self.b = np.zeros((3, 1, n, n))
        self.b[2] = b
        self.alpha = np.full((1, n, n), alpha)

    def torque(self, m, precess=True, extra=None):
        return fields.llg_torque(m, self.b + extra, self.alpha, GAMMA_LL, precess)


@pytest.mark.parametrize("x", [1.5, 3.0])
def test_boltzmann_equilibrium_langevin(x):
    """Free macrospins in B along z stay in the Boltzmann distribution, whose
    mean projection is <m_z> = coth x - 1/x, x = Msat V B / kB T, under the
    thermal field over 2.5 relaxation times.  Seeded, so the outcome is
    fixed; the statistical error of the estimate is about 0.004, the
    tolerance 0.02 (a variance wrong by the factor 1 + alpha^2 = 1.25 would
    relax the x = 3 value towards 0.60)."""
    msat, b, alpha, cell = 8e5, 0.05, 0.5, 5e-9
    n = 64
    prob = _FreeSpins(n, msat, b, alpha, cell)
    temp = np.zeros(256)
    temp[0] = msat * cell ** 3 * b / (x * KB)
    # start from the Boltzmann distribution itself (cos theta by inversion of
    # its distribution function, azimuth uniform): the dynamics must keep it
    rng = np.random.Generator(np.random.PCG64(3))
    u = rng.random((n, n))
    ct = 1.0 + np.log1p(-u * (1.0 - math.exp(-2.0 * x))) / x
    ph = 2 * math.pi * rng.random((n, n))
    st = np.sqrt(np.maximum(0.0, 1.0 - ct * ct))
    m = np.stack([st * np.cos(ph), st * np.sin(ph), ct])[:, None]
    dt = 2e-13
    tau = (1 + alpha ** 2) / (alpha * GAMMA_LL * b)
    neq = int(tau / dt)
    m = thermal.run_thermal(prob, m, dt, neq, temp, seed=99)
    acc, cnt, step = 0.0, 0, neq
    for _ in range(25):
        m = thermal.run_thermal(prob, m, dt, 84, temp, seed=99, step0=step)
        step += 84
        acc += m[2].mean()
        cnt += 1
    mz = acc / cnt
    lang = 1.0 / math.tanh(x) - 1.0 / x
    assert mz == pytest.approx(lang, abs=0.02)


def test_heun_second_order():
    """One precession period of an undamped macrospin in 0.1 T (paper figure
    figConvergence): error against dt has slope 2."""
    p = synth.material(1.0 / (4e-7 * math.pi), 0.0, alpha=0.0, bext=(0.0, 0.0, 0.1))
    prob = fields.Problem((1, 1, 1), (1e-9,) * 3, np.zeros((1, 1, 1), np.uint8), p, demag=False)
    period = 2 * math.pi / (GAMMA_LL * 0.1)
    errs, dts = [], []
    for nstep in (200, 400, 800):
        dt = period / nstep
        m = np.array([1.0, 0.0, 0.0]).reshape(3, 1, 1, 1)
        for _ in range(nstep):
            m, _ = thermal.heun_step(prob.torque, m, dt)
        errs.append(float(np.max(np.abs(m.ravel() - np.array([1.0, 0.0, 0.0])))))
        dts.append(dt)
    slope = np.polyfit(np.log(dts), np.log(errs), 1)[0]
    assert slope == pytest.approx(2.0, abs=0.3)


def test_rk12_adaptive_tracks_precession():
    p = synth.material(1.0 / (4e-7 * math.pi), 0.0, alpha=0.0, bext=(0.0, 0.0, 0.1))
    prob = fields.Problem((1, 1, 1), (1e-9,) * 3, np.zeros((1, 1, 1), np.uint8), p, demag=False)
    t_end = 2e-10
    errs = []
    for me in (1e-4, 1e-5):
        it = integrate.Integrator(prob.torque, np.array([1.0, 0.0, 0.0]).reshape(3, 1, 1, 1), "rk12", dt=1e-14,
                                  max_err=me)
        it.run(t_end)
        w = GAMMA_LL * 0.1 * t_end
        errs.append(float(np.max(np.abs(it.m.ravel() - np.array([math.cos(w), math.sin(w), 0.0])))))
        assert it.nevals == 1 + it.nsteps + it.nrejects + it.nsteps  # fresh first stage after each accept
    assert errs[1] < errs[0] and errs[0] < 0.05
