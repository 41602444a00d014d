"""Thermal fluctuations and Heun's method (oracle, FP64, CPU).

Test infrastructure: only tests/, the smoke check and the benchmark's CPU
baseline use this module.

Paper section "Thermal fluctuations" (Eq. for B_therm): every cell carries a
random field eta * sqrt(2 mu0 alpha kB T / (B_sat gamma_LL dV dt)); with
B_sat = mu0 Msat this is eta * sqrt(2 alpha kB T / (Msat gamma_LL dV dt)).
eta has three independent standard normal components, drawn anew for every
time step.  Section "Dynamics": Heun's method (RK12: second order, with the
Euler step as first-order error estimate) is the solver for finite
temperature, with a fixed time step; the random field is held constant over
the two stages of a step.

Random numbers (the paper does not fix a generator; this is the reading both
the oracle and the GPU library implement, each from the published definition):
  * Philox4x32-10 (Salmon, Moraes, Dror and Shaw, "Parallel random numbers:
    as easy as 1, 2, 3", SC 2011): counter (c0, c1, c2, c3), key (k0, k1);
    a round maps (c0..c3) to (hi(B c2) ^ c1 ^ k0, lo(B c2), hi(A c0) ^ c3 ^ k1,
    lo(A c0)) with A = 0xD2511F53, B = 0xCD9E8D57, and the key advances by
    (0x9E3779B9, 0xBB67AE85) after every round; ten rounds.
  * counter (cell index, step mod 2^32, step div 2^32, 0), key (seed mod 2^32,
    seed div 2^32), with step the number of steps taken since the generator
    was seeded;
  * the 32-bit outputs x0..x3 become uniforms u = (floor(x / 2^8) + 1/2) / 2^24
    in (0, 1) (24 bits, exact in single precision);
  * Box-Muller: eta_x = r cos(2 pi u1), eta_y = r sin(2 pi u1) with
    r = sqrt(-2 ln u0); eta_z = sqrt(-2 ln u2) cos(2 pi u3).

Parity: pinned in tests/test_oracle_thermal.py (the generator against its
published known-answer vectors; the normal moments; Heun's second order on a
precessing macrospin; the Boltzmann equilibrium of macrospins in a field,
whose mean projection is the Langevin function).
"""
import numpy as np

from .constants import GAMMA_LL, KB
from .integrate import normalize

_A, _B = 0xD2511F53, 0xCD9E8D57
_WA, _WB = 0x9E3779B9, 0xBB67AE85
_M32 = 0xFFFFFFFF


def philox4x32_10(ctr, key):
    """Philox4x32-10 of counters ctr [4, n] (integers < 2^32) under key (k0, k1).

    Returns [4, n] uint64 holding the 32-bit outputs."""
    c = [np.asarray(v, dtype=np.uint64) & _M32 for v in ctr]
    k0, k1 = int(key[0]) & _M32, int(key[1]) & _M32
    for _ in range(10):
        p0 = np.uint64(_A) * c[0]
        p1 = np.uint64(_B) * c[2]
        c = [(p1 >> np.uint64(32)) ^ c[1] ^ np.uint64(k0), p1 & np.uint64(_M32),
             (p0 >> np.uint64(32)) ^ c[3] ^ np.uint64(k1), p0 & np.uint64(_M32)]
        k0 = (k0 + _WA) & _M32
        k1 = (k1 + _WB) & _M32
    return np.stack(c)


def uniforms(x):
    """(floor(x / 2^8) + 1/2) / 2^24 for 32-bit outputs x."""
    return ((np.asarray(x, dtype=np.uint64) >> np.uint64(8)).astype(np.float64) + 0.5) / 16777216.0


def normals(ncell, step, seed):
    """eta [3, ncell] of time step `step` (standard normal, independent)."""
    cells = np.arange(ncell, dtype=np.uint64)
    z = np.zeros(ncell, dtype=np.uint64)
    ctr = [cells, z + np.uint64(step & _M32), z + np.uint64((step >> 32) & _M32), z]
    u = uniforms(philox4x32_10(ctr, (seed & _M32, (seed >> 32) & _M32)))
    r0 = np.sqrt(-2.0 * np.log(u[0]))
    r2 = np.sqrt(-2.0 * np.log(u[2]))
    return np.stack([r0 * np.cos(2 * np.pi * u[1]), r0 * np.sin(2 * np.pi * u[1]), r2 * np.cos(2 * np.pi * u[3])])


def thermal_sigma(params, temp, cell):
    """Per-region standard deviation times sqrt(dt): sqrt(2 alpha kB T /
    (Msat gamma dV)), 0 for non-magnetic regions or T = 0."""
    msat = np.asarray(params["msat"], dtype=np.float64)
    alpha = np.asarray(params["alpha"], dtype=np.float64)
    gamma = float(params.get("gamma_ll", 0.0) or GAMMA_LL)
    vol = cell[0] * cell[1] * cell[2]
    t = np.asarray(temp, dtype=np.float64)
    ok = (msat > 0) & (t > 0)
    return np.where(ok, np.sqrt(np.where(ok, 2.0 * alpha * KB * t / (np.where(ok, msat, 1.0) * gamma * vol), 0.0)), 0.0)


def thermal_field(region, params, temp, cell, dt, step, seed):
    """B_therm [3, nz, ny, nx] (tesla) of time step `step`."""
    region = np.asarray(region)
    sig = thermal_sigma(params, temp, cell)[region] / np.sqrt(dt)
    eta = normals(region.size, step, seed).reshape((3,) + region.shape)
    return eta * sig


def heun_step(f, m, dt):
    """One step of Heun's method for dm/dt = f(m): k1 = f(m), k2 = f(m + dt k1),
    m_new = m + dt (k1 + k2)/2.  Returns (normalised m_new, eps) with
    eps = dt max_cells |(k2 - k1)/2| (Heun minus Euler)."""
    k1 = f(m)
    k2 = f(m + dt * k1)
    d = 0.5 * (k2 - k1)
    eps = dt * float(np.max(np.sqrt(np.sum(d * d, axis=0))))
    return normalize(m + dt * 0.5 * (k1 + k2)), eps


def run_thermal(problem, m, dt, nsteps, temp, seed, step0=0, precess=True):
    """Fixed-step Heun run with the thermal field: step n uses
    thermal_field(..., step=step0 + n) in both stages.  Returns m."""
    m = np.asarray(m, dtype=np.float64)
    for n in range(nsteps):
        bth = thermal_field(problem.region, problem.params, temp, problem.cell, dt, step0 + n, seed)
        m, _ = heun_step(lambda x: problem.torque(x, precess=precess, extra=bth), m, dt)
    return m
