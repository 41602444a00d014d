"""Time integration of the Landau-Lifshitz equation (oracle, FP64, CPU).

Paper section "Dynamics": RK45 (Dormand-Prince, 5th order with a 4th-order
error estimate, the default), RK32 (Bogacki-Shampine, used by relax), RK12
(Heun, second order with the Euler step as error estimate) and the
adaptive step of section "Adaptive time step": the error of a step is
eps = max over cells |tau_high - tau_low| dt, compared with MaxErr and used to
rescale dt with a headroom of 0.8.  Classical fixed-step RK4 is not among the
paper's solvers; it is provided for fixed-step trajectory comparisons.

Readings of points the paper leaves open: the step factor is
headroom * (MaxErr/eps)^(1/(q+1)) with q the order of the embedded
(lower-order) solution, clamped to [0.1, 2] (2 when eps = 0); a rejected step
is retried with the new dt; the last step is clipped to land on t_end; after
each accepted step m is renormalised to unit length (stage states stay raw);
first-same-as-last reuses the last stage's torque, evaluated at the
un-normalised stage state, as the next step's first.  The step law is pinned
by what the paper fixes -- the error per step is kept close to MaxErr with
headroom 0.8 -- together with eps = C dt^(q+1): a step rejected (or accepted)
with eps = r MaxErr is followed by one at eps = 0.8^(q+1) MaxErr whatever r
(tests/test_oracle_integrate.py); the clamps are readings checked as such.
relax() is pinned by its outcome: energy not increasing, known minima, and
the residual torque band of section "Energy minimization".
"""
from fractions import Fraction as F

import numpy as np

# Butcher tableaux (rows a[s] hold the coefficients of k_1..k_s for stage s+1)
RK4 = {
    "a": [[F(1, 2)], [F(0), F(1, 2)], [F(0), F(0), F(1)]],
    "b": [F(1, 6), F(1, 3), F(1, 3), F(1, 6)],
}

BS23 = {  # Bogacki-Shampine 3(2), FSAL
    "a": [[F(1, 2)], [F(0), F(3, 4)], [F(2, 9), F(1, 3), F(4, 9)]],
    "b": [F(2, 9), F(1, 3), F(4, 9), F(0)],
    "bstar": [F(7, 24), F(1, 4), F(1, 3), F(1, 8)],
    "order_low": 2,
}

DP45 = {  # Dormand-Prince 5(4), FSAL
    "a": [
        [F(1, 5)],
        [F(3, 40), F(9, 40)],
        [F(44, 45), F(-56, 15), F(32, 9)],
        [F(19372, 6561), F(-25360, 2187), F(64448, 6561), F(-212, 729)],
        [F(9017, 3168), F(-355, 33), F(46732, 5247), F(49, 176), F(-5103, 18656)],
        [F(35, 384), F(0), F(500, 1113), F(125, 192), F(-2187, 6784), F(11, 84)],
    ],
    "b": [F(35, 384), F(0), F(500, 1113), F(125, 192), F(-2187, 6784), F(11, 84), F(0)],
    "bstar": [F(5179, 57600), F(0), F(7571, 16695), F(393, 640), F(-92097, 339200),
              F(187, 2100), F(1, 40)],
    "order_low": 4,
}

RK12 = {  # Heun with the Euler step as error estimate; not first-same-as-last
    "a": [[F(1)]],
    "b": [F(1, 2), F(1, 2)],
    "bstar": [F(1), F(0)],
    "order_low": 1,
    "fsal": False,
}

SOLVERS = {"rk12": RK12, "rk23": BS23, "rk45": DP45}


def normalize(m):
    n = np.sqrt(np.sum(m * m, axis=0))
    return m / np.where(n > 0, n, 1.0)


def rk4_step(f, m, dt):
    """One classical RK4 step of dm/dt = f(m), followed by renormalisation."""
    k = [f(m)]
    for row in RK4["a"]:
        ms = m + dt * sum(float(a) * kj for a, kj in zip(row, k) if a != 0)
        k.append(f(ms))
    m1 = m + dt * sum(float(b) * kj for b, kj in zip(RK4["b"], k))
    return normalize(m1)


def embedded_step(f, m, k1, dt, tab, t=None):
    """One attempt of an FSAL embedded pair.

    Returns (m_new_raw, k_last, eps) where m_new_raw is the higher-order
    solution (= the last stage state), k_last = f(m_new_raw) and
    eps = dt * max_cells |sum_j (b_j - b*_j) k_j|.  With a time t, f takes
    (m, t_s) with the stage time t_s = t + c_s dt, c_s the row sum of a."""
    k = [k1]
    ms = m
    for row in tab["a"]:
        ms = m + dt * sum(float(a) * kj for a, kj in zip(row, k) if a != 0)
        k.append(f(ms) if t is None else f(ms, t + dt * float(sum(row))))
    e = [float(b - bs) for b, bs in zip(tab["b"], tab["bstar"])]
    diff = sum(ej * kj for ej, kj in zip(e, k) if ej != 0)
    eps = dt * float(np.max(np.sqrt(np.sum(diff * diff, axis=0)))) if diff.size else 0.0
    return ms, k[-1], eps


def step_factor(eps, max_err, order_low, headroom=0.8):
    if eps == 0.0:
        return 2.0
    fac = headroom * (max_err / eps) ** (1.0 / (order_low + 1))
    return min(2.0, max(0.1, fac))


class Integrator:
    """Adaptive integrator state: m, t, dt, the FSAL torque and counters."""

    def __init__(self, f, m, solver="rk45", dt=1e-14, max_err=1e-5, headroom=0.8,
                 dt_min=0.0, dt_max=np.inf, timed=False):
        """timed: f takes (m, t), evaluated at each stage's time."""
        self.timed = timed
        self.f = f
        self.tab = SOLVERS[solver]
        self.m = np.asarray(m, dtype=np.float64).copy()
        self.t = 0.0
        self.dt = dt
        self.max_err = max_err
        self.headroom = headroom
        self.dt_min = dt_min
        self.dt_max = dt_max
        self.k1 = f(self.m, 0.0) if timed else f(self.m)
        self.nsteps = 0
        self.nrejects = 0
        self.nevals = 1

    def step(self, t_end=None):
        """One attempt; returns (accepted, eps)."""
        dt = self.dt
        if t_end is not None and self.t + dt > t_end:
            dt = t_end - self.t
        if self.tab.get("fsal", True):
            m_new, k_last, eps = embedded_step(self.f, self.m, self.k1, dt, self.tab,
                                               self.t if self.timed else None)
        else:
            k = [self.k1]
            for row in self.tab["a"]:
                ms = self.m + dt * sum(float(a) * kj for a, kj in zip(row, k) if a != 0)
                k.append(self.f(ms, self.t + dt * float(sum(row))) if self.timed else self.f(ms))
            m_new = self.m + dt * sum(float(b) * kj for b, kj in zip(self.tab["b"], k))
            e = [float(b - bs) for b, bs in zip(self.tab["b"], self.tab["bstar"])]
            diff = sum(ej * kj for ej, kj in zip(e, k) if ej != 0)
            eps = dt * float(np.max(np.sqrt(np.sum(diff * diff, axis=0))))
            k_last = None
        self.nevals += len(self.tab["a"])
        fac = step_factor(eps, self.max_err, self.tab["order_low"], self.headroom)
        accepted = eps <= self.max_err
        if accepted:
            self.m = normalize(m_new)
            if k_last is None:  # no first-same-as-last: the next first stage is evaluated afresh
                k_last = self.f(self.m, self.t + dt) if self.timed else self.f(self.m)
                self.nevals += 1
            self.k1 = k_last
            self.t += dt
            self.nsteps += 1
        else:
            self.nrejects += 1
        self.dt = min(self.dt_max, max(self.dt_min, dt * fac))
        return accepted, eps

    def run(self, t_end, max_steps=10 ** 9):
        while self.t < t_end and self.nsteps + self.nrejects < max_steps:
            self.step(t_end)
        return self.m


def relax(problem, m, max_err=1e-5, min_err=1e-9, block=3, max_steps=100000, dt=1e-14):
    """Energy minimisation following the paper's relax() (section "Energy minimization").

    Precession is switched off and RK23 advances m.  Energy phase: blocks of
    `block` steps until the total energy stops decreasing.  Torque phase:
    blocks until max |tau| stops decreasing; then MaxErr is halved and the
    torque phase repeats, until MaxErr drops below min_err.  Returns
    (m, energy, max_torque, steps).  Parity unpinned: judged by its outcome
    (energy does not increase, residual torque, known minima)."""
    f = lambda s: problem.torque(s, precess=False)  # noqa: E731
    it = Integrator(f, m, "rk23", dt=dt, max_err=max_err)

    def attempts():
        return it.nsteps + it.nrejects

    def advance():
        n0 = it.nsteps
        while it.nsteps < n0 + block and attempts() < max_steps:
            it.step()

    e0 = problem.energy(it.m)["total"]
    while attempts() < max_steps:
        advance()
        e1 = problem.energy(it.m)["total"]
        if e1 >= e0:
            break
        e0 = e1

    def max_torque():
        tq = f(it.m)
        return float(np.max(np.sqrt(np.sum(tq * tq, axis=0))))

    t0 = max_torque()
    while it.max_err >= min_err and attempts() < max_steps:
        while attempts() < max_steps:
            advance()
            t1 = max_torque()
            if t1 >= t0:
                break
            t0 = t1
        it.max_err /= 2.0
    return it.m, problem.energy(it.m)["total"], max_torque(), it.nsteps
