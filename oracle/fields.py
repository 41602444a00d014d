"""Effective field, Landau-Lifshitz torque and energies (oracle, FP64, CPU).

Material parameters come as a dict of 256-entry region look-up tables
(paper section "Material Regions"):
  msat[256] (A/m), aex[256] (J/m), alpha[256], ku1[256], ku2[256] (J/m^3),
  anis_u[256, 3] (unit vectors), bext[256, 3] (T),
  exch_scale[256*257//2]: the inter-region scale S(i, j) for i >= j stored at
  i*(i+1)//2 + j (a lower-triangular matrix indexed by the two regions);
  S(i, i) is taken as 1 whatever is stored there,
  gamma_ll (rad/(T s)).
The region map is a uint8 array [nz, ny, nx]; m is [3, nz, ny, nx].
"""
import math

import numpy as np

from . import demag as _demag
from .constants import GAMMA_LL


def _lut(params, key, region):
    return np.asarray(params[key], dtype=np.float64)[region]


def exchange_scale(params, ra, rb):
    """S(ra, rb) from the packed lower-triangular table; 1 inside a region."""
    hi = np.maximum(ra, rb).astype(np.int64)
    lo = np.minimum(ra, rb).astype(np.int64)
    s = np.asarray(params["exch_scale"], dtype=np.float64)[hi * (hi + 1) // 2 + lo]
    return np.where(ra == rb, 1.0, s)


def exchange_coefficient(params, ra, rb):
    """2 S 2 l1 l2 / (l1 + l2) with l = Aex/Msat (paper Eq. eqBexch).

    Inside one region this is 2 Aex/Msat (Eq. eqBexch1).  A cell with Msat = 0
    is not magnetic: the pair then has no coupling (the neighbour counts as
    missing, which is the Neumann rule of the paper)."""
    msat = np.asarray(params["msat"], dtype=np.float64)
    aex = np.asarray(params["aex"], dtype=np.float64)
    ma, mb = msat[ra], msat[rb]
    ok = (ma > 0) & (mb > 0)
    la = np.where(ok, aex[ra] / np.where(ok, ma, 1.0), 0.0)
    lb = np.where(ok, aex[rb] / np.where(ok, mb, 1.0), 0.0)
    den = la + lb
    hm = np.where(ok & (den > 0), 2.0 * la * lb / np.where(den > 0, den, 1.0), 0.0)
    return 2.0 * exchange_scale(params, ra, rb) * hm


def exchange_field(m, region, params, cell, pbc=(0, 0, 0)):
    """6-neighbour exchange field (T), paper Eqs. eqBexch1 / eqBexch.

    B(c) = sum over the existing neighbours n of c(r_c, r_n) (m_n - m_c) / D_n^2.
    A neighbour outside the grid is replaced by the cell itself (Neumann
    boundary), i.e. it contributes nothing.  Along a periodic axis (pbc > 0,
    paragraph "Periodic boundary conditions") the grid wraps around: the last
    cell and the first are neighbours."""
    m = np.asarray(m, dtype=np.float64)
    B = np.zeros_like(m)
    for axis, d, p in zip((3, 2, 1), cell, pbc):   # array axis of x, y, z
        n = m.shape[axis]
        if n < 2:
            continue
        if p > 0:
            # the faces (i, i + 1 mod n), the wrap-around face included
            nb = np.roll(m, -1, axis=axis)
            rnb = np.roll(region, -1, axis=axis - 1)
            coef = exchange_coefficient(params, region, rnb) / (d * d)
            diff = nb - m
            B += coef * diff                            # neighbour on the + side
            B -= np.roll(coef * diff, 1, axis=axis)     # neighbour on the - side
            continue
        lo = [slice(None)] * 4
        hi = [slice(None)] * 4
        lo[axis] = slice(0, n - 1)
        hi[axis] = slice(1, n)
        rlo = region[tuple(lo[1:])]
        rhi = region[tuple(hi[1:])]
        coef = exchange_coefficient(params, rlo, rhi) / (d * d)
        diff = m[tuple(hi)] - m[tuple(lo)]
        B[tuple(lo)] += coef * diff            # neighbour on the + side
        B[tuple(hi)] -= coef * diff            # neighbour on the - side
    return B * (_lut(params, "msat", region) > 0)


def _dmi_neighbours(m, region, params, cell, pbc):
    """For the in-plane directions (-x, +x, -y, +y): each cell's neighbour
    magnetisation with the boundary rule of the induced DMI (section
    "Dzyaloshinskii-Moriya interaction", Eqs. eqDMIBC1 - eqDMIBC2), and
    whether the neighbour is real.

    The paper replaces a neighbour only where it is missing at the boundary
    of the magnet.  A neighbour is therefore real when it lies inside the grid
    (or across a periodic boundary) and is magnetic (Msat > 0), whatever its
    Aex or the interface scale; a missing one is replaced by the ghost
    m + n Delta dm/di|_boundary with n = -1 on the low side and +1 on the high
    side, where, with xi = D/(2A) of the cell's region (0 where A = 0),
    dm/dx|_b = (-xi m_z, 0, xi m_x) and dm/dy|_b = (0, -xi m_z, xi m_y).
    Returns a list of (value [3, ...], real mask, sign n, axis letter)."""
    m = np.asarray(m, dtype=np.float64)
    aex = _lut(params, "aex", region)
    dind = _lut(params, "dind", region)
    xi = np.where(aex > 0, dind / (2.0 * np.where(aex > 0, aex, 1.0)), 0.0)
    out = []
    for axis, d, p, name in ((3, cell[0], pbc[0], "x"), (2, cell[1], pbc[1], "y")):
        n = m.shape[axis]
        for sgn in (-1, 1):
            nb = np.roll(m, -sgn, axis=axis)              # value at index i + sgn
            rnb = np.roll(region, -sgn, axis=axis - 1)
            idx = np.arange(n)
            inside = (idx + sgn >= 0) & (idx + sgn < n) if p == 0 else np.ones(n, bool)
            shape = [1, 1, 1]
            shape[axis - 1] = n
            inside = np.broadcast_to(inside.reshape(shape), region.shape)
            real = inside & (_lut(params, "msat", rnb) > 0)
            if name == "x":
                dm = np.stack([-xi * m[2], 0.0 * m[0], xi * m[0]])
            else:
                dm = np.stack([0.0 * m[0], -xi * m[2], xi * m[1]])
            ghost = m + sgn * d * dm
            out.append((np.where(real, nb, ghost), real, sgn, name))
    return out


def dmi_field(m, region, params, cell, pbc=(0, 0, 0)):
    """Induced (interfacial) DMI field (T), Eq. eqBDMI with central differences:
    B = 2D/Msat (dm_z/dx, dm_z/dy, -dm_x/dx - dm_y/dy), dm/di = (m_{i+1} - m_{i-1})/(2 Delta_i),
    a missing neighbour replaced by its boundary ghost (_dmi_neighbours).
    Zero without the "dind" table or where Msat = 0."""
    m = np.asarray(m, dtype=np.float64)
    if "dind" not in params:
        return np.zeros_like(m)
    msat = _lut(params, "msat", region)
    pre = np.where(msat > 0, 2.0 * _lut(params, "dind", region) / np.where(msat > 0, msat, 1.0), 0.0)
    (xm, _, _, _), (xp, _, _, _), (ym, _, _, _), (yp, _, _, _) = _dmi_neighbours(m, region, params, cell, pbc)
    dx, dy = cell[0], cell[1]
    dmz_dx = (xp[2] - xm[2]) / (2 * dx)
    dmz_dy = (yp[2] - ym[2]) / (2 * dy)
    dmx_dx = (xp[0] - xm[0]) / (2 * dx)
    dmy_dy = (yp[1] - ym[1]) / (2 * dy)
    return pre * np.stack([dmz_dx, dmz_dy, -dmx_dx - dmy_dy])


def dmi_boundary_exchange(m, region, params, cell, pbc=(0, 0, 0)):
    """The exchange field's share of the DMI boundary rule ("applied to the
    Heisenberg exchange field" as well): each missing in-plane neighbour
    contributes 2A/Msat (ghost - m)/Delta^2 of the cell's own region, where
    without DMI it contributes nothing."""
    m = np.asarray(m, dtype=np.float64)
    if "dind" not in params:
        return np.zeros_like(m)
    c_self = exchange_coefficient(params, region, region)
    B = np.zeros_like(m)
    for val, real, sgn, name in _dmi_neighbours(m, region, params, cell, pbc):
        d = cell[0] if name == "x" else cell[1]
        B += np.where(real, 0.0, c_self * (val - m) / (d * d))
    return B


def anisotropy_field_parts(m, region, params):
    """Uniaxial anisotropy field split as (Ku1 part, Ku2 part), in tesla.

    B = (2 Ku1 / Msat)(u.m) u + (4 Ku2 / Msat)(u.m)^3 u.  The paper prints
    B_sat in the denominator; Msat is the reading that has units of tesla
    and satisfies the paper's energy identity E = -Ku1 (u.m)^2 - Ku2 (u.m)^4."""
    m = np.asarray(m, dtype=np.float64)
    msat = _lut(params, "msat", region)
    u = np.moveaxis(np.asarray(params["anis_u"], dtype=np.float64)[region], -1, 0)
    inv = np.where(msat > 0, 1.0 / np.where(msat > 0, msat, 1.0), 0.0)
    um = np.sum(u * m, axis=0)
    b1 = 2.0 * _lut(params, "ku1", region) * inv * um * u
    b2 = 4.0 * _lut(params, "ku2", region) * inv * um ** 3 * u
    return b1, b2


def cubic_axes(params, region):
    """(c1, c2, c3) per cell [3, ...]: the given axes normalised, c3 = c1 x c2
    (section "Magneto-crystalline anisotropy", paragraph "Cubic")."""
    c1 = np.asarray(params["anis_c1"], dtype=np.float64)
    c2 = np.asarray(params["anis_c2"], dtype=np.float64)
    n1 = np.linalg.norm(c1, axis=-1, keepdims=True)
    n2 = np.linalg.norm(c2, axis=-1, keepdims=True)
    c1 = np.where(n1 > 0, c1 / np.where(n1 > 0, n1, 1.0), 0.0)
    c2 = np.where(n2 > 0, c2 / np.where(n2 > 0, n2, 1.0), 0.0)
    c3 = np.cross(c1, c2)
    return tuple(np.moveaxis(c[region], -1, 0) for c in (c1, c2, c3))


def cubic_anisotropy_field_parts(m, region, params):
    """Cubic anisotropy field split by constant (Kc1, Kc2, Kc3 parts), tesla,
    as the paper's equation for B_anis writes it term by term:

      -2 Kc1/Msat [((c2.m)^2 + (c3.m)^2)(c1.m) c1 + ((c1.m)^2 + (c3.m)^2)(c2.m) c2
                   + ((c1.m)^2 + (c2.m)^2)(c3.m) c3]
      -2 Kc2/Msat [(c2.m)^2 (c3.m)^2 (c1.m) c1 + (c1.m)^2 (c3.m)^2 (c2.m) c2
                   + (c1.m)^2 (c2.m)^2 (c3.m) c3]
      -4 Kc3/Msat [((c2.m)^4 + (c3.m)^4)(c1.m)^3 c1 + ((c1.m)^4 + (c3.m)^4)(c2.m)^3 c2
                   + ((c1.m)^4 + (c2.m)^4)(c3.m)^3 c3]

    params may lack the cubic keys ("kc" [256, 3], "anis_c1", "anis_c2"):
    then all three parts are zero."""
    m = np.asarray(m, dtype=np.float64)
    if "kc" not in params:
        z = np.zeros_like(m)
        return z, z, z
    c1, c2, c3 = cubic_axes(params, region)
    msat = _lut(params, "msat", region)
    inv = np.where(msat > 0, 1.0 / np.where(msat > 0, msat, 1.0), 0.0)
    kc = np.moveaxis(np.asarray(params["kc"], dtype=np.float64)[region], -1, 0)
    d1, d2, d3 = (np.sum(c * m, axis=0) for c in (c1, c2, c3))
    b1 = -2.0 * kc[0] * inv * ((d2 ** 2 + d3 ** 2) * d1 * c1 + (d1 ** 2 + d3 ** 2) * d2 * c2
                                + (d1 ** 2 + d2 ** 2) * d3 * c3)
    b2 = -2.0 * kc[1] * inv * (d2 ** 2 * d3 ** 2 * d1 * c1 + d1 ** 2 * d3 ** 2 * d2 * c2
                                + d1 ** 2 * d2 ** 2 * d3 * c3)
    b3 = -4.0 * kc[2] * inv * ((d2 ** 4 + d3 ** 4) * d1 ** 3 * c1 + (d1 ** 4 + d3 ** 4) * d2 ** 3 * c2
                                + (d1 ** 4 + d2 ** 4) * d3 ** 3 * c3)
    return b1, b2, b3


def zeeman_field(region, params):
    """Applied field B_ext of each cell's region (T), paper section "Landau-Lifshitz torque"."""
    b = np.moveaxis(np.asarray(params["bext"], dtype=np.float64)[region], -1, 0)
    return b * (_lut(params, "msat", region) > 0)


def magnetisation(m, region, params):
    """M = Msat m (A/m)."""
    return _lut(params, "msat", region) * np.asarray(m, dtype=np.float64)


class Problem:
    """A grid with its materials: evaluates B_eff, the torque and the energies.

    grid = (nx, ny, nz), cell = (dx, dy, dz) in metres; demag=False drops the
    magnetostatic term (the paper's EnableDemag = false)."""

    def __init__(self, grid, cell, region, params, demag=True, workers=None, pbc=(0, 0, 0)):
        self.grid = tuple(int(v) for v in grid)
        self.cell = tuple(float(v) for v in cell)
        self.region = np.asarray(region, dtype=np.uint8).reshape(self.grid[::-1])
        self.params = params
        self.demag = demag
        self.workers = workers
        self.pbc = tuple(int(v) for v in pbc)
        self.gamma = float(params.get("gamma_ll", 0.0) or GAMMA_LL)
        self.periodic = any(p > 0 for p in self.pbc)
        self.octant = None
        self.window = None
        if demag and self.periodic:
            self.window = _demag.tensor_window(self.grid, self.cell, self.pbc)
        elif demag:
            self.octant = _demag.tensor_octant(self.grid, self.cell)
        self.magnetic = _lut(params, "msat", self.region) > 0

    # -- field terms ---------------------------------------------------------
    def demag_field(self, m):
        if not self.demag:
            return np.zeros((3,) + self.region.shape)
        M = magnetisation(m, self.region, self.params)
        if self.periodic:
            return _demag.demag_field_fft_pbc(M, self.window, self.pbc, workers=self.workers)
        return _demag.demag_field_fft(M, self.octant, workers=self.workers)

    def terms(self, m):
        """Dict of the field terms at m: demag, exch (Heisenberg exchange plus the
        induced DMI, with the DMI boundary rule, section "Dzyaloshinskii-Moriya
        interaction": its energy is -1/2 M.B like the exchange's), anis1, anis2,
        cubic1..3, zeeman (T)."""
        b1, b2 = anisotropy_field_parts(m, self.region, self.params)
        c1, c2, c3 = cubic_anisotropy_field_parts(m, self.region, self.params)
        return {
            "demag": self.demag_field(m),
            "exch": exchange_field(m, self.region, self.params, self.cell, self.pbc)
            + dmi_boundary_exchange(m, self.region, self.params, self.cell, self.pbc)
            + dmi_field(m, self.region, self.params, self.cell, self.pbc),
            "anis1": b1,
            "anis2": b2,
            "cubic1": c1,
            "cubic2": c2,
            "cubic3": c3,
            "zeeman": zeeman_field(self.region, self.params),
        }

    excitations = ()

    def excitation_field(self, t):
        """Sum of the excitation terms f_k(t) g_k(r) at time t (section "Material
        Regions", paragraph "Time-dependent parameters"): each term is
        (g [3, nz, ny, nx] in T, a, b, omega, phi) with f(t) = a + b sin(omega t + phi)."""
        out = np.zeros((3,) + self.region.shape)
        for g, a, b, w, phi in self.excitations:
            out += (a + b * np.sin(w * t + phi)) * np.asarray(g, dtype=np.float64)
        return out

    def beff(self, m, extra=None, t=None):
        """Effective field (T); zero in cells with Msat = 0.  `extra` (e.g. the
        thermal field, section "Thermal fluctuations") is added as is; with a
        time t the excitation terms at t are added too."""
        terms = self.terms(m)
        b = terms["demag"] + terms["exch"] + terms["anis1"] + terms["anis2"] + terms["zeeman"] \
            + terms["cubic1"] + terms["cubic2"] + terms["cubic3"]
        if extra is not None:
            b = b + extra
        if t is not None and self.excitations:
            b = b + self.excitation_field(t)
        return b * self.magnetic

    def torque(self, m, precess=True, extra=None, t=None):
        """Landau-Lifshitz torque (1/s), paper Eq. eqLLG with the sign that damps.

        tau = -gamma/(1+alpha^2) [m x B + alpha m x (m x B)]; with precess=False
        (relax, section "Energy minimization") the m x B term is dropped."""
        return llg_torque(m, self.beff(m, extra, t), _lut(self.params, "alpha", self.region),
                          self.gamma, precess) * self.magnetic

    def torque_at(self, m, t):
        """The torque at time t (excitations evaluated at t)."""
        return self.torque(m, True, None, t)

    def energy(self, m):
        """Energies (J) from the fields, paper Eqs. for E_demag, E_exch, E_anis.

        E = V sum[-1/2 M.B_demag - 1/2 M.B_exch - 1/2 M.B_anis(Ku1)
                  - 1/4 M.B_anis(Ku2) - 1/4 M.B_anis(Kc1) - 1/6 M.B_anis(Kc2)
                  - 1/8 M.B_anis(Kc3) - M.B_ext], summed with math.fsum (the
        cubic weights: Eq. EanisCM)."""
        t = self.terms(m)
        M = magnetisation(m, self.region, self.params)
        vol = self.cell[0] * self.cell[1] * self.cell[2]
        dens = {
            "demag": -0.5 * np.sum(M * t["demag"], axis=0),
            "exch": -0.5 * np.sum(M * t["exch"], axis=0),
            "anis": -0.5 * np.sum(M * t["anis1"], axis=0) - 0.25 * np.sum(M * t["anis2"], axis=0)
            - 0.25 * np.sum(M * t["cubic1"], axis=0) - np.sum(M * t["cubic2"], axis=0) / 6.0
            - 0.125 * np.sum(M * t["cubic3"], axis=0),
            "zeeman": -np.sum(M * t["zeeman"], axis=0),
        }
        e = {k: vol * math.fsum(v[self.magnetic].ravel()) for k, v in dens.items()}
        e["total"] = math.fsum(e.values())
        return e


def llg_torque(m, B, alpha, gamma=GAMMA_LL, precess=True):
    """tau = -gamma/(1+alpha^2) [m x B + alpha m x (m x B)] (precession term optional)."""
    m = np.asarray(m, dtype=np.float64)
    mxb = np.cross(m, B, axis=0)
    mxmxb = np.cross(m, mxb, axis=0)
    pre = -gamma / (1.0 + alpha * alpha)
    if precess:
        return pre * (mxb + alpha * mxmxb)
    return pre * alpha * mxmxb
