"""Pins of the oracle's demagnetising tensor and convolution (CPU only).

Paper section "Magnetostatic field": cube factors of 1/3 (table tabCube),
long-range point-dipole limit (figure figLong), FFT convolution.
"""
import math
import os

import mpmath as mp
import numpy as np
import pytest

from oracle import demag
from oracle.constants import MU0
from tests.aharoni import prism_factors

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _box_average(grid, cell):
    """(1/Nc) sum over all ordered cell pairs of N(r_i - r_j): the box tensor."""
    nx, ny, nz = grid
    full = demag.tensor_full(demag.tensor_octant(grid, cell))
    cnt = np.einsum("k,j,i->kji", *[n - np.abs(np.arange(-(n - 1), n)) for n in (nz, ny, nx)])
    return full.reshape(6, -1) @ cnt.ravel() / (nx * ny * nz)


def test_self_term_trace_is_one():
    for cell in [(1, 1, 1), (1, 2, 3), (5e-9, 5e-9, 8e-9), (1, 1, 1 / 64), (8, 1, 1)]:
        t = demag.tensor_at(0.0, 0.0, 0.0, cell)
        assert abs(t["xx"] + t["yy"] + t["zz"] - 1.0) < 1e-13
        for c in ("xy", "xz", "yz"):
            assert abs(t[c]) < 1e-15


def test_self_term_equals_prism_factor():
    for cell in [(1, 2, 3), (2e-9, 3e-9, 0.5e-9), (1, 1, 0.1)]:
        t = demag.tensor_at(0.0, 0.0, 0.0, cell)
        dx, dy, dz = prism_factors(*cell)
        assert t["xx"] == pytest.approx(dx, rel=1e-12, abs=1e-14)
        assert t["yy"] == pytest.approx(dy, rel=1e-12, abs=1e-14)
        assert t["zz"] == pytest.approx(dz, rel=1e-12, abs=1e-14)


@pytest.mark.parametrize("grid,cell", [
    ((2, 2, 2), (1.0, 1.0, 1.0)),
    ((4, 4, 4), (0.25, 0.25, 0.25)),
    ((3, 4, 5), (1.0, 0.7, 1.3)),
    ((12, 12, 12), (1.0, 1.0, 1.0)),     # reaches the quadrature branch
    ((16, 8, 1), (1.0, 2.0, 2.0)),
])
def test_box_average_equals_prism(grid, cell):
    avg = _box_average(grid, cell)
    ref = prism_factors(grid[0] * cell[0], grid[1] * cell[1], grid[2] * cell[2])
    np.testing.assert_allclose(avg[:3], ref, rtol=0, atol=2e-12)
    np.testing.assert_allclose(avg[3:], 0.0, atol=1e-13)


def test_table_cube_aspects():
    """The paper's cube test (appendix script for table tabCube): a unit cube cut
    into aspect x aspect x 1 (flat) or 1 x 1 x aspect (elongated) cells.  The
    exact factor is 1/3; the paper's printed values (golden file) must lie
    within the 3-4 digits it claims of what the oracle returns."""
    golden = {}
    with open(os.path.join(GOLDEN, "tab_cube.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                a, nxx, nyy, nzz = line.split()
                golden[a] = (-float(nxx), -float(nyy), -float(nzz))
    for p in range(7):
        a = 2 ** p
        avg = _box_average((a, a, 1), (1.0 / a, 1.0 / a, 1.0))
        np.testing.assert_allclose(avg[:3], 1.0 / 3.0, rtol=0, atol=1e-9)
        if "1/%d" % a in golden:
            np.testing.assert_allclose(avg[:3], golden["1/%d" % a], rtol=2e-3)
    for p in range(4):
        a = 2 ** p
        avg = _box_average((1, 1, a), (1.0, 1.0, 1.0 / a))
        np.testing.assert_allclose(avg[:3], 1.0 / 3.0, rtol=0, atol=1e-11)
        if "%d/1" % a in golden:
            np.testing.assert_allclose(avg[:3], golden["%d/1" % a], rtol=2e-3)


def _newell_mp(comp, X, Y, Z, dx, dy, dz, dps=60):
    """Newell's closed form evaluated with 60 significant digits (mpmath)."""
    mp.mp.dps = dps

    def f(x, y, z):
        x2, y2, z2 = x * x, y * y, z * z
        r = mp.sqrt(x2 + y2 + z2)
        o = (2 * x2 - y2 - z2) * r / 6
        if x2 + z2 > 0:
            o += y * (z2 - x2) * mp.asinh(y / mp.sqrt(x2 + z2)) / 2
        if x2 + y2 > 0:
            o += z * (y2 - x2) * mp.asinh(z / mp.sqrt(x2 + y2)) / 2
        if x != 0:
            o -= x * y * z * mp.atan(y * z / (x * r))
        return o

    def g(x, y, z):
        x2, y2, z2 = x * x, y * y, z * z
        r = mp.sqrt(x2 + y2 + z2)
        o = -x * y * r / 3
        if x2 + y2 > 0:
            o += x * y * z * mp.asinh(z / mp.sqrt(x2 + y2))
        if y2 + z2 > 0:
            o += y * (3 * z2 - y2) * mp.asinh(x / mp.sqrt(y2 + z2)) / 6
        if x2 + z2 > 0:
            o += x * (3 * z2 - x2) * mp.asinh(y / mp.sqrt(x2 + z2)) / 6
        if z != 0:
            o -= z2 * z * mp.atan(x * y / (z * r)) / 6
        if y != 0:
            o -= z * y2 * mp.atan(x * z / (y * r)) / 2
        if x != 0:
            o -= z * x2 * mp.atan(y * z / (x * r)) / 2
        return o

    X, Y, Z, dx, dy, dz = (mp.mpf(v) for v in (X, Y, Z, dx, dy, dz))
    fun, (a, b, c, da, db, dc) = {
        "xx": (f, (X, Y, Z, dx, dy, dz)), "yy": (f, (Y, X, Z, dy, dx, dz)),
        "zz": (f, (Z, Y, X, dz, dy, dx)), "xy": (g, (X, Y, Z, dx, dy, dz)),
        "xz": (g, (X, Z, Y, dx, dz, dy)), "yz": (g, (Y, Z, X, dy, dz, dx)),
    }[comp]
    w = {-1: -1, 0: 2, 1: -1}
    s = mp.mpf(0)
    for p in (-1, 0, 1):
        for q in (-1, 0, 1):
            for r in (-1, 0, 1):
                s += w[p] * w[q] * w[r] * fun(a + p * da, b + q * db, c + r * dc)
    return s / (4 * mp.pi * dx * dy * dz)


@pytest.mark.parametrize("cell", [(1.0, 1.0, 1.0), (1.0, 0.6, 1.7)])
def test_tensor_against_60_digit_newell(cell):
    """Both branches, at distances from touching cells to far away, agree with
    Newell's exact formula evaluated in 60-digit arithmetic."""
    rng = np.random.default_rng(7)
    diag = math.sqrt(sum(c * c for c in cell))
    for rho in [0.5, 1.5, 2.9, 3.1, 5.0, 8.0, 15.0, 40.0, 120.0]:
        v = rng.standard_normal(3)
        v = v / np.linalg.norm(v) * rho * diag
        # snap to the lattice of cell displacements
        X, Y, Z = (round(v[i] / cell[i]) * cell[i] for i in range(3))
        t = demag.tensor_at(X, Y, Z, cell)
        scale = max(abs(float(t[c])) for c in demag.COMPONENTS)
        for comp in demag.COMPONENTS:
            ref = float(_newell_mp(comp, X, Y, Z, *cell))
            assert abs(float(t[comp]) - ref) <= 2e-11 * scale, (rho, comp, float(t[comp]), ref)


def test_branches_agree_at_switch_radius():
    cell = (1.0, 1.0, 1.0)
    diag = math.sqrt(3.0)
    for direction in [(1, 0, 0), (1, 1, 0), (1, 1, 1), (0.3, 0.2, 0.93)]:
        d = np.asarray(direction, float) / np.linalg.norm(direction) * demag.R_SW * diag
        near = demag.tensor_newell(*d, *cell)
        far = demag.tensor_quadrature(*d, *cell, int(demag.quadrature_order(demag.R_SW)))
        scale = max(abs(near[c]) for c in demag.COMPONENTS)
        for c in demag.COMPONENTS:
            assert abs(near[c] - far[c]) < 1e-11 * scale


def test_parities_and_symmetry():
    cell = (1.0, 0.8, 1.2)
    rng = np.random.default_rng(3)
    for _ in range(20):
        i, j, k = rng.integers(0, 9, 3)
        base = demag.tensor_at(i * cell[0], j * cell[1], k * cell[2], cell)
        scale = max(abs(float(base[c])) for c in demag.COMPONENTS)
        for sx, sy, sz in [(-1, 1, 1), (1, -1, 1), (1, 1, -1), (-1, -1, -1)]:
            t = demag.tensor_at(sx * i * cell[0], sy * j * cell[1], sz * k * cell[2], cell)
            for c in demag.COMPONENTS:
                px, py, pz = demag.PARITY[c]
                sign = (px if sx < 0 else 1) * (py if sy < 0 else 1) * (pz if sz < 0 else 1)
                assert t[c] == pytest.approx(sign * base[c], rel=1e-12, abs=1e-12 * scale)
    # N_ij = N_ji: xy from g(x, y, z) equals yx from g(y, x, z) (g symmetric in x, y)
    a = demag.newell_g(1.3, 0.4, 0.7)
    b = demag.newell_g(0.4, 1.3, 0.7)
    assert a == pytest.approx(b, rel=1e-14)


def test_far_field_is_point_dipole():
    """Paper figure figLong: far from a cell the kernel is the dipole field."""
    cell = (1e-9, 1e-9, 1e-9)
    V = 1e-27
    for r_cells, direction in [(300, (1, 0, 0)), (500, (0.6, 0.8, 0)), (1000, (0.48, 0.6, 0.64))]:
        u = np.asarray(direction, float)
        u /= np.linalg.norm(u)
        d = u * r_cells * 1e-9
        t = demag.tensor_at(*d, cell)
        r = np.linalg.norm(d)
        dip = -V / (4 * np.pi * r ** 3) * (3 * np.outer(u, u) - np.eye(3))
        got = np.array([[t["xx"], t["xy"], t["xz"]], [t["xy"], t["yy"], t["yz"]],
                        [t["xz"], t["yz"], t["zz"]]])
        assert np.max(np.abs(got - dip)) < 5.0 / r_cells ** 2 * np.max(np.abs(dip))


def _tiny(grid, seed):
    rng = np.random.default_rng(seed)
    nx, ny, nz = grid
    M = rng.standard_normal((3, nz, ny, nx)) * 8e5
    return M


@pytest.mark.parametrize("grid,cell", [
    ((5, 3, 2), (2e-9, 3e-9, 1e-9)),
    ((8, 8, 4), (4e-9, 4e-9, 4e-9)),
    ((7, 1, 1), (1e-9, 1e-9, 1e-9)),
    ((1, 6, 3), (1e-9, 2e-9, 1e-9)),
    ((9, 6, 1), (3e-9, 3e-9, 1e-9)),
])
def test_fft_convolution_equals_direct_sum(grid, cell):
    M = _tiny(grid, 11)
    octant = demag.tensor_octant(grid, cell)
    b_fft = demag.demag_field_fft(M, octant)
    b_dir = demag.demag_field_direct(M, octant)
    np.testing.assert_allclose(b_fft, b_dir, rtol=0, atol=1e-12 * np.max(np.abs(b_dir)))


def test_direct_sum_of_uniform_box_is_prism_field():
    """Average B of a uniformly magnetised box = -mu0 N_box M (Aharoni)."""
    grid, cell = (6, 4, 3), (1e-9, 1.5e-9, 2e-9)
    nx, ny, nz = grid
    octant = demag.tensor_octant(grid, cell)
    ref = prism_factors(nx * cell[0], ny * cell[1], nz * cell[2])
    for axis in range(3):
        M = np.zeros((3, nz, ny, nx))
        M[axis] = 1.0 / MU0          # B_sat = 1 T
        B = demag.demag_field_fft(M, octant)
        assert np.mean(B[axis]) == pytest.approx(-ref[axis], abs=1e-12)


def test_long_range_single_cell():
    """Appendix script for figure figLong: one 1 nm^3 cell with B_sat = 1 T in a
    512 x 1 x 1 grid; its field along x equals -N_xx(x) and tends to the
    dipole 2 V / (4 pi x^3) (in tesla)."""
    grid, cell = (512, 1, 1), (1e-9, 1e-9, 1e-9)
    octant = demag.tensor_octant(grid, cell)
    M = np.zeros((3, 1, 1, 512))
    M[0, 0, 0, 0] = 1.0 / MU0
    B = demag.demag_field_fft(M, octant)
    np.testing.assert_allclose(B[0, 0, 0], -octant[0, 0, 0], rtol=0, atol=1e-15)
    x = np.arange(100, 512) * 1e-9
    dip = 2e-27 / (4 * np.pi * x ** 3)
    np.testing.assert_allclose(B[0, 0, 0, 100:], dip, rtol=2e-4)
