"""Demagnetising tensor and magnetostatic convolution (oracle, FP64, CPU).

Paper: section "Magnetostatic field" -- the demag field is the discrete
convolution B_demag,i = K_ij * M_j with M = Msat m; the kernel assumes a
uniform magnetisation inside every finite-difference cell and averages the
resulting field over the destination cell ("Magnetostatic kernel").

Conventions used throughout this module
---------------------------------------
* Arrays are indexed [z, y, x] (x fastest), vector fields [3, z, y, x].
* N(d) is the dimensionless cell-averaged demagnetising tensor between two
  cells separated by d = (i dx, j dy, k dz): H = -N M, so N(0) has trace 1
  and a lone cube has N = I/3 (the paper's table "tabCube" prints -N).
  The convolution kernel of the paper is K = -mu0 N, giving B in tesla.
* Component order xx, yy, zz, xy, xz, yz.

How N(d) is evaluated
---------------------
Near a cell the cell-pair average has the closed form of Newell, Williams and
Dunlop (1993): a weighted 27-point second difference of the functions f
(diagonal) and g (off-diagonal) taken on the lattice of corner offsets.  It is
the exact value of the integral the paper evaluates numerically, but it
cancels catastrophically at large |d| (relative error ~1e-16 (|d|/a)^6).
Far away (|d| >= R_SW cell diagonals) the oracle integrates the point-dipole
tensor against the triangular density of (destination - source) positions
with Gauss-Legendre quadrature on each half of every axis, the number of
points growing as the cells get closer -- the paper's "number of integration
points chosen by distance".  Both branches approximate the same integral;
tests pin them against each other at the switch radius, against a
60-digit evaluation of Newell's formula, and against the closed forms.
"""
import numpy as np
import scipy.fft

from .constants import MU0

COMPONENTS = ("xx", "yy", "zz", "xy", "xz", "yz")
# parity of each component under d_x -> -d_x, d_y -> -d_y, d_z -> -d_z
PARITY = {
    "xx": (1, 1, 1), "yy": (1, 1, 1), "zz": (1, 1, 1),
    "xy": (-1, -1, 1), "xz": (-1, 1, -1), "yz": (1, -1, -1),
}

R_SW = 2.5  # near/far switch radius, in cell diagonals


def _safe_div(a, b):
    return a / np.where(b != 0, b, 1.0)


def newell_f(x, y, z):
    """Newell's f(x, y, z) (generator of the diagonal element along x)."""
    x = np.asarray(x, dtype=np.float64)
    x2, y2, z2 = x * x, y * y, z * z
    r = np.sqrt(x2 + y2 + z2)
    rxz = np.sqrt(x2 + z2)
    rxy = np.sqrt(x2 + y2)
    out = (2.0 * x2 - y2 - z2) * r / 6.0
    out = out + np.where(rxz > 0, 0.5 * y * (z2 - x2) * np.arcsinh(_safe_div(y, rxz)), 0.0)
    out = out + np.where(rxy > 0, 0.5 * z * (y2 - x2) * np.arcsinh(_safe_div(z, rxy)), 0.0)
    xr = x * r
    out = out - np.where(xr != 0, x * y * z * np.arctan(_safe_div(y * z, xr)), 0.0)
    return out


def newell_g(x, y, z):
    """Newell's g(x, y, z) (generator of the off-diagonal element xy)."""
    x = np.asarray(x, dtype=np.float64)
    x2, y2, z2 = x * x, y * y, z * z
    r = np.sqrt(x2 + y2 + z2)
    rxy = np.sqrt(x2 + y2)
    ryz = np.sqrt(y2 + z2)
    rxz = np.sqrt(x2 + z2)
    out = -x * y * r / 3.0
    out = out + np.where(rxy > 0, x * y * z * np.arcsinh(_safe_div(z, rxy)), 0.0)
    out = out + np.where(ryz > 0, y / 6.0 * (3.0 * z2 - y2) * np.arcsinh(_safe_div(x, ryz)), 0.0)
    out = out + np.where(rxz > 0, x / 6.0 * (3.0 * z2 - x2) * np.arcsinh(_safe_div(y, rxz)), 0.0)
    zr, yr, xr = z * r, y * r, x * r
    out = out - np.where(zr != 0, z2 * z / 6.0 * np.arctan(_safe_div(x * y, zr)), 0.0)
    out = out - np.where(yr != 0, z * y2 / 2.0 * np.arctan(_safe_div(x * z, yr)), 0.0)
    out = out - np.where(xr != 0, z * x2 / 2.0 * np.arctan(_safe_div(y * z, xr)), 0.0)
    return out


_W = {-1: -1.0, 0: 2.0, 1: -1.0}


def _newell_sum(fun, a, b, c, da, db, dc):
    """Weighted 27-point sum prod_axis (2 delta_0 - delta_{+-1}) of fun, over 4 pi da db dc."""
    s = 0.0
    for p in (-1, 0, 1):
        for q in (-1, 0, 1):
            for r in (-1, 0, 1):
                s = s + _W[p] * _W[q] * _W[r] * fun(a + p * da, b + q * db, c + r * dc)
    return s / (4.0 * np.pi * da * db * dc)


def tensor_newell(X, Y, Z, dx, dy, dz):
    """All six N components at displacements (X, Y, Z) from Newell's closed form."""
    return {
        "xx": _newell_sum(newell_f, X, Y, Z, dx, dy, dz),
        "yy": _newell_sum(newell_f, Y, X, Z, dy, dx, dz),
        "zz": _newell_sum(newell_f, Z, Y, X, dz, dy, dx),
        "xy": _newell_sum(newell_g, X, Y, Z, dx, dy, dz),
        "xz": _newell_sum(newell_g, X, Z, Y, dx, dz, dy),
        "yz": _newell_sum(newell_g, Y, Z, X, dy, dz, dx),
    }


def _half_axis_nodes(h, n):
    """Nodes and weights on [-h, h] for the triangular density (h - |s|)/h^2."""
    xi, wi = np.polynomial.legendre.leggauss(n)
    s = 0.5 * h * (1.0 + xi)
    w = 0.5 * h * wi * (h - s) / (h * h)
    return np.concatenate([-s[::-1], s]), np.concatenate([w[::-1], w])


def tensor_quadrature(X, Y, Z, dx, dy, dz, n):
    """All six N components by 2n-point-per-axis quadrature of the dipole tensor.

    N_ij(d) = -(V / 4 pi) < (3 w_i w_j - |w|^2 delta_ij) / |w|^5 >, w = d + s,
    where s is distributed as the difference of two uniform points in a cell
    (product of triangular densities) and V = dx dy dz is the source volume.
    """
    sx, wx = _half_axis_nodes(dx, n)
    sy, wy = _half_axis_nodes(dy, n)
    sz, wz = _half_axis_nodes(dz, n)
    acc = {c: 0.0 for c in COMPONENTS}
    for a in range(sx.size):
        ux = X + sx[a]
        for b in range(sy.size):
            uy = Y + sy[b]
            for c in range(sz.size):
                uz = Z + sz[c]
                r2 = ux * ux + uy * uy + uz * uz
                inv5 = r2 ** -2.5
                w = wx[a] * wy[b] * wz[c]
                acc["xx"] = acc["xx"] + w * (3.0 * ux * ux - r2) * inv5
                acc["yy"] = acc["yy"] + w * (3.0 * uy * uy - r2) * inv5
                acc["zz"] = acc["zz"] + w * (3.0 * uz * uz - r2) * inv5
                acc["xy"] = acc["xy"] + w * 3.0 * ux * uy * inv5
                acc["xz"] = acc["xz"] + w * 3.0 * ux * uz * inv5
                acc["yz"] = acc["yz"] + w * 3.0 * uy * uz * inv5
    pre = -dx * dy * dz / (4.0 * np.pi)
    return {c: pre * v for c, v in acc.items()}


def quadrature_order(rho):
    """Gauss points per half axis for a displacement of rho cell diagonals.

    Chosen so the quadrature error stays below ~1e-12 relative (measured
    against a 60-digit Newell evaluation in the tests)."""
    rho = np.asarray(rho)
    n = np.full(rho.shape, 2, dtype=np.int64)
    n[rho < 400.0] = 3
    n[rho < 50.0] = 4
    n[rho < 12.0] = 5
    n[rho < 6.0] = 6
    n[rho < 4.0] = 8
    return n


def tensor_at(X, Y, Z, cell):
    """N at displacement arrays (X, Y, Z) (metres), choosing the branch per entry."""
    dx, dy, dz = cell
    X, Y, Z = np.broadcast_arrays(*(np.asarray(v, dtype=np.float64) for v in (X, Y, Z)))
    diag = np.sqrt(dx * dx + dy * dy + dz * dz)
    rho = np.sqrt(X * X + Y * Y + Z * Z) / diag
    out = {c: np.zeros(X.shape) for c in COMPONENTS}
    near = rho < R_SW
    if near.any():
        t = tensor_newell(X[near], Y[near], Z[near], dx, dy, dz)
        for c in COMPONENTS:
            out[c][near] = t[c]
    order = quadrature_order(rho)
    for n in np.unique(order[~near]):
        sel = (~near) & (order == n)
        t = tensor_quadrature(X[sel], Y[sel], Z[sel], dx, dy, dz, int(n))
        for c in COMPONENTS:
            out[c][sel] = t[c]
    return out


def tensor_octant(grid, cell):
    """N for all displacements (i dx, j dy, k dz), 0 <= i < nx etc.

    Returns an array [6, nz, ny, nx]; other octants follow by PARITY."""
    nx, ny, nz = grid
    dx, dy, dz = cell
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    t = tensor_at(i * dx, j * dy, k * dz, cell)
    return np.stack([t[c] for c in COMPONENTS])


def tensor_full(octant):
    """Expand an octant [6, nz, ny, nx] to all displacements [6, 2nz-1, 2ny-1, 2nx-1].

    Entry [c, k + nz - 1, j + ny - 1, i + nx - 1] holds N_c(i dx, j dy, k dz)."""
    _, nz, ny, nx = octant.shape
    out = np.empty((6, 2 * nz - 1, 2 * ny - 1, 2 * nx - 1))
    for ci, c in enumerate(COMPONENTS):
        px, py, pz = PARITY[c]
        a = octant[ci]
        for sz in (1, -1):
            for sy in (1, -1):
                for sx in (1, -1):
                    sign = (px if sx < 0 else 1) * (py if sy < 0 else 1) * (pz if sz < 0 else 1)
                    kk = nz - 1 + sz * np.arange(nz)
                    jj = ny - 1 + sy * np.arange(ny)
                    ii = nx - 1 + sx * np.arange(nx)
                    out[ci][np.ix_(kk, jj, ii)] = sign * a
    return out


_PAIRS = [(0, 0, 0), (1, 1, 1), (2, 2, 2), (0, 1, 3), (1, 0, 3), (0, 2, 4), (2, 0, 4), (1, 2, 5), (2, 1, 5)]


def demag_field_fft(M, octant, workers=None):
    """B_demag = -mu0 N * M by zero-padded FFT convolution (tesla).

    M: [3, nz, ny, nx] magnetisation in A/m.  Each axis of length n > 1 is
    padded to 2n - 1, the smallest length for which the cyclic convolution
    equals the linear (aperiodic) one on the physical cells."""
    _, nz, ny, nx = M.shape
    shape = tuple(2 * n - 1 for n in (nz, ny, nx))
    full = tensor_full(octant)            # displacements -(n-1) .. (n-1)
    # roll so that displacement 0 sits at index 0 (cyclic layout)
    kern = np.roll(full, shift=(-(nz - 1), -(ny - 1), -(nx - 1)), axis=(1, 2, 3))
    khat = scipy.fft.rfftn(kern, s=shape, axes=(1, 2, 3), workers=workers)
    mhat = scipy.fft.rfftn(M, s=shape, axes=(1, 2, 3), workers=workers)
    bhat = np.zeros_like(mhat)
    for i, j, c in _PAIRS:
        bhat[i] += khat[c] * mhat[j]
    b = scipy.fft.irfftn(bhat, s=shape, axes=(1, 2, 3), workers=workers)
    return -MU0 * b[:, :nz, :ny, :nx]


def demag_field_direct(M, octant):
    """B_demag by the literal double sum over source and destination cells."""
    _, nz, ny, nx = M.shape
    full = tensor_full(octant)
    B = np.zeros_like(M, dtype=np.float64)
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                # displacement destination - source for every source cell
                sub = full[:, z + nz - 1 - np.arange(nz)[:, None, None],
                           y + ny - 1 - np.arange(ny)[None, :, None],
                           x + nx - 1 - np.arange(nx)[None, None, :]]
                for i, j, c in _PAIRS:
                    B[i, z, y, x] += np.sum(sub[c] * M[j])
    return -MU0 * B


# ---------------------------------------------------------------------------
# Periodic boundary conditions by macro geometry (paper paragraph "Periodic
# boundary conditions"): along a periodic axis the magnetisation repeats with
# the box length L = n d, and a finite number P of repetitions is counted.
# Reading (pinned by the paper's tables tabPBC1 / tabPBC2, see the tests): a
# destination cell feels every source -- the box's own cells and their images
# -- whose displacement along that axis lies within +-(n P - 1) cells, the
# window of a non-periodic grid 2 n P cells long around the destination.


def window_radius(grid, pbc):
    """Largest |displacement| (cells) per axis: n P - 1 along a periodic axis
    with P images per side, n - 1 otherwise."""
    return tuple(int(n) * int(p) - 1 if p > 0 else int(n) - 1 for n, p in zip(grid, pbc))


def tensor_window(grid, cell, pbc):
    """N at every signed displacement of the window: [6, 2Rz+1, 2Ry+1, 2Rx+1],
    entry [c, k + Rz, j + Ry, i + Rx] = N_c(i dx, j dy, k dz).

    Evaluated at the signed displacement itself (no parity folding)."""
    rx, ry, rz = window_radius(grid, pbc)
    dx, dy, dz = cell
    k, j, i = np.meshgrid(np.arange(-rz, rz + 1), np.arange(-ry, ry + 1), np.arange(-rx, rx + 1), indexing="ij")
    t = tensor_at(i * dx, j * dy, k * dz, cell)
    return np.stack([t[c] for c in COMPONENTS])


def demag_field_fft_pbc(M, window, pbc, workers=None):
    """B_demag = -mu0 N * M with periodic axes (tesla), by FFT.

    Along a periodic axis the convolution is cyclic with period n: the kernel
    of the cyclic transform (length n) at index q is the sum of N over every
    window displacement congruent to q modulo n.  A non-periodic axis is
    zero-padded to 2n - 1 as in demag_field_fft.  `window` is tensor_window's
    array for the same grid and pbc."""
    _, nz, ny, nx = M.shape
    shape = tuple(n if p > 0 else 2 * n - 1 for n, p in zip((nz, ny, nx), (pbc[2], pbc[1], pbc[0])))
    _, wz, wy, wx = window.shape
    rz, ry, rx = (wz - 1) // 2, (wy - 1) // 2, (wx - 1) // 2
    dk, dj, di = np.meshgrid(np.arange(-rz, rz + 1), np.arange(-ry, ry + 1), np.arange(-rx, rx + 1), indexing="ij")
    kern = np.zeros((6,) + shape)
    for c in range(6):
        np.add.at(kern[c], (dk % shape[0], dj % shape[1], di % shape[2]), window[c])
    khat = scipy.fft.rfftn(kern, axes=(1, 2, 3), workers=workers)
    mhat = scipy.fft.rfftn(M, s=shape, axes=(1, 2, 3), workers=workers)
    bhat = np.zeros_like(mhat)
    for i, j, c in _PAIRS:
        bhat[i] += khat[c] * mhat[j]
    b = scipy.fft.irfftn(bhat, s=shape, axes=(1, 2, 3), workers=workers)
    return -MU0 * b[:, :nz, :ny, :nx]


def demag_field_direct_pbc(M, window, pbc):
    """B_demag with periodic axes by the literal sum over source cells and
    their images: image s of source r' sits at r' + s L; it counts when the
    displacement r - r' - s L lies inside the window on every axis."""
    _, nz, ny, nx = M.shape
    _, wz, wy, wx = window.shape
    R = ((wx - 1) // 2, (wy - 1) // 2, (wz - 1) // 2)
    grid = (nx, ny, nz)
    shifts = [range(-p, p + 1) if p > 0 else range(0, 1) for p in pbc]
    B = np.zeros_like(M, dtype=np.float64)
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                for zs in range(nz):
                    for ys in range(ny):
                        for xs in range(nx):
                            for sz in shifts[2]:
                                for sy in shifts[1]:
                                    for sx in shifts[0]:
                                        d = (x - xs - sx * grid[0], y - ys - sy * grid[1], z - zs - sz * grid[2])
                                        if any(abs(d[a]) > R[a] for a in range(3)):
                                            continue
                                        n = window[:, d[2] + R[2], d[1] + R[1], d[0] + R[0]]
                                        for i, j, c in _PAIRS:
                                            B[i, z, y, x] += n[c] * M[j, zs, ys, xs]
    return -MU0 * B
