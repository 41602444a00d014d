"""Demagnetising factor of a uniformly magnetised rectangular prism.

A. Aharoni, "Demagnetizing factors for rectangular ferromagnetic prisms",
J. Appl. Phys. 83, 3432 (1998), Eq. (1): D_z of a prism with sides 2a, 2b, 2c
along x, y, z.  Written independently of the oracle's Newell functions so it
can pin them: the cell-pair tensor averaged over all pairs of cells in a box
must equal the box's own factor.  The formula is itself pinned in the tests
(a cube gives 1/3, the three factors sum to 1, film and needle limits).
"""
import math


def prism_dz(a, b, c):
    """D_z for half-sides a, b, c (any positive lengths)."""
    r = math.sqrt(a * a + b * b + c * c)
    rab = math.sqrt(a * a + b * b)
    rbc = math.sqrt(b * b + c * c)
    rac = math.sqrt(a * a + c * c)
    t = 0.0
    t += (b * b - c * c) / (2 * b * c) * math.log((r - a) / (r + a))
    t += (a * a - c * c) / (2 * a * c) * math.log((r - b) / (r + b))
    t += b / (2 * c) * math.log((rab + a) / (rab - a))
    t += a / (2 * c) * math.log((rab + b) / (rab - b))
    t += c / (2 * a) * math.log((rbc - b) / (rbc + b))
    t += c / (2 * b) * math.log((rac - a) / (rac + a))
    t += 2 * math.atan(a * b / (c * r))
    t += (a ** 3 + b ** 3 - 2 * c ** 3) / (3 * a * b * c)
    t += (a * a + b * b - 2 * c * c) / (3 * a * b * c) * r
    t += c / (a * b) * (rac + rbc)
    t -= (rab ** 3 + rbc ** 3 + rac ** 3) / (3 * a * b * c)
    return t / math.pi


def prism_factors(lx, ly, lz):
    """(D_x, D_y, D_z) of a box with full side lengths lx, ly, lz."""
    a, b, c = lx / 2, ly / 2, lz / 2
    return prism_dz(b, c, a), prism_dz(c, a, b), prism_dz(a, b, c)
