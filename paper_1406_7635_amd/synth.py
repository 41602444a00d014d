"""Seeded synthetic inputs: grids, region maps, material tables and initial m.

This module only draws inputs (numpy PCG64 generators); it computes nothing
of the micromagnetic method itself.  Both the GPU library's tests/benchmark
and the CPU oracle consume what it returns, as data.

Every builder returns a dict with keys
  grid   (nx, ny, nz)             cell  (dx, dy, dz) in metres
  region uint8 [nz, ny, nx]       params dict of 256-entry region tables
  m0     float32 [3, nz, ny, nx]  unit vectors, rounded to FP32 once
and the solver settings of the workload where it has them.
"""
import numpy as np

NREG = 256


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def empty_params(gamma_ll=1.7595e11):
    """All-zero region tables (Msat = 0 means 'no magnet') and S = 1 everywhere."""
    return {
        "msat": np.zeros(NREG), "aex": np.zeros(NREG), "alpha": np.zeros(NREG),
        "ku1": np.zeros(NREG), "ku2": np.zeros(NREG),
        "anis_u": np.tile([1.0, 0.0, 0.0], (NREG, 1)),
        "bext": np.zeros((NREG, 3)),
        "exch_scale": np.ones(NREG * (NREG + 1) // 2),
        "gamma_ll": gamma_ll,
    }


def material(msat, aex, alpha=0.0, ku1=0.0, ku2=0.0, anis_u=(1.0, 0.0, 0.0),
             bext=(0.0, 0.0, 0.0), region=0, params=None):
    """Set one region's parameters (returns the params dict)."""
    p = empty_params() if params is None else params
    p["msat"][region] = msat
    p["aex"][region] = aex
    p["alpha"][region] = alpha
    p["ku1"][region] = ku1
    p["ku2"][region] = ku2
    p["anis_u"][region] = anis_u
    p["bext"][region] = bext
    return p


def _unit(v):
    n = np.sqrt(np.sum(v * v, axis=0))
    return v / n


def random_sphere(grid, seed):
    """Unit vectors uniform on the sphere (normalised N(0,1)^3), FP32 [3, nz, ny, nx]."""
    nx, ny, nz = grid
    v = _rng(seed).standard_normal((3, nz, ny, nx))
    return _unit(v).astype(np.float32)


def uniform_m(grid, direction):
    nx, ny, nz = grid
    d = np.asarray(direction, dtype=np.float64)
    d = d / np.sqrt(np.sum(d * d))
    return np.broadcast_to(d[:, None, None, None], (3, nz, ny, nx)).astype(np.float32).copy()


def vortex(grid, cell, seed, core=10e-9, noise=0.01):
    """In-plane curl (circulation +1), core along +z, plus seeded noise.

    m = (-sin phi, cos phi, 0) sqrt(1 - mz^2) + mz z, mz = exp(-(r/core)^2),
    centred on the grid centre; then noise * N(0,1)^3 is added and the result
    is renormalised."""
    nx, ny, nz = grid
    dx, dy, _ = cell
    x = (np.arange(nx) - (nx - 1) / 2.0) * dx
    y = (np.arange(ny) - (ny - 1) / 2.0) * dy
    X, Y = np.meshgrid(x, y, indexing="xy")
    r = np.hypot(X, Y)
    phi = np.arctan2(Y, X)
    mz = np.exp(-(r / core) ** 2)
    s = np.sqrt(1.0 - mz * mz)
    v = np.stack([-np.sin(phi) * s, np.cos(phi) * s, mz])[:, None, :, :]
    v = np.broadcast_to(v, (3, nz, ny, nx)).copy()
    v += noise * _rng(seed).standard_normal(v.shape)
    return _unit(v).astype(np.float32)


def voronoi_regions(grid, cell, grain, seed):
    """3D Voronoi grains: Poisson seeds, one per grain volume grain^3.

    Each cell takes the nearest seed (FP64 distance from the cell centre);
    each seed gets a uniform random colour 0..255, reused across grains."""
    from scipy.spatial import cKDTree

    nx, ny, nz = grid
    dx, dy, dz = cell
    L = np.array([nx * dx, ny * dy, nz * dz])
    rng = _rng(seed)
    nseeds = max(1, int(round(np.prod(L) / grain ** 3)))
    pts = rng.uniform(0.0, 1.0, (nseeds, 3)) * L
    colour = rng.integers(0, NREG, nseeds)
    z, y, x = np.meshgrid((np.arange(nz) + 0.5) * dz, (np.arange(ny) + 0.5) * dy,
                          (np.arange(nx) + 0.5) * dx, indexing="ij")
    _, idx = cKDTree(pts).query(np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1))
    return colour[idx].reshape(nz, ny, nx).astype(np.uint8)


# ---------------------------------------------------------------------------
# Workloads
# ---------------------------------------------------------------------------

def parity_cube(seed=1):
    """32x32x4 cells of 4 nm, one region: Msat 8e5, Aex 1.3e-11, alpha 0.5,
    no anisotropy, no field; random m; 200 fixed RK4 steps of 1e-13 s."""
    grid, cell = (32, 32, 4), (4e-9, 4e-9, 4e-9)
    params = material(8e5, 1.3e-11, alpha=0.5)
    return {"name": "film32x32x4_rk4", "grid": grid, "cell": cell,
            "region": np.zeros(grid[::-1], dtype=np.uint8), "params": params,
            "m0": random_sphere(grid, seed), "solver": "rk4", "dt": 1e-13, "steps": 200}


def vortex_film(seed=2, n=1024):
    """n x n x 1 film of 2 nm cells: Msat 8e5, Aex 1.3e-11, alpha 0.01,
    B_ext = 10 mT along x; vortex + 1 % noise; RK45, MaxErr 1e-5, 5 ns."""
    grid, cell = (n, n, 1), (2e-9, 2e-9, 2e-9)
    params = material(8e5, 1.3e-11, alpha=0.01, bext=(0.01, 0.0, 0.0))
    return {"name": "vortex%dx%dx1_rk45" % (n, n), "grid": grid, "cell": cell,
            "region": np.zeros(grid[::-1], dtype=np.uint8), "params": params,
            "m0": vortex(grid, cell, seed), "solver": "rk45", "max_err": 1e-5, "t_end": 5e-9}


def grains(seed=3, grid=(256, 256, 64), smooth=False):
    """256x256x64 cells of 3 nm, 256 regions from a 3D Voronoi of mean grain
    (20 nm)^3: Msat ~ U(6e5, 1e6), Ku1 ~ U(0, 5e5) with random easy axes,
    Aex 1.5e-11, inter-region exchange scaled by 0.9."""
    cell = (3e-9, 3e-9, 3e-9)
    region = voronoi_regions(grid, cell, 20e-9, seed)
    rng = _rng(10 * seed)
    p = empty_params()
    p["msat"][:] = rng.uniform(6e5, 1e6, NREG)
    p["aex"][:] = 1.5e-11
    p["alpha"][:] = 0.01
    p["ku1"][:] = rng.uniform(0.0, 5e5, NREG)
    p["anis_u"][:] = _unit(rng.standard_normal((3, NREG))).T
    p["exch_scale"][:] = 0.9
    if smooth:
        tilt = 0.2 * rng.standard_normal((NREG, 3))
        d = _unit((np.array([0.0, 0.0, 1.0]) + tilt).T).T
        m0 = _unit(np.moveaxis(d[region], -1, 0)).astype(np.float32)
    else:
        m0 = random_sphere(grid, 10 * seed + 1)
    return {"name": "grains%dx%dx%d" % grid, "grid": grid, "cell": cell, "region": region,
            "params": p, "m0": m0, "solver": "rk45", "max_err": 1e-5}


def paper_bench(n):
    """The paper's throughput workload: n x n x 1 of 4 nm cells, Msat 8e5,
    Aex 13e-12, alpha 0.01, B_ext = (0, 10 mT, 0), m = (1, 0, 0), RK45."""
    grid, cell = (n, n, 1), (4e-9, 4e-9, 4e-9)
    params = material(8e5, 13e-12, alpha=0.01, bext=(0.0, 0.01, 0.0))
    return {"name": "paperbench%d" % n, "grid": grid, "cell": cell,
            "region": np.zeros(grid[::-1], dtype=np.uint8), "params": params,
            "m0": uniform_m(grid, (1, 0, 0)), "solver": "rk45", "max_err": 1e-5}


def random_problem(grid, cell, seed, nregions=3, ku=True, field=True, vacuum=False):
    """Small multi-region problem for parity tests: random materials per region,
    random S, random anisotropy axes and fields; optional vacuum cells."""
    rng = _rng(seed)
    nx, ny, nz = grid
    region = rng.integers(0, nregions, (nz, ny, nx)).astype(np.uint8)
    p = empty_params()
    p["msat"][:nregions] = rng.uniform(4e5, 1.2e6, nregions)
    p["aex"][:nregions] = rng.uniform(5e-12, 2e-11, nregions)
    p["alpha"][:nregions] = rng.uniform(0.01, 0.5, nregions)
    if ku:
        p["ku1"][:nregions] = rng.uniform(-5e5, 5e5, nregions)
        p["ku2"][:nregions] = rng.uniform(-2e5, 2e5, nregions)
        p["anis_u"][:nregions] = _unit(rng.standard_normal((3, nregions))).T
    if field:
        p["bext"][:nregions] = rng.uniform(-0.1, 0.1, (nregions, 3))
    p["exch_scale"][:] = rng.uniform(0.2, 1.2, p["exch_scale"].shape)
    if vacuum:
        p["msat"][nregions - 1] = 0.0
    return {"name": "random%dx%dx%d" % grid, "grid": grid, "cell": cell, "region": region,
            "params": p, "m0": random_sphere(grid, seed + 1000)}


def ensemble(n=512, seed=4, sizes=(32, 64, 128, 256), layers=(1, 2), t_end=1e-9):
    """Ensemble of n independent simulations: nx, ny drawn independently from
    `sizes`, nz from `layers`, cubic cells of U(2, 5) nm, one region with Msat
    ~ U(4e5, 1.2e6), Aex ~ U(5e-12, 2e-11), alpha ~ U(0.005, 0.5), no applied
    field, m0 random on the sphere (member i from sub-seed 1000 seed + i);
    DP45 with MaxErr 1e-5 to t_end.  Returns the list of member dicts."""
    rng = _rng(seed)
    members = []
    for i in range(n):
        nx, ny = (int(v) for v in rng.choice(sizes, 2))
        nz = int(rng.choice(layers))
        d = float(rng.uniform(2e-9, 5e-9))
        p = material(float(rng.uniform(4e5, 1.2e6)), float(rng.uniform(5e-12, 2e-11)),
                     alpha=float(rng.uniform(0.005, 0.5)))
        grid = (nx, ny, nz)
        members.append({"name": "member%d" % i, "grid": grid, "cell": (d, d, d),
                        "region": np.zeros((nz, ny, nx), dtype=np.uint8), "params": p,
                        "m0": random_sphere(grid, 1000 * seed + i), "solver": "rk45", "max_err": 1e-5,
                        "t_end": t_end})
    return members


# Spectral neural operator (the surrogate of the magnetostatic field): 32
# channels, kept modes kx = 0..15, ky = -8..7, four layers.  Flat weight order:
# P[32][3], p[32], then per layer R[16 ky][16 kx][32 o][32 c][re, im], W[32][32],
# b[32], then Q[3][32], q[3].
SNO_C, SNO_KX, SNO_KY, SNO_LAYERS = 32, 16, 16, 4
SNO_NWEIGHTS = SNO_C * 3 + SNO_C + SNO_LAYERS * (SNO_KY * SNO_KX * SNO_C * SNO_C * 2 + SNO_C * SNO_C + SNO_C) \
    + 3 * SNO_C + 3


def sno_random_weights(seed, scale=1.0):
    """Seeded surrogate weights in the flat order above: pointwise weights
    N(0, 1/fan_in), spectral weights N(0, 1) / C per real and imaginary part,
    small biases; float32."""
    rng = _rng(seed)
    c = SNO_C
    parts = [rng.standard_normal((c, 3)) / np.sqrt(3.0) * scale, 0.1 * rng.standard_normal(c)]
    for _ in range(SNO_LAYERS):
        parts.append(rng.standard_normal((SNO_KY, SNO_KX, c, c, 2)) * scale / c)
        parts.append(rng.standard_normal((c, c)) / np.sqrt(c) * scale)
        parts.append(0.1 * rng.standard_normal(c))
    parts += [rng.standard_normal((3, c)) / np.sqrt(c) * scale, 0.01 * rng.standard_normal(3)]
    out = np.concatenate([np.ravel(a) for a in parts]).astype(np.float32)
    assert out.size == SNO_NWEIGHTS
    return out


def film_textures(n, seed=5, grid=(256, 256), cell=4e-9, msat=8e5, aex=1.3e-11):
    """Seeded magnetisation textures on an nx x ny x 1 film, FP32 [n, 3, 1, ny, nx]:
    a mixture of (i) domains (2-6 random directions over a smooth partition
    of the plane, walls of width about pi l_ex, l_ex = sqrt(2 Aex/(mu0 Msat^2))),
    (ii) vortices with random centre, chirality and polarity, (iii) spirals
    with wavelength 8-256 nm along a random direction, each with added
    N(0, s^2) noise, s ~ U(0, 0.1), and renormalised."""
    rng = _rng(seed)
    nx, ny = grid
    y, x = np.mgrid[0:ny, 0:nx].astype(np.float64)
    x = (x + 0.5) * cell
    y = (y + 0.5) * cell
    lex = np.sqrt(2 * aex / (4e-7 * np.pi * msat * msat))
    width = np.pi * lex
    out = np.empty((n, 3, 1, ny, nx), dtype=np.float32)
    for i in range(n):
        kind = i % 3
        if kind == 0:
            k = int(rng.integers(2, 7))
            cx = rng.uniform(0, nx * cell, k)
            cy = rng.uniform(0, ny * cell, k)
            u = _unit(rng.standard_normal((3, k)))
            d = np.sqrt((x[None] - cx[:, None, None]) ** 2 + (y[None] - cy[:, None, None]) ** 2)
            w = np.exp(-(d - d.min(axis=0)) / width)
            m = np.einsum("ck,kyx->cyx", u, w / w.sum(axis=0))
        elif kind == 1:
            cx, cy = rng.uniform(0.2, 0.8) * nx * cell, rng.uniform(0.2, 0.8) * ny * cell
            chir = rng.choice([-1.0, 1.0])
            pol = rng.choice([-1.0, 1.0])
            rc = rng.uniform(1.0, 3.0) * lex
            phi = np.arctan2(y - cy, x - cx)
            r2 = (x - cx) ** 2 + (y - cy) ** 2
            mz = pol * np.exp(-r2 / (rc * rc))
            s = np.sqrt(np.maximum(0.0, 1 - mz * mz))
            m = np.stack([-chir * np.sin(phi) * s, chir * np.cos(phi) * s, mz])
        else:
            lam = np.exp(rng.uniform(np.log(8e-9), np.log(256e-9)))
            th = rng.uniform(0, 2 * np.pi)
            ph = 2 * np.pi * (np.cos(th) * x + np.sin(th) * y) / lam + rng.uniform(0, 2 * np.pi)
            a = _unit(rng.standard_normal(3))
            b = _unit(np.cross(a, rng.standard_normal(3)))
            m = a[:, None, None] * np.cos(ph)[None] + b[:, None, None] * np.sin(ph)[None]
        m = m + rng.uniform(0, 0.1) * rng.standard_normal(m.shape)
        out[i, :, 0] = _unit(m).astype(np.float32)
    return out
