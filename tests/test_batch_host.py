"""Ensemble entry points, host side only (no call reaches the GPU): argument
validation of mm_batch_create, and the seeded ensemble workload."""
import ctypes
import os

import numpy as np
import pytest

from paper_1406_7635_amd import build as mmbuild
from paper_1406_7635_amd import mm, synth


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(mm.LIB_PATH):
        mmbuild.build()
    return mm.load()


def _create(lib, grids, region=0x1000):
    n = len(grids)
    g = (mm.Grid * max(n, 1))()
    p = (mm.Params * max(n, 1))()
    for i, (nx, ny, nz, *rest) in enumerate(grids):
        pbc = rest[0] if rest else (0, 0, 0)
        g[i] = mm.Grid(nx, ny, nz, 2e-9, 2e-9, 2e-9, (ctypes.c_int32 * 3)(*pbc))
        p[i] = mm.params_struct(synth.material(8e5, 1.3e-11, alpha=0.1))
    h = ctypes.c_void_p()
    return lib.mm_batch_create(ctypes.byref(h), n, g, p, ctypes.c_void_p(region), None)


def test_batch_create_rejects_before_touching_the_device(lib):
    assert _create(lib, [], region=0x1000) == -1                     # n = 0
    assert _create(lib, [(64, 64, 1)], region=0) == -1               # no region map
    assert _create(lib, [(64, 64, 1), (600, 64, 1)]) == -4           # nx > 512
    assert _create(lib, [(64, 64, 9)]) == -4                         # nz > 8
    assert _create(lib, [(16, 64, 1)]) == -4                         # padded x length 32 < 64
    assert _create(lib, [(64, 64, 1, (1, 0, 0))]) == -4              # periodic
    assert _create(lib, [(0, 64, 1)]) == -1


def test_ensemble_workload_is_seeded_and_in_range():
    a = synth.ensemble(n=64, seed=4)
    b = synth.ensemble(n=64, seed=4)
    assert len(a) == 64
    for x, y in zip(a, b):
        assert x["grid"] == y["grid"] and np.array_equal(x["m0"], y["m0"])
        nx, ny, nz = x["grid"]
        assert nx in (32, 64, 128, 256) and ny in (32, 64, 128, 256) and nz in (1, 2)
        d = x["cell"][0]
        assert x["cell"] == (d, d, d) and 2e-9 <= d <= 5e-9
        p = x["params"]
        assert 4e5 <= p["msat"][0] <= 1.2e6 and 5e-12 <= p["aex"][0] <= 2e-11 and 0.005 <= p["alpha"][0] <= 0.5
        assert np.all(p["msat"][1:] == 0) and not np.any(x["region"])
        assert np.allclose(np.sum(x["m0"].astype(np.float64) ** 2, axis=0), 1.0, atol=1e-6)
    # both axis sizes and both layer counts occur, drawn independently
    grids = [m["grid"] for m in synth.ensemble(n=512, seed=4)]
    assert len({g[0] for g in grids}) == 4 and len({g[1] for g in grids}) == 4 and len({g[2] for g in grids}) == 2
    assert any(g[0] != g[1] for g in grids)
