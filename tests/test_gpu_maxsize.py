"""The largest transform lengths the library serves (padded length 4096,
sixteen points per thread) along each axis, and the largest periodic x
(2048 cells, the size limit of every axis) transformed without padding,
against the FP64 oracle: B_eff and the torque
over every cell (1e-5), then three accepted Dormand-Prince attempts at a
fixed step against the oracle's embedded steps (m within 2e-6).
"""
import numpy as np
import pytest

from oracle import fields as ofields
from oracle import integrate as ointegrate
from paper_1406_7635_amd import mm, synth
from tests.gpu_helpers import log, rel_inf, to_np

pytestmark = pytest.mark.gpu

CASES = [
    ((2048, 3, 1), (0, 0, 0), 4096),   # x padded to 4096
    ((5, 2048, 1), (0, 0, 0), 4096),   # y padded to 4096
    ((3, 2, 2048), (0, 0, 0), 4096),   # z padded to 4096
    ((2048, 2, 1), (1, 0, 0), 2048),   # periodic x of 2048 cells, unpadded (fused pass)
]


@pytest.mark.parametrize("grid,pbc,plen", CASES, ids=[str(c[0]) + str(c[1]) for c in CASES])
def test_maximum_lengths(gpu, grid, pbc, plen):
    import torch

    case = synth.random_problem(grid, (2e-9, 2e-9, 2e-9), seed=sum(grid) + 3, nregions=3, vacuum=True)
    ctx = mm.Context(case["grid"], case["cell"], case["region"], case["params"], pbc=pbc)
    prob = ofields.Problem(case["grid"], case["cell"], case["region"], case["params"], pbc=pbc)
    info = ctx.info()
    assert max(info["px"], info["py"], info["pz"]) == plen
    m = torch.from_numpy(np.ascontiguousarray(case["m0"])).to("cuda:0")
    m_ref = case["m0"].astype(np.float64)
    eb = rel_inf(to_np(ctx.beff(m)), prob.beff(m_ref))
    et = rel_inf(to_np(ctx.torque(m)), prob.torque(m_ref))
    log("max length", grid, pbc, "B_eff %.2e torque %.2e" % (eb, et))
    assert eb < 1e-5 and et < 1e-5
    f = prob.torque
    k1 = f(m_ref)
    t, dt = 0.0, 1e-14
    opts = mm.solver_opts(max_err=1.0)
    for _ in range(3):  # the error estimate is not compared: FP32 leaves it tens of per cent off here
        acc, t, _, err = ctx.rk45_step(m, t, dt, opts)
        assert acc
        ms, k1, eps = ointegrate.embedded_step(f, m_ref, k1, dt, ointegrate.DP45)
        m_ref = ointegrate.normalize(ms)
        d = float(np.max(np.abs(to_np(m) - m_ref)))
        log("  DP45 |dm| %.2e err %.3e / %.3e" % (d, err, eps))
        assert d < 2e-6
    ctx.close()
