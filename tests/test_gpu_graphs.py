"""Graph replay of mm_run's attempts (opt-in) against direct launches: the same
attempts, bit for bit, with eager work and synchronisations between the
replays (DP45 through the fused x passes, RK23 on a 3D grid, Heun with the
thermal field through the fused local passes)."""
import numpy as np
import pytest

from paper_1406_7635_amd import mm, synth
from tests.gpu_helpers import log, make_ctx, to_np

pytestmark = pytest.mark.gpu


def _run(case, graphs, solver, demag=True, temp=None):
    import torch

    ctx, m = make_ctx(case, demag=demag)
    ctx.set_run_graphs(graphs)
    if temp is not None:
        ctx.set_temperature(temp, 5)
    t, dt = 0.0, 2e-14
    outs = []
    for _ in range(3):
        t, dt, st = ctx.run(m, float("inf"), t=t, dt=dt, solver=solver, max_attempts=24)
        ctx.beff(m)                      # eager work between replays
        torch.cuda.synchronize()
        outs.append((to_np(m), t, dt, st["steps"], st["rejects"]))
    ctx.close()
    return outs


@pytest.mark.parametrize("grid,solver,demag,temp", [((64, 48, 1), 45, True, None), ((33, 20, 3), 23, True, None),
                                                    ((40, 30, 1), 12, False, 300.0), ((40, 30, 1), 12, True, 300.0)])
def test_graph_replays_equal_direct_launches(gpu, grid, solver, demag, temp):
    case = synth.random_problem(grid, (3e-9, 3e-9, 3e-9), seed=sum(grid), nregions=2)
    log("graph replay", grid, solver, demag, temp)
    a = _run(case, True, solver, demag, temp)
    b = _run(case, False, solver, demag, temp)
    for (ma, ta, da, sa, ra), (mb, tb, db, sb, rb) in zip(a, b):
        assert np.array_equal(ma, mb)
        assert (ta, da, sa, ra) == (tb, db, sb, rb)
