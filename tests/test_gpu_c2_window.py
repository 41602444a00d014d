"""The 1024 x 1024 x 1 vortex film over its first 140 ps of Dormand-Prince
(about 1030 accepted steps) against the oracle's trajectory.

tests/golden/c2_window.txt holds the FP64 oracle's average magnetisation at
the output times k * 5 ps (k = 1..10), then every 10 ps up to 140 ps, and m at
2048 seeded cells at 140 ps (written by tests/golden/make_c2_window.py from the
oracle alone).  The
library runs the same schedule (first step 1e-14 s, MaxErr 1e-5, headroom
0.8, each segment clipped onto its output time).  Checked: <m>(t) within
1e-4 at every output time, m at the sampled cells within 1e-3, unit length
kept, and B_eff / torque of the evolved state (the library's own, after 140 ps)
against the oracle's evaluation of that same state within 1e-5.
"""
import os

import numpy as np
import pytest

from paper_1406_7635_amd import synth
from tests.gpu_helpers import log, make_pair, rel_inf, to_np

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c2_window.txt")


def _golden():
    means, cells = [], []
    for line in open(GOLDEN):
        w = line.split()
        if not w or w[0].startswith("#"):
            continue
        if w[0] == "mean":
            means.append((float(w[1]), int(w[2]), int(w[3]), np.array([float(v) for v in w[4:7]])))
        elif w[0] == "cell":
            cells.append((int(w[1]), int(w[2]), np.array([float(v) for v in w[3:6]])))
    return means, cells


@pytest.mark.skipif(not os.path.exists(GOLDEN), reason="tests/golden/c2_window.txt not generated")
def test_c2_window(gpu):
    means, cells = _golden()
    case = synth.vortex_film(seed=2, n=1024)
    ctx, prob, m = make_pair(case)
    prob.workers = -1
    t, dt = 0.0, 1e-14
    steps = 0
    for t_out, ns, nr, mref in means:
        t, dt, st = ctx.run(m, t_out, t=t, dt=dt, max_attempts=100000, opts=None)
        steps += st["steps"]
        assert t == pytest.approx(t_out, rel=1e-12)
        mean = to_np(m).reshape(3, -1).mean(axis=1)
        d = float(np.max(np.abs(mean - mref)))
        log("t %.1e steps %d (oracle %d) |<m> - <m>_ref| %.2e" % (t_out, steps, ns, d))
        assert d < 1e-4
    got = to_np(m)
    ys = np.array([c[0] for c in cells])
    xs = np.array([c[1] for c in cells])
    ref = np.stack([c[2] for c in cells], axis=1)
    dm = float(np.max(np.abs(got[:, 0, ys, xs] - ref)))
    log("sampled cells at %.3g s: max |m - m_ref| %.2e" % (t, dm))
    assert dm < 1e-3
    assert np.allclose(np.sum(got * got, axis=0), 1.0, atol=1e-5)
    # fields of the evolved state: the library's own B_eff and torque against
    # the oracle's evaluation of the same (FP32) state
    b = to_np(ctx.beff(m))
    tau = to_np(ctx.torque(m))
    assert rel_inf(b, prob.beff(got)) < 1e-5
    assert rel_inf(tau, prob.torque(got)) < 1e-5
    ctx.close()
