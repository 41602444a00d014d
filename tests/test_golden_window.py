"""Integrity of the stored trajectory window (tests/golden/c2_window.txt) that
the GPU test of the 1024 x 1024 x 1 vortex film compares against.

The file is the FP64 oracle's Dormand-Prince run written by
tests/golden/make_c2_window.py.  Checked here, on the CPU: the output schedule
(every 5 ps up to 50 ps, then every 10 ps), accepted-step counts that grow,
unit-length magnetisation at the sampled cells (the stepper renormalises m on
every accepted step, section "Dynamics"), the cell sample being the
generator's seeded draw, and the direction of the motion: in a field along +x
the damped precession turns the in-plane vortex towards +x, so <m_x> grows
at every output time (a sign slip in the Zeeman term or the damping term
would turn it away).
"""
import importlib.util
import os

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden", "c2_window.txt")


def _generator():
    spec = importlib.util.spec_from_file_location("make_c2_window", os.path.join(HERE, "golden", "make_c2_window.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _read():
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
def test_window_schedule_and_steps():
    means, _ = _read()
    times = np.array([m[0] for m in means])
    expect = [k * 5e-12 for k in range(1, 11)] + [k * 1e-11 for k in range(6, 6 + len(means) - 10)]
    assert len(means) >= 11
    assert np.allclose(times, expect, rtol=1e-9, atol=0.0)
    steps = np.array([m[1] for m in means])
    rejects = np.array([m[2] for m in means])
    assert np.all(np.diff(steps) > 0) and steps[0] > 0
    assert np.all(rejects >= 0) and np.all(np.diff(rejects) >= 0)
    # the window spans about a thousand accepted steps
    assert steps[-1] >= 1000


@pytest.mark.skipif(not os.path.exists(GOLDEN), reason="tests/golden/c2_window.txt not generated")
def test_window_magnetisation():
    means, cells = _read()
    mean = np.stack([m[3] for m in means])
    assert np.all(np.linalg.norm(mean, axis=1) <= 1.0)
    assert np.all(np.diff(mean[:, 0]) > 0) and mean[0, 0] > 0
    gen = _generator()
    ys, xs = gen.sample_cells()
    assert len(cells) == gen.NSAMPLE
    assert np.array_equal([c[0] for c in cells], ys)
    assert np.array_equal([c[1] for c in cells], xs)
    m = np.stack([c[2] for c in cells])
    assert np.allclose(np.linalg.norm(m, axis=1), 1.0, atol=1e-8)
