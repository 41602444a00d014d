"""Checkpoint and resume (mm_state_save / mm_state_load): a run resumed in a
fresh context from a saved state, the saved m and the returned (t, dt)
continues bit for bit like the uninterrupted run -- Dormand-Prince with the
FSAL derivative carried over, and Heun at finite temperature with the
thermal generator's step counter carried over; malformed states are refused.
"""
import numpy as np
import pytest

from paper_1406_7635_amd import mm, synth
from tests.gpu_helpers import log

pytestmark = pytest.mark.gpu


def _ctx(case):
    return mm.Context(case["grid"], case["cell"], case["region"], case["params"])


def test_dp45_resume_bit_identical(gpu):
    import torch

    case = synth.random_problem((64, 48, 2), (2e-9, 2e-9, 2e-9), seed=21, nregions=3)
    a = _ctx(case)
    m = torch.from_numpy(case["m0"]).cuda()
    t, dt, _ = a.run(m, float("inf"), dt=1e-14, max_attempts=25)
    saved_m = m.clone()
    state = a.state_save()
    t_a, dt_a, st_a = a.run(m, float("inf"), t=t, dt=dt, max_attempts=25)
    b = _ctx(case)
    m_b = saved_m.clone()
    b.state_load(state, m_b)
    t_b, dt_b, st_b = b.run(m_b, float("inf"), t=t, dt=dt, max_attempts=25)
    log("resume DP45: t %.6e / %.6e, steps %d / %d" % (t_a, t_b, st_a["steps"], st_b["steps"]))
    assert torch.equal(m, m_b)
    assert t_a == t_b and dt_a == dt_b and st_a["steps"] == st_b["steps"] and st_a["evals"] == st_b["evals"]
    # without the saved state the resumed run re-evaluates the first stage at
    # the normalised state and drifts at rounding level
    c = _ctx(case)
    m_c = saved_m.clone()
    c.run(m_c, float("inf"), t=t, dt=dt, max_attempts=25)
    log("resume without the state: max |dm| %.2e" % float((m_c - m).abs().max()))
    for x in (a, b, c):
        x.close()


def test_thermal_heun_resume_bit_identical(gpu):
    import torch

    case = synth.random_problem((32, 32, 1), (4e-9, 4e-9, 4e-9), seed=5, nregions=2)
    a = _ctx(case)
    a.set_temperature(300.0, seed=77)
    m = torch.from_numpy(case["m0"]).cuda()
    t, dt, _ = a.run(m, float("inf"), dt=1e-13, solver=12, max_attempts=20)
    saved_m = m.clone()
    state = a.state_save()
    a.run(m, float("inf"), t=t, dt=dt, solver=12, max_attempts=20)
    b = _ctx(case)
    b.set_temperature(300.0, seed=77)
    m_b = saved_m.clone()
    b.state_load(state, m_b)
    b.run(m_b, float("inf"), t=t, dt=dt, solver=12, max_attempts=20)
    assert torch.equal(m, m_b)
    a.close()
    b.close()


def test_bad_state_refused(gpu):
    import torch

    case = synth.random_problem((16, 16, 1), (2e-9, 2e-9, 2e-9), seed=2)
    a = _ctx(case)
    m = torch.from_numpy(case["m0"]).cuda()
    a.run(m, float("inf"), dt=1e-14, max_attempts=3)
    state = a.state_save()
    with pytest.raises(mm.MMError):
        a.state_load(state[:20], m)
    with pytest.raises(mm.MMError):
        a.state_load(b"\\0" * len(state), m)
    other = synth.random_problem((16, 8, 1), (2e-9, 2e-9, 2e-9), seed=2)
    b = _ctx(other)
    with pytest.raises(mm.MMError):
        b.state_load(state, torch.from_numpy(other["m0"]).cuda())
    a.close()
    b.close()
