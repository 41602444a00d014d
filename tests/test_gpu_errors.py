"""Failure paths of the C ABI (include/mm.h): every status the library
raises is driven here through the ctypes binding, on the GPU.

* a NaN in m spreads through the magnetostatic convolution to every cell;
  the embedded error estimate is then not finite and the run stops with
  MM_ENONFINITE (single context and ensemble member alike);
* a dt_min above the step the controller needs stops with MM_ESTEP, while a
  run whose last, clipped step is shorter than dt_min ends normally;
* relax with too small a step budget returns MM_ENOTCONVERGED;
* sizes the library does not serve give MM_EUNSUPPORTED at creation;
* null pointers give MM_EINVAL;
* creating and destroying a context many times leaves device memory flat.
"""
import ctypes

import numpy as np
import pytest

from paper_1406_7635_amd import mm, synth
from tests.gpu_helpers import log, make_ctx

pytestmark = pytest.mark.gpu

ENONFINITE, ESTEP, ENOTCONVERGED, EUNSUPPORTED, EINVAL = -5, -6, -7, -4, -1


def _status(fn, *args):
    with pytest.raises(mm.MMError) as ei:
        fn(*args)
    return ei.value.status


def _film(n=32, nz=1):
    return synth.random_problem((n, n - 8, nz), (3e-9, 3e-9, 3e-9), seed=11, nregions=2)


@pytest.mark.parametrize("solver", [45, 23, 12])
def test_nan_in_m_gives_enonfinite(gpu, solver):
    case = _film()
    ctx, m = make_ctx(case)
    m[0, 0, 3, 5] = float("nan")
    log("NaN in m, solver", solver)
    st = _status(ctx.run, m, 1e-9, 0.0, 1e-14, solver)
    assert st == ENONFINITE
    ctx.close()


def test_nan_in_m_single_step(gpu):
    ctx, m = make_ctx(_film())
    m[2, 0, 0, 0] = float("nan")
    assert _status(ctx.rk45_step, m, 0.0, 1e-14) == ENONFINITE
    ctx.close()


def test_nan_in_ensemble_member(gpu):
    import torch

    members = synth.ensemble(n=6, seed=4)
    b = mm.Batch(members)
    m = b.pack([c["m0"] for c in members])
    b.member(m, 3)[0, 0, 1, 7] = float("nan")   # x component of a cell of member 3
    b.start(45, 0.0, 1e-14, 1e-11, mm.solver_opts(max_err=1e-5))
    b.run(m, 200)
    torch.cuda.synchronize()
    s = b.stats_all()
    log("ensemble statuses", list(s["status"]))
    assert s["status"][3] == ENONFINITE
    assert all(s["status"][i] == 0 for i in range(6) if i != 3)
    b.close()


def test_dt_min_above_needed_step_gives_estep(gpu):
    case = synth.vortex_film(seed=2, n=32)
    ctx, m = make_ctx(case)
    # the vortex takes steps of ~1e-13 s at MaxErr 1e-7: from dt0 = 1e-13 s the
    # step law proposes at most 2e-13 s, below dt_min = 5e-13 s
    o = mm.solver_opts(max_err=1e-7, dt_min=5e-13)
    st = _status(ctx.run, m, 1e-9, 0.0, 1e-13, 45, 10 ** 6, o)
    assert st == ESTEP
    ctx.close()


def test_short_clipped_last_step_ends_normally(gpu):
    """A run whose last step is clipped to a remainder below dt_min reaches
    t_end with MM_OK: dt_min judges the step law's proposals, not the clip."""
    case = _film()
    ctx, m = make_ctx(case)
    o = mm.solver_opts(max_err=1e-5, dt_min=1e-15, dt_max=1e-13)
    t_end = 10 * 1e-13 + 3e-17   # ten full steps, then a 3e-17 s remainder
    t, dt, st = ctx.run(m, t_end, dt=1e-13, solver=45, opts=o)
    log("clipped run: t", t, "steps", st["steps"])
    assert t == t_end and st["steps"] >= 11
    ctx.close()


def test_relax_step_cap_gives_enotconverged(gpu):
    case = _film()
    ctx, m = make_ctx(case)
    e, tq, n = ctypes.c_double(), ctypes.c_double(), ctypes.c_int64()
    o = mm.solver_opts(max_err=1e-5, precess=False)
    st = mm.load().mm_relax(ctx._h, mm._ptr(m), ctypes.byref(o), 1e-9, 5, ctypes.byref(e), ctypes.byref(tq),
                            ctypes.byref(n))
    assert st == ENOTCONVERGED
    r = ctx.relax(m, max_steps=5)
    assert not r["converged"]
    ctx.close()


@pytest.mark.parametrize("grid,pbc", [((2049, 4, 1), (0, 0, 0)), ((8, 4097, 1), (0, 0, 0)),
                                      ((4, 4, 3000), (0, 0, 0)), ((64, 64, 1), (0, 0, 1 << 21)),
                                      ((1024, 1024, 1), (64, 64, 0))])
def test_unsupported_sizes_at_create(gpu, grid, pbc):
    nx, ny, nz = grid
    region = np.zeros((nz, ny, nx), np.uint8)
    st = _status(mm.Context, grid, (1e-9,) * 3, region, synth.material(8e5, 1e-11), False, None, pbc)
    assert st == EUNSUPPORTED


def test_null_pointers_give_einval(gpu):
    import torch

    lib = mm.load()
    case = _film()
    ctx, m = make_ctx(case)
    out = torch.empty_like(m)
    null = ctypes.c_void_p(0)
    g = mm.Grid(8, 8, 1, 1e-9, 1e-9, 1e-9, (ctypes.c_int32 * 3)(0, 0, 0))
    p = mm.params_struct(synth.material(8e5, 1e-11))
    h = ctypes.c_void_p()
    reg = torch.zeros((1, 8, 8), dtype=torch.uint8, device="cuda:0")
    assert lib.mm_create(None, ctypes.byref(g), ctypes.byref(p), mm._ptr(reg), null) == EINVAL
    assert lib.mm_create(ctypes.byref(h), None, ctypes.byref(p), mm._ptr(reg), null) == EINVAL
    assert lib.mm_create(ctypes.byref(h), ctypes.byref(g), None, mm._ptr(reg), null) == EINVAL
    assert lib.mm_create(ctypes.byref(h), ctypes.byref(g), ctypes.byref(p), null, null) == EINVAL
    assert lib.mm_beff(null, mm._ptr(m), mm._ptr(out), null) == EINVAL
    assert lib.mm_beff(ctx._h, null, mm._ptr(out), null) == EINVAL
    assert lib.mm_beff(ctx._h, mm._ptr(m), null, null) == EINVAL
    assert lib.mm_torque(ctx._h, mm._ptr(m), null, 1) == EINVAL
    assert lib.mm_llg_torque(ctx._h, mm._ptr(m), null, mm._ptr(out), 1) == EINVAL
    t, dt = ctypes.c_double(0.0), ctypes.c_double(1e-14)
    assert lib.mm_run(ctx._h, null, 45, 1e-12, 10, ctypes.byref(t), ctypes.byref(dt), None, None) == EINVAL
    assert lib.mm_run(ctx._h, mm._ptr(m), 45, 1e-12, 10, None, ctypes.byref(dt), None, None) == EINVAL
    assert lib.mm_run(ctx._h, mm._ptr(m), 44, 1e-12, 10, ctypes.byref(t), ctypes.byref(dt), None, None) == EINVAL
    acc, err = ctypes.c_int32(), ctypes.c_double()
    assert lib.mm_rk45_step(ctx._h, null, ctypes.byref(t), ctypes.byref(dt), None, ctypes.byref(acc),
                            ctypes.byref(err)) == EINVAL
    assert lib.mm_energy(ctx._h, mm._ptr(m), None) == EINVAL
    assert lib.mm_max_torque(ctx._h, null, 1, ctypes.byref(err)) == EINVAL
    assert lib.mm_relax(null, mm._ptr(m), None, 1e-9, 10, None, None, None) == EINVAL
    assert lib.mm_rk4_step(ctx._h, mm._ptr(m), float("nan"), 1) == EINVAL
    assert lib.mm_get_info(ctx._h, None) == EINVAL
    lib.mm_destroy(null)   # a null context is ignored
    ctx.close()


def test_create_destroy_cycles_keep_memory_flat(gpu):
    import torch

    case = _film(48, 2)
    ctx, m = make_ctx(case)
    ctx.beff(m)
    ctx.close()
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    for i in range(100):
        c = mm.Context(case["grid"], case["cell"], case["region"], case["params"])
        if i % 10 == 0:
            c.beff(m)
        c.close()
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    log("free before / after 100 cycles (MiB):", free0 >> 20, free1 >> 20)
    assert abs(free0 - free1) < (8 << 20)
