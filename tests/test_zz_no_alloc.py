"""mm_beff_noalloc (the allocation-free B_eff entry point) against mm_beff.

Both run the same kernels on the same inputs; the only difference is where
the FFT spectrum lives (the context's buffer or the library's static per-GPU
array), so the fields must agree bit for bit.  Two calls in a row through the
static array, the second on a smaller grid, show that nothing of a previous
call's spectrum leaks into the next.  Device memory must not change across
the calls, and a grid whose spectrum exceeds the array is refused before any
work is enqueued.
"""
import ctypes

import numpy as np
import pytest

from paper_1406_7635_amd import synth
from tests.gpu_helpers import log, make_ctx

pytestmark = pytest.mark.gpu


def _same(a, b):
    return bool(np.array_equal(a.cpu().numpy(), b.cpu().numpy()))


def test_noalloc_matches_beff_twice(gpu):
    import torch

    from paper_1406_7635_amd import mm

    big = synth.vortex_film(seed=2, n=1024)          # 1024 x 1024 x 1, the largest film that fits the array
    small = synth.random_problem((40, 24, 3), (2e-9, 2e-9, 2e-9), seed=7, nregions=4, vacuum=True)
    log("noalloc: contexts 1024x1024x1 and 40x24x3")
    cb, mb = make_ctx(big)
    cs, ms = make_ctx(small)
    ref_b, ref_bd = cb.beff(mb, want_demag=True)
    ref_s, ref_sd = cs.beff(ms, want_demag=True)
    out_b, out_bd = cb.new_field(), cb.new_field()
    out_s, out_sd = cs.new_field(), cs.new_field()
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    cb.beff_noalloc(mb, out_b, out_bd)                # first call: the larger grid
    cs.beff_noalloc(ms, out_s, out_sd)                # second call: the smaller grid
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    log("noalloc: free device memory before %d after %d" % (free0, free1))
    assert _same(out_b, ref_b) and _same(out_bd, ref_bd)
    assert _same(out_s, ref_s) and _same(out_sd, ref_sd)
    assert free1 == free0
    # and once more in the other order, without the demag output
    out_s2, out_b2 = cs.new_field(), cb.new_field()
    cs.beff_noalloc(ms, out_s2)
    cb.beff_noalloc(mb, out_b2)
    assert _same(out_s2, ref_s) and _same(out_b2, ref_b)
    cb.close()
    cs.close()


def test_noalloc_thin3d_and_no_demag(gpu):
    """The thin-3D column pass (2-4 layers) and a grid without demag."""
    for grid, demag in (((64, 48, 2), True), ((33, 20, 4), True), ((50, 30, 1), False)):
        case = synth.random_problem(grid, (2.5e-9, 2e-9, 3e-9), seed=sum(grid), nregions=3)
        log("noalloc:", grid, "demag" if demag else "no demag")
        ctx, m = make_ctx(case, demag=demag)
        ref = ctx.beff(m)
        out = ctx.new_field()
        ctx.beff_noalloc(m, out)
        assert _same(out, ref)
        ctx.close()


def test_noalloc_refuses_oversize_grid(gpu):
    """A spectrum larger than the static array: MM_ESCRATCH, nothing enqueued."""
    from paper_1406_7635_amd import mm

    case = synth.random_problem((1500, 1100, 1), (2e-9, 2e-9, 2e-9), seed=3, nregions=1, ku=False, field=False)
    log("noalloc: oversize 1500x1100x1")
    # built without the (large) kernel initialisation, then demag switched on:
    # the size check comes before every other state check
    ctx = mm.Context(case["grid"], case["cell"], case["region"], case["params"], demag=False)
    assert mm.load().mm_set_demag(ctx._h, 1) == 0
    m = ctx.new_field()
    out = ctx.new_field()
    st = mm.load().mm_beff_noalloc(ctx._h, ctypes.c_void_p(m.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                   ctypes.c_void_p(0))
    assert mm.STATUS[st] == "MM_ESCRATCH"
    ctx.close()
