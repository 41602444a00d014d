"""Matrix-core DFT stages of the y convolution (BF16 / FP16 split precision)
against the FP64 oracle at the benchmark size (1024 x 1024 x 1, padded y
length 2048).  The relative error of B_demag (max over cells of |B - B_ref|
over max |B_ref|) must stay within 1e-4; the FP32 path is checked beside it.
"""
import numpy as np
import pytest

from oracle import demag as odemag
from oracle.constants import MU0
from paper_1406_7635_amd import synth
from tests.gpu_helpers import log, make_ctx, make_pair, rel_inf, to_np

pytestmark = pytest.mark.gpu

PRECS = ("bf16", "fp16")


@pytest.fixture(scope="module")
def film():
    case = synth.vortex_film(seed=2, n=1024)
    ctx, prob, m = make_pair(case)
    prob.workers = -1
    ref = prob.demag_field(case["m0"].astype(np.float64))
    yield case, ctx, m, ref
    ctx.close()


@pytest.mark.parametrize("prec", PRECS)
def test_film_demag_error(gpu, film, prec):
    case, ctx, m, ref = film
    ctx.set_conv_precision(prec)
    _, bd = ctx.beff(m, want_demag=True)
    err = rel_inf(to_np(bd), ref)
    ctx.set_conv_precision("fp32")
    _, bd32 = ctx.beff(m, want_demag=True)
    err32 = rel_inf(to_np(bd32), ref)
    log("film 1024 demag rel error", prec, "%.3e" % err, "fp32 %.3e" % err32)
    assert err < 1e-4
    assert err32 < 1e-5


@pytest.mark.parametrize("prec", PRECS)
def test_impulse_response(gpu, prec):
    """One magnetised cell (an impulse) in a vacuum film: B_demag is the kernel
    column -mu0 N(r - r0) M, exact from the oracle's tensor at any cell."""
    grid, cell = (1024, 1024, 1), (2e-9, 2e-9, 2e-9)
    region = np.zeros((1, 1024, 1024), dtype=np.uint8)
    y0, x0 = 517, 301
    region[0, y0, x0] = 1
    p = synth.material(8e5, 1.3e-11, alpha=0.01, region=1)
    case = {"grid": grid, "cell": cell, "region": region, "params": p,
            "m0": synth.uniform_m(grid, (0.6, -0.48, 0.64))}
    ctx, m = make_ctx(case)
    ctx.set_conv_precision(prec)
    _, bd = ctx.beff(m, want_demag=True)
    bd = to_np(bd)[:, 0]
    rng = np.random.Generator(np.random.PCG64(11))
    ys = np.concatenate([[y0, y0, y0 + 1, y0 - 3, 0, 1023], rng.integers(0, 1024, 60)])
    xs = np.concatenate([[x0, x0 + 1, x0, x0 + 5, 0, 1023], rng.integers(0, 1024, 60)])
    N = odemag.tensor_at((xs - x0) * cell[0], (ys - y0) * cell[1], np.zeros(len(xs)), cell)
    M = 8e5 * case["m0"][:, 0, y0, x0].astype(np.float64)
    ref = -MU0 * np.stack([N["xx"] * M[0] + N["xy"] * M[1] + N["xz"] * M[2],
                           N["xy"] * M[0] + N["yy"] * M[1] + N["yz"] * M[2],
                           N["xz"] * M[0] + N["yz"] * M[1] + N["zz"] * M[2]])
    got = bd[:, ys, xs]
    err = rel_inf(got, ref)
    log("impulse", prec, "%.3e" % err)
    assert err < 1e-4
    ctx.close()


def test_precision_switch_rejects_other_grids(gpu):
    case = synth.random_problem((40, 24, 3), (2e-9, 2e-9, 2e-9), seed=3)
    ctx, _ = make_ctx(case)
    from paper_1406_7635_amd import mm
    with pytest.raises(mm.MMError):
        ctx.set_conv_precision("bf16")
    ctx.set_conv_precision("fp32")
    ctx.close()


@pytest.mark.parametrize("prec", PRECS)
def test_periodic_film_demag_error(gpu, prec):
    """The matrix-core column pass with periodic images (the images live in
    the kernel only): a 96 x 1024 film periodic along x (2 images per side)
    against the FP64 oracle's image sum, within 1e-4."""
    import torch

    from oracle import fields as ofields
    from paper_1406_7635_amd import mm

    case = synth.random_problem((96, 1024, 1), (3e-9, 3e-9, 3e-9), seed=9, nregions=2)
    pbc = (2, 0, 0)
    ctx = mm.Context(case["grid"], case["cell"], case["region"], case["params"], pbc=pbc)
    prob = ofields.Problem(case["grid"], case["cell"], case["region"], case["params"], pbc=pbc, workers=-1)
    ref = prob.demag_field(case["m0"].astype(np.float64))
    m = torch.from_numpy(case["m0"]).cuda()
    ctx.set_conv_precision(prec)
    _, bd = ctx.beff(m, want_demag=True)
    err = rel_inf(to_np(bd), ref)
    log("periodic film demag rel error", prec, "%.3e" % err)
    assert err < 1e-4
    ctx.close()
