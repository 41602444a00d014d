"""The surrogate's forward pass on the GPU (mm_sno_*) against the FP64 oracle
of the same network (oracle/sno.py) with the same BF16-rounded weights: a
ragged grid (rows not a multiple of the 16-row tile, nx not a power of two)
and the 256 x 256 grid of the surrogate workload."""
import numpy as np
import pytest

from oracle import sno
from paper_1406_7635_amd import mm, synth
from tests.gpu_helpers import log, rel_inf, to_np

pytestmark = pytest.mark.gpu


def bf16_round(w):
    """FP32 -> nearest-even BF16, returned as FP32 values."""
    b = np.asarray(w, dtype=np.float32).view(np.uint32).astype(np.uint64)
    b = ((b + 0x7FFF + ((b >> 16) & 1)) >> 16) << 16
    return b.astype(np.uint32).view(np.float32)


@pytest.mark.parametrize("grid", [(96, 40), (256, 256)])
def test_sno_forward_matches_oracle(gpu, grid):
    import torch

    nx, ny = grid
    w = bf16_round(synth.sno_random_weights(11))
    m = synth.random_sphere((nx, ny, 1), 12)
    log("surrogate forward %dx%d against the oracle" % (nx, ny))
    s = mm.Surrogate(nx, ny, w, out_scale=2.5)
    got = to_np(s(torch.from_numpy(m).to("cuda:0")))[:, 0]
    ref = 2.5 * sno.forward(w.astype(np.float64), m)
    err = rel_inf(got, ref)
    log("  rel %.2e" % err)
    assert err < 1e-4
    s.close()


def test_sno_weights_replace_and_reject_bad_counts(gpu):
    import torch

    nx, ny = 64, 32
    m = torch.from_numpy(synth.random_sphere((nx, ny, 1), 3)).to("cuda:0")
    w1 = bf16_round(synth.sno_random_weights(1))
    w2 = bf16_round(synth.sno_random_weights(2))
    s = mm.Surrogate(nx, ny, w1, 1.0)
    a = to_np(s(m)).copy()
    s.set_weights(w2)
    b = to_np(s(m))
    s.set_weights(w1)
    c = to_np(s(m))
    assert not np.array_equal(a, b) and np.array_equal(a, c)
    with pytest.raises(mm.MMError):
        s.set_weights(w1[:-1])
    with pytest.raises(mm.MMError):
        mm.Surrogate(16, 32, w1, 1.0)  # nx below two kept-mode spans
    s.close()


MU0 = 4e-7 * np.pi


def film(nx=64, ny=48, seed=3):
    params = synth.material(8e5, 1.3e-11, alpha=0.05, bext=(0.01, 0.0, 0.0))
    region = np.zeros((1, ny, nx), dtype=np.uint8)
    m0 = synth.film_textures(1, seed=seed, grid=(nx, ny), cell=4e-9)[0]
    return (nx, ny, 1), (4e-9, 4e-9, 4e-9), region, params, m0


def test_surrogate_stages_match_hybrid_oracle_step(gpu):
    """One Dormand-Prince step whose stages 2-6 take B_demag from the
    surrogate and whose last stage is exact, against the same step in FP64
    (oracle fields, oracle surrogate, the oracle's embedded step)."""
    import torch

    from oracle import fields as ofields
    from oracle import integrate as ointegrate

    grid, cell, region, params, m0 = film()
    nx, ny, _ = grid
    scale = MU0 * 8e5
    w = bf16_round(synth.sno_random_weights(13, scale=0.5))
    ctx = mm.Context(grid, cell, region, params)
    s = mm.Surrogate(nx, ny, w, scale)
    ctx.set_surrogate(s, tol=1e30)
    m = torch.from_numpy(m0).to("cuda:0")
    dt = 2e-14
    t, _, st = ctx.run(m, dt, dt=dt, max_attempts=1, opts=mm.solver_opts(max_err=1e3))
    stats = ctx.surrogate_stats()
    log("surrogate step: t %.3e, stats %s" % (t, stats))
    assert t == dt and stats["surrogate_steps"] == 1 and stats["fallbacks"] == 0

    exact = ofields.Problem(grid, cell, region, params)
    local = ofields.Problem(grid, cell, region, params, demag=False)
    alpha = np.asarray(params["alpha"])[region]
    calls = [0]

    def f(ms):
        calls[0] += 1
        if calls[0] <= 5:
            b = local.beff(ms) + scale * sno.forward(w.astype(np.float64), ms)[:, None] * local.magnetic
            return ofields.llg_torque(ms, b, alpha, local.gamma) * local.magnetic
        return exact.torque(ms)

    m64 = m0.astype(np.float64)
    ms, _, _ = ointegrate.embedded_step(f, m64, exact.torque(m64), dt, ointegrate.DP45)
    ref = ointegrate.normalize(ms)
    got = to_np(m)
    err = float(np.max(np.abs(got - ref)))
    log("  |dm| against the hybrid FP64 step: %.2e" % err)
    assert err < 1e-5
    bd = exact.demag_field(ms)
    err_ref = float(np.max(np.linalg.norm(scale * sno.forward(w.astype(np.float64), ms)[:, None] - bd, axis=0))
                    / np.max(np.linalg.norm(bd, axis=0)))
    log("  surrogate error at the new state: %.4e (oracle %.4e)" % (stats["last_err"], err_ref))
    assert stats["last_err"] == pytest.approx(err_ref, rel=1e-3)
    ctx.close()
    s.close()


@pytest.mark.parametrize("corrupt", ["nan", "random"])
def test_surrogate_fallback_reproduces_the_plain_trajectory(gpu, corrupt):
    """Weights that miss the tolerance (NaN, or an untrained network): the
    first surrogate attempt is rejected with dt kept and the run continues on
    the exact path, so the trajectory is the plain path's, bit for bit."""
    import torch

    grid, cell, region, params, m0 = film(seed=4)
    nx, ny, _ = grid
    w = synth.sno_random_weights(17)
    if corrupt == "nan":
        w = np.full_like(w, np.nan)
    plain = mm.Context(grid, cell, region, params)
    hyb = mm.Context(grid, cell, region, params)
    s = mm.Surrogate(nx, ny, w, MU0 * 8e5)
    hyb.set_surrogate(s, tol=1e-4)
    m1 = torch.from_numpy(m0).to("cuda:0")
    m2 = m1.clone()
    t_end = 4e-13
    t1, dt1, s1 = plain.run(m1, t_end, dt=1e-14)
    t2, dt2, s2 = hyb.run(m2, t_end, dt=1e-14)
    stats = hyb.surrogate_stats()
    log("fallback (%s): plain steps %d, hybrid steps %d, stats %s" % (corrupt, s1["steps"], s2["steps"], stats))
    assert stats["fallbacks"] == 1 and stats["surrogate_steps"] == 0
    assert (t1, dt1, s1["steps"]) == (t2, dt2, s2["steps"])
    assert np.array_equal(to_np(m1), to_np(m2))
    for c in (plain, hyb):
        c.close()
    s.close()
