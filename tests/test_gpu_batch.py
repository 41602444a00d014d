"""Ensemble (mm_batch_*) parity.

Per member the ensemble runs the single-grid arithmetic with another
schedule, so every member is checked against its own single-grid context
(the plain path the other GPU tests pin to the FP64 oracle), small members
also directly against the oracle, and the ensemble at its full size (512
members, about 1e7 cells) on sampled members.  Graph replays are checked
against direct launches with eager work between the replays, and tuned
persistent grids and tile shapes against one wide workgroup per tile.
"""
import math

import numpy as np
import pytest

from oracle import fields as ofields
from paper_1406_7635_amd import mm, synth
from tests.gpu_helpers import log, rel_inf, to_np

pytestmark = pytest.mark.gpu

# one member per padded-length class: px, py in 64 ... 1024, pz in 1, 4, 8, 16
SHAPES = [(17, 33, 1), (40, 20, 2), (64, 64, 1), (100, 70, 2), (130, 33, 3), (32, 256, 1),
          (200, 129, 1), (33, 40, 5), (512, 24, 1), (48, 300, 2)]


def mixed_members(seed=11, shapes=SHAPES):
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for i, g in enumerate(shapes):
        cell = tuple(float(v) for v in rng.uniform(2e-9, 5e-9, 3))
        case = synth.random_problem(g, cell, seed + 17 * i, nregions=3, vacuum=(i % 4 == 3))
        out.append(case)
    return out


def single_ctx(case):
    return mm.Context(case["grid"], case["cell"], case["region"], case["params"])


def test_batch_beff_matches_single_contexts(gpu):
    import torch

    members = mixed_members()
    log("batch B_eff: %d members of every padded class" % len(members))
    b = mm.Batch(members)
    m = b.pack([c["m0"] for c in members])
    beff = b.beff(m)
    torch.cuda.synchronize()
    for i, case in enumerate(members):
        ctx = single_ctx(case)
        ref = to_np(ctx.beff(torch.from_numpy(case["m0"]).to("cuda:0")))
        got = to_np(b.member(beff, i))
        err = rel_inf(got, ref)
        log("  member %d %s: rel %.2e" % (i, case["grid"], err))
        assert err < 1e-6
        ctx.close()
    b.close()


def test_batch_beff_small_members_vs_oracle(gpu):
    members = mixed_members(seed=5, shapes=[(17, 20, 1), (24, 18, 2), (20, 19, 3)])
    log("batch B_eff of small members against the FP64 oracle")
    b = mm.Batch(members)
    m = b.pack([c["m0"] for c in members])
    beff = b.beff(m)
    for i, case in enumerate(members):
        prob = ofields.Problem(case["grid"], case["cell"], case["region"], case["params"])
        ref = prob.beff(case["m0"].astype(np.float64))
        err = rel_inf(to_np(b.member(beff, i)), ref)
        log("  member %d %s: rel %.2e" % (i, case["grid"], err))
        assert err < 1e-5
    b.close()


def run_single(case, t_end, attempts):
    import torch

    ctx = single_ctx(case)
    m = torch.from_numpy(case["m0"]).to("cuda:0")
    t, dt, st = ctx.run(m, t_end, dt=1e-14, max_attempts=attempts)
    out = to_np(m)
    ctx.close()
    return out, t, st


def test_batch_run_matches_single_contexts(gpu):
    members = mixed_members(seed=21)
    t_end = 3e-13
    log("batch DP45 to %.1e s against single-grid runs" % t_end)
    b = mm.Batch(members)
    m = b.pack([c["m0"] for c in members])
    b.start(45, 0.0, 1e-14, t_end)
    na, act = b.run(m, 2000)
    assert act == 0
    for i, case in enumerate(members):
        ref, t, st = run_single(case, t_end, 2000)
        s = b.stats(i)
        got = to_np(b.member(m, i))
        err = float(np.max(np.abs(got - ref)))
        log("  member %d %s: steps %d/%d rejects %d/%d |dm| %.2e" % (i, case["grid"], s["steps"], st["steps"],
                                                                      s["rejects"], st["rejects"], err))
        assert s["status"] == 0
        assert s["t"] == pytest.approx(t_end, rel=1e-12)
        assert s["steps"] == st["steps"] and s["rejects"] == st["rejects"]
        assert err < 1e-5
        assert np.allclose(np.sum(got * got, axis=0)[case["params"]["msat"][case["region"]] > 0], 1.0, atol=1e-5)
    b.close()


def _run_chunks(b, members, graph, eager_between):
    b.set_graph(graph)
    m = b.pack([c["m0"] for c in members])
    b.start(45, 0.0, 1e-14, float("inf"))
    outs = []
    for _ in range(4):
        b.run(m, 3)
        outs.append(to_np(m))
        if eager_between:
            b.beff(m)  # eager work between two replays
    stats = [b.stats(i) for i in range(len(members))]
    return outs, stats


def test_batch_graph_replays_match_direct_launches(gpu):
    members = mixed_members(seed=31, shapes=SHAPES[:6])
    log("batch: graph replays against direct launches")
    b = mm.Batch(members)
    direct, st_d = _run_chunks(b, members, graph=False, eager_between=False)
    graph, st_g = _run_chunks(b, members, graph=True, eager_between=True)
    for k, (x, y) in enumerate(zip(direct, graph)):
        assert np.array_equal(x, y), "replay chunk %d differs" % k
    for a, c in zip(st_d, st_g):
        assert (a["steps"], a["rejects"], a["t"], a["dt"]) == (c["steps"], c["rejects"], c["t"], c["dt"])
    b.close()


def test_batch_tuned_grids_same_result(gpu):
    members = mixed_members(seed=41, shapes=SHAPES[:8])
    log("batch: autotuned persistent grids against one workgroup per tile")
    b = mm.Batch(members)
    m = b.pack([c["m0"] for c in members])
    b.start(45, 0.0, 1e-14, float("inf"))
    b.run(m, 6)
    ref = to_np(m)
    grids = b.autotune(m)
    log("  tuned grids", grids)
    for name, g in grids.items():
        assert g >= 0 and g % 8 == 0, name  # 0: a pass no member uses
    # a small persistent grid as well: every workgroup walks many tiles
    b.set_grid("x", 8)
    m2 = b.pack([c["m0"] for c in members])
    b.start(45, 0.0, 1e-14, float("inf"))
    b.run(m2, 6)
    assert np.array_equal(to_np(m2), ref)
    b.close()


def test_batch_tile_shapes_same_result(gpu):
    """The narrow tile shapes of the x passes and of the 2D y convolution (a
    quarter of the row pairs or columns per work item) run the same
    arithmetic per row and column as the wide ones: bit-identical states in
    every combination, also on a small persistent grid and after the
    autotuner's choice of shape and grid; the narrow shape is refused when a
    member's padded length exceeds 512."""
    members = mixed_members(seed=43, shapes=SHAPES[:8])
    log("batch: tile shapes")
    b = mm.Batch(members)

    def run():
        m = b.pack([c["m0"] for c in members])
        b.start(45, 0.0, 1e-14, float("inf"))
        b.run(m, 6)
        return to_np(m)

    ref = run()
    for tx, tc in (("narrow", "wide"), ("wide", "narrow"), ("narrow", "narrow")):
        b.set_tile("x", tx)
        b.set_tile("conv2d", tc)
        assert (b.get_tile("x"), b.get_tile("conv2d")) == (tx, tc)
        assert np.array_equal(run(), ref), (tx, tc)
    b.set_grid("x", 8)
    b.set_grid("conv2d", 16)
    assert np.array_equal(run(), ref)
    m = b.pack([c["m0"] for c in members])
    grids = b.autotune(m)
    tiles = {p: b.get_tile(p) for p in ("x", "conv2d")}
    log("  tuned", grids, tiles)
    assert np.array_equal(run(), ref)
    with pytest.raises(mm.MMError):
        b.set_tile("y", "narrow")
    b.close()
    big = mixed_members(seed=44, shapes=[(17, 33, 1), (512, 24, 1)])  # px 1024
    b = mm.Batch(big)
    with pytest.raises(mm.MMError):
        b.set_tile("x", "narrow")
    b.set_tile("conv2d", "narrow")  # py 64 and 128: served
    b.close()


def test_batch_full_ensemble_sampled_members(gpu):
    """The 512-member ensemble of the throughput workload: a few attempts of
    every member, then sampled members against their single-grid runs."""
    members = synth.ensemble(n=512, seed=4)
    ncell = sum(int(np.prod(c["grid"])) for c in members)
    log("full ensemble: %d members, %d cells" % (len(members), ncell))
    b = mm.Batch(members)
    m = b.pack([c["m0"] for c in members])
    b.start(45, 0.0, 1e-14, members[0]["t_end"])
    attempts = 4
    na, act = b.run(m, attempts)
    assert na == attempts and act == len(members)
    sizes = [int(np.prod(c["grid"])) for c in members]
    pick = sorted({int(np.argmin(sizes)), int(np.argmax(sizes)), 7, 300, 511,
                   next(i for i, c in enumerate(members) if c["grid"][2] == 2)})
    for i in pick:
        ref, t, st = run_single(members[i], members[i]["t_end"], attempts)
        got = to_np(b.member(m, i))
        s = b.stats(i)
        err = float(np.max(np.abs(got - ref)))
        log("  member %d %s: steps %d/%d |dm| %.2e" % (i, members[i]["grid"], s["steps"], st["steps"], err))
        assert s["steps"] == st["steps"] and s["rejects"] == st["rejects"]
        assert err < 1e-5
        assert math.isfinite(s["dt"]) and s["dt"] > 0
    b.close()
