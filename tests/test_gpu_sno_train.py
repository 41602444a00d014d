"""The surrogate's hand-written training kernels (mm_sno_train_*) against
the FP64 oracle of the network (oracle/sno.py).

The backward pass is pinned by finite differences of the oracle's loss, not
by any second implementation of the gradient: for each parameter group
(lift P, p; per layer R, W, b; projection Q, q) the GPU's gradient projected
on a random direction within the group must equal the central difference
(L(w + e v) - L(w - e v)) / 2e of the oracle's FP64 loss, and so must a few
single components.  A wrong sign, a missing conjugate, a dropped w_kx / N
factor or a transposed weight in any of the backward kernels fails one of
them.  Also: the loss itself, and Adam steps lowering it on a fixed batch."""
import numpy as np
import pytest

from oracle import sno as osno
from paper_1406_7635_amd import mm, synth
from tests.gpu_helpers import log

pytestmark = pytest.mark.gpu

NX, NY, B = 32, 16, 2


def oracle_loss(w, m, t):
    """Mean over the batch of ||y_b - t_b|| / ||t_b|| with the oracle's FP64 forward pass."""
    tot = 0.0
    for b in range(m.shape[0]):
        y = osno.forward(w, m[b])
        tot += np.linalg.norm(y - t[b]) / np.linalg.norm(t[b])
    return tot / m.shape[0]


def groups():
    c, lw = 32, osno.KY * osno.KX * 32 * 32 * 2 + 32 * 32 + 32
    out = [("P", 0, 96), ("p", 96, 128)]
    for l in range(osno.NLAYER):
        base = 128 + l * lw
        out += [("R%d" % l, base, base + osno.KY * osno.KX * c * c * 2),
                ("W%d" % l, base + osno.KY * osno.KX * c * c * 2, base + osno.KY * osno.KX * c * c * 2 + c * c),
                ("b%d" % l, base + osno.KY * osno.KX * c * c * 2 + c * c, base + lw)]
    q0 = 128 + osno.NLAYER * lw
    out += [("Q", q0, q0 + 96), ("q", q0 + 96, q0 + 99)]
    assert out[-1][2] == osno.weight_count()
    return out


@pytest.fixture(scope="module")
def problem(gpu):
    import torch

    w = synth.sno_random_weights(11, scale=0.7)
    rng = np.random.Generator(np.random.PCG64(12))
    m = synth.film_textures(B, seed=13, grid=(NX, NY), cell=4e-9)[:, :, 0].astype(np.float32)
    t = (0.3 * rng.standard_normal((B, 3, NY, NX))).astype(np.float32)
    tr = mm.SurrogateTrainer(NX, NY, B, w)
    md, td = torch.from_numpy(m).cuda(), torch.from_numpy(t).cuda()
    loss, g = tr.grad(md, td)
    yield w.astype(np.float64), m.astype(np.float64), t.astype(np.float64), loss, g.cpu().numpy().astype(np.float64)
    tr.close()


def test_loss_matches_oracle(problem):
    w, m, t, loss, _ = problem
    ref = oracle_loss(w, m, t)
    log("surrogate loss GPU %.9f oracle %.9f" % (loss, ref))
    assert loss == pytest.approx(ref, rel=2e-6)


@pytest.mark.parametrize("name,lo,hi", groups(), ids=[g[0] for g in groups()])
def test_gradient_direction_matches_finite_difference(problem, name, lo, hi):
    w, m, t, _, g = problem
    rng = np.random.Generator(np.random.PCG64(lo + 7))
    v = np.zeros_like(w)
    v[lo:hi] = rng.standard_normal(hi - lo)
    eps = 1e-4 / max(1.0, np.linalg.norm(v[lo:hi]) / np.sqrt(hi - lo))
    fd = (oracle_loss(w + eps * v, m, t) - oracle_loss(w - eps * v, m, t)) / (2 * eps)
    got = float(np.dot(g, v))
    scale = max(abs(fd), np.linalg.norm(g[lo:hi]) * np.linalg.norm(v[lo:hi]) / np.sqrt(hi - lo))
    log("grad %-3s  <g,v> %.6e  finite difference %.6e  rel %.1e" % (name, got, fd, abs(got - fd) / scale))
    assert abs(got - fd) <= 2e-3 * scale


@pytest.mark.parametrize("name,lo,hi", [g for g in groups() if g[0] in ("P", "p", "R0", "W3", "b1", "Q", "q")],
                         ids=[g[0] for g in groups() if g[0] in ("P", "p", "R0", "W3", "b1", "Q", "q")])
def test_gradient_components_match_finite_difference(problem, name, lo, hi):
    w, m, t, _, g = problem
    rng = np.random.Generator(np.random.PCG64(hi))
    gmax = float(np.max(np.abs(g[lo:hi])))
    for i in rng.choice(np.arange(lo, hi), size=min(3, hi - lo), replace=False):
        e = np.zeros_like(w)
        e[i] = 1e-4 * max(1.0, abs(w[i]))
        fd = (oracle_loss(w + e, m, t) - oracle_loss(w - e, m, t)) / (2 * e[i])
        assert abs(g[i] - fd) <= 2e-3 * max(abs(fd), 1e-2 * gmax), (name, i, g[i], fd)


def test_adam_steps_lower_the_loss(gpu):
    import torch

    n, b = 64, 4
    w = synth.sno_random_weights(3, scale=0.5)
    m = synth.film_textures(b, seed=21, grid=(n, n), cell=4e-9)[:, :, 0]
    ctx = mm.Context((n, n, 1), (4e-9,) * 3, np.zeros((1, n, n), np.uint8), synth.material(8e5, 1.3e-11))
    md = torch.from_numpy(np.ascontiguousarray(m)).cuda()
    td = torch.empty_like(md)
    for k in range(b):
        _, bd = ctx.beff(md[k].unsqueeze(1).contiguous(), want_demag=True)
        td[k] = bd[:, 0] / (4e-7 * np.pi * 8e5)
    tr = mm.SurrogateTrainer(n, n, b, w)
    losses = [tr.step(md, td, 3e-3) for _ in range(60)]
    log("Adam on a fixed batch: loss %.4f -> %.4f" % (losses[0], losses[-1]))
    assert np.all(np.isfinite(losses)) and losses[-1] < 0.5 * losses[0]
    wf = tr.weights()
    assert np.all(np.isfinite(wf)) and not np.array_equal(wf, w)
    tr.close()
    ctx.close()
