"""Train the spectral-neural-operator surrogate of the magnetostatic field
(offline; the trained weights are what the library's mm_sno_* kernels run).

    python -m paper_1406_7635_amd.sno_train --out weights.npy [--pairs N] [--steps K]

(the committed data/sno_film256_bf16.npy came from --pairs 2048 --steps 4000)

Training pairs: seeded film textures (synth.film_textures) and their B_demag
from the library's exact FP32 convolution (mm_beff), in units of mu0 Msat.
The model below is the network of include/mm.h written with torch's real
FFTs so that autograd can train it; its forward pass is checked against the
FP64 oracle of the same network by the CPU tests.  The weights are saved as
the BF16 bit patterns (uint16) of the flat array in include/mm.h's order.
"""
import argparse
import math
import os
import sys
import time

import numpy as np

C, KX, KY, NLAYER = 32, 16, 16, 4
MU0 = 4e-7 * math.pi
# weights trained by this script for the 256 x 256 x 1 film of 4 nm cells
# (Msat 8e5 A/m, Aex 1.3e-11 J/m): 2048 pairs, 4000 steps, seed 5
TRAINED = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data", "sno_film256_bf16.npy")


def save_weights(path, w):
    """The flat weights as their BF16 bit patterns (uint16)."""
    b = bf16_values(w).view(np.uint32)
    np.save(path, (b >> 16).astype(np.uint16))


def load_weights(path=TRAINED):
    """Flat FP32 weights from a file written by save_weights."""
    return (np.load(path).astype(np.uint32) << 16).view(np.float32)


def make_model(torch):
    nn = torch.nn

    class Sno(nn.Module):
        def __init__(self):
            super().__init__()
            self.P = nn.Parameter(torch.randn(C, 3) / math.sqrt(3.0))
            self.p = nn.Parameter(torch.zeros(C))
            self.R = nn.ParameterList([nn.Parameter(torch.randn(KY, KX, C, C, 2) / (C * 4)) for _ in range(NLAYER)])
            self.W = nn.ParameterList([nn.Parameter(torch.randn(C, C) / math.sqrt(C)) for _ in range(NLAYER)])
            self.b = nn.ParameterList([nn.Parameter(torch.zeros(C)) for _ in range(NLAYER)])
            self.Q = nn.Parameter(torch.randn(3, C) / math.sqrt(C))
            self.q = nn.Parameter(torch.zeros(3))

        def forward(self, m):
            """m [B, 3, ny, nx] -> prediction [B, 3, ny, nx]."""
            ny, nx = m.shape[-2:]
            h = torch.einsum("cj,bjyx->bcyx", self.P, m) + self.p[None, :, None, None]
            rows = torch.cat([torch.arange(ny - KY // 2, ny), torch.arange(0, KY // 2)]).to(m.device)
            for r, w, b in zip(self.R, self.W, self.b):
                hh = torch.fft.rfft2(h)[:, :, rows, :KX]  # [B, C, KY, KX], row j <-> ky = j - KY/2
                rc = torch.complex(r[..., 0], r[..., 1])
                gh = torch.einsum("jkoc,bcjk->bojk", rc, hh)
                full = torch.zeros(h.shape[0], C, ny, nx // 2 + 1, dtype=gh.dtype, device=m.device)
                full[:, :, rows, :KX] = gh
                g = torch.fft.irfft2(full, s=(ny, nx))
                h = torch.nn.functional.gelu(g + torch.einsum("oc,bcyx->boyx", w, h) + b[None, :, None, None])
            return torch.einsum("jc,bcyx->bjyx", self.Q, h) + self.q[None, :, None, None]

        def flat(self):
            parts = [self.P, self.p]
            for r, w, b in zip(self.R, self.W, self.b):
                parts += [r, w, b]
            parts += [self.Q, self.q]
            return torch.cat([t.detach().reshape(-1).double().cpu() for t in parts]).numpy()

        def load_flat(self, flat):
            flat = torch.as_tensor(np.asarray(flat, dtype=np.float64))
            o = 0
            for t in [self.P, self.p] + [x for trip in zip(self.R, self.W, self.b) for x in trip] + [self.Q, self.q]:
                n = t.numel()
                with torch.no_grad():
                    t.copy_(flat[o:o + n].reshape(t.shape).to(t.dtype))
                o += n
            return self

    return Sno()


def bf16_values(w):
    """FP32 -> nearest-even BF16 values (as FP32)."""
    b = np.asarray(w, dtype=np.float32).view(np.uint32).astype(np.uint64)
    b = ((b + 0x7FFF + ((b >> 16) & 1)) >> 16) << 16
    return b.astype(np.uint32).view(np.float32)


def make_pairs(n, seed, grid=(256, 256), cell=4e-9, msat=8e5, aex=1.3e-11, batch=64):
    """Textures and their exact FP32 B_demag / (mu0 Msat), both [n, 3, ny, nx]."""
    import torch

    from paper_1406_7635_amd import mm, synth

    nx, ny = grid
    params = synth.material(msat, aex, alpha=0.01)
    ctx = mm.Context((nx, ny, 1), (cell, cell, cell), np.zeros((1, ny, nx), np.uint8), params)
    xs = torch.empty((n, 3, ny, nx), dtype=torch.float32, device="cuda")
    ys = torch.empty_like(xs)
    for i0 in range(0, n, batch):
        tex = synth.film_textures(min(batch, n - i0), seed=seed * 1000003 + i0, grid=grid, cell=cell, msat=msat,
                                  aex=aex)
        for k in range(tex.shape[0]):
            m = torch.from_numpy(tex[k]).cuda()
            _, bd = ctx.beff(m, want_demag=True)
            xs[i0 + k] = m[:, 0]
            ys[i0 + k] = bd[:, 0] / (MU0 * msat)
    torch.cuda.synchronize()
    ctx.close()
    return xs, ys


def train(pairs=2048, steps=3000, batch=16, lr=3e-3, seed=5, log=print):
    import torch

    torch.manual_seed(seed)
    t0 = time.time()
    xs, ys = make_pairs(pairs, seed)
    nval = max(16, pairs // 16)
    xv, yv, xt, yt = xs[:nval], ys[:nval], xs[nval:], ys[nval:]
    log("pairs: %d (%.1f s)" % (pairs, time.time() - t0))
    model = make_model(torch).cuda()
    opt = torch.optim.Adam(model.parameters(), lr=lr)
    sched = torch.optim.lr_scheduler.OneCycleLR(opt, max_lr=lr, total_steps=steps, pct_start=0.1)
    gen = torch.Generator(device="cuda").manual_seed(seed)

    def rel(pred, y):
        return (torch.linalg.vector_norm(pred - y, dim=(1, 2, 3)) / torch.linalg.vector_norm(y, dim=(1, 2, 3))).mean()

    for step in range(steps):
        idx = torch.randint(0, xt.shape[0], (batch,), device="cuda", generator=gen)
        loss = rel(model(xt[idx]), yt[idx])
        opt.zero_grad(set_to_none=True)
        loss.backward()
        opt.step()
        sched.step()
        if step % 250 == 0 or step == steps - 1:
            with torch.no_grad():
                v = rel(model(xv), yv).item()
                vinf = ((model(xv) - yv).abs().amax(dim=(1, 2, 3)) / yv.abs().amax(dim=(1, 2, 3))).max().item()
            log("step %5d  train %.4f  val rel-L2 %.4f  val max rel-inf %.4f  (%.0f s)"
                % (step, loss.item(), v, vinf, time.time() - t0))
    return bf16_values(model.flat())


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--pairs", type=int, default=2048)
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--seed", type=int, default=5)
    a = ap.parse_args()
    w = train(a.pairs, a.steps, seed=a.seed, log=lambda s: print(s, flush=True))
    os.makedirs(os.path.dirname(os.path.abspath(a.out)), exist_ok=True)
    save_weights(a.out, w)
    print("saved", a.out, w.size, flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
