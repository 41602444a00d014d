"""Spectral neural operator (the surrogate of the magnetostatic field): its
forward pass written out in FP64 (oracle, CPU).

Test infrastructure: only tests/, the smoke check and the benchmark's CPU
baseline use this module.

The network maps the magnetisation m (3 channels on an nx x ny grid) to a
prediction of B_demag in units of mu0 Msat.  It is not part of the paper's
method; it is the learned stand-in for the convolution whose exact form the
paper computes in section "Magnetostatic field".  Definition:

  lift        h0_c(r) = sum_j P[c, j] m_j(r) + p[c],                c < C
  layer l     hhat_c(kx, ky) = sum_{x,y} h_c(x, y) exp(-2 pi i (kx x/nx + ky y/ny))
              for the kept modes kx = 0 .. KX-1, ky = -KY/2 .. KY/2-1;
              ghat_o(k) = sum_c R[l, ky + KY/2, kx, o, c] hhat_c(k)   (complex R);
              g_o(x, y) = Re sum_k w_kx ghat_o(k) exp(+2 pi i (kx x/nx + ky y/ny)) / (nx ny),
              w_0 = 1, w_kx = 2 otherwise (the real inverse of a spectrum that is
              zero outside the kept modes);
              h_o <- GELU(g_o + sum_c W[l, o, c] h_c + b[l, o]),
              GELU(z) = z (1 + erf(z / sqrt 2)) / 2;
  project     y_j(r) = sum_c Q[j, c] h_c(r) + q[j],                   j < 3.

The weights travel as one flat array in the order P, p, then per layer R
(real and imaginary interleaved, index [ky][kx][o][c][re/im]), W, b, then Q,
q (`unpack` / `pack`).

Parity: pinned in tests/test_oracle_sno.py (the truncated transforms against
numpy's real FFTs, a pure mode against its closed form, brute-force pointwise
layers, translation equivariance).
"""
import math

import numpy as np
from scipy.special import erf

C, KX, KY, NLAYER = 32, 16, 16, 4


def weight_count(c=C, kx=KX, ky=KY, nlayer=NLAYER):
    return c * 3 + c + nlayer * (ky * kx * c * c * 2 + c * c + c) + 3 * c + 3


def unpack(flat, c=C, kx=KX, ky=KY, nlayer=NLAYER):
    """Named weight arrays (FP64) from the flat array."""
    w = np.asarray(flat, dtype=np.float64).ravel()
    if w.size != weight_count(c, kx, ky, nlayer):
        raise ValueError("expected %d weights, got %d" % (weight_count(c, kx, ky, nlayer), w.size))
    o = 0

    def take(shape):
        nonlocal o
        n = int(np.prod(shape))
        a = w[o:o + n].reshape(shape)
        o += n
        return a

    out = {"P": take((c, 3)), "p": take((c,)), "R": [], "W": [], "b": []}
    for _ in range(nlayer):
        r = take((ky, kx, c, c, 2))
        out["R"].append(r[..., 0] + 1j * r[..., 1])
        out["W"].append(take((c, c)))
        out["b"].append(take((c,)))
    out["Q"] = take((3, c))
    out["q"] = take((3,))
    return out


def pack(w):
    """Flat array from the named weights (inverse of unpack)."""
    parts = [w["P"].ravel(), w["p"].ravel()]
    for r, wl, bl in zip(w["R"], w["W"], w["b"]):
        parts.append(np.stack([r.real, r.imag], axis=-1).ravel())
        parts.append(wl.ravel())
        parts.append(bl.ravel())
    parts += [w["Q"].ravel(), w["q"].ravel()]
    return np.concatenate(parts)


def gelu(z):
    """z Phi(z) with the exact normal distribution function (erf form)."""
    return 0.5 * z * (1.0 + erf(z / math.sqrt(2.0)))


def mode_matrices(nx, ny, kx=KX, ky=KY):
    """Forward transform matrices of the kept modes: Fx[kx, x] =
    exp(-2 pi i kx x / nx), Fy[j, y] = exp(-2 pi i (j - KY/2) y / ny)."""
    x = np.arange(nx)
    y = np.arange(ny)
    kxs = np.arange(kx)
    kys = np.arange(ky) - ky // 2
    fx = np.exp(-2j * np.pi * np.outer(kxs, x) / nx)
    fy = np.exp(-2j * np.pi * np.outer(kys, y) / ny)
    return fx, fy


def forward_modes(h, fx, fy):
    """hhat[c, j, kx] = sum_{y,x} h[c, y, x] Fy[j, y] Fx[kx, x] for fields h[c, ny, nx]."""
    return np.einsum("jy,cyx,kx->cjk", fy, h, fx, optimize=True)


def inverse_modes(g_hat, fx, fy, nx, ny):
    """Real field of a spectrum that is zero outside the kept modes:
    g[c, y, x] = Re sum_{j,kx} w_kx ghat[c, j, kx] conj(Fy[j, y]) conj(Fx[kx, x]) / (nx ny)."""
    wk = np.full(fx.shape[0], 2.0)
    wk[0] = 1.0
    z = np.einsum("cjk,jy,kx->cyx", g_hat * wk[None, None, :], np.conj(fy), np.conj(fx), optimize=True)
    return z.real / (nx * ny)


def forward(flat_weights, m):
    """Prediction y[3, ny, nx] for m[3, ny, nx] (or [3, 1, ny, nx])."""
    w = unpack(flat_weights)
    m = np.asarray(m, dtype=np.float64)
    if m.ndim == 4:
        m = m[:, 0]
    _, ny, nx = m.shape
    fx, fy = mode_matrices(nx, ny)
    h = np.einsum("cj,jyx->cyx", w["P"], m) + w["p"][:, None, None]
    for r, wl, bl in zip(w["R"], w["W"], w["b"]):
        hh = forward_modes(h, fx, fy)
        gh = np.einsum("jkoc,cjk->ojk", r, hh)
        g = inverse_modes(gh, fx, fy, nx, ny)
        h = gelu(g + np.einsum("oc,cyx->oyx", wl, h) + bl[:, None, None])
    return np.einsum("jc,cyx->jyx", w["Q"], h) + w["q"][:, None, None]
