"""Pins of the surrogate's FP64 forward pass (oracle/sno.py): the truncated
transforms against numpy's real 2D FFTs, a pure mode against its closed form,
the pointwise part against a brute-force per-pixel evaluation, translation
equivariance, and GELU against known values of the normal distribution."""
import math

import numpy as np

from oracle import sno
from paper_1406_7635_amd import synth


def test_weight_layout_round_trip():
    w = synth.sno_random_weights(3).astype(np.float64)
    assert w.size == sno.weight_count() == synth.SNO_NWEIGHTS
    assert np.array_equal(sno.pack(sno.unpack(w)), w)
    u = sno.unpack(w)
    # R[l][ky][kx][o][c] real and imaginary parts interleaved after P, p
    off = 32 * 3 + 32
    assert u["R"][0][2, 5, 7, 11].real == w[off + (((2 * 16 + 5) * 32 + 7) * 32 + 11) * 2]
    assert u["R"][0][2, 5, 7, 11].imag == w[off + (((2 * 16 + 5) * 32 + 7) * 32 + 11) * 2 + 1]


def test_gelu_known_values():
    # Phi(1) = 0.841344746068543, Phi(-1) = 0.158655253931457 (standard normal)
    assert abs(sno.gelu(1.0) - 0.8413447460685429) < 1e-15
    assert abs(sno.gelu(-1.0) + 0.15865525393145707) < 1e-15
    assert sno.gelu(0.0) == 0.0
    x = np.linspace(-6, 6, 25)
    assert np.allclose(sno.gelu(x) - sno.gelu(-x), x, atol=1e-14)


def test_truncated_transforms_match_numpy_real_fft():
    rng = np.random.Generator(np.random.PCG64(1))
    ny, nx = 48, 64
    h = rng.standard_normal((3, ny, nx))
    fx, fy = sno.mode_matrices(nx, ny)
    hh = sno.forward_modes(h, fx, fy)
    ref = np.fft.rfft2(h, axes=(1, 2))
    for j in range(sno.KY):
        ky = j - sno.KY // 2
        assert np.allclose(hh[:, j, :], ref[:, ky % ny, :sno.KX], rtol=1e-12, atol=1e-10)
    g_hat = rng.standard_normal((3, sno.KY, sno.KX)) + 1j * rng.standard_normal((3, sno.KY, sno.KX))
    full = np.zeros((3, ny, nx // 2 + 1), dtype=np.complex128)
    for j in range(sno.KY):
        full[:, (j - sno.KY // 2) % ny, :sno.KX] = g_hat[:, j, :]
    ref_inv = np.fft.irfft2(full, s=(ny, nx), axes=(1, 2))
    assert np.allclose(sno.inverse_modes(g_hat, fx, fy, nx, ny), ref_inv, rtol=1e-12, atol=1e-14)


def test_pure_mode_passes_an_identity_layer():
    """A cosine at a kept mode through R = identity at that mode, W = 0, b = 0:
    the spectral branch returns the same cosine."""
    ny = nx = 32
    fx, fy = sno.mode_matrices(nx, ny)
    y, x = np.mgrid[0:ny, 0:nx]
    for kx0, ky0 in ((3, -5), (0, 2), (15, 7), (1, -8)):
        h = np.cos(2 * np.pi * (kx0 * x / nx + ky0 * y / ny))[None]
        hh = sno.forward_modes(h, fx, fy)
        keep = np.zeros_like(hh)
        keep[:, ky0 + sno.KY // 2, kx0] = hh[:, ky0 + sno.KY // 2, kx0]
        if kx0 == 0:  # the conjugate mode -ky0 is kept too
            keep[:, -ky0 + sno.KY // 2, 0] = hh[:, -ky0 + sno.KY // 2, 0] if -ky0 < sno.KY // 2 else 0
        g = sno.inverse_modes(keep, fx, fy, nx, ny)
        expect = h if (kx0 > 0 or -ky0 < sno.KY // 2) else 0.5 * h
        assert np.allclose(g, expect, atol=1e-12), (kx0, ky0)


def test_pointwise_part_brute_force():
    """With every spectral weight zero the network is a per-pixel MLP:
    evaluate it cell by cell with plain loops."""
    w = sno.unpack(synth.sno_random_weights(5).astype(np.float64))
    for r in w["R"]:
        r[...] = 0
    flat = sno.pack(w)
    rng = np.random.Generator(np.random.PCG64(2))
    m = rng.standard_normal((3, 4, 4))
    got = sno.forward(flat, m)
    for yy in range(4):
        for xx in range(4):
            h = [sum(w["P"][c][j] * m[j, yy, xx] for j in range(3)) + w["p"][c] for c in range(32)]
            for layer in range(4):
                z = [sum(w["W"][layer][o][c] * h[c] for c in range(32)) + w["b"][layer][o] for o in range(32)]
                h = [0.5 * v * (1.0 + math.erf(v / math.sqrt(2.0))) for v in z]
            for j in range(3):
                ref = sum(w["Q"][j][c] * h[c] for c in range(32)) + w["q"][j]
                assert abs(got[j, yy, xx] - ref) < 1e-12 * max(1.0, abs(ref))


def test_translation_equivariance():
    flat = synth.sno_random_weights(7).astype(np.float64)
    rng = np.random.Generator(np.random.PCG64(3))
    m = rng.standard_normal((3, 32, 32))
    a = sno.forward(flat, np.roll(m, (5, -3), axis=(1, 2)))
    b = np.roll(sno.forward(flat, m), (5, -3), axis=(1, 2))
    assert np.allclose(a, b, atol=1e-11)
