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
