"""Shared helpers of the GPU parity tests: build a library context and the
oracle problem from the same seeded inputs, and compare fields."""
import sys

import numpy as np

from oracle import fields as ofields


def log(*args):
    print(*args, flush=True)
    sys.stdout.flush()


def make_pair(case, demag=True):
    """(GPU context, oracle problem, m0 tensor on cuda:0) for a synth case."""
    import torch

    from paper_1406_7635_amd import mm

    ctx = mm.Context(case["grid"], case["cell"], case["region"], case["params"], demag=demag)
    prob = ofields.Problem(case["grid"], case["cell"], case["region"], case["params"], demag=demag)
    m = torch.from_numpy(np.ascontiguousarray(case["m0"])).to("cuda:0")
    return ctx, prob, m


def make_ctx(case, demag=True):
    """(GPU context, m0 tensor on cuda:0) without the oracle problem (whose
    demagnetising tensor would be built for nothing)."""
    import torch

    from paper_1406_7635_amd import mm

    ctx = mm.Context(case["grid"], case["cell"], case["region"], case["params"], demag=demag)
    return ctx, torch.from_numpy(np.ascontiguousarray(case["m0"])).to("cuda:0")


def rel_inf(got, ref):
    """max |got - ref| / max |ref| over all cells and components."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    scale = np.max(np.abs(ref))
    return float(np.max(np.abs(got - ref)) / (scale if scale > 0 else 1.0))


def to_np(t):
    return t.detach().cpu().numpy().astype(np.float64)
