"""Shared helpers of the GPU tests (device context, tensor transfer)."""
import numpy as np

from oracle import fullgrid
from paper_2403_04946_amd import tt


def make_ctx():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return tt.Context(0)


def upload(ctx, cores, caps=None):
    d, n = len(cores), cores[0].shape[1]
    ranks = [1] + [c.shape[2] for c in cores]
    if caps is None:
        caps = ranks
    elif np.isscalar(caps):
        caps = [1] + [max(int(caps), r) for r in ranks[1:-1]] + [1]
    t = tt.Tensor(ctx, d, n, caps)
    t.set_cores(cores)
    return t


def full(t):
    return fullgrid.tt_to_full(t.get_cores())


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(np.asarray(b).ravel()), 1e-300))
