"""Host <-> device helpers shared by the GPU tests (uint16 frames travel as
their int16 bit pattern, which every torch build can copy)."""

import sys

import numpy as np


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def to_dev(torch, a, dev):
    a = np.ascontiguousarray(a)
    if a.dtype == np.uint16:
        return torch.from_numpy(a.view(np.int16)).to(dev).view(torch.uint16)
    return torch.from_numpy(a).to(dev)


def to_host(torch, t):
    if t.dtype == torch.uint16:
        return t.view(torch.int16).cpu().numpy().view(np.uint16)
    return t.cpu().numpy()


def full(torch, shape, val, dtype, dev):
    if dtype == torch.uint16:
        return torch.full(shape, val, dtype=torch.int16, device=dev).view(torch.uint16)
    return torch.full(shape, val, dtype=dtype, device=dev)


def same(torch, a, b):
    """Bitwise equality of two device tensors of the same pixel type."""
    if a.dtype == torch.uint16:
        return torch.equal(a.view(torch.int16), b.view(torch.int16))
    return torch.equal(a, b)
