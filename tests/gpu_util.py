"""Helpers shared by the GPU tests: seeded inputs on the device and the
comparison metric (global relative L2 difference)."""
import numpy as np

from paper_1612_02750_amd import synth


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def to_dev(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def to_host(t):
    return t.detach().cpu().numpy()


def gauge(dims, kind="haar", seed=0, eps=0.3):
    if kind == "haar":
        return synth.haar_gauge(dims, seed)
    if kind == "weak":
        return synth.weak_gauge(dims, eps, seed)
    if kind == "unit":
        return synth.unit_gauge(dims)
    raise ValueError(kind)


def half_vol(dims):
    return int(np.prod(dims)) // 2
