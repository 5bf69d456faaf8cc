"""Helpers shared by the GPU tests: seeded inputs on the device and the
comparison metric: the larger of the global relative L2 difference and the
largest per-site difference relative to the largest per-site value."""
import numpy as np

from paper_1612_02750_amd import synth


def _site_axes(a):
    """Trailing axes that make up one site's value: a 3x3 link matrix, a colour
    3-vector, or a single element."""
    if a.ndim >= 3 and a.shape[-2:] == (3, 3):
        return 2
    if a.ndim >= 2 and a.shape[-1] == 3:
        return 1
    return 0


def rel_global(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def rel_site(a, b):
    """max over sites |a_x - b_x| / max over sites |b_x| (2-norm over a site's
    colours or link elements): an error confined to a few sites (a boundary
    slice, one tile) is not diluted by the volume as in the global norm."""
    a = np.asarray(a)
    b = np.asarray(b)
    k = _site_axes(b)
    d = np.abs(a - b) ** 2
    r = np.abs(b) ** 2
    if k:
        d = d.sum(axis=tuple(range(-k, 0)))
        r = r.sum(axis=tuple(range(-k, 0)))
    return float(np.sqrt(d.max()) / np.sqrt(r.max()))


def rel(a, b):
    """The comparison metric of every parity test: max(global, per-site)."""
    return max(rel_global(a, b), rel_site(a, b))


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
