"""Shared helpers of the GPU parity tests (argument plumbing only)."""
import numpy as np


def rel_l2(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def rel_max(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    mb = np.abs(b).max()
    return np.abs(a - b).max() / (mb if mb > 0 else 1.0)


def to_dev(torch, a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def load_state(ch, u, v, w, p=None):
    import torch
    ch.field(0).copy_(torch.from_numpy(np.ascontiguousarray(u)))
    ch.field(1).copy_(torch.from_numpy(np.ascontiguousarray(v)))
    ch.field(2).copy_(torch.from_numpy(np.ascontiguousarray(w)))
    if p is not None:
        ch.field(3).copy_(torch.from_numpy(np.ascontiguousarray(p)))
    torch.cuda.synchronize()


def fields(ch):
    import torch
    torch.cuda.synchronize()
    return {name: ch.field(k).cpu().numpy().copy() for k, name in enumerate(["u", "v", "w", "p", "nut", "b"])}
