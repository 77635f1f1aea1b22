"""Helpers shared by the GPU tests (torch device tensors <-> numpy)."""

import numpy as np


def torch_mod():
    import torch
    return torch


def to_dev(a):
    torch = torch_mod()
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.complex128)).to("cuda")


def to_host(t):
    torch = torch_mod()
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def rel_max(a, b):
    """max |a - b| / max |b|"""
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def announce(msg):
    print(f"[gpu-case] {msg}", flush=True)
