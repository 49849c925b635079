"""Helpers shared by the GPU tests: device transfer and oracle-side references."""
import numpy as np


def dev():
    import torch
    return torch.device("cuda:0")


def to_dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to(dev())


def to_np(t):
    return t.detach().cpu().numpy()


def log(msg):
    print(f"[gpu-test] {msg}", flush=True)
