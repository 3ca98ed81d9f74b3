"""Helpers shared by the GPU tests (no method arithmetic here)."""
import numpy as np


def dev(a, dtype):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype).cuda().contiguous()


def host(t):
    return t.detach().cpu().double().numpy()


def torch_dtype(precision):
    import torch
    return torch.float64 if precision == "fp64" else torch.float32


def say(*a):
    print("[gpu-case]", *a, flush=True)
