"""Helpers for the GPU tests: device tensors and the comparison metric."""
import numpy as np


def dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).to("cuda:0")


def host(t):
    return t.detach().to("cpu").numpy()


def maxabs(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b)))) if np.size(a) else 0.0


def announce(msg):
    print(f"[gpu-test] {msg}", flush=True)
