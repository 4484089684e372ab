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


def check_tune_report(rep, nvar):
    """Stage 1 times nvar variants on the plans' current cuts; stage 2 the
    best of them again with its plan cut at half and at twice its work-item
    length (one or two more entries).  The chosen entry is the fastest."""
    v = rep["variants"]
    assert nvar + 1 <= len(v) <= nvar + 2 and 0 <= rep["chosen"] < len(v)
    assert all(x["ms"] > 0 for x in v)
    assert v[rep["chosen"]]["ms"] == min(x["ms"] for x in v)
    assert {x["plan"] for x in v[:nvar]} == {"fused", "two_visit"}
    b = min(range(nvar), key=lambda i: v[i]["ms"])
    for x in v[nvar:]:
        assert (x["plan"], x["occupancy"], x["skip_zero"]) == (v[b]["plan"], v[b]["occupancy"], v[b]["skip_zero"])
        assert x["item_blocks"] in (v[b]["item_blocks"] // 2, 2 * v[b]["item_blocks"])
