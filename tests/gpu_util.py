"""Shared helpers of the GPU tests: run the HIP solver through the C ABI on
seeded inputs and compare with the CPU oracle."""
import sys

import numpy as np

from paper_1606_08740_amd import aar, inputs


def say(msg: str) -> None:
    """Name the case before a GPU step (flushed, so it survives a crash)."""
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def to_dev(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda:0")


def gpu_solve(prob, params, b, x0=None):
    import torch
    s = aar.Solver([prob], params)
    bt = to_dev(b)
    xt = to_dev(np.zeros(prob.size) if x0 is None else x0)
    res = s.solve(bt, xt)
    torch.cuda.synchronize()
    out = xt.cpu().numpy()
    log = s.residual_log() if params.flags & aar.AAR_FLAG_RECORD_RESIDUALS else None
    s.close()
    return out, res, log


def params(**kw):
    p = inputs.Params()
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def rel_err(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def mean_free(v):
    return v - v.mean()
