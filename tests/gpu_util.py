"""Helpers for the GPU parity tests: host <-> device column transfer and the
per-item scales the tolerances need."""

import numpy as np
import torch

DEV = "cuda:0"


def gpu(cols, dtype):
    """numpy columns -> contiguous GPU tensors of ``dtype``."""
    return tuple(torch.from_numpy(np.ascontiguousarray(c, dtype=np.float64)).to(DEV).to(dtype).contiguous()
                 for c in cols)


def host(t):
    if isinstance(t, (tuple, list)):
        return tuple(host(x) for x in t)
    return t.detach().to("cpu").numpy()


def widened(cols, dtype):
    """The values the GPU actually sees, as float64 (exact for FP32)."""
    np_dtype = np.float32 if dtype == torch.float32 else np.float64
    return tuple(np.asarray(c, dtype=np_dtype).astype(np.float64) for c in cols)


def event_abs_scale(cart, offsets):
    """Per event: S_abs = (sum|E_i|)^2 + (sum|px_i|)^2 + (sum|py_i|)^2 + (sum|pz_i|)^2
    and sum|c_i| per component (rounding scales of sums and their mass)."""
    sums = []
    for c in cart:
        cs = np.concatenate([[0.0], np.cumsum(np.abs(c))])
        sums.append(np.maximum(cs[offsets[1:]] - cs[offsets[:-1]], 0.0))
    S = sums[3] ** 2 + sums[0] ** 2 + sums[1] ** 2 + sums[2] ** 2
    return S, sums
