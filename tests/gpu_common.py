"""Helpers shared by the GPU tests (not collected: no test_ prefix)."""
import math
import sys

import numpy as np

import oracle as O


def cuda(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).to("cuda")


def host(t):
    return t.detach().to("cpu").numpy()


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def max_rel(a, b):
    """Largest element-wise error, relative to the largest reference element."""
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.abs(a - b).max() / np.abs(b).max())


def oracle_params(info) -> O.Params:
    """The K~ the plan realises, handed to the oracle (parameters only)."""
    return O.Params(d=info["d"], nu=info["nu"], t_min=info["t_min"], t_max=info["t_max"],
                    n_t=info["n_t"], s_min=info["s_min"], s_max=info["s_max"],
                    n_sigma=info["n_sigma"], dw=info["dw"], M=info["M"],
                    center=tuple(info["center"]), scale=info["scale"])


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()
