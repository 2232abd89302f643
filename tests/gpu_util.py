"""Helpers for the GPU tests: device copies of seeded inputs and the entrywise rounding bound."""
import numpy as np

U32 = 2.0 ** -24


def gamma(n: int) -> float:
    """gamma_n = n u / (1 - n u) for binary32 (u = 2^-24): bound on n accumulated roundings."""
    return n * U32 / (1 - n * U32)


def dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def say(msg: str):
    print(msg, flush=True)
