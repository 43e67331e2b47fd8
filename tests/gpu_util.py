"""Helpers for the GPU tests: device tensors from seeded host arrays."""
import numpy as np

import synthgen


def dev(a: np.ndarray):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def host(t) -> np.ndarray:
    return t.detach().to("cpu").numpy()


def uniform(seed, r, c):
    return synthgen.uniform_pm1(seed, r, c)


def ints(seed, r, c, lo=-1, hi=1):
    return synthgen.int_range(seed, r, c, lo, hi)


def empty_dev(r, c, fill=np.nan):
    import torch
    return torch.full((r, c), float(fill), dtype=torch.float32, device="cuda")


def say(msg: str):
    print(msg, flush=True)
