"""Helpers for the GPU tests: moving numpy arrays to and from the device."""
import numpy as np


def dev():
    import torch
    return torch.device("cuda:0")


def to_dev(a: np.ndarray):
    import torch
    a = np.ascontiguousarray(a)
    view = {np.dtype(np.uint64): np.int64, np.dtype(np.uint32): np.int32}.get(a.dtype)
    if view is not None:
        a = a.view(view)
    return torch.from_numpy(a).to(dev())


def empty(m, kind):
    import torch
    dt = {"u32": torch.int32, "u8": torch.uint8, "u64": torch.int64}[kind]
    return torch.empty(m, dtype=dt, device=dev())


def to_np(t, kind):
    a = t.cpu().numpy()
    return a.view({"u32": np.uint32, "u8": np.uint8, "u64": np.uint64}[kind])


def announce(msg):
    print(msg, flush=True)
