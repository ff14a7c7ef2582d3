"""Helpers shared by the GPU tests: device transfers and comparisons."""
import numpy as np


def dev(a, dtype=None):
    """NumPy complex array -> contiguous torch tensor on cuda:0."""
    import torch
    a = np.ascontiguousarray(a)
    if dtype is not None:
        a = a.astype(dtype)
    return torch.from_numpy(a).to("cuda")


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def arena(nbytes):
    import torch
    return torch.zeros(int(nbytes), dtype=torch.uint8, device="cuda")


def max_rel(got, ref):
    """max |got - ref| / max |ref| over all entries."""
    got = np.asarray(got, dtype=np.complex128)
    ref = np.asarray(ref, dtype=np.complex128)
    return float(np.max(np.abs(got - ref)) / max(np.max(np.abs(ref)), 1e-300))


def l2_rel(got, ref):
    got = np.asarray(got, dtype=np.complex128)
    ref = np.asarray(ref, dtype=np.complex128)
    return float(np.linalg.norm(got - ref) / np.linalg.norm(ref))


def banner(msg):
    """Name the case on stdout before a GPU step (flushed)."""
    print("[gpu-case] " + msg, flush=True)
