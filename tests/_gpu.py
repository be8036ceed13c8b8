"""Helpers shared by the GPU tests (test code only)."""
import numpy as np
import torch

TOL = {  # parity bars on ||dpsi|| and |dF| (the stated accuracy targets)
    "c64": 1e-6,
    "c128": 1e-10,
}


def tdtype(name):
    return torch.complex64 if name == "c64" else torch.complex128


def to_dev(v, name):
    return torch.from_numpy(np.ascontiguousarray(v)).to(device="cuda", dtype=tdtype(name))


def to_host(t):
    return t.detach().to("cpu").to(torch.complex128).numpy()


def rel_err(got, want):
    return float(np.linalg.norm(got - want) / max(np.linalg.norm(want), 1e-300))
