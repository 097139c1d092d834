"""Helpers shared by the GPU parity tests (inputs only; no method arithmetic)."""

import numpy as np


def perturbed(O, p, seed, amp=0.02):
    """Free stream plus a seeded perturbation of every coefficient, scaled with
    sqrt(|E|) so the physical perturbation is O(amp) everywhere."""
    rng = np.random.default_rng(seed)
    u = O.freestream(p)
    vol, *_ = O.geometry()
    return u + amp * rng.uniform(-1, 1, u.shape) * np.sqrt(vol)[:, None, None]


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def to_host(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def rel_err(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))
