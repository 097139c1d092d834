"""Helpers shared by the GPU parity tests (inputs only; no method arithmetic)."""

import numpy as np


def perturbed(O, p, seed, amp=0.02):
    """Free stream plus a seeded perturbation: coefficient i of every variable
    gets amp * sqrt(|E|) * 4^(-deg_i) * U(-1, 1), deg_i the largest 1D degree of
    mode i, so the physical perturbation stays O(amp) at every order.  The
    state is checked to be physical (finite oracle residual)."""
    import oracle
    rng = np.random.default_rng(seed)
    u = O.freestream(p)
    vol, *_ = O.geometry()
    deg = oracle.modes(O.dim, p)[:, : O.dim].max(axis=1)
    scale = np.sqrt(vol)[:, None, None] * (0.25 ** deg)[None, None, :]
    u = u + amp * rng.uniform(-1, 1, u.shape) * scale
    assert np.all(np.isfinite(O.residual(p, u))), "perturbed state is not physical"
    return u


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def to_host(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def rel_err(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))
