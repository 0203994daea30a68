"""Helpers for the GPU parity tests: device tensors, and the oracle side of
each comparison.  Everything here runs only when a HIP device is present."""
import numpy as np

import synth


def dev(a, dtype=None):
    import torch
    t = torch.as_tensor(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda().contiguous()


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def empty(shape, dtype):
    import torch
    return torch.empty(shape, dtype=dtype, device="cuda")


def zeros(shape, dtype):
    import torch
    return torch.zeros(shape, dtype=dtype, device="cuda")


def real_np(ctx):
    return np.float64 if ctx.precision == 0 else np.float32


def small_scenario(name="c1", precision="fp64", **kw):
    """A generator scenario shrunk to oracle-friendly sizes."""
    base = {"c1": synth.c1, "c2": synth.c2}[name](precision=precision)
    return synth.shrink(base, **kw) if kw else base


def rel_err(a, b, floor=1e-3):
    return np.abs(a - b) / np.maximum(np.abs(b), floor)


def separable_field(scen, seed, M=None):
    """Correlated wind fields W[m, g, c] for a scenario's grid, built by
    applying the three 1-D Cholesky factors along their axes (the Kronecker
    product without forming the G x G matrix).  Test input only."""
    from oracle import wind as owind
    ax, ay, az = owind.grid_axes(scen["box"], scen["grid"])
    Lx, Ly, Lz = (owind.axis_factor(a, scen["wind_ell"], scen["wind_nugget"]) for a in (ax, ay, az))
    M = scen["M"] if M is None else M
    nx, ny, nz = (int(n) for n in scen["grid"])
    Z = np.random.default_rng(seed).standard_normal((nx, ny, nz, M, 2))
    # one axis at a time: (Lx kron Ly kron Lz) Z without the G x G matrix
    W = np.tensordot(Lx, Z, axes=(1, 0))                            # a j k m q
    W = np.moveaxis(np.tensordot(Ly, W, axes=(1, 1)), 0, 1)         # a b k m q
    W = np.moveaxis(np.tensordot(Lz, W, axes=(1, 2)), 0, 2)         # a b c m q
    W = W * scen["wind_sigma"]
    W = W.reshape(nx * ny * nz, M, 2).transpose(1, 0, 2).copy()
    return W + np.asarray(scen["wind_mean"])[None, None, :]
