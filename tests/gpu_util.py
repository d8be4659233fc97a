"""Helpers for the GPU tests: run the HIP path through the C-ABI binding and
the oracle on the same seeded inputs."""
import sys

import numpy as np

from oracle import oracle as O
from paper_1710_10420_amd.inputs import uniform_at


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def torch_mod():
    import torch
    return torch


def gpu_prs():
    from paper_1710_10420_amd import prs
    return prs


def params_pair(shape, deta, m=1.0, W0=10.0, alpha=3.0, dx=1.0, diag_every=0, eta0=1.0, beta=0.0,
                precision=None):
    prs = gpu_prs()
    kw = {} if precision is None else {"precision": precision}
    gp = prs.make_params(shape, deta=deta, m=m, W0=W0, alpha=alpha, dx=dx, diag_every=diag_every,
                         eta0=eta0, beta=beta, **kw)
    op = O.params(shape, deta=deta, m=m, W0=W0, alpha=alpha, dx=dx, eta0=eta0, beta=beta)
    return gp, op


def to_dev(a):
    torch = torch_mod()
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32).reshape(-1)).cuda()


def host(t):
    return t.detach().cpu().numpy().reshape(-1)


def gpu_run(gp, phi0, steps, dphi0=None, tiling=None, diag=True):
    """Run the HIP path from a host initial field; returns (phi, dphi, records, sim)."""
    prs = gpu_prs()
    sim = prs.Sim(gp, phi0=to_dev(phi0), dphi0=None if dphi0 is None else to_dev(dphi0))
    if tiling is not None:
        sim.set_tiling(*tiling)
    recs = sim.step_n(steps, diag=diag)
    phi, dphi = sim.state()
    return host(phi), host(dphi), recs, sim


def rel_linf(a, ref):
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.max(np.abs(np.asarray(a, dtype=np.float64) - ref)) / max(np.max(np.abs(ref)), 1e-300))


def assert_stats_match(g, o, rel=1e-12, ctx=""):
    """Counts bit for bit, FP64 sums to summation-order rounding."""
    assert g["links_dir"] == o["links_dir"], (ctx, g, o)
    assert g["links"] == o["links"], ctx
    assert g["wall_sites"] == o["wall_sites"], ctx
    assert g["nonfinite"] == o["nonfinite"], ctx
    assert g["step"] == o["step"], ctx
    for key in ("area_density", "gv2"):
        a, b = g[key], o[key]
        assert abs(a - b) <= rel * max(abs(b), 1e-300), (ctx, key, a, b)


def patch_indices(shape, center, half):
    """Linear site indices of a periodic cube of side 2*half+1 centred at
    `center` (x, y[, z]), in numpy layout (z, y, x)."""
    D = len(shape)
    offs = np.arange(-half, half + 1)
    axes = [(center[d] + offs) % shape[d] for d in range(D)]
    grids = np.meshgrid(*reversed(axes), indexing="ij")   # z, y, x
    grids = list(reversed(grids))                          # x, y, z
    idx = np.zeros(grids[0].shape, dtype=np.int64)
    stride = 1
    for d in range(D):
        idx += grids[d].astype(np.int64) * stride
        stride *= shape[d]
    return idx


def oracle_patch(op_full, shape, seed, center, steps, h):
    """Evolve the periodic patch around `center` with the oracle; the inner
    cube of half-width h is exact after `steps` steps (its dependence cone
    stays inside the patch).  Returns (indices of the inner cube, values)."""
    half = steps + h
    idx = patch_indices(shape, center, half)
    D = len(shape)
    side = 2 * half + 1
    op = O.params((side,) * D, deta=op_full.deta, alpha=op_full.alpha, m=op_full.m,
                  W0=op_full.W0, dx=op_full.dx, eta0=op_full.eta0)
    phi0 = uniform_at(seed, idx.reshape(-1)).astype(np.float64)
    phi, _, _ = O.run(op, phi0, np.zeros_like(phi0), steps)
    sl = tuple(slice(steps, steps + 2 * h + 1) for _ in range(D))
    return idx[sl].reshape(-1), phi.reshape(idx.shape)[sl].reshape(-1)
