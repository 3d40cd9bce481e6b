"""Helpers for the GPU parity tests: run the HIP path through the C ABI binding and return
numpy arrays in caller order; compare against the oracle with the stated tolerances."""
from __future__ import annotations

import numpy as np


def to_np(t):
    return t.detach().cpu().numpy()


def make_ctx(n_cap, seg_cap=1, **cfg):
    import paper_2007_03097_amd as sph
    return sph.Context(max(int(n_cap), 1), seg_cap, **cfg)


def tuned(ctx, pa, dt=1e-4):
    """Leaf and group sizes (and waves per CU) the benchmark uses for this workload (the
    package's tuning file); returns (leaf, group)."""
    import paper_2007_03097_amd as sph
    sph.sph_autotune(ctx.h, pa, dt, sph.TUNING_CACHE)
    return sph.sph_get_tuning(ctx.h)[:2]


def parts(ps, with_accel=False):
    import paper_2007_03097_amd as sph
    return sph.ParticleArrays.from_numpy(ps, with_accel=with_accel)


def gpu_keys_order(ctx, pa, box=None):
    import torch
    import paper_2007_03097_amd as sph
    n = pa.n
    keys = torch.zeros(max(n, 1), dtype=torch.int64, device="cuda")
    order = torch.zeros(max(n, 1), dtype=torch.int64, device="cuda")
    sph.sph_build_tree(ctx.h, pa, box=box, keys_out=keys, order_out=order)
    torch.cuda.synchronize()
    return to_np(keys)[:n].view(np.uint64), to_np(order)[:n]


def gpu_tree(ctx):
    import torch
    import paper_2007_03097_amd as sph
    cap = 24 * ctx.n_capacity + 64
    key = torch.zeros(cap, dtype=torch.int64, device="cuda")
    lev = torch.zeros(cap, dtype=torch.int32, device="cuda")
    leaf = torch.zeros(cap, dtype=torch.int32, device="cuda")
    st = torch.zeros(cap, dtype=torch.int64, device="cuda")
    ct = torch.zeros(cap, dtype=torch.int64, device="cuda")
    nn = sph.sph_tree_nodes(ctx.h, cap, key, lev, leaf, st, ct)
    return dict(key=to_np(key)[:nn].view(np.uint64), level=to_np(lev)[:nn], leaf=to_np(leaf)[:nn].astype(bool),
                start=to_np(st)[:nn], count=to_np(ct)[:nn])


def gpu_neighbors(ctx, n):
    import torch
    import paper_2007_03097_amd as sph
    off = torch.zeros(n + 1, dtype=torch.int64, device="cuda")
    total = sph.sph_find_neighbors(ctx.h, off, None, 0)
    idx = torch.zeros(max(total, 1), dtype=torch.int32, device="cuda")
    sph.sph_find_neighbors(ctx.h, off, idx, total)
    return to_np(off), to_np(idx)[:total].astype(np.int64)


def gpu_density(ctx, n):
    import torch
    import paper_2007_03097_amd as sph
    out = [torch.zeros(max(n, 1), dtype=torch.float64, device="cuda") for _ in range(4)]
    sph.sph_compute_density(ctx.h, *out)
    torch.cuda.synchronize()
    return [to_np(o)[:n] for o in out]


def gpu_forces(ctx, n, thermo=None):
    import torch
    import paper_2007_03097_amd as sph
    out = [torch.zeros(max(n, 1), dtype=torch.float64, device="cuda") for _ in range(4)]
    kw = {}
    if thermo is not None:
        kw = {k: torch.as_tensor(v, dtype=torch.float64, device="cuda") for k, v in zip(("rho", "P", "cs"), thermo)}
    sph.sph_compute_forces(ctx.h, *out, **kw)
    torch.cuda.synchronize()
    return [to_np(o)[:n] for o in out]


def gpu_gravity(ctx, n):
    """g and phi in caller order; sph_sync surfaces any device-side error (e.g. a walk list
    overflow) as an exception instead of leaving partial sums."""
    import torch
    import paper_2007_03097_amd as sph
    out = [torch.zeros(max(n, 1), dtype=torch.float64, device="cuda") for _ in range(4)]
    sph.sph_compute_gravity(ctx.h, *out)
    sph.sph_sync(ctx.h)
    torch.cuda.synchronize()
    return [to_np(o)[:n] for o in out]


def rel_err(got, ref, scale):
    """max_a |got_a - ref_a| / scale_a (scale > 0)."""
    scale = np.where(scale > 0, scale, 1e-300)
    return float(np.max(np.abs(got - ref) / scale)) if got.size else 0.0


def vec_rel_err(g3, r3, scale):
    d = np.sqrt(sum((a - b) ** 2 for a, b in zip(g3, r3)))
    scale = np.where(scale > 0, scale, 1e-300)
    return float(np.max(d / scale)) if d.size else 0.0
