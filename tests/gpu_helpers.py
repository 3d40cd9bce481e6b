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


def state_from(pa):
    """The state sph_step wrote back (caller order), as numpy arrays."""
    st = {k: to_np(pa[k]).copy() for k in ("x", "y", "z", "vx", "vy", "vz", "m", "h", "u")}
    for k in ("ax", "ay", "az", "dudt"):
        if pa[k] is not None:
            st[k] = to_np(pa[k]).copy()
    return st


STEP_FIELDS = ("x", "y", "z", "vx", "vy", "vz", "u", "h", "ax", "ay", "az", "dudt")


def step_scales(start, ref, dt, thermo=False):
    """Per-particle scale of each field after one kick-drift-kick step from `start` (the
    shared starting state, with its accelerations) to the oracle's `ref` (which carries the
    absolute-sum scales Sa, Su of its force pass): the sum of the magnitudes of what enters the
    field's update, so an error in the accelerations of size tol * Sa moves the field by at
    most about tol times this scale.
      x:  |x0| + |dt v'|,  v' = v0 + dt/2 a0
      v:  |v'| + dt/2 (Sa0 + Sa)            (Sa0 when the start carries it)
      u:  |u'| + dt/2 (Su0 + Su),  u' = u0 + dt/2 du0
          (thermokinetic: e' = e0 + dt/2 de0 and u = e - v^2/2 adds |v| S_v + v^2/2)
      a, du/dt: Sa, Su;  h: h."""
    half = 0.5 * dt
    sa0 = start.get("Sa", 0.0)
    su0 = start.get("Su", 0.0)
    vh = [start[v] + half * start[a] for v, a in (("vx", "ax"), ("vy", "ay"), ("vz", "az"))]
    sc = {}
    for k, v in zip(("x", "y", "z"), vh):
        sc[k] = np.abs(start[k]) + np.abs(dt * v)
    for k, v in zip(("vx", "vy", "vz"), vh):
        sc[k] = np.abs(v) + half * (sa0 + ref["Sa"])
    if thermo:
        e0 = start["u"] + 0.5 * (start["vx"] ** 2 + start["vy"] ** 2 + start["vz"] ** 2)
        eh = e0 + half * start["dudt"]
        vmag = np.sqrt(ref["vx"] ** 2 + ref["vy"] ** 2 + ref["vz"] ** 2)
        sv = np.sqrt(sum(v * v for v in vh)) + half * (sa0 + ref["Sa"])
        sc["u"] = np.abs(eh) + half * (su0 + ref["Su"]) + vmag * sv + 0.5 * vmag ** 2
    else:
        uh = start["u"] + half * start["dudt"]
        sc["u"] = np.abs(uh) + half * (su0 + ref["Su"])
    sc["h"] = np.abs(ref["h"])
    for k in ("ax", "ay", "az"):
        sc[k] = ref["Sa"]
    sc["dudt"] = ref["Su"]
    return sc


def step_errors(got, ref, start, dt, thermo=False):
    """|got - ref| / scale per particle and field (see step_scales); 0/0 counts as 0."""
    sc = step_scales(start, ref, dt, thermo)
    out = {}
    for k in STEP_FIELDS:
        d = np.abs(got[k] - ref[k])
        s = sc[k]
        out[k] = np.where(s > 0, d / np.where(s > 0, s, 1.0), np.where(d > 0, np.inf, 0.0))
    return out
