#!/usr/bin/env python3
"""Benchmark: pair interactions/s (density + force) and steps/s of the SPH + octree hot path
on one MI355X, FP64 and FP32-compensated, on the 3D Sod-type tube workload.

Workload: 987,840 particles in [0,1] x [0,0.1]^2 (two lattices with spacing ratio 2:1:
rho = 1, P = 1 left; rho = 0.125, P = 0.1 right), gamma = 5/3, adaptive h = 1.2 (m/rho)^(1/3),
Monaghan viscosity alpha = 1, beta = 2, kick-drift-kick leapfrog at dt = 0.25 min(h/c).
One benchmark step = one full leapfrog step: bounding box, keys, radix sort, reorder,
octree + moments, neighbour lists, density + EOS, forces, kicks.  Inputs are resident in
HBM before the timed region.

value = (density pairs + force pairs per step) * steps / wall time of the timed steps (FP64).
The FP32C form, per-kernel event timings, the roofline of the dominant kernel and a CPU
reference baseline are reported in the same JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6     # MI355X FP64 vector, 256 CU x 64 lanes x 2 flop x 2.4 GHz
HBM_PEAK_GBS = 8000.0
# leaf size, group size and waves per CU chosen by sph_autotune on MI355X, keyed by workload;
# missing keys are tuned on the spot (and appended to that file)
TUNING_CACHE = os.path.join(ROOT, "paper_2007_03097_amd", "tuning_gfx950.json")  # = paper_2007_03097_amd.TUNING_CACHE

# Algorithmic operation counts per true ordered pair, one flop per IEEE add, subtract,
# multiply, divide, square root or comparison of the definitions (predicate 10; density
# predicate + 15; force predicate + 56 with the viscosity), and algorithmic bytes per particle
# of the pair passes (each particle's record read once, its results written once).
FLOP_PRED_PAIR = 10      # neighbour predicate, per true pair (tested candidates are not counted)
FLOP_DENS_PAIR = 25      # density, per true pair (self included)
FLOP_FORCE_PAIR = 66     # momentum + energy with the viscosity, per b != a
BYTES_DENS_PART = 80     # x, y, z, h, m, u read; rho, P, c, h_next... written (FP64)
BYTES_FORCE_PART = 120   # x, y, z, h, v, m, rho, P, c read; a, du/dt written (FP64)


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed hardware-counter summary, or None
    when there is none or the kernel's source has changed since the counters were taken.
    Summary lines read: 'traffic: <kernel, spaces removed> <source files, comma-separated>
    <sha256 of their concatenated contents> <bytes per launch>'."""
    import hashlib
    prof = os.path.join(ROOT, "profiles")
    if not os.path.isdir(prof):
        return None
    for fn in sorted(os.listdir(prof)):
        if not fn.endswith(".md"):
            continue
        for line in open(os.path.join(prof, fn)):
            f = line.split()
            if len(f) == 5 and f[0] == "traffic:" and f[1] == kernel.replace(" ", ""):
                srcs = [os.path.join(ROOT, s) for s in f[2].split(",")]
                if all(os.path.isfile(s) for s in srcs):
                    h = hashlib.sha256(b"".join(open(s, "rb").read() for s in srcs)).hexdigest()
                    if h == f[3]:
                        return float(f[4])
    return None


def device_dt(ps, courant=0.25, seg=False, **cfg):
    """courant x the device time-step bound (sph_timestep: min h/c, and sqrt(eps/|a|) with
    gravity) of the primed initial state, on a copy of the particles; one value per set when
    seg, else the smallest."""
    import paper_2007_03097_amd as sph
    ctx = sph.Context(ps.n, max(ps.n_seg, 1), **cfg)
    pa = sph.ParticleArrays.from_numpy(ps)
    sph.sph_step(ctx.h, pa, 1e-12, 0, 0)
    b = sph.sph_timestep(ctx.h, max(ps.n_seg, 1))
    ctx.close()
    return courant * b if seg else courant * float(b.min())


def pass_times(ctx, reps):
    """Event timings (seconds) of one neighbour-list, density and force pass on the state of
    the last sph_build_tree (torch's current stream, the one the context launches on)."""
    import torch
    import paper_2007_03097_amd as sph
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    sph.sph_compute_density(ctx.h, None, None, None, None)
    torch.cuda.synchronize()
    ev[0].record()
    for _ in range(reps):
        sph.sph_find_neighbors(ctx.h, count=False)
    ev[1].record()
    for _ in range(reps):
        sph.sph_compute_density(ctx.h, None, None, None, None)
    ev[2].record()
    for _ in range(reps):
        sph.sph_compute_forces(ctx.h, None, None, None, None)
    ev[3].record()
    torch.cuda.synchronize()
    return tuple(ev[i].elapsed_time(ev[i + 1]) / reps * 1e-3 for i in range(3))


def pass_rooflines(n, pairs_dens, pairs_force, t_dens, t_force):
    """ALU fraction (algorithmic flops at the FP64 peak) and HBM fraction (algorithmic bytes
    at 8 TB/s) of the density and force passes; the larger is the roofline fraction."""
    out = {}
    for name, t, pairs, fpp, bpp in (("density", t_dens, pairs_dens, FLOP_DENS_PAIR, BYTES_DENS_PART),
                                     ("forces", t_force, pairs_force, FLOP_FORCE_PAIR, BYTES_FORCE_PART)):
        alu = pairs * fpp / t / 1e12 / FP64_PEAK_TFLOPS
        hbm = n * bpp / t / 1e9 / HBM_PEAK_GBS
        out[name] = {"ms": t * 1e3, "alu_frac": alu, "hbm_frac": hbm, "frac": max(alu, hbm),
                     "flop_per_pair": fpp, "bytes_per_particle": bpp}
    return out


def run_gpu(ps, prec, steps, warmup, reps, autotune=True, energy_form=0, key_curve=0):
    import torch
    import paper_2007_03097_amd as sph
    n = ps.n
    dt = device_dt(ps, adaptive_h=1)
    ctx = sph.Context(n, adaptive_h=1, precision=prec, energy_form=energy_form, key_curve=key_curve)
    pa = sph.ParticleArrays.from_numpy(ps)
    if autotune:
        sph.sph_autotune(ctx.h, pa, dt, TUNING_CACHE)    # leaf size, group size, waves per CU (untimed here)
    sph.sph_step(ctx.h, pa, dt, max(warmup, 1), 0)       # load, prime, warm up, capture graphs
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    diag = sph.sph_step(ctx.h, pa, dt, steps, sph.SPH_STEP_RESUME)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    # pair counts of the final state (the tube evolves little over the timed steps)
    sph.sph_build_tree(ctx.h, pa)
    total = sph.sph_find_neighbors(ctx.h, None, None, 0)
    pairs_dens, pairs_force = total, total - n
    # per-kernel timing with events on the stream the kernels run on (torch's current stream,
    # which is the null stream the context launches on): each call below launches one kernel
    t_list, t_dens, t_force = pass_times(ctx, reps)
    leaf, group, waves = sph.sph_get_tuning(ctx.h)
    final = {k: pa[k].cpu().numpy() for k in ("x", "y", "z", "vx", "vy", "vz", "h", "u")}
    ctx.close()
    return dict(ms_per_step=wall / steps * 1e3, wall=wall, pairs_dens=pairs_dens, pairs_force=pairs_force,
                value=(pairs_dens + pairs_force) * steps / wall, steps_per_s=steps / wall,
                t_list=t_list, t_dens=t_dens, t_force=t_force,
                pass_rate=(pairs_dens + pairs_force) / (t_dens + t_force),
                diag=diag.tolist(), leaf=leaf, group=group, waves=waves, dt=dt, final=final)


def fp32c_field_errors(ps):
    """FP32C against FP64 on one state (both through the library, the FP64 path being the one
    that matches the oracle to 1e-12): per field, median / p99 / max over particles of
    |x_fp32c - x_fp64| / rms(x_fp64), the acceleration as a vector."""
    import numpy as np
    import torch
    import paper_2007_03097_amd as sph
    res = {}
    for prec in (0, 1):
        ctx = sph.Context(ps.n, adaptive_h=1, precision=prec)
        pa = sph.ParticleArrays.from_numpy(ps)
        sph.sph_autotune(ctx.h, pa, 1e-4, TUNING_CACHE)
        sph.sph_build_tree(ctx.h, pa)
        out = [torch.zeros(ps.n, dtype=torch.float64, device="cuda") for _ in range(8)]
        sph.sph_compute_density(ctx.h, *out[:4])
        sph.sph_compute_forces(ctx.h, *out[4:])
        res[prec] = [o.cpu().numpy() for o in out]
        ctx.close()
    stats = {}
    a64 = np.stack(res[0][4:7], 1)
    a32 = np.stack(res[1][4:7], 1)
    fields = {"rho": (res[1][0], res[0][0]), "P": (res[1][1], res[0][1]), "h_next": (res[1][3], res[0][3]),
              "du_dt": (res[1][7], res[0][7])}
    for k, (x32, x64) in fields.items():
        e = np.abs(x32 - x64) / np.sqrt(np.mean(x64 ** 2))
        stats[k] = [float(np.median(e)), float(np.quantile(e, 0.99)), float(e.max())]
    e = np.linalg.norm(a32 - a64, axis=1) / np.sqrt(np.mean(np.sum(a64 ** 2, axis=1)))
    stats["a"] = [float(np.median(e)), float(np.quantile(e, 0.99)), float(e.max())]
    return stats


def _pairs(ctx, pa, n):
    import paper_2007_03097_amd as sph
    sph.sph_build_tree(ctx.h, pa)
    total = sph.sph_find_neighbors(ctx.h, None, None, 0)
    return total + (total - n)


def run_polytrope(ps, steps, prec, scheme=0, eps=0.01, sizes=None, cap=2048):
    """Self-gravitating set (theta = 0.5, Plummer eps, G = 1), adaptive h: the n = 1 polytrope
    (eps = 0.01) or the Evrard sphere (eps = 0.005); scheme 0 = quadrupole particle-cell walk,
    1 = symmetric node-node (FMM) gravity.  Leaf and group sizes from the autotuner, or the
    given (leaf, group).  dt = 0.25 min(h/c, sqrt(eps/|a|)) on the primed initial state.  Also
    times one gravity pass on the final state (HIP events on the context's stream)."""
    import numpy as np
    import torch
    import paper_2007_03097_amd as sph
    n = ps.n
    cfg = dict(adaptive_h=1, precision=prec, G=1.0, soft_eps=eps, theta=0.5, nbr_capacity=cap,
               gravity_scheme=scheme)
    if sizes:
        cfg.update(leaf_size=sizes[0], group_size=sizes[1])
    ctx = sph.Context(n, **cfg)
    pa = sph.ParticleArrays.from_numpy(ps, with_accel=True)
    if not sizes:
        sph.sph_autotune(ctx.h, pa, 1e-4, TUNING_CACHE)
    sph.sph_step(ctx.h, pa, 1e-9, 0, 0)                  # prime: accelerations of the initial state
    dt = 0.25 * float(sph.sph_timestep(ctx.h, 1)[0])     # device bound: min(h/c, sqrt(eps/|a|))
    sph.sph_step(ctx.h, pa, dt, 1, sph.SPH_STEP_PRIMED)  # warm up, capture graphs
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sph.sph_step(ctx.h, pa, dt, steps, sph.SPH_STEP_RESUME)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    sph.sph_build_tree(ctx.h, pa)
    total = sph.sph_find_neighbors(ctx.h, None, None, 0)
    pairs = total + (total - n)
    t_list, t_dens, t_force = pass_times(ctx, 5)
    g = [torch.zeros(n, dtype=torch.float64, device="cuda") for _ in range(3)]
    sph.sph_compute_gravity(ctx.h, *g)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(3):
        sph.sph_compute_gravity(ctx.h, *g)
    e1.record()
    torch.cuda.synchronize()
    grav_ms = e0.elapsed_time(e1) / 3
    grav = None
    if scheme == 0:   # terms of the particle-cell walk, counted on the device during the last pass
        cells, pp = sph.sph_gravity_counts(ctx.h)
        grav = {"cells_per_particle": cells / n, "pairs_per_particle": pp / n,
                "cell_terms_per_s": cells / (grav_ms * 1e-3), "pair_terms_per_s": pp / (grav_ms * 1e-3)}
    leaf, group, waves = sph.sph_get_tuning(ctx.h)
    ctx.close()
    del g
    torch.cuda.empty_cache()
    out = dict(ms_per_step=wall / steps * 1e3, steps_per_s=steps / wall, value=pairs * steps / wall, dt=dt,
               leaf_size=leaf, group_size=group, waves_per_cu=waves, gravity_ms=grav_ms,
               lists_ms=t_list * 1e3, pass_rate=pairs / (t_dens + t_force),
               passes=pass_rooflines(n, total, total - n, t_dens, t_force))
    if grav:
        out["gravity_terms"] = grav
    return out


def run_ensemble(steps):
    """256 independent boxes: one batched context (all boxes in one graph-captured step,
    FP32C) against a loop of per-box FP64 contexts."""
    import torch
    import paper_2007_03097_amd as sph
    from workloads import ensemble
    ps = ensemble(256, seed=1004)
    so = ps.seg_offsets
    n = ps.n
    dts = device_dt(ps, seg=True)       # each box by its own 0.25 min(h/c)
    dt = float(dts.min())
    out = {"n_particles": n, "n_boxes": 256, "dt_min": dt, "dt_max": float(dts.max())}
    # batched, FP32C and FP64
    for prec, key in ((1, "batched_fp32c"), (0, "batched_fp64")):
        ctx = sph.Context(n, seg_capacity=256, precision=prec)
        pa = sph.ParticleArrays.from_numpy(ps)
        pa.seg_dt = dts
        sph.sph_autotune(ctx.h, pa, dt, TUNING_CACHE)
        sph.sph_step(ctx.h, pa, dt, 1, 0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sph.sph_step(ctx.h, pa, dt, steps, sph.SPH_STEP_RESUME)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        pairs = _pairs(ctx, pa, n)
        out[key] = {"ms_per_step": wall / steps * 1e3, "value": pairs * steps / wall,
                    "leaf_size": sph.sph_get_tuning(ctx.h)[0], "group_size": sph.sph_get_tuning(ctx.h)[1],
                    "waves_per_cu": sph.sph_get_tuning(ctx.h)[2]}
        ctx.close()
        del pa
        torch.cuda.empty_cache()
    # per-box FP64 loop
    ctxs, pas = [], []
    for b in range(256):
        sub = ps.subset(slice(int(so[b]), int(so[b + 1])))
        ctx = sph.Context(sub.n, precision=0)
        pa = sph.ParticleArrays.from_numpy(sub)
        sph.sph_step(ctx.h, pa, float(dts[b]), 1, 0)
        ctxs.append(ctx)
        pas.append(pa)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        for b, ctx in enumerate(ctxs):
            sph.sph_step(ctx.h, None, float(dts[b]), 1, sph.SPH_STEP_RESUME)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    pairs = sum(_pairs(c, p, p.n) for c, p in zip(ctxs, pas))
    out["per_box_fp64_loop"] = {"ms_per_step": wall / steps * 1e3, "value": pairs * steps / wall}
    out["batched_fp32c_speedup_vs_loop"] = out["batched_fp32c"]["value"] / out["per_box_fp64_loop"]["value"]
    for c in ctxs:
        c.close()
    torch.cuda.empty_cache()
    return out


def run_sweeps():
    """Gravity time and accuracy against the opening angle (n = 1 polytrope, 262,144
    particles; the theta = 0 result of the quadrupole walk -- the direct sum -- is the
    reference), for the quadrupole particle-cell walk and the node-node (FMM) scheme, and
    time against N at theta = 0.5 (both gravity schemes and the SPH passes), with power-law
    fits."""
    import numpy as np
    import torch
    import paper_2007_03097_amd as sph
    from workloads import polytrope_n1

    def timed(fn, reps=3):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    out = {"metric": "gravity time and accuracy vs opening angle; time vs N", "data": "synthetic",
           "workload": "n = 1 polytrope, G = 1, eps = 0.01, quadrupole cells, FP64"}
    ps = polytrope_n1(262144, seed=1003)
    n = ps.n
    pa = sph.ParticleArrays.from_numpy(ps)
    ref = None
    rows = []
    for theta in (0.0, 0.2, 0.3, 0.4, 0.5, 0.6, 0.7, 0.8, 0.9, 1.0):
        ctx = sph.Context(n, G=1.0, soft_eps=0.01, theta=theta)
        sph.sph_build_tree(ctx.h, pa)
        g = [torch.zeros(n, dtype=torch.float64, device="cuda") for _ in range(3)]
        ms = timed(lambda: sph.sph_compute_gravity(ctx.h, *g), reps=1 if theta == 0.0 else 3)
        gv = torch.stack(g, 1).cpu().numpy()
        if ref is None:
            ref = gv
        e = np.linalg.norm(gv - ref, axis=1) / np.linalg.norm(ref, axis=1)
        rows.append({"theta": theta, "gravity_ms": ms, "rms_rel_err": float(np.sqrt((e ** 2).mean())),
                     "p99_rel_err": float(np.quantile(e, 0.99))})
        print(json.dumps(rows[-1]), file=sys.stderr, flush=True)
        ctx.close()
    out["theta_sweep_n262144"] = rows
    rows = []
    for theta in (0.0, 0.1, 0.2, 0.3, 0.4, 0.5, 0.6, 0.7, 0.8, 0.9, 1.0):
        ctx = sph.Context(n, G=1.0, soft_eps=0.01, theta=theta, gravity_scheme=1)
        sph.sph_build_tree(ctx.h, pa)
        g = [torch.zeros(n, dtype=torch.float64, device="cuda") for _ in range(3)]
        ms = timed(lambda: sph.sph_compute_gravity(ctx.h, *g), reps=1 if theta < 0.15 else 3)
        gv = torch.stack(g, 1).cpu().numpy()
        e = np.linalg.norm(gv - ref, axis=1) / np.linalg.norm(ref, axis=1)
        rows.append({"theta": theta, "gravity_ms": ms, "rms_rel_err": float(np.sqrt((e ** 2).mean())),
                     "p99_rel_err": float(np.quantile(e, 0.99))})
        print(json.dumps(rows[-1]), file=sys.stderr, flush=True)
        ctx.close()
    out["fmm_theta_sweep_n262144"] = rows
    del pa
    rows = []
    for n in (65536, 262144, 1048576, 4194304):
        ps = polytrope_n1(n, seed=1003)
        pa = sph.ParticleArrays.from_numpy(ps)
        ctx = sph.Context(n, G=1.0, soft_eps=0.01, theta=0.5, nbr_capacity=2048)
        sph.sph_build_tree(ctx.h, pa)
        g = [torch.zeros(n, dtype=torch.float64, device="cuda") for _ in range(3)]
        tg = timed(lambda: sph.sph_compute_gravity(ctx.h, *g))
        cf = sph.Context(n, G=1.0, soft_eps=0.01, theta=0.5, gravity_scheme=1)
        sph.sph_build_tree(cf.h, pa)
        tfmm = timed(lambda: sph.sph_compute_gravity(cf.h, *g))
        cf.close()
        tl = timed(lambda: sph.sph_find_neighbors(ctx.h, count=False))
        td = timed(lambda: sph.sph_compute_density(ctx.h, None, None, None, None))
        tf = timed(lambda: sph.sph_compute_forces(ctx.h, None, None, None, None))
        rows.append({"n": n, "gravity_ms": tg, "fmm_gravity_ms": tfmm, "lists_ms": tl, "density_ms": td,
                     "forces_ms": tf})
        print(json.dumps(rows[-1]), file=sys.stderr, flush=True)
        ctx.close()
        del pa, g
        torch.cuda.empty_cache()
    out["n_sweep_theta0.5"] = rows
    ns = np.array([r["n"] for r in rows], dtype=float)
    for key in ("gravity_ms", "fmm_gravity_ms", "lists_ms", "density_ms", "forces_ms"):
        t = np.array([r[key] for r in rows])
        out[f"{key}_exponent"] = float(np.polyfit(np.log(ns[1:]), np.log(t[1:]), 1)[0])
        out[f"{key}_per_nlogn_ns"] = [float(x * 1e6 / (m * np.log2(m))) for x, m in zip(t, ns)]
    return out


def measure_peaks():
    """Sustained rates measured on this GPU: FP64 and unpacked-FP32 FMA chains (the library's
    probe) and a 1 GiB device-to-device copy (read + write bytes)."""
    import torch
    import paper_2007_03097_amd as sph
    s = torch.cuda.current_stream()
    out = {}
    nt, iters, reps = 256 * 8192, 2048, 5
    buf = torch.empty(nt, dtype=torch.float64, device="cuda")
    for kind, name in ((0, "fp64_fma_tflops"), (1, "fp32_fma_tflops")):
        sph.sph_peak_probe(kind, buf, iters, s.cuda_stream)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        for _ in range(reps):
            sph.sph_peak_probe(kind, buf, iters, s.cuda_stream)
        e1.record(s)
        torch.cuda.synchronize()
        out[name] = 16.0 * iters * nt / (e0.elapsed_time(e1) / reps * 1e-3) / 1e12
    del buf
    nb = 1 << 30
    src = torch.empty(nb, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        dst.copy_(src)
    e1.record(s)
    torch.cuda.synchronize()
    out["copy_tb_per_s"] = 2.0 * nb / (e0.elapsed_time(e1) / reps * 1e-3) / 1e12
    del src, dst
    torch.cuda.empty_cache()
    return out


def cpu_baseline(ps, reps=10):
    """The CPU FP64 reference on a bounded sample: the slab 0.42 < x < 0.58 of the same tube
    (both lattices and the interface).  Brute-force neighbours are built once (reported,
    not counted); density + force pair throughput is the baseline."""
    import numpy as np
    import oracle
    sel = np.nonzero((ps.x > 0.42) & (ps.x < 0.58))[0]
    sub = ps.subset(sel)
    t0 = time.perf_counter()
    csr = oracle.neighbors(sub.x, sub.y, sub.z, sub.h)
    t_nbr = time.perf_counter() - t0
    pairs = int(csr[0][-1]) + int(csr[0][-1] - sub.n)
    times = []
    for _ in range(reps):
        t0 = time.perf_counter()
        rho, P, c, _ = oracle.density(sub.fields(), csr)
        oracle.forces(sub.fields(), rho, P, c, csr)
        times.append(time.perf_counter() - t0)
    best = float(np.median(times))
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    # direct-sum gravity on 1,024 sampled targets of a 262,144-particle n = 1 polytrope
    from workloads import lattice_box, polytrope_n1
    pp = polytrope_n1(262144, seed=1003)
    tg = np.sort(np.random.default_rng(3).choice(pp.n, 1024, replace=False))
    t0 = time.perf_counter()
    oracle.gravity_direct(pp.x, pp.y, pp.z, pp.m, 1.0, 0.01, targets=tg)
    t_grav = time.perf_counter() - t0
    # whole KDK steps of the 4,096-particle jittered lattice (brute-force neighbours each step)
    lb = lattice_box(16)
    prm = oracle.Params()
    st = oracle.prime(lb.fields(), prm)
    ts = []
    for _ in range(5):
        t0 = time.perf_counter()
        st = oracle.kdk_step(st, 0.0178, prm)
        ts.append(time.perf_counter() - t0)
    t_steps = float(np.median(ts))
    # whole KDK steps of one box of the 256-box ensemble (its largest, 64,000 particles), median of 3
    from workloads import ensemble
    en = ensemble(256, seed=1004)
    b = int(np.argmax(np.diff(en.seg_offsets)))
    box = en.subset(slice(int(en.seg_offsets[b]), int(en.seg_offsets[b + 1])))
    stb = oracle.prime(box.fields(), prm)
    dtb = 0.25 * float(oracle.dt_bound(stb)[0])
    tb = []
    for _ in range(3):
        t0 = time.perf_counter()
        stb = oracle.kdk_step(stb, dtb, prm)
        tb.append(time.perf_counter() - t0)
    return dict(value=pairs / best, unit="pair interactions/s", cores=cores, kind="oracle", cpu_model=model,
                sample=f"slab 0.42<x<0.58 of the tube: {sub.n} particles, {pairs} density+force pairs; "
                       f"median of {reps}: {best:.3f} s; brute-force neighbour search {t_nbr:.1f} s not counted",
                neighbor_search_s=t_nbr,
                gravity_direct={"value": tg.size * (pp.n - 1) / t_grav, "unit": "particle-particle interactions/s",
                                "sample": f"1,024 targets of a 262,144-particle polytrope, {t_grav:.2f} s"},
                steps_per_s_lattice_4096={"value": 1.0 / t_steps, "unit": "steps/s",
                                          "sample": f"median of 5 KDK steps of the 4,096-particle lattice, "
                                                    f"{t_steps:.3f} s each"},
                steps_per_s_ensemble_box={"value": 1.0 / float(np.median(tb)), "unit": "steps/s",
                                          "sample": f"median of 3 KDK steps of the ensemble's {box.n}-particle box"},
                tube_steps_note="whole KDK steps of the 987,840-particle tube are not timed: its brute-force "
                                "neighbour search alone takes minutes per step on these cores")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--ny", type=int, default=56, help="tube lattice resolution (56 -> 987,840 particles)")
    ap.add_argument("--reps", type=int, default=20, help="repetitions of the per-kernel timing")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="skip the polytrope and ensemble workloads")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default leaf size, group size and grids")
    ap.add_argument("--sweep", action="store_true",
                    help="instead of the benchmark: gravity time/accuracy vs theta and time vs N (one JSON line)")
    ap.add_argument("--polytrope", action="store_true",
                    help="instead of the benchmark: the 4M polytrope with both gravity schemes, FP64 and FP32C "
                         "(one JSON line; --steps timed steps each)")
    ap.add_argument("--evrard", action="store_true",
                    help="instead of the benchmark: the 16M Evrard sphere, FP32C and FP64, quadrupole gravity "
                         "(one JSON line; --steps timed steps each)")
    ap.add_argument("--copy-calib-mib", type=int, default=0,
                    help="first run one device-to-device copy of this many MiB (hardware-counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU path is not built.",
              file=sys.stderr)
        sys.exit(2)
    import torch
    from workloads import sod_tube
    assert torch.cuda.is_available(), "needs a GPU"
    if args.sweep:
        print(json.dumps(run_sweeps()), flush=True)
        return
    if args.polytrope:
        from workloads import polytrope_n1
        pp = polytrope_n1(4194304, seed=1003)
        out = {"workload": "n = 1 polytrope, 4,194,304 particles, G = 1, eps = 0.01, theta = 0.5, adaptive h",
               "steps": args.steps}
        for scheme, name in ((0, "quadrupole"), (1, "node_node")):
            out[name] = {"fp64": run_polytrope(pp, args.steps, 0, scheme),
                         "fp32c": run_polytrope(pp, args.steps, 1, scheme)}
        print(json.dumps(out), flush=True)
        return
    if args.evrard:
        from workloads import evrard
        pe = evrard(16777216, seed=1005)
        out = {"workload": "Evrard sphere, 16,777,216 particles, u = 0.05, G = 1, eps = 0.005, theta = 0.5, "
                           "adaptive h, quadrupole gravity, leaf 32 / group 64", "steps": args.steps}
        for prec, key in ((1, "fp32c"), (0, "fp64")):
            out[key] = run_polytrope(pe, args.steps, prec, 0, eps=0.005, sizes=(32, 64), cap=256)
        print(json.dumps(out), flush=True)
        return
    if args.copy_calib_mib > 0:
        src = torch.empty(args.copy_calib_mib << 20, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    ps = sod_tube(args.ny)
    r64 = run_gpu(ps, 0, args.steps, args.warmup, args.reps, not args.no_autotune)
    r32 = run_gpu(ps, 1, args.steps, args.warmup, args.reps, not args.no_autotune)
    n = ps.n
    kernels = {"k_nbr_lists": (r64["t_list"], r64["pairs_dens"], FLOP_PRED_PAIR),
               "k_density<false>": (r64["t_dens"], r64["pairs_dens"], FLOP_DENS_PAIR),
               "k_forces<false, false>": (r64["t_force"], r64["pairs_force"], FLOP_FORCE_PAIR)}
    rooflines = {}
    for name, (t, pairs, fpp) in kernels.items():
        ach = pairs * fpp / t / 1e12
        rooflines[name] = {"bound": "alu", "achieved": ach, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                           "frac": ach / FP64_PEAK_TFLOPS, "traffic": None,
                           "per_launch": {"pairs": pairs, "flop_per_pair": fpp, "avg_ms": t * 1e3}}
    dom = max(kernels, key=lambda k: kernels[k][0])
    peaks = measure_peaks()
    for name in rooflines:
        rooflines[name]["traffic"] = measured_traffic(name)
        rooflines[name]["measured_peak"] = peaks["fp64_fma_tflops"]
        rooflines[name]["frac_measured"] = rooflines[name]["achieved"] / peaks["fp64_fma_tflops"]
    roof = dict(rooflines[dom], kernel=dom)
    extra = {}
    if not args.no_extra:
        from workloads import polytrope_n1
        pp = polytrope_n1(4194304, seed=1003)
        extra["polytrope_4m_gravity"] = {"n_particles": pp.n, "fp64": run_polytrope(pp, 10, 0),
                                         "fp32c": run_polytrope(pp, 10, 1)}
        extra["polytrope_4m_fmm_gravity"] = {"n_particles": pp.n, "fp64": run_polytrope(pp, 10, 0, scheme=1),
                                             "fp32c": run_polytrope(pp, 10, 1, scheme=1)}
        del pp
        extra["ensemble_256"] = run_ensemble(10)
        tk = {}
        for prec, key in ((0, "fp64"), (1, "fp32c")):
            r = run_gpu(ps, prec, args.steps, args.warmup, 2, not args.no_autotune, energy_form=1)
            tk[key] = {"ms_per_step": r["ms_per_step"], "steps_per_s": r["steps_per_s"], "value": r["value"],
                       "forces_ms": r["t_force"] * 1e3}
        extra["thermokinetic_tube"] = tk
        hk = {}
        for prec, key in ((0, "fp64"), (1, "fp32c")):
            r = run_gpu(ps, prec, args.steps, args.warmup, args.reps, not args.no_autotune, key_curve=1)
            hk[key] = {"ms_per_step": r["ms_per_step"], "steps_per_s": r["steps_per_s"], "value": r["value"],
                       "kernel_ms": {"nbr_lists": r["t_list"] * 1e3, "density": r["t_dens"] * 1e3,
                                     "forces": r["t_force"] * 1e3}}
        extra["hilbert_keys_tube"] = hk
        from workloads import evrard
        pe = evrard(16777216, seed=1005)
        extra["evrard_16m_fp32c"] = dict(run_polytrope(pe, 20, 1, 0, eps=0.005, sizes=(32, 64), cap=256),
                                         n_particles=pe.n, timed_steps=20)
        del pe
    # FP32C error per field on the benchmark workload's evolved state (after the timed steps)
    ev = ps.copy()
    for k, v in r64["final"].items():
        setattr(ev, k, v)
    fp32c_err = fp32c_field_errors(ev)
    cpu = None if args.no_cpu else cpu_baseline(ps)
    out = {
        "metric": "pair interactions/sec (density+force) and steps/sec, FP64 vs FP32-comp, 1 GPU",
        "value": r64["value"], "unit": "pair interactions/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": r64["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"3D Sod-type tube, {n} particles, adaptive h, Monaghan AV, KDK leapfrog",
                   "n_particles": n, "dt": r64["dt"], "leaf_size": r64["leaf"], "group_size": r64["group"],
                   "waves_per_cu": r64["waves"], "fp32c_leaf_size": r32["leaf"], "fp32c_group_size": r32["group"],
                   "fp32c_waves_per_cu": r32["waves"]},
        "steps_per_s": r64["steps_per_s"],
        "pairs_per_step": r64["pairs_dens"] + r64["pairs_force"],
        "pass_rate": r64["pass_rate"],
        "kernel_ms": {"nbr_lists": r64["t_list"] * 1e3, "density": r64["t_dens"] * 1e3,
                      "forces": r64["t_force"] * 1e3},
        "fp32c": {"value": r32["value"], "ms_per_step": r32["ms_per_step"], "steps_per_s": r32["steps_per_s"],
                  "pass_rate": r32["pass_rate"], "speedup_vs_fp64": r32["value"] / r64["value"],
                  "pass_speedup_vs_fp64": r32["pass_rate"] / r64["pass_rate"],
                  "kernel_ms": {"nbr_lists": r32["t_list"] * 1e3, "density": r32["t_dens"] * 1e3,
                                "forces": r32["t_force"] * 1e3},
                  "error_vs_fp64_median_p99_max": fp32c_err,
                  "error_note": "per particle |x_fp32c - x_fp64| / rms(x_fp64) on the evolved tube (FP64 matches "
                                "the oracle to 1e-12 of each particle's absolute-sum scale)"},
        "pass_rooflines": pass_rooflines(n, r64["pairs_dens"], r64["pairs_force"], r64["t_dens"], r64["t_force"]),
        "roofline": roof,
        "rooflines_pair_kernels": rooflines,
        "device_peaks_measured": peaks,
        "cpu_baseline": cpu,
        **extra,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
