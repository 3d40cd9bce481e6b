"""Full-size parity on sampled outputs, in the configuration the benchmark times.

* The 3D Sod-type tube (987,840 particles, default leaf and group sizes): keys, order and
  octree bit-exact for every particle; neighbour sets bit-exact and FP64 density within
  1e-12 for 2048 sampled targets (brute force over all particles); forces for the same
  targets within 1e-12 given the GPU's rho, P, c of their neighbours (a layered check:
  those values come from the density field whose sample passed).
* The n = 1 polytrope at 4,194,304 particles: theta = 0.5 quadrupole gravity within 1e-3
  RMS relative of the direct sum on 1024 sampled targets; the node-node scheme conserves
  momentum and angular momentum to rounding over all particles and keeps its first-order
  accuracy on the same targets.
* The batched ensemble (256 boxes, 4,879,340 particles, one context as the benchmark runs
  it): keys and order bit-exact; per-set neighbour sets bit-exact and density, forces
  (layered) for sampled targets across many sets, FP64 within 1e-12 and FP32C within the
  stated 2e-6 budget.
* The Evrard-style sphere at 16,777,216 particles (FP32C as configured, and FP64): keys and
  order bit-exact; sampled neighbour sets bit-exact, density and forces (layered) within
  the FP64 / FP32C bounds; theta = 0.5 gravity within 1e-3 RMS of the direct sum.
"""
import math

import numpy as np
import pytest

from workloads import ensemble, evrard, polytrope_n1, sod_tube

from gpu_helpers import gpu_density, gpu_gravity, gpu_keys_order, gpu_tree, make_ctx, parts, rel_err, to_np, tuned

pytestmark = pytest.mark.gpu


def test_sod_full_size_sampled(orc):
    import torch
    import paper_2007_03097_amd as sph
    ps = sod_tube(56)
    n = ps.n
    assert n == 987840
    ctx = make_ctx(n, adaptive_h=1)
    pa = parts(ps)
    leaf, group = tuned(ctx, pa)
    k, o = gpu_keys_order(ctx, pa)
    print(f"\nfull-size tube: n={n} leaf {leaf} group {group}", flush=True)
    assert np.array_equal(k, orc.keys(ps.x, ps.y, ps.z))
    assert np.array_equal(o, orc.order(k))
    t = gpu_tree(ctx)
    ref = orc.octree(k[o], leaf)
    assert len(t["key"]) == len(ref["key"])
    assert np.array_equal(np.sort(t["key"]), np.sort(ref["key"]))
    off = torch.zeros(n + 1, dtype=torch.int64, device="cuda")
    total = sph.sph_find_neighbors(ctx.h, off, None, 0)
    idx = torch.zeros(total, dtype=torch.int32, device="cuda")
    sph.sph_find_neighbors(ctx.h, off, idx, total)
    off, idx = to_np(off), to_np(idx)
    rng = np.random.default_rng(5)
    tg = np.sort(rng.choice(n, 2048, replace=False))
    tg = np.unique(np.concatenate([tg, np.nonzero(np.abs(ps.x - 0.5) < 0.004)[0][::97]]))  # interface
    roff, ridx = orc.neighbors(ps.x, ps.y, ps.z, ps.h, targets=tg)
    for j, a in enumerate(tg):
        assert np.array_equal(idx[off[a]:off[a + 1]], ridx[roff[j]:roff[j + 1]]), a
    rho, P, c, hn = gpu_density(ctx, n)
    r_rho, r_P, r_c, r_hn = orc.density(ps.fields(), (roff, ridx), targets=tg)
    assert rel_err(rho[tg], r_rho, r_rho) <= 1e-12
    assert rel_err(hn[tg], r_hn, r_hn) <= 1e-12
    ax, ay, az, du = (np.zeros(n) for _ in range(4))
    outs = [torch.zeros(n, dtype=torch.float64, device="cuda") for _ in range(4)]
    sph.sph_compute_forces(ctx.h, *outs)
    ax, ay, az, du = [to_np(x) for x in outs]
    r_ax, r_ay, r_az, r_du, Sa, Su = orc.forces(ps.fields(), rho, P, c, (roff, ridx), targets=tg)
    d = np.sqrt((ax[tg] - r_ax) ** 2 + (ay[tg] - r_ay) ** 2 + (az[tg] - r_az) ** 2)
    assert np.all(d <= 1e-12 * Sa)
    assert np.all(np.abs(du[tg] - r_du) <= 1e-12 * Su + 1e-300)


def test_sod_full_size_evolved_sampled(orc, capsys):
    """The tube after five resident steps (graph replays, the benchmark's dt and tuning), when
    the pressure jump has set the gas moving and the viscosity and du/dt are active: on the
    returned state, neighbour sets bit-exact and FP64 density within 1e-12 for 2048 sampled
    targets plus the interface region, forces (layered) within 1e-12 of each target's
    absolute-sum scale; FP32C density and forces on the same state within 2e-6 (median and max
    printed per field)."""
    import torch
    import paper_2007_03097_amd as sph
    ps = sod_tube(56)
    n = ps.n
    ctx = make_ctx(n, adaptive_h=1)
    pa = parts(ps, with_accel=True)
    tuned(ctx, pa)
    sph.sph_step(ctx.h, pa, 1e-12, 0, 0)                 # prime
    dt = 0.25 * sph.sph_timestep(ctx.h, 1)[0]
    pa = parts(ps, with_accel=True)
    sph.sph_step(ctx.h, pa, dt, 5, 0)
    ev = ps.copy()
    for k in ("x", "y", "z", "vx", "vy", "vz", "h", "u"):
        setattr(ev, k, to_np(pa[k]).copy())
    vmax = np.sqrt(ev.vx ** 2 + ev.vy ** 2 + ev.vz ** 2).max()
    print(f"\nevolved tube: dt {dt:.3e}, 5 steps, max |v| {vmax:.3e}", flush=True)
    assert vmax > 1e-3
    rng = np.random.default_rng(6)
    tg = np.sort(rng.choice(n, 2048, replace=False))
    tg = np.unique(np.concatenate([tg, np.nonzero(np.abs(ev.x - 0.5) < 0.01)[0][::41]]))
    roff, ridx = orc.neighbors(ev.x, ev.y, ev.z, ev.h, targets=tg)
    results = {}
    for prec in (0, 1):
        c2 = make_ctx(n, adaptive_h=1, precision=prec)
        pe = parts(ev)
        tuned(c2, pe)
        gpu_keys_order(c2, pe)
        if prec == 0:
            off = torch.zeros(n + 1, dtype=torch.int64, device="cuda")
            total = sph.sph_find_neighbors(c2.h, off, None, 0)
            idx = torch.zeros(total, dtype=torch.int32, device="cuda")
            sph.sph_find_neighbors(c2.h, off, idx, total)
            off, idx = to_np(off), to_np(idx)
            for j, a in enumerate(tg):
                assert np.array_equal(idx[off[a]:off[a + 1]], ridx[roff[j]:roff[j + 1]]), a
        rho, P, c, hn = gpu_density(c2, n)
        outs = [torch.zeros(n, dtype=torch.float64, device="cuda") for _ in range(4)]
        sph.sph_compute_forces(c2.h, *outs)
        results[prec] = (rho, P, c, hn, [to_np(x) for x in outs])
        c2.close()
    rho, P, c, hn, (ax, ay, az, du) = results[0]
    r_rho, r_P, r_c, r_hn = orc.density(ev.fields(), (roff, ridx), targets=tg)
    assert rel_err(rho[tg], r_rho, r_rho) <= 1e-12
    assert rel_err(hn[tg], r_hn, r_hn) <= 1e-12
    r_ax, r_ay, r_az, r_du, Sa, Su = orc.forces(ev.fields(), rho, P, c, (roff, ridx), targets=tg)
    d = np.sqrt((ax[tg] - r_ax) ** 2 + (ay[tg] - r_ay) ** 2 + (az[tg] - r_az) ** 2)
    assert np.all(d <= 1e-12 * Sa)
    assert np.all(np.abs(du[tg] - r_du) <= 1e-12 * Su + 1e-300)
    # the viscosity really acts on this state: without it the sampled forces change
    n_ax, _, _, n_du, _, _ = orc.forces(ev.fields(), rho, P, c, (roff, ridx), alpha=0.0, beta=0.0, targets=tg)
    assert np.abs(n_ax - r_ax).max() > 1e-6 * np.abs(r_ax).max() and np.abs(r_du).max() > 0.0
    # FP32C on the same state against the oracle (its density by brute force, its forces given
    # the FP64 density field that passed above)
    f_rho, _, _, f_hn, (fx, fy, fz, fdu) = results[1]
    e = dict(rho=np.abs(f_rho[tg] - r_rho) / r_rho, h_next=np.abs(f_hn[tg] - r_hn) / r_hn,
             a=np.sqrt((fx[tg] - r_ax) ** 2 + (fy[tg] - r_ay) ** 2 + (fz[tg] - r_az) ** 2) / Sa,
             du=np.abs(fdu[tg] - r_du) / np.where(Su > 0, Su, 1.0))
    with capsys.disabled():
        print("evolved tube FP32C vs oracle median/p99/max: " + "  ".join(
            f"{k} {np.median(v):.1e}/{np.percentile(v, 99):.1e}/{v.max():.1e}" for k, v in e.items()), flush=True)
    for k, v in e.items():
        assert np.median(v) <= 2e-7 and v.max() <= 2e-6, k


def test_polytrope_4m_gravity_sampled(orc, capsys):
    n = 4194304
    ps = polytrope_n1(n, seed=1003)
    for prec in (0, 1):
        ctx = make_ctx(n, G=1.0, soft_eps=0.01, theta=0.5, precision=prec, adaptive_h=1, nbr_capacity=2048)
        pa = parts(ps)
        tuned(ctx, pa)
        gpu_keys_order(ctx, pa)
        gx, gy, gz, phi = gpu_gravity(ctx, n)
        rng = np.random.default_rng(7)
        tg = np.sort(rng.choice(n, 1024, replace=False))
        dx, dy, dz, dp = orc.gravity_direct(ps.x, ps.y, ps.z, ps.m, 1.0, 0.01, targets=tg)
        gd = np.sqrt(dx ** 2 + dy ** 2 + dz ** 2)
        e = np.sqrt((gx[tg] - dx) ** 2 + (gy[tg] - dy) ** 2 + (gz[tg] - dz) ** 2) / gd
        rms = math.sqrt((e ** 2).mean())
        with capsys.disabled():
            print(f"\n4M polytrope gravity prec={prec}: RMS {rms:.3e} median {np.median(e):.2e} max {e.max():.2e}",
                  flush=True)
        assert rms <= 1e-3
        ctx.close()


def test_polytrope_4m_fmm_sampled(orc, capsys):
    """The symmetric node-node gravity at 4,194,304 particles as the benchmark runs it (theta
    = 0.5, the tuned leaf size, FP64 and FP32C): linear and angular momentum of the
    gravitational forces over all particles at rounding level (1e-13 FP64, 1e-8 FP32C, of
    sum m|g| and sum m|r||g|), and the first-order accuracy the oracle shows at small N on
    1024 sampled targets against the direct sum (RMS below 0.1)."""
    import paper_2007_03097_amd as sph
    n = 4194304
    ps = polytrope_n1(n, seed=1003)
    rng = np.random.default_rng(7)
    tg = np.sort(rng.choice(n, 1024, replace=False))
    dx, dy, dz, dp = orc.gravity_direct(ps.x, ps.y, ps.z, ps.m, 1.0, 0.01, targets=tg)
    gd = np.sqrt(dx ** 2 + dy ** 2 + dz ** 2)
    pos = np.stack([ps.x, ps.y, ps.z], axis=1)
    rn = np.linalg.norm(pos, axis=1)
    for prec, bound in ((0, 1e-13), (1, 1e-8)):
        ctx = make_ctx(n, G=1.0, soft_eps=0.01, theta=0.5, precision=prec, adaptive_h=1, nbr_capacity=2048,
                       gravity_scheme=sph.SPH_GRAVITY_FMM)
        pa = parts(ps)
        leaf, _ = tuned(ctx, pa)
        gpu_keys_order(ctx, pa)
        gx, gy, gz, phi = gpu_gravity(ctx, n)
        g = np.stack([gx, gy, gz], axis=1)
        gn = np.linalg.norm(g, axis=1)
        P = np.linalg.norm((ps.m[:, None] * g).sum(axis=0)) / (ps.m * gn).sum()
        Lm = np.linalg.norm((ps.m[:, None] * np.cross(pos, g)).sum(axis=0)) / (ps.m * rn * gn).sum()
        e = np.sqrt((gx[tg] - dx) ** 2 + (gy[tg] - dy) ** 2 + (gz[tg] - dz) ** 2) / gd
        rms = math.sqrt((e ** 2).mean())
        with capsys.disabled():
            print(f"\n4M polytrope node-node gravity prec={prec} leaf {leaf}: |P|/S {P:.1e} |L|/S {Lm:.1e} "
                  f"RMS {rms:.3e} median {np.median(e):.2e}", flush=True)
        assert P <= bound and Lm <= bound
        assert rms <= 0.1
        ctx.close()


def _sampled_sph(orc, ctx, ps, tg, seg, prec, say):
    """Neighbour sets of the targets bit-exact; density and (layered) forces within the
    FP64 or FP32C bound."""
    import torch
    import paper_2007_03097_amd as sph
    n = ps.n
    off = torch.zeros(n + 1, dtype=torch.int64, device="cuda")
    total = sph.sph_find_neighbors(ctx.h, off, None, 0)
    idx = torch.zeros(total, dtype=torch.int32, device="cuda")
    sph.sph_find_neighbors(ctx.h, off, idx, total)
    off, idx = to_np(off), to_np(idx)
    roff, ridx = orc.neighbors(ps.x, ps.y, ps.z, ps.h, targets=tg, seg=seg)
    for j, a in enumerate(tg):
        assert np.array_equal(idx[off[a]:off[a + 1]], ridx[roff[j]:roff[j + 1]]), a
    say(f"neighbour sets of {tg.size} targets bit-exact ({total} pairs in all)")
    rho, P, c, hn = gpu_density(ctx, n)
    r_rho, r_P, r_c, r_hn = orc.density(ps.fields(), (roff, ridx), targets=tg)
    outs = [torch.zeros(n, dtype=torch.float64, device="cuda") for _ in range(4)]
    sph.sph_compute_forces(ctx.h, *outs)
    ax, ay, az, du = [to_np(x) for x in outs]
    r_ax, r_ay, r_az, r_du, Sa, Su = orc.forces(ps.fields(), rho, P, c, (roff, ridx), targets=tg)
    e_rho = np.abs(rho[tg] - r_rho) / r_rho
    e_a = np.sqrt((ax[tg] - r_ax) ** 2 + (ay[tg] - r_ay) ** 2 + (az[tg] - r_az) ** 2) / Sa
    e_u = np.abs(du[tg] - r_du) / np.maximum(Su, 1e-300)
    say(f"prec={prec}: max rel. err rho {e_rho.max():.2e} a {e_a.max():.2e} du {e_u.max():.2e}")
    bound = 1e-12 if prec == 0 else 2e-6
    assert e_rho.max() <= bound and e_a.max() <= bound and e_u.max() <= bound


@pytest.mark.timeout(900)
def test_ensemble_full_size_sampled(orc, capsys):
    def say(s):
        with capsys.disabled():
            print(f"\n[ensemble] {s}", flush=True)
    ps = ensemble(256, seed=1004)
    n, so = ps.n, ps.seg_offsets
    seg = orc.seg_ids(n, so)
    rng = np.random.default_rng(11)
    tg = np.sort(rng.choice(n, 1536, replace=False))
    k_ref = orc.keys(ps.x, ps.y, ps.z, seg_offsets=so)
    o_ref = orc.order(k_ref)
    say(f"n={n} in 256 sets, oracle keys and order ready")
    for prec in (0, 1):
        ctx = make_ctx(n, seg_cap=256, precision=prec)
        pa = parts(ps)
        leaf, group = tuned(ctx, pa)
        k, o = gpu_keys_order(ctx, pa)
        say(f"prec={prec}: leaf {leaf} group {group}")
        assert np.array_equal(k, k_ref) and np.array_equal(o, o_ref)
        say(f"prec={prec}: keys and order bit-exact")
        _sampled_sph(orc, ctx, ps, tg, seg, prec, say)
        ctx.close()


@pytest.mark.timeout(1200)
def test_evrard_16m_sampled(orc, capsys):
    import math as _m

    def say(s):
        with capsys.disabled():
            print(f"\n[evrard] {s}", flush=True)
    n = 16777216
    ps = evrard(n, seed=1005)
    say(f"n={n} generated")
    k_ref = orc.keys(ps.x, ps.y, ps.z)
    o_ref = orc.order(k_ref)
    say("oracle keys and order ready")
    rng = np.random.default_rng(13)
    r = np.sqrt(ps.x ** 2 + ps.y ** 2 + ps.z ** 2)
    tg = np.unique(np.concatenate([rng.choice(n, 384, replace=False), np.argsort(r)[:64:4]]))  # + the centre
    gt = np.sort(rng.choice(n, 256, replace=False))
    dx, dy, dz, dp = orc.gravity_direct(ps.x, ps.y, ps.z, ps.m, 1.0, 0.005, targets=gt)
    gd = np.sqrt(dx ** 2 + dy ** 2 + dz ** 2)
    say("oracle direct gravity on 256 targets ready")
    for prec in (1, 0):
        ctx = make_ctx(n, precision=prec, adaptive_h=1, G=1.0, soft_eps=0.005, theta=0.5, nbr_capacity=256)
        k, o = gpu_keys_order(ctx, parts(ps))
        assert np.array_equal(k, k_ref) and np.array_equal(o, o_ref)
        say(f"prec={prec}: keys and order bit-exact")
        _sampled_sph(orc, ctx, ps, tg, None, prec, say)
        gx, gy, gz, phi = gpu_gravity(ctx, n)
        e = np.sqrt((gx[gt] - dx) ** 2 + (gy[gt] - dy) ** 2 + (gz[gt] - dz) ** 2) / gd
        rms = _m.sqrt((e ** 2).mean())
        say(f"prec={prec}: gravity RMS {rms:.3e} median {np.median(e):.2e} max {e.max():.2e}")
        assert rms <= 1e-3
        ctx.close()
