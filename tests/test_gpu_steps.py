"""GPU parity of the resident leapfrog step (sph_step) against the oracle's step.

* Batched ensembles: independent sets of uneven size, each stepping by its own dt, in one
  captured step (graphs on and off), FP64 and FP32C.  Each step's keys and key order are
  checked bit for bit against the oracle's keys of the returned positions with each set's
  own box (the per-set box, L and S derived inside the step); each set's fields against the
  oracle's step of that set alone, per particle: FP64 within 1e-12 of the particle's own
  scale, FP32C within the stated budget (median, p99 and max printed per field).
* FP32C steps on the lattice and the small tube, against the oracle's FP64 step from the
  same state, per field.
* The time-step bound (sph_timestep, diagnostics entry 9) and the gravitational energy
  (entry 8) against the oracle.
* Regression: a context handed a new workspace, or autotuned and then given another set
  layout of the same size, steps like a fresh eager context (no stale captured graph).
"""
import numpy as np
import pytest

from workloads import ensemble, lattice_box, polytrope_n1, sod_tube

from gpu_helpers import STEP_FIELDS, gpu_gravity, gpu_keys_order, make_ctx, parts, state_from, step_errors, to_np

pytestmark = pytest.mark.gpu

TOL = 1e-12
# FP32C: pair arithmetic in FP32 with Kahan sums; per-particle error against the FP64 oracle
# relative to each field's scale (gpu_helpers.step_scales).
FP32C_MAX = 2e-6
FP32C_MEDIAN = 2e-7


def _box(st, a, b):
    return {k: v[a:b].copy() for k, v in st.items() if isinstance(v, np.ndarray) and v.shape[:1] == (len(st["x"]),)}


def _gpu_keys(ctx, n):
    import torch
    import paper_2007_03097_amd as sph
    keys = torch.zeros(max(n, 1), dtype=torch.int64, device="cuda")
    order = torch.zeros(max(n, 1), dtype=torch.int64, device="cuda")
    sph.sph_key_order(ctx.h, keys, order)
    return to_np(keys)[:n].view(np.uint64), to_np(order)[:n]


def _stats(name, errs, capsys, tag):
    with capsys.disabled():
        print(f"\n{tag} {name}: " + "  ".join(
            f"{k} {np.median(e):.1e}/{np.percentile(e, 99):.1e}/{e.max():.1e}" for k, e in errs.items()
            if k not in ("y", "z", "vy", "vz", "ay", "az")), flush=True)


def _small_ensemble(seed=41):
    # six jittered-lattice sets of 8^3 .. 21^3 particles (uneven sizes, densities, energies)
    return ensemble(n_boxes=6, seed=seed, n_min=500, n_max=9300, side_lo=8, side_hi=21)


@pytest.mark.parametrize("graph", ["1", "0"])
@pytest.mark.parametrize("prec", [0, 1])
def test_batched_step_lockstep(orc, prec, graph, monkeypatch, capsys):
    """Segmented, graph-captured steps of a small ensemble, each set by its own dt, in
    lockstep with the oracle's step of each set alone (3 steps)."""
    import paper_2007_03097_amd as sph
    monkeypatch.setenv("SPH_NO_GRAPH", "0" if graph == "1" else "1")
    ps = _small_ensemble()
    so = ps.seg_offsets
    nb = len(so) - 1
    prm = orc.Params()
    prim = [orc.prime(_box(ps.fields(), so[i], so[i + 1]), prm) for i in range(nb)]
    dts = np.array([0.25 * orc.dt_bound(p)[0] for p in prim])
    assert len(set(np.round(dts, 12))) > 1           # the sets really step by different dt
    ctx = make_ctx(ps.n, seg_cap=8, precision=prec, group_size=32)
    pa = parts(ps, with_accel=True)
    pa.seg_dt = dts
    # step 0 starts from the oracle's priming (FP64) or from the GPU's own (FP32C: its
    # accelerations enter the predictors, so only that start makes the same step)
    flags = 0
    if prec == 1:
        sph.sph_step(ctx.h, pa, 1.0, 0, 0)
        flags = sph.SPH_STEP_PRIMED
    worst = {k: [] for k in STEP_FIELDS}
    for step in range(3):
        start = None if (step == 0 and prec == 0) else state_from(pa)
        print(f"[batched lockstep] prec={prec} graph={graph} step {step}", flush=True)
        sph.sph_step(ctx.h, pa, 1.0, 1, flags)   # dt argument unused: seg_dt given
        got = state_from(pa)
        # the step's keys: per-set box of the returned positions, 18 bits + set number
        k, o = _gpu_keys(ctx, ps.n)
        assert np.array_equal(k, orc.keys(got["x"], got["y"], got["z"], seg_offsets=so)), step
        assert np.array_equal(o, orc.order(k)), step
        for i in range(nb):
            a, b = so[i], so[i + 1]
            st_i = prim[i] if start is None else _box(start, a, b)
            ref = orc.kdk_step(st_i, dts[i], prm)
            e = step_errors(_box(got, a, b), ref, st_i, dts[i])
            for kf in STEP_FIELDS:
                worst[kf].append(e[kf])
            if prec == 0:
                for kf, ek in e.items():
                    assert ek.max() <= TOL, (step, i, kf, float(ek.max()))
        flags = sph.SPH_STEP_PRIMED
    errs = {kf: np.concatenate(v) for kf, v in worst.items()}
    _stats(f"prec={prec} graph={graph}", errs, capsys, "batched step median/p99/max")
    if prec == 1:
        for kf, e in errs.items():
            assert np.median(e) <= FP32C_MEDIAN and e.max() <= FP32C_MAX, kf
    # the time-step bound of each set after the last step, against the oracle's
    if prec == 0:
        bd = sph.sph_timestep(ctx.h, nb)
        for i in range(nb):
            ref = orc.kdk_step(_box(start, so[i], so[i + 1]), dts[i], prm)
            assert abs(bd[i] - orc.dt_bound(ref)[0]) <= TOL * bd[i], i


@pytest.mark.parametrize("case,adaptive,dt", [("lattice", 0, 0.0178), ("tube", 1, 4.0e-4)])
def test_fp32c_step_lockstep(orc, case, adaptive, dt, capsys):
    """FP32C steps against the oracle's FP64 step from the same state (3 steps): per field
    median <= 2e-7 and max <= 2e-6 of each particle's scale."""
    import paper_2007_03097_amd as sph
    ps = lattice_box(16) if case == "lattice" else sod_tube(8)
    ctx = make_ctx(ps.n, adaptive_h=adaptive, precision=1)
    pa = parts(ps, with_accel=True)
    prm = orc.Params(adaptive_h=bool(adaptive))
    # lockstep from the GPU's own primed state: the FP32C accelerations of the input state
    # enter the predictors, so a step from the oracle's FP64 priming would not be the same step
    sph.sph_step(ctx.h, pa, dt, 0, 0)
    allerr = {k: [] for k in STEP_FIELDS}
    for step in range(3):
        start = state_from(pa)
        sph.sph_step(ctx.h, pa, dt, 1, sph.SPH_STEP_PRIMED)
        ref = orc.kdk_step(start, dt, prm)
        e = step_errors(state_from(pa), ref, start, dt)
        for k in STEP_FIELDS:
            allerr[k].append(e[k])
    errs = {k: np.concatenate(v) for k, v in allerr.items()}
    _stats(case, errs, capsys, "FP32C step median/p99/max")
    for k, e in errs.items():
        assert np.median(e) <= FP32C_MEDIAN and e.max() <= FP32C_MAX, k


def test_timestep_bound_and_potential_energy(orc):
    """With self-gravity (theta = 0, the direct sum): the time-step bound of the primed state
    (min of h/c and the free-fall term) and E_grav = sum m phi / 2 equal the oracle's."""
    import paper_2007_03097_amd as sph
    ps = polytrope_n1(3000, seed=23)
    G, eps = 1.0, 0.01
    ctx = make_ctx(ps.n, G=G, soft_eps=eps, theta=0.0, adaptive_h=1, nbr_capacity=1024)
    pa = parts(ps)
    d = sph.sph_step(ctx.h, pa, 1e-3, 0, 0)         # prime only
    prm = orc.Params(adaptive_h=True, G=G, soft_eps=eps)
    st = orc.prime(ps.fields(), prm)
    ref_b = orc.dt_bound(st, eps)[0]
    assert abs(d[9] - ref_b) <= TOL * ref_b
    assert abs(sph.sph_timestep(ctx.h, 1)[0] - ref_b) <= TOL * ref_b
    # the free-fall term decides somewhere (else this would only test h/c)
    a = np.sqrt(st["ax"] ** 2 + st["ay"] ** 2 + st["az"] ** 2)
    assert np.min(np.sqrt(eps / a)) < np.min(st["h"] / st["cs"])
    _, _, _, phi, sg = orc.gravity_direct(ps.x, ps.y, ps.z, ps.m, G, eps, scale=True)
    eg = orc.diagnostics(st, phi)[8]
    assert abs(d[8] - eg) <= TOL * 0.5 * np.sum(ps.m * np.abs(phi))
    # without gravity the bound is h/c alone; nsteps = 0 with SPH_STEP_PRIMED has no density
    ctx2 = make_ctx(ps.n, adaptive_h=1, nbr_capacity=1024)
    pa2 = parts(ps, with_accel=True)
    d2 = sph.sph_step(ctx2.h, pa2, 1e-3, 0, 0)
    st2 = orc.prime(ps.fields(), orc.Params(adaptive_h=True))
    assert abs(d2[9] - orc.dt_bound(st2)[0]) <= TOL * d2[9]
    d3 = sph.sph_step(ctx2.h, pa2, 1e-3, 0, sph.SPH_STEP_PRIMED)
    assert np.isnan(d3[9])
    with pytest.raises(sph.SPHError):
        sph.sph_timestep(ctx2.h, 1)


def _step_fresh(ps, steps, no_graph, monkeypatch, **cfg):
    import paper_2007_03097_amd as sph
    monkeypatch.setenv("SPH_NO_GRAPH", "1" if no_graph else "0")
    ctx = make_ctx(ps.n, **cfg)
    pa = parts(ps, with_accel=True)
    sph.sph_step(ctx.h, pa, 4e-4, steps, 0)
    out = state_from(pa)
    ctx.close()
    return out


def test_new_workspace_recaptures_the_step(monkeypatch):
    """A context handed a second workspace steps like a fresh eager context: the graphs
    captured with the first workspace's pointers are dropped, not replayed."""
    import torch
    import paper_2007_03097_amd as sph
    ps = sod_tube(8)
    ref = _step_fresh(ps, 2, True, monkeypatch, adaptive_h=1)
    monkeypatch.setenv("SPH_NO_GRAPH", "0")
    ctx = make_ctx(ps.n, adaptive_h=1)
    pa = parts(ps, with_accel=True)
    sph.sph_step(ctx.h, pa, 4e-4, 2, 0)        # captures with workspace 1
    ws2 = torch.empty_like(ctx.ws)
    sph.sph_set_workspace(ctx.h, ws2)
    old = ctx.ws
    ctx.ws = ws2
    old.fill_(0xFF)                            # stale pointers would now read garbage
    pa = parts(ps, with_accel=True)
    sph.sph_step(ctx.h, pa, 4e-4, 2, 0)
    got = state_from(pa)
    for k in got:
        assert np.array_equal(got[k], ref[k]), k


def test_same_size_new_layout_recaptures_the_step(monkeypatch, tmp_path):
    """After autotuning on one set layout, a set of the same size but other segment offsets
    steps like a fresh eager context (the table version only ever increases)."""
    import paper_2007_03097_amd as sph
    a = ensemble(n_boxes=4, seed=51, n_min=500, n_max=4000, side_lo=8, side_hi=16)
    b = a.copy()
    so = a.seg_offsets.copy()
    so[1:-1] = np.sort(np.random.default_rng(3).choice(np.arange(1, a.n), len(so) - 2, replace=False))
    b.seg_offsets = so
    cap = dict(seg_cap=8, nbr_capacity=1024)   # the new sets may join overlapping boxes
    monkeypatch.setenv("SPH_NO_GRAPH", "0")
    ctx = make_ctx(a.n, **cap)
    sph.sph_autotune(ctx.h, parts(a), 1e-3, str(tmp_path / "t.json"))
    pa = parts(b, with_accel=True)
    sph.sph_step(ctx.h, pa, 4e-4, 2, 0)
    got = state_from(pa)
    lf, gs, _ = sph.sph_get_tuning(ctx.h)
    ref = _step_fresh(b, 2, True, monkeypatch, leaf_size=lf, group_size=gs, **cap)
    for k in got:
        assert np.array_equal(got[k], ref[k]), k


def test_step_reports_a_state_turned_nonfinite(monkeypatch):
    """A state that turns non-finite during the steps is reported: one particle with negative
    thermal energy has a NaN sound speed, so its viscous pairs (and the accelerations) are NaN,
    and the kick-drift that applies them raises SPH_E_NONFINITE, with graphs and without."""
    import paper_2007_03097_amd as sph
    for no_graph in ("0", "1"):
        monkeypatch.setenv("SPH_NO_GRAPH", no_graph)
        ps = lattice_box(8, seed=3, v_sigma=0.1)
        ps.u[100] = -1.0
        ctx = make_ctx(ps.n)
        with pytest.raises(sph.SPHError) as e:
            sph.sph_step(ctx.h, parts(ps), 1e-4, 2, 0)
        assert e.value.status == -6
        ok = lattice_box(8, seed=3, v_sigma=0.1)
        ctx2 = make_ctx(ok.n)
        sph.sph_step(ctx2.h, parts(ok), 1e-4, 2, 0)  # the same set with u > 0 steps cleanly


@pytest.mark.parametrize("no_graph", [False, True])
def test_run_of_steps_equals_single_steps(monkeypatch, no_graph):
    """Inside a run the closing half kick of a step is applied at the start of the next one (the
    two kicks of the leapfrog's joint, with the same accelerations); the state after one call of
    three steps is bit for bit that of three calls of one step, with adaptive h, both energy
    equations and both precisions."""
    import paper_2007_03097_amd as sph
    monkeypatch.setenv("SPH_NO_GRAPH", "1" if no_graph else "0")
    ps = sod_tube(6)
    for cfg in (dict(adaptive_h=1), dict(adaptive_h=1, energy_form=sph.SPH_ENERGY_THERMOKINETIC),
                dict(adaptive_h=0, precision=1)):
        runs = []
        for split in (False, True):
            ctx = make_ctx(ps.n, **cfg)
            pa = parts(ps, with_accel=True)
            if split:
                sph.sph_step(ctx.h, pa, 4e-4, 1, 0)
                sph.sph_step(ctx.h, pa, 4e-4, 1, sph.SPH_STEP_RESUME)
                sph.sph_step(ctx.h, pa, 4e-4, 1, sph.SPH_STEP_RESUME)
            else:
                sph.sph_step(ctx.h, pa, 4e-4, 3, 0)
            runs.append(state_from(pa))
            ctx.close()
        for k in STEP_FIELDS:
            assert np.array_equal(runs[0][k], runs[1][k]), (cfg, k)


@pytest.mark.parametrize("no_graph", [False, True])
def test_run_with_gravity_keeps_the_final_potential(monkeypatch, no_graph):
    """Inside a run of steps only the last step's gravity pass evaluates the potential, which
    nothing but the energy diagnostic reads: the state and the diagnostics (E_grav included)
    after one call of three steps are bit for bit those of three calls of one step, in both
    precisions and with both gravity schemes, and a gravity pass through the API after the run
    returns the potential again (equal to that of a fresh context on the same particles)."""
    import paper_2007_03097_amd as sph
    monkeypatch.setenv("SPH_NO_GRAPH", "1" if no_graph else "0")
    ps = polytrope_n1(3000, seed=23)
    for prec, scheme in ((0, 0), (1, 0), (0, 1), (1, 1)):
        cfg = dict(G=1.0, soft_eps=0.01, theta=0.5, adaptive_h=1, nbr_capacity=1024, precision=prec,
                   gravity_scheme=scheme)
        runs, diags = [], []
        for split in (False, True):
            ctx = make_ctx(ps.n, **cfg)
            pa = parts(ps, with_accel=True)
            if split:
                sph.sph_step(ctx.h, pa, 1e-3, 1, 0)
                sph.sph_step(ctx.h, pa, 1e-3, 1, sph.SPH_STEP_RESUME)
                d = sph.sph_step(ctx.h, pa, 1e-3, 1, sph.SPH_STEP_RESUME)
            else:
                d = sph.sph_step(ctx.h, pa, 1e-3, 3, 0)
                gpu_keys_order(ctx, pa)
                after = gpu_gravity(ctx, ps.n)
                fresh = make_ctx(ps.n, **cfg)
                gpu_keys_order(fresh, pa)
                ref = gpu_gravity(fresh, ps.n)
                fresh.close()
                for a, b in zip(after, ref):
                    assert np.array_equal(a, b), (prec, scheme)
                assert np.all(ref[3] < 0.0)  # the potential was evaluated
            runs.append(state_from(pa))
            diags.append(np.asarray(d, dtype=np.float64))
            ctx.close()
        for k in STEP_FIELDS:
            assert np.array_equal(runs[0][k], runs[1][k]), (prec, scheme, k)
        assert np.array_equal(diags[0], diags[1], equal_nan=True), (prec, scheme)
        assert np.isfinite(diags[0][8]) and diags[0][8] < 0.0  # E_grav of the final state
