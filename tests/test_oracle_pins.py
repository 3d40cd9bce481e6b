"""Pins for the CPU FP64 reference (oracle/): every function is checked against something
other than itself -- the paper's worked example (Fig. 1), closed forms, library routines,
exact invariants of the discrete equations, and finite differences of an independent
quantity.  These tests run on the CPU only."""
import math
import os

import numpy as np
import pytest
from scipy import integrate

from workloads import fig1_points, lattice_box, polytrope_n1, uniform_random

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------------------- kernel
def test_kernel_normalisation(orc):
    """M4 spline in 3D integrates to one: 4 pi int_0^2 W q^2 dq with W = w/pi (h = 1)."""
    val = sum(integrate.quad(lambda q: 4.0 * math.pi * orc.w(q) / math.pi * q * q, a, b, epsabs=1e-15,
                             epsrel=1e-14)[0] for a, b in ((0.0, 1.0), (1.0, 2.0)))
    assert abs(val - 1.0) < 1e-13


def test_kernel_shape(orc):
    """Continuity at q = 1, 2; w(0) = 1; compact support."""
    assert orc.w(0.0) == 1.0
    assert abs(orc.w(1.0 - 1e-12) - orc.w(1.0)) < 1e-11
    assert orc.w(2.0) == 0.0 and orc.w(2.5) == 0.0
    assert abs(orc.w(1.0) - 0.25) < 1e-15


def test_kernel_gradient_matches_finite_difference(orc):
    """g(q) = w'(q)/q, checked against central differences of w."""
    for q in np.linspace(0.05, 1.95, 39):
        if abs(q - 1.0) < 1e-3:
            continue
        d = 1e-6
        fd = (orc.w(q + d) - orc.w(q - d)) / (2 * d)
        assert abs(orc.dw_over_q(q) * q - fd) < 1e-8


# ---------------------------------------------------------------------------- keys / order
def _key_to_fig(key, level):
    s = "1"
    for i in range(level):
        s += str((int(key) >> (3 * (level - 1 - i))) & 7)
    return s


def test_fig1_tree(orc):
    """Fig. 1: ten particles, one per leaf; the leaf and internal keys of the right panel."""
    x, y, z, box = fig1_points()
    k = orc.keys(x, y, z, box=box)
    o = orc.order(k)
    t = orc.octree(k[o], leaf_cap=1)
    got_leaf = sorted(_key_to_fig(kk, lv) for kk, lv, lf in zip(t["key"], t["level"], t["leaf"]) if lf)
    got_int = sorted(_key_to_fig(kk, lv) for kk, lv, lf in zip(t["key"], t["level"], t["leaf"]) if not lf)
    lines = dict(l.split(":", 1) for l in open(os.path.join(GOLDEN, "fig1_tree.txt")) if not l.startswith("#"))
    assert got_leaf == sorted(lines["leaves"].split())
    assert got_int == sorted(lines["internal"].split())


def test_key_bit_interleave_hand_cases(orc):
    """Single-axis unit steps give digits 1 (x), 2 (y), 4 (z) in the lowest digit; a point
    at the far corner gets all 63 digit bits set."""
    box = np.array([0.0, 0.0, 0.0, 1.0, 1.0, 1.0])
    q = 1.0 / 2 ** 21
    pts = np.array([[0, 0, 0], [q, 0, 0], [0, q, 0], [0, 0, q], [1, 1, 1], [0.5, 0, 0]], dtype=float)
    k = orc.keys(pts[:, 0], pts[:, 1], pts[:, 2], box=box)
    s = np.uint64(1 << 63)
    assert list(k - s) == [0, 1, 2, 4, (1 << 63) - 1, 1 << 60]


def test_key_segments(orc):
    """Segmented sets: sentinel, segment number in bits 54..62, 18 bits per axis."""
    ps = uniform_random(300, seed=3)
    so = np.array([0, 100, 100, 300])
    k = orc.keys(ps.x, ps.y, ps.z, seg_offsets=so)
    seg = (k >> np.uint64(54)) & np.uint64(511)
    assert (k >> np.uint64(63)).all()
    assert (seg[:100] == 0).all() and (seg[100:] == 2).all()
    assert (k & np.uint64((1 << 54) - 1)).max() < (1 << 54)


def test_hilbert_index_is_a_hilbert_curve(orc):
    """Skilling's Hilbert index on 2^b grids (b = 1..4): a bijection onto 0 .. 8^b - 1 that
    starts at the origin, moves to a face neighbour at every step, and maps every octree
    cell (equal leading 3-bit digits) onto an aligned cube -- the properties that make it a
    Hilbert curve and make octree cells contiguous runs of keys."""
    import itertools
    for b in (1, 2, 3, 4):
        N = 1 << b
        at = {}
        for x, y, z in itertools.product(range(N), repeat=3):
            at[orc.hilbert(x, y, z, b)] = (x, y, z)
        assert sorted(at) == list(range(N ** 3))
        assert at[0] == (0, 0, 0)
        for h in range(N ** 3 - 1):
            assert sum(abs(p - q) for p, q in zip(at[h], at[h + 1])) == 1, (b, h)
        for lev in range(1, b + 1):
            sh = 3 * (b - lev)
            cells = {}
            for h, c in at.items():
                cells.setdefault(h >> sh, set()).add(tuple(v >> (b - lev) for v in c))
            assert all(len(s) == 1 for s in cells.values())


def test_hilbert_keys_give_the_same_octree_cells(orc):
    """The octree over Hilbert-sorted keys has the same cells (as particle sets, per level)
    as the one over Morton-sorted keys; keys keep the sentinel and segment prefix."""
    ps = uniform_random(3000, seed=31, h=0.05)
    ps.x[:40] = ps.x[0]; ps.y[:40] = ps.y[0]; ps.z[:40] = ps.z[0]   # a run of equal keys
    cells = []
    for curve in ("morton", "hilbert"):
        k = orc.keys(ps.x, ps.y, ps.z, curve=curve)
        assert np.all(k >> np.uint64(63) == 1)
        o = orc.order(k)
        t = orc.octree(k[o], 8)
        cells.append(sorted((int(l), tuple(sorted(o[s:s + c].tolist())))
                            for l, s, c in zip(t["level"], t["start"], t["count"])))
    assert cells[0] == cells[1]
    so = np.array([0, 1000, 3000])
    kh = orc.keys(ps.x, ps.y, ps.z, seg_offsets=so, curve="hilbert")
    assert np.all((kh[1000:] >> np.uint64(54)) & np.uint64(511) == 1) and np.all(kh >> np.uint64(63) == 1)


def test_order_matches_lexsort(orc):
    """Stable order by (key, caller index) equals numpy.lexsort, including many ties."""
    rng = np.random.default_rng(7)
    k = rng.integers(0, 50, size=5000).astype(np.uint64) | np.uint64(1 << 63)
    assert (orc.order(k) == np.lexsort((np.arange(k.size), k))).all()


# ---------------------------------------------------------------------------- octree
def _octree_by_levels(sorted_keys, cap, min_level=0):
    """Independent construction: level by level, a cell is a node iff its parent cell is a
    node that is refined (more than cap particles, or below min_level)."""
    body = sorted_keys & np.uint64((1 << 63) - 1)
    nodes = set()
    refined_prev = None
    for lv in range(22):
        pref = body >> np.uint64(3 * (21 - lv))
        uniq, cnt = np.unique(pref, return_counts=True)
        parent = uniq >> np.uint64(3) if lv > 0 else uniq
        refined = set()
        for p, u, c in zip(parent, uniq, cnt):
            if lv == 0 or int(p) in refined_prev:
                leaf = (lv >= min_level and c <= cap) or lv == 21
                nodes.add((lv, int(u), bool(leaf)))
                if not leaf:
                    refined.add(int(u))
        refined_prev = refined
    return nodes


@pytest.mark.parametrize("cap,min_level", [(1, 0), (4, 0), (16, 0), (16, 3)])
def test_octree_matches_level_construction(orc, cap, min_level):
    ps = polytrope_n1(3000, seed=11)
    k = np.sort(orc.keys(ps.x, ps.y, ps.z))
    k[100:110] = k[100]  # a run of equal keys
    k = np.sort(k)
    t = orc.octree(k, leaf_cap=cap, min_level=min_level)
    mask = np.uint64((1 << 63) - 1)
    got = set()
    for kk, lv, lf in zip(t["key"], t["level"], t["leaf"]):
        got.add((int(lv), int(np.uint64(kk) & ~np.uint64(1 << (3 * int(lv))) & mask) if lv > 0 else 0, bool(lf)))
    assert got == _octree_by_levels(k, cap, min_level)
    # leaves partition the sorted range in order
    leaves = [(s, c) for s, c, lf in zip(t["start"], t["count"], t["leaf"]) if lf]
    pos = 0
    for s, c in leaves:
        assert s == pos
        pos += c
    assert pos == k.size


# ---------------------------------------------------------------------------- neighbours
# Closed lattice sums of an infinite cubic lattice with h = hfac dx (m = dx^3 = rho0 = 1):
# rho/rho0 = sum over integer vectors n with |n| < 2 hfac of w(|n|/hfac) / (pi hfac^3), self
# included, and the number of such vectors.  The values were computed independently of this
# repository's code (high-precision sums of the M4 kernel); the short ones carry 5 digits.
LATTICE_SUMS = {1.0: (0.99997, 27, 5e-6), 1.2: (1.000809548358436, 57, 1e-13), 1.3: (0.99726, 81, 5e-6),
                1.5: (1.00179, 93, 5e-6)}


@pytest.mark.parametrize("hfac", sorted(LATTICE_SUMS))
def test_lattice_density_and_neighbour_count(orc, hfac):
    """A perfect lattice recovers rho0 up to the closed lattice sum; interior particles have
    exactly as many neighbours as integer vectors inside radius 2 hfac (self included)."""
    ps = lattice_box(16, jitter=0.0, v_sigma=0.0)
    dx = 1.0 / 16
    ps.h = np.full(ps.n, hfac * dx)
    csr = orc.neighbors(ps.x, ps.y, ps.z, ps.h)
    rho, P, c, hn = orc.density(ps.fields(), csr)
    e = 2 * hfac * dx
    inner = ((ps.x > e) & (ps.x < 1 - e) & (ps.y > e) & (ps.y < 1 - e) & (ps.z > e) & (ps.z < 1 - e))
    ref, cnt, rtol = LATTICE_SUMS[hfac]
    assert inner.sum() > 0
    assert (np.diff(csr[0])[inner] == cnt).all()
    assert np.allclose(rho[inner], ref, rtol=rtol, atol=0)


def test_neighbours_match_kdtree(orc):
    """Constant h: the neighbour sets equal scipy's cKDTree ball query of radius 2h (no exact
    ties in random data)."""
    from scipy.spatial import cKDTree
    ps = uniform_random(2000, seed=5, h=(0.04, 0.04))
    off, idx = orc.neighbors(ps.x, ps.y, ps.z, ps.h)
    tree = cKDTree(np.stack([ps.x, ps.y, ps.z], axis=1))
    ref = tree.query_ball_point(np.stack([ps.x, ps.y, ps.z], axis=1), r=0.08)
    for a in range(ps.n):
        assert list(idx[off[a]:off[a + 1]]) == sorted(ref[a])


def test_neighbours_symmetric_variable_h(orc):
    ps = uniform_random(1500, seed=6, h=(0.01, 0.06))
    off, idx = orc.neighbors(ps.x, ps.y, ps.z, ps.h)
    pairs = set()
    for a in range(ps.n):
        for b in idx[off[a]:off[a + 1]]:
            pairs.add((a, int(b)))
    assert all((b, a) in pairs for a, b in pairs)
    assert all((a, a) in pairs for a in range(ps.n))


def test_neighbours_segments(orc):
    ps = uniform_random(400, seed=8, h=0.1)
    so = np.array([0, 150, 400])
    seg = orc.seg_ids(ps.n, so)
    off, idx = orc.neighbors(ps.x, ps.y, ps.z, ps.h, seg=seg)
    for a in range(ps.n):
        assert (seg[idx[off[a]:off[a + 1]]] == seg[a]).all()


# ---------------------------------------------------------------------------- EOS
def test_eos_closed_form(orc):
    """u = 1, gamma = 5/3: P = 2 rho / 3, c = sqrt(10/9); h_next^3 rho / m = 1.2^3."""
    ps = lattice_box(8)
    csr = orc.neighbors(ps.x, ps.y, ps.z, ps.h)
    rho, P, c, hn = orc.density(ps.fields(), csr)
    assert np.allclose(P / rho, 2.0 / 3.0, rtol=1e-15)
    assert np.allclose(c, math.sqrt(10.0 / 9.0), rtol=1e-15)
    assert np.allclose(hn ** 3 * rho / ps.m, 1.2 ** 3, rtol=1e-14)


# ---------------------------------------------------------------------------- forces
def _random_state(orc, n=300, seed=21, v_sigma=0.5):
    ps = uniform_random(n, seed=seed, h=(0.08, 0.16), v_sigma=v_sigma)
    csr = orc.neighbors(ps.x, ps.y, ps.z, ps.h)
    rho, P, c, _ = orc.density(ps.fields(), csr)
    return ps, csr, rho, P, c


def test_momentum_and_angular_momentum_conserved(orc):
    """Pair terms are antisymmetric and central (Sec. 1: conservation to machine precision):
    sum m a = 0 and sum m r x a = 0 to rounding, viscosity included."""
    ps, csr, rho, P, c = _random_state(orc)
    ax, ay, az, du, Sa, Su = orc.forces(ps.fields(), rho, P, c, csr)
    scale = (ps.m * Sa).sum()
    assert abs((ps.m * ax).sum()) < 1e-14 * scale
    assert abs((ps.m * ay).sum()) < 1e-14 * scale
    assert abs((ps.m * az).sum()) < 1e-14 * scale
    r = np.stack([ps.x, ps.y, ps.z], axis=1)
    a = np.stack([ax, ay, az], axis=1)
    L = (ps.m[:, None] * np.cross(r, a)).sum(axis=0)
    assert np.abs(L).max() < 1e-13 * scale


def test_energy_rate_vanishes(orc):
    """dE/dt = sum m v.a + sum m du/dt = 0 for the semi-discrete system (viscous terms cancel
    pairwise through the 1/2 in eq. (5))."""
    ps, csr, rho, P, c = _random_state(orc)
    ax, ay, az, du, Sa, Su = orc.forces(ps.fields(), rho, P, c, csr)
    dE = (ps.m * (ps.vx * ax + ps.vy * ay + ps.vz * az)).sum() + (ps.m * du).sum()
    vmag = np.sqrt(ps.vx ** 2 + ps.vy ** 2 + ps.vz ** 2)
    scale = (ps.m * (vmag * Sa + Su)).sum()
    assert abs(dE) < 1e-14 * scale
    # the viscosity is active in this state
    _, _, _, du0, _, _ = orc.forces(ps.fields(), rho, P, c, csr, alpha=0.0, beta=0.0)
    assert np.abs(du - du0).max() > 1e-3 * np.abs(du).max()


def test_thermokinetic_rate_is_thermal_plus_kinetic(orc):
    """Eq. (8) against eq. (5) and (6): per particle, de_a/dt = du_a/dt + v_a . dv_a/dt (no
    gravity) -- the pressure parts recombine as P_a v_b/rho_a^2 + P_b v_a/rho_b^2 and the
    viscous parts as (v_a + v_b)/2 Pi_ab.  A swapped P_a/P_b, a wrong sign or a dropped
    viscous half breaks it."""
    ps, csr, rho, P, c = _random_state(orc)
    ax, ay, az, du, Sa, Su = orc.forces(ps.fields(), rho, P, c, csr)
    de, Se = orc.dedt(ps.fields(), rho, P, c, csr)
    vmag = np.sqrt(ps.vx ** 2 + ps.vy ** 2 + ps.vz ** 2)
    ref = du + ps.vx * ax + ps.vy * ay + ps.vz * az
    assert np.all(np.abs(de - ref) <= 1e-13 * (Se + Su + vmag * Sa))
    assert np.abs(de).max() > 1e-3 * np.abs(Se).max()       # the rate is not trivially zero


def test_thermokinetic_rate_conserves_total_energy(orc):
    """Eq. (8)'s pair terms are antisymmetric: sum m_a de_a/dt = 0 to rounding, viscosity
    included; with v = 0 every term vanishes."""
    ps, csr, rho, P, c = _random_state(orc)
    de, Se = orc.dedt(ps.fields(), rho, P, c, csr)
    assert abs((ps.m * de).sum()) < 1e-14 * (ps.m * Se).sum()
    z = np.zeros(ps.n)
    de0, _ = orc.dedt(ps.fields(), rho, P, c, csr, vel=(z, z, z))
    assert np.all(de0 == 0.0)


def test_thermokinetic_kdk_conserves_energy_each_step(orc):
    """With e = u + v^2/2 integrated by the kick-drift-kick, sum m e changes only by rounding
    per step (sum m de/dt = 0 at every evaluation), while the eq. (5) integrator's error is
    of third order in dt; momentum is conserved to rounding in both."""
    ps = lattice_box(8, v_sigma=0.05, jitter=0.2)
    prm = orc.Params(adaptive_h=False, thermokinetic=True)
    st = orc.prime(ps.fields(), prm)
    E0 = orc.diagnostics(st)
    for _ in range(3):
        st = orc.kdk_step(st, 0.02, prm)
        E = orc.diagnostics(st)
        assert abs((E[6] + E[7]) - (E0[6] + E0[7])) <= 1e-13 * (E0[6] + E0[7])
        assert np.abs(E[:3] - E0[:3]).max() < 1e-15
    st5 = orc.kdk_step(orc.prime(ps.fields(), orc.Params(adaptive_h=False)), 0.02, orc.Params(adaptive_h=False))
    E5 = orc.diagnostics(st5)
    assert abs((E5[6] + E5[7]) - (E0[6] + E0[7])) > 1e-10 * (E0[6] + E0[7])


def test_thermokinetic_step_agrees_with_thermal_to_third_order(orc):
    """Both energy forms discretise the same equations, so one step of each differs by the
    local error only: the difference in u and v falls by ~2^3 per halving of dt (a predictor
    or EOS-input mistake in either form leaves a second-order difference)."""
    ps = lattice_box(8, v_sigma=0.05, jitter=0.2)
    pt, pk = orc.Params(adaptive_h=False), orc.Params(adaptive_h=False, thermokinetic=True)
    st_t, st_k = orc.prime(ps.fields(), pt), orc.prime(ps.fields(), pk)
    diffs = []
    for dt in (0.02, 0.01, 0.005):
        a, b = orc.kdk_step(st_t, dt, pt), orc.kdk_step(st_k, dt, pk)
        diffs.append(max(np.abs(a["u"] - b["u"]).max(), np.abs(a["vx"] - b["vx"]).max()))
    assert 7.0 < diffs[0] / diffs[1] < 20.0 and 7.0 < diffs[1] / diffs[2] < 20.0


def _thermal_energy(orc, ps, K, gamma):
    csr = orc.neighbors(ps.x, ps.y, ps.z, ps.h)
    rho, _, _, _ = orc.density(ps.fields(), csr)
    return (ps.m * K * rho ** (gamma - 1) / (gamma - 1)).sum()


def test_pressure_force_is_energy_gradient(orc):
    """Without viscosity, m_a dv_a/dt from eq. (6) is -dE_th/dr_a at fixed entropy
    (E_th = sum m_b u_b(rho_b)), checked by central differences of the density sum."""
    gamma = 5.0 / 3.0
    ps = uniform_random(120, seed=31, h=(0.15, 0.25), v_sigma=0.0)
    csr = orc.neighbors(ps.x, ps.y, ps.z, ps.h)
    rho, P, c, _ = orc.density(ps.fields(), csr)
    K = P / rho ** gamma
    ax, ay, az, du, Sa, _ = orc.forces(ps.fields(), rho, P, c, csr)
    for a in [0, 17, 55, 99]:
        for comp, acc in (("x", ax), ("y", ay), ("z", az)):
            d = 1e-6
            p1, p2 = ps.copy(), ps.copy()
            getattr(p1, comp)[a] += d
            getattr(p2, comp)[a] -= d
            grad = (_thermal_energy(orc, p1, K, gamma) - _thermal_energy(orc, p2, K, gamma)) / (2 * d)
            assert abs(ps.m[a] * acc[a] + grad) < 1e-6 * ps.m[a] * Sa[a]


def test_energy_equation_is_compression_rate(orc):
    """Without viscosity, eq. (5) is du_a/dt = (P_a/rho_a^2) d rho_a/dt, with d rho_a/dt from
    central differences of the density sum along the velocity field (eq. (4))."""
    ps = uniform_random(150, seed=41, h=(0.15, 0.25), v_sigma=1.0)
    csr = orc.neighbors(ps.x, ps.y, ps.z, ps.h)
    rho, P, c, _ = orc.density(ps.fields(), csr)
    _, _, _, du, _, Su = orc.forces(ps.fields(), rho, P, c, csr, alpha=0.0, beta=0.0)
    d = 1e-6
    p1, p2 = ps.copy(), ps.copy()
    for comp, v in (("x", ps.vx), ("y", ps.vy), ("z", ps.vz)):
        getattr(p1, comp)[:] += d * v
        getattr(p2, comp)[:] -= d * v
    r1 = orc.density(p1.fields(), orc.neighbors(p1.x, p1.y, p1.z, p1.h))[0]
    r2 = orc.density(p2.fields(), orc.neighbors(p2.x, p2.y, p2.z, p2.h))[0]
    drho = (r1 - r2) / (2 * d)
    assert np.all(np.abs(du - P / rho ** 2 * drho) < 1e-6 * (Su + 1e-300))


def test_viscosity_structure(orc):
    """Monaghan viscosity: zero for receding pairs; for an approaching pair it decelerates
    along the line of centres, heats both particles, and its linear part scales with alpha
    and with the mean sound speed."""
    h = np.array([0.5, 0.5])
    base = dict(x=np.array([0.0, 0.6]), y=np.zeros(2), z=np.zeros(2), h=h, m=np.ones(2))
    rho, P = np.ones(2), np.ones(2)
    c = np.ones(2)
    csr = (np.array([0, 2, 4]), np.array([0, 1, 0, 1]))

    def run(vx, alpha=1.0, beta=0.0, cc=c):
        st = dict(base, vx=np.array(vx), vy=np.zeros(2), vz=np.zeros(2))
        return orc.forces(st, rho, P, cc, csr, alpha=alpha, beta=beta)

    a_off = run([1.0, -1.0], alpha=0.0)
    a_on = run([1.0, -1.0])
    dv = a_on[0][0] - a_off[0][0]
    assert dv < 0 and a_on[3][0] > 0 and a_on[3][1] > 0          # decelerates, heats
    assert a_on[1][0] == 0 and a_on[2][0] == 0                   # along the line of centres
    dv2 = run([1.0, -1.0], alpha=2.0)[0][0] - a_off[0][0]
    assert abs(dv2 - 2 * dv) < 1e-14 * abs(dv)
    dvc = run([1.0, -1.0], cc=2 * c)[0][0] - a_off[0][0]
    assert abs(dvc - 2 * dv) < 1e-14 * abs(dv)
    rec = run([-1.0, 1.0])
    rec0 = run([-1.0, 1.0], alpha=0.0)
    assert rec[0][0] == rec0[0][0] and rec[3][0] == rec0[3][0]


def test_lattice_forces_vanish(orc):
    """Perfect lattice, v = 0, uniform u: interior accelerations cancel by symmetry and
    du/dt is exactly zero everywhere."""
    ps = lattice_box(16, jitter=0.0, v_sigma=0.0)
    dx = 1.0 / 16
    csr = orc.neighbors(ps.x, ps.y, ps.z, ps.h)
    rho, P, c, _ = orc.density(ps.fields(), csr)
    ax, ay, az, du, Sa, Su = orc.forces(ps.fields(), rho, P, c, csr)
    inner = ((ps.x > 4.8 * dx) & (ps.x < 1 - 4.8 * dx) & (ps.y > 4.8 * dx) & (ps.y < 1 - 4.8 * dx)
             & (ps.z > 4.8 * dx) & (ps.z < 1 - 4.8 * dx))
    amag = np.sqrt(ax ** 2 + ay ** 2 + az ** 2)
    assert (amag[inner] <= 1e-13 * Sa[inner]).all()
    assert (du == 0).all()


# ---------------------------------------------------------------------------- gravity
def test_direct_gravity_two_body(orc):
    """Two bodies: g = -G m r/(r^2 + eps^2)^{3/2}, phi = -G m/sqrt(r^2 + eps^2)."""
    x, y, z, m = np.array([0.0, 3.0]), np.array([0.0, 4.0]), np.zeros(2), np.array([2.0, 5.0])
    gx, gy, gz, phi = orc.gravity_direct(x, y, z, m, G=1.5, eps=0.3)
    s = math.sqrt(25 + 0.09)
    assert abs(gx[0] - 1.5 * 5 * 3 / s ** 3) < 1e-15 and abs(gy[0] - 1.5 * 5 * 4 / s ** 3) < 1e-15
    assert abs(phi[1] + 1.5 * 2 / s) < 1e-15
    assert gz[0] == 0


def test_direct_gravity_momentum(orc):
    ps = polytrope_n1(2000, seed=3)
    gx, gy, gz, _ = orc.gravity_direct(ps.x, ps.y, ps.z, ps.m, G=1.0, eps=0.01)
    gm = np.sqrt(gx ** 2 + gy ** 2 + gz ** 2)
    for g in (gx, gy, gz):
        assert abs((ps.m * g).sum()) < 1e-13 * (ps.m * gm).sum()


def test_quadrupole_equals_textbook_form(orc):
    """eps = 0: the expansion equals the traceless quadrupole potential
    phi = -G (M/R + R.Q.R / (2 R^5)), Q = sum m (3 y y^T - |y|^2 I); its field equals minus
    the finite-difference gradient of that potential."""
    rng = np.random.default_rng(2)
    p = rng.normal(size=(25, 3)) * 0.2
    m = rng.uniform(0.5, 1.5, size=25)
    mom = orc.moments(p[:, 0], p[:, 1], p[:, 2], m)
    Rc = mom[1:4]
    y = p - Rc
    Q = (m[:, None, None] * (3 * y[:, :, None] * y[:, None, :] - (y * y).sum(1)[:, None, None] * np.eye(3))).sum(0)

    def phi_tb(pt):
        R = pt - Rc
        r = np.linalg.norm(R)
        return -(mom[0] / r + R @ Q @ R / (2 * r ** 5))

    for pt in [np.array([2.0, 0.5, -1.0]), np.array([-3.0, 1.0, 0.2])]:
        g, phi = orc.quad_field(mom, pt, G=1.0, eps=0.0)
        assert abs(phi - phi_tb(pt)) < 1e-14 * abs(phi)
        d = 1e-5
        fd = np.array([-(phi_tb(pt + d * e) - phi_tb(pt - d * e)) / (2 * d) for e in np.eye(3)])
        assert np.abs(g - fd).max() < 1e-8 * np.linalg.norm(g)


def test_quadrupole_softened_gradient_and_order(orc):
    """eps > 0: the field is minus the gradient of the expansion potential, and the error
    against the direct softened sum falls as the third power of the distance ratio
    (doubling the distance divides the relative error by about 8)."""
    rng = np.random.default_rng(4)
    p = rng.normal(size=(40, 3)) * 0.1
    m = rng.uniform(0.5, 1.5, size=40)
    mom = orc.moments(p[:, 0], p[:, 1], p[:, 2], m)
    eps = 0.05
    pt = np.array([1.0, 0.7, -0.4])
    g, phi = orc.quad_field(mom, pt, G=1.0, eps=eps)
    d = 1e-5
    fd = np.array([-(orc.quad_field(mom, pt + d * e, 1.0, eps)[1] - orc.quad_field(mom, pt - d * e, 1.0, eps)[1])
                   / (2 * d) for e in np.eye(3)])
    assert np.abs(g - fd).max() < 1e-8 * np.linalg.norm(g)
    errs = []
    for s in (2.0, 4.0, 8.0):
        q = mom[1:4] + s * np.array([0.6, 0.64, 0.48])
        allp = np.vstack([p, q])
        gx, gy, gz, _ = orc.gravity_direct(allp[:, 0], allp[:, 1], allp[:, 2], np.append(m, 0.0), 1.0, eps,
                                           targets=np.array([40]))
        gq, _ = orc.quad_field(mom, q, 1.0, eps)
        gd = np.array([gx[0], gy[0], gz[0]])
        errs.append(np.linalg.norm(gq - gd) / np.linalg.norm(gd))
    assert 7.0 < errs[0] / errs[1] < 20.0 and 7.0 < errs[1] / errs[2] < 20.0


def _sorted_tree(orc, ps, leaf_cap, gsize):
    k = orc.keys(ps.x, ps.y, ps.z)
    o = orc.order(k)
    ks = k[o]
    t = orc.octree(ks, leaf_cap)
    L = max(np.ptp(ps.x), np.ptp(ps.y), np.ptp(ps.z))
    gstart = np.arange(0, ps.n, gsize)
    gcount = np.minimum(gsize, ps.n - gstart)
    return o, t, L, gstart, gcount


def test_tree_gravity_theta_zero_is_direct(orc):
    """theta_MAC = 0 reduces the tree sum to the exact direct sum (Sec. 2.2.2)."""
    ps = polytrope_n1(1500, seed=9)
    o, t, L, gs, gc = _sorted_tree(orc, ps, 8, 32)
    xs, ys, zs, ms = ps.x[o], ps.y[o], ps.z[o], ps.m[o]
    gx, gy, gz, phi = orc.tree_gravity(xs, ys, zs, ms, t, L, 0.0, 1.0, 0.01, gs, gc)
    dx, dy, dz, dp = orc.gravity_direct(xs, ys, zs, ms, 1.0, 0.01)
    assert np.abs(gx - dx).max() < 1e-12 * np.abs(dx).max()
    assert np.abs(phi - dp).max() < 1e-12 * np.abs(dp).max()


def test_tree_gravity_theta_half_accuracy(orc):
    """theta = 0.5 with quadrupoles: RMS relative error against the direct sum <= 1e-3, and
    the error falls as theta decreases (Sec. 3.2: approaches N-body as the MAC decreases)."""
    ps = polytrope_n1(8192, seed=10)
    o, t, L, gs, gc = _sorted_tree(orc, ps, 16, 32)
    xs, ys, zs, ms = ps.x[o], ps.y[o], ps.z[o], ps.m[o]
    dx, dy, dz, _ = orc.gravity_direct(xs, ys, zs, ms, 1.0, 0.01)
    gd = np.sqrt(dx ** 2 + dy ** 2 + dz ** 2)
    rms = []
    for th in (0.5, 0.3):
        gx, gy, gz, _ = orc.tree_gravity(xs, ys, zs, ms, t, L, th, 1.0, 0.01, gs, gc)
        e = np.sqrt((gx - dx) ** 2 + (gy - dy) ** 2 + (gz - dz) ** 2) / gd
        rms.append(math.sqrt((e ** 2).mean()))
    assert rms[0] <= 1e-3
    assert rms[1] < rms[0]


# ---------------------------------------------------------------------------- node-node (FMM) gravity
def _fmm_setup(orc, ps, leaf_cap, min_level=0):
    k = orc.keys(ps.x, ps.y, ps.z)
    o = orc.order(k)
    t = orc.octree(k[o], leaf_cap, min_level)
    box = orc.bbox(ps.x, ps.y, ps.z)
    return o, t, box, orc.scale(box, 21)


def test_fmm_theta_zero_is_direct(orc):
    """theta_MAC = 0 accepts no node pair: eq. (10) reduces to the exact particle sum (Sec.
    2.2.2); the mutual recursion must still reach every pair exactly once."""
    ps = polytrope_n1(1500, seed=9)
    o, t, box, S = _fmm_setup(orc, ps, 8)
    xs, ys, zs, ms = ps.x[o], ps.y[o], ps.z[o], ps.m[o]
    r = orc.fmm_gravity(xs, ys, zs, ms, t, box, S, 0.0, 1.3, 0.01)
    dx, dy, dz, dp = orc.gravity_direct(xs, ys, zs, ms, 1.3, 0.01)
    assert np.all(r["cover"] == ps.n - 1)
    d = np.sqrt((r["gx"] - dx) ** 2 + (r["gy"] - dy) ** 2 + (r["gz"] - dz) ** 2)
    assert np.all(d <= 1e-13 * r["sg"])
    assert np.all(np.abs(r["phi"] - dp) <= 1e-13 * r["sp"])


@pytest.mark.parametrize("theta", [0.3, 0.5, 1.0])
def test_fmm_partition_and_conservation(orc, theta):
    """The node-pair recursion partitions all particle pairs (every particle is reached by
    each other one exactly once), and the symmetric node-node terms conserve linear momentum
    and -- at first order, with central forces between centres of mass -- angular momentum
    to rounding (Sec. 2.2.2).  The particle-cell quadrupole walk misses both by ~1e-4."""
    ps = polytrope_n1(6000, seed=31)
    o, t, box, S = _fmm_setup(orc, ps, 12)
    xs, ys, zs, ms = ps.x[o], ps.y[o], ps.z[o], ps.m[o]
    r = orc.fmm_gravity(xs, ys, zs, ms, t, box, S, theta, 1.0, 0.01)
    assert np.all(r["cover"] == ps.n - 1)
    g = np.stack([r["gx"], r["gy"], r["gz"]], axis=1)
    pos = np.stack([xs, ys, zs], axis=1)
    gn = np.linalg.norm(g, axis=1)
    P = (ms[:, None] * g).sum(axis=0)
    Lm = (ms[:, None] * np.cross(pos, g)).sum(axis=0)
    assert np.linalg.norm(P) <= 1e-14 * (ms * gn).sum()
    assert np.linalg.norm(Lm) <= 1e-14 * (ms * np.linalg.norm(pos, axis=1) * gn).sum()


def test_fmm_two_clusters_closed_form(orc):
    """Two compact clusters in opposite corners of the root cell.  With leaf capacity 8 and
    leaves from level 2, the level-2 cells holding the clusters pass the opening test for
    theta > 1/3 (3 T^2 = 48 < 432 theta^2 in half-finest-cell units) but not below.  Above,
    each particle feels its own cluster directly plus Newton's point-mass attraction of the
    other cluster's mass at its centre of mass, evaluated at its own cluster's centre of mass,
    and the first-order potential; below, everything is the direct sum."""
    rng = np.random.default_rng(5)
    a = rng.uniform(0.0, 0.01, size=(8, 3))
    b = rng.uniform(0.99, 1.0, size=(8, 3))
    a[0] = 0.0
    b[0] = 1.0
    p = np.vstack([a, b])
    m = rng.uniform(0.5, 2.0, size=16)
    ps = uniform_random(16, seed=1)
    ps.x, ps.y, ps.z = [np.ascontiguousarray(p[:, i]) for i in range(3)]
    ps.m = m
    o, t, box, S = _fmm_setup(orc, ps, 8, min_level=2)
    assert o[:8].max() < 8 <= o[8:].min()  # cluster A sorts first
    G, eps = 1.7, 0.003
    xs, ys, zs, ms = ps.x[o], ps.y[o], ps.z[o], ps.m[o]
    pos = np.stack([xs, ys, zs], axis=1)
    dx, dy, dz, dp = orc.gravity_direct(xs, ys, zs, ms, G, eps)
    r = orc.fmm_gravity(xs, ys, zs, ms, t, box, S, 0.3, G, eps)
    assert np.allclose(r["gx"], dx, rtol=0, atol=1e-13 * np.abs(dx).max())
    assert np.allclose(r["phi"], dp, rtol=0, atol=1e-13 * np.abs(dp).max())
    r = orc.fmm_gravity(xs, ys, zs, ms, t, box, S, 0.5, G, eps)
    for own, other in ((slice(0, 8), slice(8, 16)), (slice(8, 16), slice(0, 8))):
        jx, jy, jz, jp = orc.gravity_direct(xs[own], ys[own], zs[own], ms[own], G, eps)
        MA, MB = ms[own].sum(), ms[other].sum()
        RA = (ms[own, None] * pos[own]).sum(axis=0) / MA
        RB = (ms[other, None] * pos[other]).sum(axis=0) / MB
        R = RA - RB
        s = math.sqrt(R @ R + eps * eps)
        gfar = -G * MB * R / s ** 3
        want_g = np.stack([jx, jy, jz], axis=1) + gfar
        want_p = jp - G * MB / s - (pos[own] - RA) @ gfar
        got_g = np.stack([r["gx"][own], r["gy"][own], r["gz"][own]], axis=1)
        assert np.abs(got_g - want_g).max() <= 1e-12 * np.abs(want_g).max()
        assert np.abs(r["phi"][own] - want_p).max() <= 1e-12 * np.abs(want_p).max()


def test_fmm_error_orders(orc):
    """First order in the Taylor expansion of the potential: the acceleration (constant
    across a node) errs at first order in the opening angle, the potential (with its linear
    term) at second order.  Halving theta from 1 to 0.5 must shrink the RMS acceleration
    error by 1.6-3x and the potential error by at least 3x (a tidal term in the acceleration
    would make the first ratio ~4, a missing linear potential term the second ~2); at 0.25
    the error keeps falling."""
    ps = polytrope_n1(8192, seed=10)
    o, t, box, S = _fmm_setup(orc, ps, 16)
    xs, ys, zs, ms = ps.x[o], ps.y[o], ps.z[o], ps.m[o]
    dx, dy, dz, dp = orc.gravity_direct(xs, ys, zs, ms, 1.0, 0.01)
    gd = np.sqrt(dx ** 2 + dy ** 2 + dz ** 2)
    eg, ep = [], []
    for th in (1.0, 0.5, 0.25):
        r = orc.fmm_gravity(xs, ys, zs, ms, t, box, S, th, 1.0, 0.01)
        e = np.sqrt((r["gx"] - dx) ** 2 + (r["gy"] - dy) ** 2 + (r["gz"] - dz) ** 2) / gd
        eg.append(math.sqrt((e ** 2).mean()))
        ep.append(math.sqrt((((r["phi"] - dp) / dp) ** 2).mean()))
    assert eg[1] < 0.1
    assert 1.6 < eg[0] / eg[1] < 3.0
    assert ep[0] / ep[1] > 3.0
    assert eg[2] < eg[1] and ep[2] < ep[1]


# ---------------------------------------------------------------------------- integrator
def test_kdk_momentum_and_energy_order(orc):
    """KDK leapfrog: momentum is conserved to rounding; the one-step energy error falls by
    at least 2^3 when dt is halved (local error of third order or better; a wrong half
    kick or a missing predictor makes it first or second order)."""
    ps = lattice_box(8, v_sigma=0.05, jitter=0.2)
    prm = orc.Params(adaptive_h=False)
    st0 = orc.prime(ps.fields(), prm)
    E0 = orc.diagnostics(st0)
    errs = []
    for dt in (0.02, 0.01, 0.005):
        st1 = orc.kdk_step(st0, dt, prm)
        E1 = orc.diagnostics(st1)
        errs.append(abs((E1[6] + E1[7]) - (E0[6] + E0[7])))
        assert np.abs(E1[:3] - E0[:3]).max() < 1e-15
    assert 7.0 < errs[0] / errs[1] < 20.0 and 7.0 < errs[1] / errs[2] < 20.0


# ---------------------------------------------------------------------------- diagnostics, time step
def test_diagnostics_rigid_rotation_closed_form(orc):
    """Rigid rotation v = w z_hat x r of a cell-centred n^3 lattice with spacing dx and equal
    masses m: L_z = w m sum (x^2 + y^2) = w m 2 n^2 dx^2 (n^3/3 - n/12) (the 1D sum of
    ((i + 1/2) dx)^2), L_x = L_y = 0, P = 0 about the lattice centre, E_kin = w L_z / 2."""
    n, dx, w, m = 10, 0.1, 0.7, 0.3
    c = (np.arange(n) + 0.5) * dx - 0.5 * n * dx   # centred on the origin
    X, Y, Z = (a.ravel() for a in np.meshgrid(c, c, c, indexing="ij"))
    st = dict(x=X, y=Y, z=Z, vx=-w * Y, vy=w * X, vz=np.zeros_like(X), m=np.full(X.size, m), u=np.ones(X.size))
    d = orc.diagnostics(st)
    s1 = dx * dx * (n ** 3 / 12.0 - n / 12.0)         # sum_i (i + 1/2 - n/2)^2 dx^2
    Lz = w * m * 2 * n * n * s1
    assert np.allclose(d[:3], 0.0, atol=1e-13)
    assert np.allclose(d[3:5], 0.0, atol=1e-13)
    assert abs(d[5] - Lz) <= 1e-13 * Lz
    assert abs(d[6] - 0.5 * w * Lz) <= 1e-13 * Lz
    assert d[7] == pytest.approx(m * X.size, rel=1e-15)
    # L about a shifted origin picks up r0 x P = 0 (P = 0), so it is unchanged
    st2 = dict(st, x=X + 3.0, vx=st["vx"], vy=st["vy"])
    st2["vx"] = -w * Y
    st2["vy"] = w * X
    assert abs(orc.diagnostics(st2)[5] - Lz) <= 1e-12 * Lz


def test_diagnostics_two_body_potential_energy(orc):
    """E_grav = sum m phi / 2 of two softened point masses is -G m1 m2 / sqrt(r^2 + eps^2)."""
    G, eps, m1, m2, r = 1.3, 0.05, 0.4, 0.9, 0.37
    x, y, z = np.array([0.1, 0.1 + r]), np.zeros(2), np.zeros(2)
    m = np.array([m1, m2])
    _, _, _, phi = orc.gravity_direct(x, y, z, m, G, eps)
    st = dict(x=x, y=y, z=z, vx=np.zeros(2), vy=np.zeros(2), vz=np.zeros(2), m=m, u=np.zeros(2))
    eg = orc.diagnostics(st, phi)[8]
    assert eg == pytest.approx(-G * m1 * m2 / math.sqrt(r * r + eps * eps), rel=1e-15)


def test_gravity_absolute_sum_scale(orc):
    """The direct sum's absolute-sum scale: for two bodies it is |g|; for a body midway between
    two equal masses the pulls cancel (g = 0) while the scale is twice one pull."""
    G, eps = 1.0, 0.01
    x, y, z = np.array([0.0, 0.5]), np.zeros(2), np.zeros(2)
    m = np.array([1.0, 2.0])
    gx, gy, gz, phi, sg = orc.gravity_direct(x, y, z, m, G, eps, scale=True)
    assert np.allclose(sg, np.abs(gx), rtol=1e-15)
    x3 = np.array([-1.0, 0.0, 1.0])
    gx, _, _, _, sg = orc.gravity_direct(x3, np.zeros(3), np.zeros(3), np.ones(3), G, eps, scale=True)
    one = G * 1.0 / (1.0 + eps * eps) ** 1.5
    assert abs(gx[1]) <= 1e-16 and sg[1] == pytest.approx(2 * one, rel=1e-14)


def test_dt_bound_closed_forms(orc):
    """Time-step bound min(h/c, sqrt(eps/|a|)): the sound speed c = sqrt(gamma (gamma - 1) u)
    does not depend on rho, so a jittered lattice with one h and one u gives exactly
    h / sqrt(gamma (gamma - 1) u) (10/9 for u = 1); two sets with their own u give one value
    each; with gravity, two distant bodies (no hydro neighbours) are limited by the
    free-fall term sqrt(eps / |a|) with |a| = G m r / (r^2 + eps^2)^(3/2)."""
    prm = orc.Params()
    ps = lattice_box(8, seed=5)
    st = orc.prime(ps.fields(), prm)
    assert orc.dt_bound(st)[0] == pytest.approx(ps.h[0] / math.sqrt(10.0 / 9.0), rel=1e-14)
    # two sets: the second one hotter (u = 4 -> c doubles, bound halves)
    a, b = lattice_box(6, seed=6), lattice_box(6, seed=7)
    xs = {k: np.concatenate([getattr(a, k), getattr(b, k) + (5.0 if k == "x" else 0.0)])
          for k in ("x", "y", "z", "vx", "vy", "vz", "m", "h", "u")}
    xs["u"][a.n:] = 4.0
    so = [0, a.n, a.n + b.n]
    st2 = orc.prime(xs, prm, seg=orc.seg_ids(a.n + b.n, so))
    bd = orc.dt_bound(st2, seg_offsets=so)
    assert bd[0] == pytest.approx(a.h[0] / math.sqrt(10.0 / 9.0), rel=1e-14)
    assert bd[1] == pytest.approx(b.h[0] / math.sqrt(40.0 / 9.0), rel=1e-14)
    # gravity: two bodies 0.5 apart, h = 0.2 (no hydro pairs: r > h_a + h_b), softening 0.01
    G, eps, r = 1.0, 0.01, 0.5
    two = dict(x=np.array([0.0, r]), y=np.zeros(2), z=np.zeros(2), vx=np.zeros(2), vy=np.zeros(2), vz=np.zeros(2),
               m=np.array([0.5, 0.5]), h=np.full(2, 0.2), u=np.full(2, 1.0))
    st3 = orc.prime(two, orc.Params(G=G, soft_eps=eps))
    acc = G * 0.5 * r / (r * r + eps * eps) ** 1.5
    assert orc.dt_bound(st3, eps)[0] == pytest.approx(math.sqrt(eps / acc), rel=1e-14)
    assert math.sqrt(eps / acc) < 0.2 / math.sqrt(10.0 / 9.0)   # the gravity term decides
    assert orc.dt_bound(st3, 0.0)[0] == pytest.approx(0.2 / math.sqrt(10.0 / 9.0), rel=1e-14)


def test_kdk_per_set_step_sizes(orc):
    """Independent sets stepped with their own dt (one value per particle) evolve exactly as
    each set stepped alone with its scalar dt."""
    prm = orc.Params()
    a, b = lattice_box(6, seed=8, v_sigma=0.1), lattice_box(5, seed=9, v_sigma=0.1)
    fa, fb = a.fields(), b.fields()
    both = {k: np.concatenate([fa[k], fb[k]]) for k in fa}   # overlapping, but separate sets
    so = [0, a.n, a.n + b.n]
    seg = orc.seg_ids(a.n + b.n, so)
    st = orc.prime(both, prm, seg=seg)
    dts = np.concatenate([np.full(a.n, 0.01), np.full(b.n, 0.004)])
    s2 = orc.kdk_step(st, dts, prm, seg=seg)
    ra = orc.kdk_step(orc.prime(fa, prm), 0.01, prm)
    rb = orc.kdk_step(orc.prime(fb, prm), 0.004, prm)
    for k in ("x", "vx", "u", "h", "ax", "dudt"):
        assert np.array_equal(s2[k][:a.n], ra[k]), k
        assert np.array_equal(s2[k][a.n:], rb[k]), k


def test_tree_gravity_counts_closed_form(orc):
    """Counted terms: at theta = 0 no cell is accepted and every ordered pair is summed once
    (n (n - 1), the direct sum); at theta = 0.5 accepted cells replace part of the pairs."""
    ps = polytrope_n1(3000, seed=11)
    o, t, L, gs, gc = _sorted_tree(orc, ps, 8, 32)
    xs, ys, zs, ms = ps.x[o], ps.y[o], ps.z[o], ps.m[o]
    *_, (nc, npair) = orc.tree_gravity(xs, ys, zs, ms, t, L, 0.0, 1.0, 0.01, gs, gc, counts=True)
    assert nc == 0 and npair == ps.n * (ps.n - 1)
    *_, (nc, npair) = orc.tree_gravity(xs, ys, zs, ms, t, L, 0.5, 1.0, 0.01, gs, gc, counts=True)
    assert nc > 0 and 0 < npair < ps.n * (ps.n - 1)
