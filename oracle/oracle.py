"""Python side of the CPU FP64 reference (TEST INFRASTRUCTURE ONLY).

Thin numpy wrappers around ``oracle.c`` plus the leapfrog step, written in the order the
method takes its steps.  Brute-force O(N^2) neighbours; use ``targets`` to sample large
sets.  Every array is float64 (or int64 for indices) in caller order unless stated.

Parity pins: tests/test_oracle_pins.py.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_d = ctypes.POINTER(ctypes.c_double)
_i64 = ctypes.POINTER(ctypes.c_int64)
_i32 = ctypes.POINTER(ctypes.c_int32)
_u64 = ctypes.POINTER(ctypes.c_uint64)
I64, I32, DBL = ctypes.c_int64, ctypes.c_int32, ctypes.c_double


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc (no FMA contraction, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-shared", "-fPIC",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = ctypes.CDLL(_LIB)
        L.orc_keys.argtypes = [I64, _d, _d, _d, I32, _i64, _d, _u64]
        L.orc_keys_hilbert.argtypes = [I64, _d, _d, _d, I32, _i64, _d, _u64]
        L.orc_hilbert.argtypes = [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_int]
        L.orc_hilbert.restype = ctypes.c_uint64
        L.orc_order.argtypes = [I64, _u64, _i64]
        L.orc_octree.argtypes = [I64, _u64, ctypes.c_int, ctypes.c_int, I64, _u64, _i32, _i32, _i64, _i64]
        L.orc_octree.restype = I64
        L.orc_nbr_count.argtypes = [I64, _d, _d, _d, _d, _i32, I64, _i64, _i64]
        L.orc_nbr_fill.argtypes = [I64, _d, _d, _d, _d, _i32, I64, _i64, _i64, _i64]
        L.orc_w.argtypes = [DBL]
        L.orc_w.restype = DBL
        L.orc_dw_over_q.argtypes = [DBL]
        L.orc_dw_over_q.restype = DBL
        L.orc_density.argtypes = [_d, _d, _d, _d, _d, _d, DBL, DBL, I64, _i64, _i64, _i64, _d, _d, _d, _d]
        L.orc_forces.argtypes = [_d] * 11 + [DBL, DBL, DBL, I64, _i64, _i64, _i64] + [_d] * 6
        L.orc_dedt.argtypes = [_d] * 11 + [DBL, DBL, DBL, I64, _i64, _i64, _i64] + [_d] * 2
        L.orc_gravity_direct.argtypes = [I64, _d, _d, _d, _d, DBL, DBL, I64, _i64, _d, _d, _d, _d, _d]
        L.orc_moments.argtypes = [I64, I64, _i64, _d, _d, _d, _d, _d]
        L.orc_quad_field.argtypes = [_d, DBL, DBL, DBL, DBL, DBL, _d, _d]
        L.orc_tree_gravity.argtypes = ([I64, I64, _i32, _i32, _i64, _i64, _d, _d, _d, _d, DBL, DBL, DBL, DBL,
                                        I64, _i64, _i64, _d, _d, _d, _d, _i64])
        L.orc_fmm_gravity.argtypes = ([I64, I64, _i32, _i32, _i64, _i64, _d, _d, _d, _d, _d, DBL, ctypes.c_int, DBL,
                                       DBL, DBL, _d, _d, _d, _d, _d, _d, _i64])
        L.orc_fmm_gravity.restype = ctypes.c_int
        L.orc_bbox.argtypes = [I64, I64, _d, _d, _d, _d]
        L.orc_scale.argtypes = [_d, ctypes.c_int]
        L.orc_scale.restype = DBL
        _lib = L
    return _lib


def _p(a, t=_d):
    return None if a is None else a.ctypes.data_as(t)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ii(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.int64)


# ---------------------------------------------------------------------------------------
# Keys, order, tree (Sec. 2.1 "Tree topology", Fig. 1)

def keys(x, y, z, seg_offsets=None, box=None, curve="morton"):
    """Sentinel-prefixed keys of the quantised positions: the Morton bit interleave
    (Fig. 1), or the Hilbert index (curve="hilbert")."""
    x, y, z = _f64(x), _f64(y), _f64(z)
    n = x.size
    out = np.empty(n, dtype=np.uint64)
    nseg = 1 if seg_offsets is None else len(seg_offsets) - 1
    so = _ii(seg_offsets)
    bx = None if box is None else _f64(box)
    fn = lib().orc_keys_hilbert if curve == "hilbert" else lib().orc_keys
    fn(n, _p(x), _p(y), _p(z), nseg, _p(so, _i64), _p(bx), _p(out, _u64))
    return out


def hilbert(kx, ky, kz, bits):
    """Hilbert index of one grid cell (for pins)."""
    return int(lib().orc_hilbert(int(kx), int(ky), int(kz), int(bits)))


def order(k):
    k = np.ascontiguousarray(k, dtype=np.uint64)
    out = np.empty(k.size, dtype=np.int64)
    lib().orc_order(k.size, _p(k, _u64), _p(out, _i64))
    return out


def octree(sorted_keys, leaf_cap, min_level=0):
    """Pre-order node list: dict of arrays key, level, leaf, start, count."""
    k = np.ascontiguousarray(sorted_keys, dtype=np.uint64)
    n = k.size
    cap = max(64, 2 * n + 22 * (n // max(1, leaf_cap + 1) + 1) + 64)
    nkey = np.empty(cap, np.uint64)
    nlev = np.empty(cap, np.int32)
    nleaf = np.empty(cap, np.int32)
    nst = np.empty(cap, np.int64)
    ncnt = np.empty(cap, np.int64)
    m = lib().orc_octree(n, _p(k, _u64), int(leaf_cap), int(min_level), cap, _p(nkey, _u64), _p(nlev, _i32),
                         _p(nleaf, _i32), _p(nst, _i64), _p(ncnt, _i64))
    if m < 0:
        raise RuntimeError("octree capacity exceeded")
    return dict(key=nkey[:m], level=nlev[:m], leaf=nleaf[:m].astype(bool), start=nst[:m], count=ncnt[:m])


def bbox(x, y, z):
    out = np.empty(6)
    x, y, z = _f64(x), _f64(y), _f64(z)
    lib().orc_bbox(0, x.size, _p(x), _p(y), _p(z), _p(out))
    return out


def scale(box6, bits):
    b = _f64(box6)
    return lib().orc_scale(_p(b), int(bits))


# ---------------------------------------------------------------------------------------
# Neighbours: brute force, lists sorted by caller index, self included

def seg_ids(n, seg_offsets):
    if seg_offsets is None or len(seg_offsets) <= 2:
        return None
    s = np.empty(n, np.int32)
    for i in range(len(seg_offsets) - 1):
        s[seg_offsets[i]:seg_offsets[i + 1]] = i
    return s


def neighbors(x, y, z, h, targets=None, seg=None):
    """CSR (offsets int64[ntgt+1], idx int64[nnz]) of the neighbour sets of the targets."""
    x, y, z, h = _f64(x), _f64(y), _f64(z), _f64(h)
    n = x.size
    tg = _ii(targets)
    nt = n if tg is None else tg.size
    sg = None if seg is None else np.ascontiguousarray(seg, dtype=np.int32)
    cnt = np.empty(nt, np.int64)
    lib().orc_nbr_count(n, _p(x), _p(y), _p(z), _p(h), _p(sg, _i32), nt, _p(tg, _i64), _p(cnt, _i64))
    off = np.zeros(nt + 1, np.int64)
    np.cumsum(cnt, out=off[1:])
    idx = np.empty(int(off[-1]), np.int64)
    lib().orc_nbr_fill(n, _p(x), _p(y), _p(z), _p(h), _p(sg, _i32), nt, _p(tg, _i64), _p(off, _i64),
                       _p(idx, _i64))
    return off, idx


# ---------------------------------------------------------------------------------------
# Density + EOS (eq. (7), (9)); forces (eq. (5), (6)); gravity (eq. (10))

def w(q):
    return lib().orc_w(float(q))


def dw_over_q(q):
    return lib().orc_dw_over_q(float(q))


def density(ps_or_arrays, csr, gamma=5.0 / 3.0, h_coeff=1.2, targets=None):
    """Returns rho, P, c, h_next indexed by target."""
    x, y, z, h, m, u = (_f64(ps_or_arrays[k]) for k in ("x", "y", "z", "h", "m", "u"))
    off, idx = csr
    tg = _ii(targets)
    nt = x.size if tg is None else tg.size
    rho, P, c, hn = (np.empty(nt) for _ in range(4))
    lib().orc_density(_p(x), _p(y), _p(z), _p(h), _p(m), _p(u), gamma, h_coeff, nt, _p(tg, _i64),
                      _p(_ii(off), _i64), _p(_ii(idx), _i64), _p(rho), _p(P), _p(c), _p(hn))
    return rho, P, c, hn


def forces(ps_or_arrays, rho, P, c, csr, alpha=1.0, beta=2.0, eps_av=0.01, targets=None, vel=None):
    """Returns ax, ay, az, dudt, Sa, Su indexed by target.  rho, P, c indexed by particle.
    vel: optional (vx, vy, vz) overriding the state's velocities (the KDK predictor)."""
    x, y, z, h, m = (_f64(ps_or_arrays[k]) for k in ("x", "y", "z", "h", "m"))
    vx, vy, vz = (_f64(v) for v in (vel if vel is not None else
                                     (ps_or_arrays["vx"], ps_or_arrays["vy"], ps_or_arrays["vz"])))
    rho, P, c = _f64(rho), _f64(P), _f64(c)
    off, idx = csr
    tg = _ii(targets)
    nt = x.size if tg is None else tg.size
    out = [np.empty(nt) for _ in range(6)]
    lib().orc_forces(_p(x), _p(y), _p(z), _p(vx), _p(vy), _p(vz), _p(h), _p(m), _p(rho), _p(P), _p(c),
                     alpha, beta, eps_av, nt, _p(tg, _i64), _p(_ii(off), _i64), _p(_ii(idx), _i64),
                     *[_p(o) for o in out])
    return tuple(out)


def dedt(ps_or_arrays, rho, P, c, csr, alpha=1.0, beta=2.0, eps_av=0.01, targets=None, vel=None):
    """Eq. (8), thermokinetic energy rate: returns dedt, Se indexed by target.  rho, P, c
    indexed by particle; vel: optional (vx, vy, vz) overriding the state's velocities."""
    x, y, z, h, m = (_f64(ps_or_arrays[k]) for k in ("x", "y", "z", "h", "m"))
    vx, vy, vz = (_f64(v) for v in (vel if vel is not None else
                                     (ps_or_arrays["vx"], ps_or_arrays["vy"], ps_or_arrays["vz"])))
    rho, P, c = _f64(rho), _f64(P), _f64(c)
    off, idx = csr
    tg = _ii(targets)
    nt = x.size if tg is None else tg.size
    de, se = np.empty(nt), np.empty(nt)
    lib().orc_dedt(_p(x), _p(y), _p(z), _p(vx), _p(vy), _p(vz), _p(h), _p(m), _p(rho), _p(P), _p(c),
                   alpha, beta, eps_av, nt, _p(tg, _i64), _p(_ii(off), _i64), _p(_ii(idx), _i64), _p(de), _p(se))
    return de, se


def gravity_direct(x, y, z, m, G=1.0, eps=0.0, targets=None, scale=False):
    """Direct softened sums (eq. (10) with every cell opened): gx, gy, gz, phi, and with
    scale=True also the absolute-sum scale |G| sum_b m_b |r_ab| / s_ab^3 of each target."""
    x, y, z, m = _f64(x), _f64(y), _f64(z), _f64(m)
    tg = _ii(targets)
    nt = x.size if tg is None else tg.size
    gx, gy, gz, phi = (np.empty(nt) for _ in range(4))
    sg = np.empty(nt) if scale else None
    lib().orc_gravity_direct(x.size, _p(x), _p(y), _p(z), _p(m), G, eps, nt, _p(tg, _i64), _p(gx), _p(gy),
                             _p(gz), _p(phi), _p(sg))
    return (gx, gy, gz, phi, sg) if scale else (gx, gy, gz, phi)


def moments(x, y, z, m, idx=None):
    x, y, z, m = _f64(x), _f64(y), _f64(z), _f64(m)
    out = np.empty(10)
    ii = _ii(idx)
    k = x.size if ii is None else ii.size
    lib().orc_moments(0, k, _p(ii, _i64), _p(x), _p(y), _p(z), _p(m), _p(out))
    return out


def quad_field(mom10, p, G=1.0, eps=0.0):
    mo = _f64(mom10)
    g = np.empty(3)
    phi = np.empty(1)
    lib().orc_quad_field(_p(mo), float(p[0]), float(p[1]), float(p[2]), G, eps, _p(g), _p(phi))
    return g, float(phi[0])


def tree_gravity(xs, ys, zs, ms, tree, L, theta, G, eps, gstart, gcount, counts=False):
    """Tree gravity over particles already in sorted order; tree from octree().  counts=True
    also returns (cell terms, particle-particle terms) evaluated."""
    xs, ys, zs, ms = _f64(xs), _f64(ys), _f64(zs), _f64(ms)
    n = xs.size
    lev = np.ascontiguousarray(tree["level"], np.int32)
    leaf = np.ascontiguousarray(tree["leaf"], np.int32)
    st, ct = _ii(tree["start"]), _ii(tree["count"])
    gs, gc = _ii(gstart), _ii(gcount)
    gx, gy, gz, phi = (np.empty(n) for _ in range(4))
    cnt = np.zeros(2, np.int64)
    lib().orc_tree_gravity(n, lev.size, _p(lev, _i32), _p(leaf, _i32), _p(st, _i64), _p(ct, _i64), _p(xs), _p(ys),
                           _p(zs), _p(ms), L, theta, G, eps, gs.size, _p(gs, _i64), _p(gc, _i64), _p(gx), _p(gy),
                           _p(gz), _p(phi), _p(cnt, _i64))
    if counts:
        return gx, gy, gz, phi, (int(cnt[0]), int(cnt[1]))
    return gx, gy, gz, phi


def fmm_gravity(xs, ys, zs, ms, tree, lo, S, theta, G, eps, bits=21):
    """Symmetric node-node gravity (Sec. 2.2.2, eq. (10)) over particles already in key order;
    tree from octree(), lo/S the key quantisation.  Returns dict of g (x, y, z), phi, the
    absolute-sum scales sg, sp and cover (other particles reached, n - 1 when every pair is
    accounted for exactly once)."""
    xs, ys, zs, ms = _f64(xs), _f64(ys), _f64(zs), _f64(ms)
    n = xs.size
    lev = np.ascontiguousarray(tree["level"], np.int32)
    leaf = np.ascontiguousarray(tree["leaf"], np.int32)
    st, ct = _ii(tree["start"]), _ii(tree["count"])
    lo3 = _f64(np.asarray(lo, dtype=np.float64)[:3])
    out = {k: np.empty(n) for k in ("gx", "gy", "gz", "phi", "sg", "sp")}
    cover = np.empty(n, np.int64)
    r = lib().orc_fmm_gravity(n, lev.size, _p(lev, _i32), _p(leaf, _i32), _p(st, _i64), _p(ct, _i64), _p(xs), _p(ys),
                              _p(zs), _p(ms), _p(lo3), float(S), int(bits), float(theta), float(G), float(eps),
                              _p(out["gx"]), _p(out["gy"]), _p(out["gz"]), _p(out["phi"]), _p(out["sg"]),
                              _p(out["sp"]), _p(cover, _i64))
    if r != 0:
        raise RuntimeError("fmm_gravity: malformed tree")
    out["cover"] = cover
    return out


# ---------------------------------------------------------------------------------------
# Leapfrog (kick-drift-kick) with velocity and energy predictors, lagged adaptive h

class Params:
    """thermokinetic: evolve e = u + v^2/2 with eq. (8) instead of u with eq. (5); the state
    keeps the thermal u, and its "dudt" entry holds de/dt."""

    def __init__(self, gamma=5.0 / 3.0, alpha=1.0, beta=2.0, eps_av=0.01, h_coeff=1.2, adaptive_h=False,
                 G=0.0, soft_eps=0.0, thermokinetic=False):
        self.gamma, self.alpha, self.beta, self.eps_av = gamma, alpha, beta, eps_av
        self.h_coeff, self.adaptive_h, self.G, self.soft_eps = h_coeff, adaptive_h, G, soft_eps
        self.thermokinetic = thermokinetic


def accelerations(st: dict, prm: Params, vel=None, u=None, seg=None):
    """Hydro (+ direct gravity) accelerations for the whole set, as a dict: ax, ay, az, dudt,
    rho, P, c, h_next, and the absolute-sum scales Sa (of the acceleration) and Su (of dudt):
    each the sum of its terms' magnitudes, gravity's included.  u overrides the state's thermal
    energy in the EOS.  Thermokinetic: dudt is de/dt of eq. (8), plus v . g with gravity (the
    work of gravity on e = u + v^2/2)."""
    csr = neighbors(st["x"], st["y"], st["z"], st["h"], seg=seg)
    d = dict(st)
    if u is not None:
        d["u"] = u
    rho, P, c, hn = density(d, csr, prm.gamma, prm.h_coeff)
    ax, ay, az, du, Sa, Su = forces(d, rho, P, c, csr, prm.alpha, prm.beta, prm.eps_av, vel=vel)
    if prm.thermokinetic:
        du, Su = dedt(d, rho, P, c, csr, prm.alpha, prm.beta, prm.eps_av, vel=vel)
    if prm.G != 0.0:
        gx, gy, gz, _, sg = gravity_direct(st["x"], st["y"], st["z"], st["m"], prm.G, prm.soft_eps, scale=True)
        ax, ay, az = ax + gx, ay + gy, az + gz
        Sa = Sa + sg
        if prm.thermokinetic:
            v = vel if vel is not None else (st["vx"], st["vy"], st["vz"])
            du = du + (v[0] * gx + v[1] * gy + v[2] * gz)
            Su = Su + np.sqrt(v[0] ** 2 + v[1] ** 2 + v[2] ** 2) * sg
    return dict(ax=ax, ay=ay, az=az, dudt=du, rho=rho, P=P, c=c, h_next=hn, Sa=Sa, Su=Su)


def prime(st: dict, prm: Params, seg=None):
    """Accelerations at t = 0 and, for adaptive h, h <- h_coeff (m / rho)^(1/3).  The result
    also carries rho, cs (the sound speed) and the scales Sa, Su of that pass."""
    st = {k: np.array(v, dtype=np.float64) for k, v in st.items()}
    r = accelerations(st, prm, seg=seg)
    st.update(ax=r["ax"], ay=r["ay"], az=r["az"], dudt=r["dudt"], rho=r["rho"], cs=r["c"], Sa=r["Sa"], Su=r["Su"])
    if prm.adaptive_h:
        st["h"] = r["h_next"]
    return st


def kdk_step(st: dict, dt, prm: Params, seg=None):
    """One step from a primed state (dict with x..u, ax, ay, az, dudt).  dt is a number, or an
    array of one step size per particle (independent sets stepping by their own dt).  The
    result also carries rho, cs and the scales Sa, Su of the step's force pass."""
    if prm.thermokinetic:
        return _kdk_step_thermokinetic(st, dt, prm, seg)
    s = {k: np.array(v, dtype=np.float64) for k, v in st.items()}
    half = 0.5 * dt
    vhx, vhy, vhz = s["vx"] + half * s["ax"], s["vy"] + half * s["ay"], s["vz"] + half * s["az"]
    uh = s["u"] + half * s["dudt"]
    s["x"], s["y"], s["z"] = s["x"] + dt * vhx, s["y"] + dt * vhy, s["z"] + dt * vhz
    vpx, vpy, vpz = vhx + half * s["ax"], vhy + half * s["ay"], vhz + half * s["az"]
    up = uh + half * s["dudt"]
    r = accelerations(s, prm, vel=(vpx, vpy, vpz), u=up, seg=seg)
    s["vx"], s["vy"], s["vz"] = vhx + half * r["ax"], vhy + half * r["ay"], vhz + half * r["az"]
    s["u"] = uh + half * r["dudt"]
    s.update(ax=r["ax"], ay=r["ay"], az=r["az"], dudt=r["dudt"], rho=r["rho"], cs=r["c"], Sa=r["Sa"], Su=r["Su"])
    if prm.adaptive_h:
        s["h"] = r["h_next"]
    return s


def _kdk_step_thermokinetic(st: dict, dt, prm: Params, seg=None):
    """The same kick-drift-kick with the total energy e = u + v^2/2 in place of u:
    e' = e + dt/2 de; predictor e^ = e' + dt/2 de and u^ = e^ - |v^|^2/2 for the EOS;
    e = e' + dt/2 de_new; the returned state holds u = e - |v|^2/2."""
    s = {k: np.array(v, dtype=np.float64) for k, v in st.items()}
    half = 0.5 * dt
    e = s["u"] + 0.5 * (s["vx"] ** 2 + s["vy"] ** 2 + s["vz"] ** 2)
    vhx, vhy, vhz = s["vx"] + half * s["ax"], s["vy"] + half * s["ay"], s["vz"] + half * s["az"]
    eh = e + half * s["dudt"]
    s["x"], s["y"], s["z"] = s["x"] + dt * vhx, s["y"] + dt * vhy, s["z"] + dt * vhz
    vpx, vpy, vpz = vhx + half * s["ax"], vhy + half * s["ay"], vhz + half * s["az"]
    ep = eh + half * s["dudt"]
    up = ep - 0.5 * (vpx ** 2 + vpy ** 2 + vpz ** 2)
    r = accelerations(s, prm, vel=(vpx, vpy, vpz), u=up, seg=seg)
    s["vx"], s["vy"], s["vz"] = vhx + half * r["ax"], vhy + half * r["ay"], vhz + half * r["az"]
    e = eh + half * r["dudt"]
    s["u"] = e - 0.5 * (s["vx"] ** 2 + s["vy"] ** 2 + s["vz"] ** 2)
    s.update(ax=r["ax"], ay=r["ay"], az=r["az"], dudt=r["dudt"], rho=r["rho"], cs=r["c"], Sa=r["Sa"], Su=r["Su"])
    if prm.adaptive_h:
        s["h"] = r["h_next"]
    return s


def dt_bound(st: dict, eps=0.0, seg_offsets=None):
    """Time-step bound of a state that carries h, cs and the accelerations: per set, the
    minimum over its particles of min(h/c, sqrt(eps/|a|)); the second term only for eps > 0
    and |a| > 0.  One value per set (seg_offsets), or one for the whole state."""
    b = st["h"] / st["cs"]
    if eps > 0.0:
        a = np.sqrt(st["ax"] ** 2 + st["ay"] ** 2 + st["az"] ** 2)
        with np.errstate(divide="ignore"):
            g = np.where(a > 0.0, np.sqrt(eps / np.where(a > 0.0, a, 1.0)), np.inf)
        b = np.minimum(b, g)
    so = [0, b.size] if seg_offsets is None else list(seg_offsets)
    return np.array([b[so[i]:so[i + 1]].min() if so[i + 1] > so[i] else np.inf for i in range(len(so) - 1)])


def diagnostics(st: dict, phi=None):
    """[Px, Py, Pz, Lx, Ly, Lz, Ekin, Eth, Egrav] summed over all particles."""
    m = st["m"]
    v = np.stack([st["vx"], st["vy"], st["vz"]])
    r = np.stack([st["x"], st["y"], st["z"]])
    P = (m * v).sum(axis=1)
    L = (m * np.cross(r.T, v.T).T).sum(axis=1)
    ek = 0.5 * (m * (v * v).sum(axis=0)).sum()
    eth = (m * st["u"]).sum()
    eg = 0.0 if phi is None else 0.5 * (m * phi).sum()
    return np.array([*P, *L, ek, eth, eg])
