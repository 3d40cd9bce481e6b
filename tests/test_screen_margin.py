"""The neighbour kernel's FP32 screen, emulated on the CPU: whenever the screen decides a pair
(|d'| > M), its decision equals the FP64 predicate fl(fl(fl(dx dx) + fl(dy dy)) + fl(dz dz)) <
fl(t t).  Screen: offsets from the group origin o formed in FP64 and rounded to FP32,
r2' = fma(dx', dx', fma(dy', dy', dz' dz')), t' = fl(h_a' + h_b'), d' = fma(t', t', -r2'),
M = fma(t2', 2^-19, me) with t2' = fl(t'^2), me = 2^-21 E^2 + 2^-100 rounded up, E the largest
per-axis offset of a target from o.  The kernel decides with the tile margin M' = fma(fl(fl(|h_a'| + hm)^2), 2^-19, me),
hm the largest |h'| of the tile's 64 sources, which is at least M for each of the tile's pairs.
The fused operations are emulated by one FP64 evaluation rounded to FP32 (the FP32 product is
exact in FP64)."""
import numpy as np

f32 = np.float32


def _fma32(a, b, c):
    return (a.astype(np.float64) * b.astype(np.float64) + c.astype(np.float64)).astype(f32)


def _screen(ta, sb, ha, hb, o, E, tile=0):
    """tile > 0: margins from the largest |h| of each run of `tile` consecutive sources."""
    a = (ta - o).astype(f32)
    b = (sb - o).astype(f32)
    d = (a - b).astype(f32)
    r2 = _fma32(d[:, 0], d[:, 0], _fma32(d[:, 1], d[:, 1], (d[:, 2] * d[:, 2]).astype(f32)))
    tt = (ha.astype(f32) + hb.astype(f32)).astype(f32)
    t2 = (tt * tt).astype(f32)
    me = f32((np.ldexp(E * E, -21) + 2.0 ** -100) * (1 + 2.0 ** -20))
    M = _fma32(t2, np.full_like(t2, f32(2.0 ** -19)), np.full_like(t2, me))
    if tile:
        hbf = np.abs(hb.astype(f32))
        pad = (-len(hbf)) % tile
        hm = np.repeat(np.concatenate([hbf, np.zeros(pad, f32)]).reshape(-1, tile).max(1), tile)[:len(hbf)]
        tx = (np.abs(ha.astype(f32)) + hm).astype(f32)
        Mt = _fma32((tx * tx).astype(f32), np.full_like(t2, f32(2.0 ** -19)), np.full_like(t2, me))
        assert np.all(Mt >= M)  # the tile margin bounds every pair's own margin
        M = Mt
    dd = _fma32(tt, tt, -r2)
    hit = dd > M
    undecided = ~(np.abs(dd) > M)
    return hit, undecided


def _exact(ta, sb, ha, hb):
    d = ta - sb
    r2 = d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]
    r2 = r2 + d[:, 2] * d[:, 2]
    t = ha + hb
    return r2 < t * t


def test_screen_never_contradicts_fp64():
    rng = np.random.default_rng(5)
    checked = undecided_total = 0
    for scale, origin in ((1e-3, 0.3), (1.0, 10.0), (1e-6, 1.0), (1e5, -3e5), (3e-2, 0.0)):
        n = 200_000
        o = origin + rng.uniform(-1, 1, size=3) * scale
        E = scale * rng.uniform(0.1, 4.0)
        ta = o + rng.uniform(-E, E, size=(n, 3))
        ta[0] = o
        dirn = rng.normal(size=(n, 3))
        dirn /= np.linalg.norm(dirn, axis=1, keepdims=True)
        r = E * 10.0 ** rng.uniform(-1, 0.5, size=n)  # supports comparable to the group extent
        sb = ta + dirn * r[:, None]
        dist = np.sqrt(((ta - sb) ** 2).sum(1))
        # supports at, a few ulps around, and log-uniformly away from the separation
        rel = np.where(rng.random(n) < 0.25, rng.integers(-8, 9, size=n) * 2.0 ** -52,
                       np.sign(rng.normal(size=n)) * 10.0 ** rng.uniform(-16, -2, size=n))
        ha = 0.5 * dist * (1 + rel) * rng.uniform(0.7, 1.0, size=n)
        hb = dist * (1 + rel) - ha
        Eo = np.max(np.abs(ta - o))
        hit, und = _screen(ta, sb, ha, hb, o, Eo)
        ex = _exact(ta, sb, ha, hb)
        assert np.array_equal(hit[~und], ex[~und])
        checked += int((~und).sum())
        undecided_total += int(und.sum())
    assert checked > 150_000 and undecided_total > 100_000  # both paths exercised


def test_screen_decides_ordinary_pairs():
    """On a lattice-like neighbourhood away from exact ties almost every pair is decided."""
    rng = np.random.default_rng(6)
    s = 1.0 / 56
    o = np.array([0.2, 0.05, 0.05])
    ta = o + rng.uniform(0, 4 * s, size=(100_000, 3))
    sb = ta + rng.uniform(-4 * s, 4 * s, size=(100_000, 3))
    h = np.full(100_000, 1.2 * s)
    hit, und = _screen(ta, sb, h, h, o, 4 * s)
    assert und.mean() < 1e-3
    assert np.array_equal(hit[~und], _exact(ta, sb, h, h)[~und])


def test_tile_margin_keeps_the_screen_exact():
    """With the per-tile margin (largest |h| of 64 consecutive sources, whose h vary by a factor
    of up to 30) decided pairs still agree with the FP64 predicate, and ordinary pairs stay
    decided."""
    rng = np.random.default_rng(7)
    for scale, origin in ((1e-3, 0.3), (1.0, 10.0), (3e-2, 0.0)):
        n = 128_000
        o = origin + rng.uniform(-1, 1, size=3) * scale
        E = scale * rng.uniform(0.1, 4.0)
        ta = o + rng.uniform(-E, E, size=(n, 3))
        dirn = rng.normal(size=(n, 3))
        dirn /= np.linalg.norm(dirn, axis=1, keepdims=True)
        r = E * 10.0 ** rng.uniform(-1, 0.5, size=n)
        sb = ta + dirn * r[:, None]
        dist = np.sqrt(((ta - sb) ** 2).sum(1))
        rel = np.where(rng.random(n) < 0.25, rng.integers(-8, 9, size=n) * 2.0 ** -52,
                       np.sign(rng.normal(size=n)) * 10.0 ** rng.uniform(-16, -2, size=n))
        ha = 0.5 * dist * (1 + rel) * rng.uniform(0.05, 1.0, size=n)
        hb = dist * (1 + rel) - ha
        Eo = np.max(np.abs(ta - o))
        hit, und = _screen(ta, sb, ha, hb, o, Eo, tile=64)
        ex = _exact(ta, sb, ha, hb)
        assert np.array_equal(hit[~und], ex[~und])
        assert (~und).sum() > 0.1 * n and und.sum() > 0.1 * n  # both paths exercised
    # ordinary neighbourhoods with h varying within a tile are still decided almost always
    sp = 1.0 / 56
    o = np.array([0.2, 0.05, 0.05])
    ta = o + rng.uniform(0, 4 * sp, size=(128_000, 3))
    sb = ta + rng.uniform(-4 * sp, 4 * sp, size=(128_000, 3))
    ha = sp * rng.uniform(0.6, 1.8, size=128_000)
    hb = sp * rng.uniform(0.6, 1.8, size=128_000)
    hit, und = _screen(ta, sb, ha, hb, o, 4 * sp, tile=64)
    assert und.mean() < 2e-3
    assert np.array_equal(hit[~und], _exact(ta, sb, ha, hb)[~und])
