"""Thin binding of the C ABI (include/sph.h) for torch tensors.

Each ``sph_*`` function marshals its arguments and calls the function of the same name in
libsph_gfx950.so; tensors must be contiguous CUDA/HIP tensors of the stated dtype.  The
``Context`` class only bundles a context handle with its workspace tensor.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import _abi
from ._abi import SPHError, sph_config, sph_particles

FIELDS = ("x", "y", "z", "vx", "vy", "vz", "m", "h", "u")
ACCEL = ("ax", "ay", "az", "dudt")


def _lib():
    return _abi.load()


def _ptr(t, dtype=None):
    if t is None:
        return None
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError("expected a torch tensor")
    if not t.is_cuda:
        raise ValueError("tensor must be on the GPU")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"expected {dtype}, got {t.dtype}")
    return ctypes.c_void_p(t.data_ptr())


def _check(ctx, status):
    if status != 0:
        msg = _lib().sph_last_error(ctx)
        raise SPHError(status, msg.decode() if msg else "")


class ParticleArrays:
    """Device arrays (float64, caller order) of a particle set plus optional segments."""

    def __init__(self, x, y, z, vx, vy, vz, m, h, u, seg_offsets=None, ax=None, ay=None, az=None, dudt=None,
                 seg_dt=None):
        import torch
        self.t = dict(x=x, y=y, z=z, vx=vx, vy=vy, vz=vz, m=m, h=h, u=u, ax=ax, ay=ay, az=az, dudt=dudt)
        self.n = int(x.shape[0])
        self.seg = None if seg_offsets is None else np.ascontiguousarray(seg_offsets, dtype=np.int64)
        self.seg_dt = None if seg_dt is None else np.ascontiguousarray(seg_dt, dtype=np.float64)
        self._dtype = torch.float64

    @classmethod
    def from_numpy(cls, ps, device="cuda", with_accel=False):
        import torch
        f = {k: torch.as_tensor(np.ascontiguousarray(getattr(ps, k)), dtype=torch.float64, device=device)
             for k in FIELDS}
        acc = {k: torch.zeros(ps.n, dtype=torch.float64, device=device) for k in ACCEL} if with_accel else {}
        return cls(**f, **acc, seg_offsets=ps.seg_offsets)

    def struct(self) -> sph_particles:
        s = sph_particles()
        s.n = self.n
        if self.seg is not None and self.seg.size > 2:
            s.n_seg = self.seg.size - 1
            self._seg_c = self.seg.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
            s.seg_offsets = self._seg_c
        else:
            s.n_seg = 1
            s.seg_offsets = None
        for k in FIELDS + ACCEL:
            p = _ptr(self.t[k], self._dtype)
            setattr(s, k, p.value if p is not None else None)
        if self.seg_dt is not None:
            self._seg_dt_c = self.seg_dt.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
            s.seg_dt = self._seg_dt_c
        else:
            s.seg_dt = None
        return s

    def __getitem__(self, k):
        return self.t[k]


# ---------------------------------------------------------------------------------------
def sph_config_default(**overrides) -> sph_config:
    c = sph_config()
    _lib().sph_config_default(ctypes.byref(c))
    for k, v in overrides.items():
        if not hasattr(c, k):
            raise AttributeError(k)
        setattr(c, k, v)
    return c


def sph_create(cfg: sph_config, n_capacity: int, seg_capacity: int = 1):
    h = ctypes.c_void_p()
    st = _lib().sph_create(ctypes.byref(cfg), int(n_capacity), int(seg_capacity), ctypes.byref(h))
    if st != 0:
        raise SPHError(st, "sph_create rejected the configuration")
    return h


def sph_destroy(ctx):
    _check(ctx, _lib().sph_destroy(ctx))


def sph_workspace_size(ctx) -> int:
    b = ctypes.c_size_t()
    _check(ctx, _lib().sph_workspace_size(ctx, ctypes.byref(b)))
    return int(b.value)


def sph_set_workspace(ctx, ws):
    _check(ctx, _lib().sph_set_workspace(ctx, _ptr(ws), ws.numel() * ws.element_size()))


def sph_build_tree(ctx, parts: ParticleArrays, box=None, keys_out=None, order_out=None):
    import torch
    s = parts.struct()
    bx = None
    if box is not None:
        bx_np = np.ascontiguousarray(box, dtype=np.float64)
        bx = bx_np.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    if keys_out is not None and keys_out.element_size() != 8:
        raise TypeError("keys_out must have 8-byte elements (int64 or uint64)")
    _check(ctx, _lib().sph_build_tree(ctx, ctypes.byref(s), bx, _ptr(keys_out), _ptr(order_out, torch.int64)))


def sph_tree_nodes(ctx, capacity: int, key=None, level=None, leaf=None, start=None, count=None) -> int:
    n = ctypes.c_int64()
    _check(ctx, _lib().sph_tree_nodes(ctx, int(capacity), _ptr(key), _ptr(level), _ptr(leaf), _ptr(start), _ptr(count),
                                      ctypes.byref(n)))
    return int(n.value)


def sph_find_neighbors(ctx, offsets_out=None, idx_out=None, capacity: int = 0, count: bool = True) -> int:
    """count=False with no outputs only (re)builds the device lists (asynchronous)."""
    import torch
    tot = ctypes.c_int64()
    _check(ctx, _lib().sph_find_neighbors(ctx, _ptr(offsets_out, torch.int64), _ptr(idx_out, torch.int32),
                                          int(capacity), ctypes.byref(tot) if count else None))
    return int(tot.value) if count else -1


def sph_compute_density(ctx, rho, P, cs, h_next=None):
    _check(ctx, _lib().sph_compute_density(ctx, _ptr(rho), _ptr(P), _ptr(cs), _ptr(h_next)))


def sph_compute_forces(ctx, ax, ay, az, dudt, rho=None, P=None, cs=None):
    _check(ctx, _lib().sph_compute_forces(ctx, _ptr(rho), _ptr(P), _ptr(cs), _ptr(ax), _ptr(ay), _ptr(az),
                                          _ptr(dudt)))


def sph_compute_gravity(ctx, gx, gy, gz, phi=None):
    _check(ctx, _lib().sph_compute_gravity(ctx, _ptr(gx), _ptr(gy), _ptr(gz), _ptr(phi)))


def sph_step(ctx, parts: ParticleArrays | None, dt: float, nsteps: int, flags: int = 0) -> np.ndarray:
    """Returns the 10 diagnostics (momenta, angular momenta, energies, time-step bound)."""
    diag = np.zeros(10)
    s = parts.struct() if parts is not None else None
    _check(ctx, _lib().sph_step(ctx, ctypes.byref(s) if s is not None else None, float(dt), int(nsteps), int(flags),
                                diag.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    return diag


def sph_step_noalloc(ctx, parts: ParticleArrays | None, dt: float, nsteps: int, flags: int = 0) -> np.ndarray:
    """sph_step in the library's static device scratch (allocates nothing; see sph.h)."""
    diag = np.zeros(10)
    s = parts.struct() if parts is not None else None
    _check(ctx, _lib().sph_step_noalloc(ctx, ctypes.byref(s) if s is not None else None, float(dt), int(nsteps),
                                        int(flags), diag.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    return diag


# Leaf size, group size and waves per CU measured by sph_autotune on MI355X, keyed by
# workload (n, sets, precision, gravity, adaptive h); sph_autotune reads a key when present.
TUNING_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning_gfx950.json")


def sph_autotune(ctx, parts: ParticleArrays, dt: float, cache_path: str | None = None):
    s = parts.struct()
    _check(ctx, _lib().sph_autotune(ctx, ctypes.byref(s), float(dt), cache_path.encode() if cache_path else None))


def sph_get_tuning(ctx):
    """(leaf_size, group_size, waves_per_cu) of the context."""
    a, b, w = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check(ctx, _lib().sph_get_tuning(ctx, ctypes.byref(a), ctypes.byref(b), ctypes.byref(w)))
    return int(a.value), int(b.value), int(w.value)


def sph_timestep(ctx, n_seg: int = 1) -> np.ndarray:
    """Time-step bound min(h/c, sqrt(eps/|a|)) of each set of the resident state."""
    out = np.zeros(n_seg)
    _check(ctx, _lib().sph_timestep(ctx, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    return out


def sph_gravity_counts(ctx):
    """(cell terms, particle-particle terms) of the last particle-cell gravity pass."""
    c, p = ctypes.c_int64(), ctypes.c_int64()
    _check(ctx, _lib().sph_gravity_counts(ctx, ctypes.byref(c), ctypes.byref(p)))
    return int(c.value), int(p.value)


def sph_key_order(ctx, keys_out=None, order_out=None):
    import torch
    if keys_out is not None and keys_out.element_size() != 8:
        raise TypeError("keys_out must have 8-byte elements (int64 or uint64)")
    _check(ctx, _lib().sph_key_order(ctx, _ptr(keys_out), _ptr(order_out, torch.int64)))


def sph_sync(ctx):
    _check(ctx, _lib().sph_sync(ctx))


def sph_last_error(ctx) -> str:
    m = _lib().sph_last_error(ctx)
    return m.decode() if m else ""


def sph_peak_probe(kind: int, out, iters: int, stream=None):
    """FMA-chain probe (kind 0 FP64, 1 FP32) over out.numel() threads; asynchronous."""
    import torch
    st = _lib().sph_peak_probe(int(kind), _ptr(out, torch.float64), out.numel(), int(iters),
                               ctypes.c_void_p(stream) if stream else None)
    if st != 0:
        raise SPHError(st, "sph_peak_probe rejected its arguments or failed to launch")


# ---------------------------------------------------------------------------------------
class Context:
    """A context handle plus its workspace tensor (allocated once, as uint8 on the GPU)."""

    def __init__(self, n_capacity: int, seg_capacity: int = 1, device="cuda", **cfg):
        import torch
        self.cfg = sph_config_default(**cfg)
        self.h = sph_create(self.cfg, n_capacity, seg_capacity)
        nbytes = sph_workspace_size(self.h)
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=device)
        sph_set_workspace(self.h, self.ws)
        self.n_capacity = n_capacity

    def close(self):
        if self.h is not None:
            sph_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
