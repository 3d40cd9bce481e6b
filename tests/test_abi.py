"""CPU-side checks of the C ABI: the library loads next to torch's HIP runtime, exports every
function include/sph.h declares, and validates arguments on the host (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "sph.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(sph_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    from paper_2007_03097_amd import _abi
    lib = _abi.load()
    decl = _declared()
    assert len(decl) >= 20
    for name in decl:
        assert hasattr(lib, name), name
    assert sorted(_abi.EXPORTS) == decl


def test_single_hip_runtime_loaded():
    from paper_2007_03097_amd import _abi
    _abi.load()
    maps = open("/proc/self/maps").read()
    libs = {l.split()[-1] for l in maps.splitlines() if "libamdhip64" in l}
    assert len(libs) == 1, libs


def test_host_validation_without_gpu():
    import paper_2007_03097_amd as sph
    from paper_2007_03097_amd import _abi
    cfg = sph.sph_config_default()
    assert abs(cfg.gamma - 5.0 / 3.0) < 1e-15 and cfg.leaf_size == 16 and cfg.group_size == 32
    h = sph.sph_create(cfg, 1000, 1)
    n = sph.sph_workspace_size(h)
    assert n > 1000 * 8 * 30
    sph.sph_destroy(h)
    for bad in (dict(gamma=1.0), dict(theta=1.5), dict(group_size=12), dict(leaf_size=0 - 1), dict(nbr_capacity=8),
                dict(precision=3), dict(soft_eps=-1.0)):
        with pytest.raises(sph.SPHError):
            sph.sph_create(sph.sph_config_default(**bad), 10, 1)
    with pytest.raises(sph.SPHError):
        sph.sph_create(cfg, -1, 1)
    with pytest.raises(sph.SPHError):
        sph.sph_create(cfg, 10, 513)
    with pytest.raises(sph.SPHError):  # the octree's node indices would overflow 32 bits
        sph.sph_create(cfg, 600_000_000, 1)
    for bad in (dict(gravity_scheme=2), dict(key_curve=5), dict(energy_form=-1), dict(waves_per_cu=-1),
                dict(waves_per_cu=33)):
        with pytest.raises(sph.SPHError):
            sph.sph_create(sph.sph_config_default(**bad), 10, 1)
    lib = _abi.load()
    # calls on a context without workspace fail with SPH_E_NOMEM / SPH_E_STATE, no GPU touched
    h = sph.sph_create(cfg, 10, 1)
    p = _abi.sph_particles()
    p.n, p.n_seg = 5, 1
    assert lib.sph_build_tree(h, ctypes.byref(p), None, None, None) in (_abi.SPH_E_ARG, _abi.SPH_E_NOMEM)
    assert lib.sph_compute_forces(h, None, None, None, None, None, None, None) in (_abi.SPH_E_STATE, _abi.SPH_E_ARG)
    assert lib.sph_step(h, None, -1.0, 1, 0, None) == _abi.SPH_E_ARG
    # per-set step sizes must be positive (checked before anything is launched)
    bad_dt = (ctypes.c_double * 1)(0.0)
    p.seg_dt = ctypes.cast(bad_dt, ctypes.POINTER(ctypes.c_double))
    assert lib.sph_step(h, ctypes.byref(p), 1e-3, 1, 0, None) == _abi.SPH_E_ARG
    assert b"seg_dt" in lib.sph_last_error(h)
    bound = (ctypes.c_double * 1)()
    assert lib.sph_timestep(h, bound) == _abi.SPH_E_STATE   # no resident state yet
    assert lib.sph_timestep(None, bound) == _abi.SPH_E_ARG
    assert lib.sph_key_order(h, None, None) == _abi.SPH_E_STATE
    c1, c2 = ctypes.c_int64(), ctypes.c_int64()
    assert lib.sph_gravity_counts(h, ctypes.byref(c1), ctypes.byref(c2)) == _abi.SPH_E_STATE   # gravity off
    assert lib.sph_gravity_counts(None, ctypes.byref(c1), ctypes.byref(c2)) == _abi.SPH_E_ARG
    # the allocation-free step refuses contexts larger than its scratch before touching the GPU
    big = sph.sph_create(cfg, 1_000_000, 1)
    assert lib.sph_step_noalloc(big, None, 1e-3, 1, 0, None) == _abi.SPH_E_CAPACITY
    assert b"scratch" in lib.sph_last_error(big)
    sph.sph_destroy(big)
    assert lib.sph_last_error(h)
    assert lib.sph_destroy(None) == 0
    sph.sph_destroy(h)
    # the peak probe validates before launching
    for args in ((2, 1, 256, 1), (0, None, 256, 1), (1, 1, 100, 1), (0, 1, 0, 1), (0, 1, 256, 0)):
        assert lib.sph_peak_probe(args[0], args[1], args[2], args[3], None) == _abi.SPH_E_ARG


def test_workspace_scales_with_capacity():
    import paper_2007_03097_amd as sph
    cfg = sph.sph_config_default()
    a = sph.sph_create(cfg, 10000, 1)
    b = sph.sph_create(cfg, 20000, 1)
    wa, wb = sph.sph_workspace_size(a), sph.sph_workspace_size(b)
    assert 1.8 < wb / wa < 2.2
    sph.sph_destroy(a)
    sph.sph_destroy(b)
