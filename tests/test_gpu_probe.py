"""The FMA-chain peak probe computes what it states: out[i] is the sum of 8 chains
a <- a * m + b started at a_c = 1e-3 (c + 1) + 1e-9 t (t = thread index in its workgroup),
which after n links equals m^n a_c + b (1 - m^n) / (1 - m)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("kind,tol", [(0, 1e-12), (1, 2e-5)])
def test_peak_probe_closed_form(kind, tol):
    import torch
    import paper_2007_03097_amd as sph
    nt, iters = 512, 97
    out = torch.full((nt,), float("nan"), dtype=torch.float64, device="cuda")
    sph.sph_peak_probe(kind, out, iters)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    t = np.arange(nt) % 256
    m = 0.9999999 if kind == 0 else float(np.float32(0.9999999))
    b = 1e-7 if kind == 0 else float(np.float32(1e-7))
    mn = m ** iters
    want = np.zeros(nt)
    for c in range(8):
        a0 = 1e-3 * (c + 1) + 1e-9 * t
        if kind == 1:
            a0 = a0.astype(np.float32).astype(np.float64)
        want += mn * a0 + b * (1.0 - mn) / (1.0 - m)
    assert np.max(np.abs(got - want) / np.abs(want)) < tol


def test_peak_probe_rejects_bad_sizes():
    import torch
    import paper_2007_03097_amd as sph
    out = torch.zeros(300, dtype=torch.float64, device="cuda")
    with pytest.raises(sph.SPHError):
        sph.sph_peak_probe(0, out, 10)
