"""GPU tests of the measurement probes: the streaming HBM probe moves the
bytes it is asked to, and the hardware square root and reciprocal lie within
the 2 ulps that the contraction lookup's fall-back margin assumes."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


def _lib():
    import paper_2210_04847_amd as nacc
    return nacc._lib


def _ulps(got, exact):
    """|got - exact| in units of the last place of the correctly rounded
    value (exact in FP64)."""
    rounded = exact.astype(np.float32)
    return np.abs(got.astype(np.float64) - exact) / np.spacing(np.abs(rounded)).astype(np.float64)


def test_hardware_sqrt_and_reciprocal_within_two_ulps():
    lib = _lib()
    rng = np.random.default_rng(77)
    n = 1 << 22
    # squared norms the lookups see (points out to 1e4 and beyond), norms
    # near 1 (where the contraction starts), and their reciprocals' range
    x = np.exp(rng.uniform(np.log(1e-6), np.log(1e12), n)).astype(np.float32)
    x[: n // 8] = (1.0 + rng.uniform(-1e-3, 1e-3, n // 8)).astype(np.float32)
    xd = torch.from_numpy(x).cuda()
    s = torch.empty_like(xd)
    r = torch.empty_like(xd)
    lib.probe_fast_sqrt_rcp(xd, s, r)
    torch.cuda.synchronize()
    x64 = x.astype(np.float64)
    e_sqrt = _ulps(s.cpu().numpy(), np.sqrt(x64))
    e_rcp = _ulps(r.cpu().numpy(), 1.0 / x64)
    print(f"hardware sqrt within {e_sqrt.max():.3f} ulp, reciprocal within {e_rcp.max():.3f} ulp")
    assert e_sqrt.max() <= 2.0 and e_rcp.max() <= 2.0


def test_hbm_probe_copies():
    lib = _lib()
    n = 1 << 20
    src = torch.arange(n, dtype=torch.int32, device="cuda")
    dst = torch.zeros(n, dtype=torch.int32, device="cuda")
    lib.probe_hbm(lib.PROBE_COPY, src, dst, n * 4, 64)
    torch.cuda.synchronize()
    assert torch.equal(src, dst)
    lib.probe_hbm(lib.PROBE_WRITE, None, dst, n * 4, 64)
    torch.cuda.synchronize()
    assert int(dst.abs().sum().item()) == 0
