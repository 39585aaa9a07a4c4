"""The allocation-free filter (chebyshev_filter_noalloc) against
chebyshev_filter, through the C ABI.

Both run the same kernels on the same inputs; only the place of the KB
coefficients differs (the library's fixed device scratch instead of the
handle's), so the filtered blocks must be identical.  Two calls in a row,
the second smaller (fewer vectors, another precision and degree), check that
what the first call left in the shared scratch does not leak into the
second; the library's count of its own device allocations must not move.
"""
import numpy as np
import pytest

from oracle import chfsi as OC
from synth.cluster import random_block

from gpu_system import build, to_rows

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def system():
    return build()


def _filter(B, H, name, X, W, degree, a, b, a0):
    code = B.CHF_F64 if X.dtype == torch.float64 else B.CHF_F32
    B.call(name, H.handle, code, B._ptr(X), X.stride(0), X.shape[1], degree, a, b, a0, B._ptr(W), W.stride(0),
           B._stream())


def test_noalloc_filter_equals_filter_on_two_calls(system):
    s = system
    B, H = s["B"], s["Hg"]
    v0 = random_block(s["g"].n, 1, 3001)[:, 0]
    b, tmin, _ = OC.lanczos_bound(s["Ho"].apply, v0, 10)
    a, a0 = tmin + 0.1 * (b - tmin), tmin
    cases = [(torch.float64, 64, 9, 2800), (torch.float32, 24, 4, 2801)]   # second call smaller
    for dtype, m, degree, seed in cases:
        X = to_rows(s, random_block(s["g"].n, m, seed), dtype)
        ref = X.clone()
        _filter(B, H, "chebyshev_filter", ref, torch.zeros_like(ref), degree, a, b, a0)
        W = torch.zeros_like(X)
        torch.cuda.synchronize()
        before = B.device_allocations()
        _filter(B, H, "chebyshev_filter_noalloc", X, W, degree, a, b, a0)
        torch.cuda.synchronize()
        assert B.device_allocations() == before
        assert torch.equal(X, ref), (dtype, m)
    # a narrower work block takes column blocks, as in chebyshev_filter
    X = to_rows(s, random_block(s["g"].n, 40, 2802), torch.float64)
    ref = X.clone()
    _filter(B, H, "chebyshev_filter", ref, torch.zeros_like(ref), 5, a, b, a0)
    _filter(B, H, "chebyshev_filter_noalloc", X, torch.zeros((H.n_rows, 16), dtype=torch.float64, device="cuda"), 5,
            a, b, a0)
    assert torch.equal(X, ref)


def test_noalloc_filter_checks_arguments(system):
    s = system
    B, H = s["B"], s["Hg"]
    buf = torch.zeros((H.n_rows, 64), dtype=torch.float64, device="cuda")
    with pytest.raises(B.ChfError) as e:     # X and work overlap
        _filter(B, H, "chebyshev_filter_noalloc", buf[:, :32], buf[:, 16:48], 3, 0.0, 1.0, -1.0)
    assert e.value.code == -1
    X = torch.zeros((H.n_rows, 16), dtype=torch.float64, device="cuda")
    with pytest.raises(B.ChfError) as e:     # bounds out of order
        _filter(B, H, "chebyshev_filter_noalloc", X, torch.zeros_like(X), 3, 1.0, 0.0, -1.0)
    assert e.value.code == -1
