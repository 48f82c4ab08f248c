"""rs_dense_inverse_noalloc against rs_dense_inverse through the C-ABI: the
same kernels on the library's static scratch array instead of pool memory,
so the results are bitwise equal.  Two calls in a row, the second smaller
(the array keeps the first call's contents), a singular matrix between them
(the flag must be cleared by the next call), sizes beyond the maximum, and
the pool unchanged by the calls."""
import numpy as np
import pytest
import torch

from paper_1812_03952_amd import rsolve as rs
from gpu_util import dev

pytestmark = pytest.mark.gpu


def _mat(n, seed):
    rng = np.random.default_rng(seed)
    a = rng.standard_normal((n, n))
    a[np.arange(n), np.arange(n)] += 0.5 * n ** 0.5      # well conditioned, still pivots
    return a


def _both(a):
    n = a.shape[0]
    da = dev(a)
    ref = torch.empty(n, n, dtype=torch.float64, device="cuda")
    got = torch.full((n, n), float("nan"), dtype=torch.float64, device="cuda")
    rs.dense_inverse(da, ref)
    torch.cuda.synchronize()
    live0 = rs.pool_usage()
    rs.dense_inverse_noalloc(da, got)
    assert rs.pool_usage() == live0
    return ref.cpu().numpy(), got.cpu().numpy()


@pytest.mark.parametrize("sizes", [(300, 120), (1024, 37), (150, 7)])
def test_noalloc_matches_allocating_entry_point(sizes):
    for k, n in enumerate(sizes):
        print(f"dense_inverse_noalloc n={n}", flush=True)
        a = _mat(n, 10 + k)
        ref, got = _both(a)
        assert np.array_equal(got, ref)
        assert np.allclose(got @ a, np.eye(n), atol=1e-9)


def test_noalloc_singular_then_regular_and_limits():
    n = 64
    a = _mat(n, 3)
    a[:, 17] = 0.0                  # a zero column stays exactly zero: zero pivot
    da = dev(a)
    out = torch.empty(n, n, dtype=torch.float64, device="cuda")
    with pytest.raises(rs.RsError) as e:
        rs.dense_inverse(da, out)
    assert e.value.status == -4
    with pytest.raises(rs.RsError) as e:
        rs.dense_inverse_noalloc(da, out)
    assert e.value.status == -4
    b = _mat(40, 4)                                           # smaller, regular: flag cleared
    ref, got = _both(b)
    assert np.array_equal(got, ref)
    big = torch.zeros(rs.DENSE_NOALLOC_MAX + 1, rs.DENSE_NOALLOC_MAX + 1, dtype=torch.float64, device="cuda")
    with pytest.raises(rs.RsError) as e:
        rs.dense_inverse_noalloc(big, big)
    assert e.value.status == -1
    # d_a and d_inv may alias
    c = _mat(33, 5)
    dc = dev(c)
    ref = torch.empty_like(dc)
    rs.dense_inverse(dc, ref)
    rs.dense_inverse_noalloc(dc, dc)
    assert torch.equal(dc, ref)
