"""The inner product that allocates nothing (mpk_dot_noalloc) against the
workspace form (mpk_dot): same kernels and reduction tree, so the results
must be identical bit for bit, on two calls in a row (the second with a
smaller input, which must not see the first call's partials), real and
complex, in every precision; sizes past the fixed scratch are rejected."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mpk():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2504_14498_amd import mpk as m
    m.library()
    return m


def vec(rng, n, C, K):
    x = np.zeros((n, C, K))
    v = rng.uniform(-1, 1, (n, C))
    for k in range(K):
        x[:, :, k] = v
        v = v * rng.uniform(0.5, 1.0, (n, C)) * 2.0 ** -53
    return x


@pytest.mark.parametrize("C,K", [(1, 1), (1, 2), (1, 3), (1, 4), (2, 2), (2, 4)])
def test_noalloc_dot_matches_workspace_dot(mpk, C, K):
    import torch
    rng = np.random.default_rng(10 * C + K)
    nmax = mpk.dot_noalloc_max_elements(C, K)
    assert nmax >= (1 << 24) // (C * K)
    for n in (min(nmax, 3_000_017), 1_001):       # the second call is smaller
        a = torch.as_tensor(vec(rng, n, C, K)).cuda()
        b = torch.as_tensor(vec(rng, n, C, K)).cuda()
        out = torch.full((C, K), float("nan"), dtype=torch.float64, device="cuda")
        mpk.dot_noalloc(a, b, out)
        ref = mpk.dot(a, b)
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), ref.cpu().numpy()), (n, C, K)


def test_noalloc_dot_rejects_sizes_past_the_scratch(mpk):
    import torch
    a = torch.zeros((1, 1, 2), dtype=torch.float64, device="cuda")
    out = torch.zeros((1, 2), dtype=torch.float64, device="cuda")
    nmax = mpk.dot_noalloc_max_elements(1, 2)
    st = mpk._lib().mpk_dot_noalloc(2, 0, nmax + 1, mpk._ptr(a), mpk._ptr(a), mpk._ptr(out),
                                   None)
    assert st == -3
