"""The allocation-free dense inverse against the workspace entry point: two
calls in a row (the second smaller, so the static scratch still holds the
first call's larger matrix), each bitwise equal to the workspace version
(same kernels on the same input), and the size limit."""
import numpy as np
import pytest

from gpu_common import require_gpu

pytestmark = pytest.mark.gpu


def test_noalloc_dense_inverse_matches_the_workspace_entry_point():
    require_gpu()
    from paper_1808_04338_amd._lib import DP_E_INVALID, DpError
    from paper_1808_04338_amd.sim import dense_inverse_noalloc, dense_inverse_selftest

    rng = np.random.default_rng(7)
    for n in (300, 45):
        A = rng.standard_normal((n, n)) + n * np.eye(n)
        perm = np.arange(n)
        for b0 in range(0, n, 32):
            perm[b0:b0 + 32] = b0 + rng.permutation(min(32, n - b0))
        A = A[perm]  # pivot swaps inside the 32-row panels run
        X = dense_inverse_noalloc(A)
        Y = dense_inverse_selftest(A)
        assert np.array_equal(X, Y), n
        assert np.abs(X @ A - np.eye(n)).max() <= 1e-12 * n
    with pytest.raises(DpError) as e:
        dense_inverse_noalloc(np.eye(1025))
    assert e.value.code == DP_E_INVALID
