"""The entry point that allocates no device memory (ddqmc_dev_binom_noalloc,
samples staged in the library's static scratch) against the allocating one
(ddqmc_dev_binom): the same samples, on two calls in a row, the second with
a smaller input, so that it runs over what the first left in the scratch;
the same errors."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dq():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_1802_05931_amd as m
    return m


@pytest.mark.parametrize("n,p,mode", [(1000, 0.3, 0), (2 ** 31 - 1, 1e-6, 0), (400, 0.1, 1),
                                      (1000, 3.05, 2)])
def test_noalloc_equals_alloc_twice(dq, n, p, mode):
    first, second = 1 << 20, 3000  # the scratch's largest input, then a smaller one
    a1 = dq.dev_binom(n, p, mode, 17, first)
    b1 = dq.dev_binom_noalloc(n, p, mode, 17, first)
    assert np.array_equal(a1, b1)
    a2 = dq.dev_binom(n, p, mode, 23, second)
    b2 = dq.dev_binom_noalloc(n, p, mode, 23, second)
    assert np.array_equal(a2, b2)
    assert not np.array_equal(b2, b1[:second])  # another seed: the scratch was rewritten


def test_noalloc_limits(dq):
    with pytest.raises(dq.DDQMCError) as e:
        dq.dev_binom_noalloc(10, 0.5, 0, 1, (1 << 20) + 1)
    assert e.value.code == -1
    with pytest.raises(dq.DDQMCError) as e:
        dq.dev_binom_noalloc(10, 1.5, 0, 1, 10)
    assert e.value.code == -1
    assert len(dq.dev_binom_noalloc(10, 0.5, 0, 1, 0)) == 0
