"""The scan decides most quiet tests from a single-precision estimate of the
no-event probability g = prod_k (1 - p_k)^n_k (Sec. III.B) and relies on its
relative error staying below 2e-7 + 2e-6 n (n = n_R + n_I <= 1024, every
p_k <= 1/2, estimate >= 2^-30), with a decision band of 1e-5 (1 + n).

Here the estimate is formed as the device forms it, in float32 (numpy's
log2 / exp2 stand in for the device's, both within a few ulps), over random
inputs across that whole domain, and compared with the oracle's fp64 product.
"""
import numpy as np


def _estimate(p4, nR, nI):
    one = np.float32(1.0)
    lr = np.float32(0.0)
    li = np.float32(0.0)
    for k in range(4):
        lr = np.float32(lr + np.log2(one - np.float32(p4[k])))
        li = np.float32(li + np.log2(one - np.float32(p4[k])))
    E = np.float32(np.float32(nR) * lr + np.float32(nI) * li)
    return float(np.exp2(E)), float(E)


def test_estimate_error_within_the_stated_bound(orc):
    rng = np.random.default_rng(8)
    worst = 0.0
    checked = 0
    for i in range(6000):
        scale = [0.5, 0.05, 0.005][i % 3]
        p4 = rng.uniform(0, scale, 4) * (rng.random(4) < 0.9)
        n_tot = int(rng.integers(1, 1025)) if i % 2 else int(rng.integers(1, 40))
        nR = int(rng.integers(0, n_tot + 1))
        nI = n_tot - nR
        ga, E = _estimate(p4, nR, nI)
        if not E > -30.0:
            continue  # left to the exact product
        g = orc.no_event_prob(np.tile(p4, 2), [nR] * 4 + [nI] * 4)
        rel = abs(ga / g - 1.0)
        bound = 2e-7 + 2e-6 * n_tot
        assert rel < bound, (p4, nR, nI, rel, bound)
        assert bound < 1e-5 * (1 + n_tot)  # the band covers the bound
        worst = max(worst, rel / bound)
        checked += 1
    assert checked > 3000
    print(f"worst error / bound = {worst:.3f} over {checked} cases")
