"""Pins of the oracle's random-number and elementary-function pieces.

* Philox4x32-10 against the published known-answer vectors of Salmon et al.
  (SC'11, Random123 distribution), and against rocRAND's own engine over
  many keys and counters (the counter's carry across 32-bit words included).
* The 53-bit uniform construction: values on the 2^-53 grid in [0, 1), moments.
* det_log / det_exp (only +,-,*,/) against the C library's log / exp.
"""
import ctypes
import math
import os
import shutil
import subprocess

import numpy as np
import pytest


KAT = [  # (counter, key, output) -- Random123 philox4x32_10 known answers
    ((0, 0, 0, 0), (0, 0), (0x6627e8d5, 0xe169c58d, 0xbc57ac4c, 0x9b00dbd8)),
    ((0xffffffff,) * 4, (0xffffffff,) * 2, (0x408f276d, 0x41c83b0e, 0xa20bc7c6, 0x6d5451fd)),
    ((0x243f6a88, 0x85a308d3, 0x13198a2e, 0x03707344), (0xa4093822, 0x299f31d0),
     (0xd16cfe09, 0x94fdcceb, 0x5001e420, 0x24126ea1)),
]


@pytest.mark.parametrize("ctr,key,out", KAT)
def test_philox_known_answers(orc, ctr, key, out):
    assert tuple(int(x) for x in orc.philox(ctr, key)) == out


@pytest.fixture(scope="module")
def rocrand_philox(tmp_path_factory):
    """rocRAND's header-only Philox engine built for the host (tests/rocrand_philox.cpp)."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    if not shutil.which(hipcc) or not os.path.exists("/opt/rocm/include/rocrand"):
        pytest.skip("hipcc or the rocRAND headers are missing")
    src = os.path.join(os.path.dirname(__file__), "rocrand_philox.cpp")
    so = str(tmp_path_factory.mktemp("rocrand") / "rocrand_philox.so")
    subprocess.run([hipcc, "-x", "hip", "--offload-arch=gfx950", "-O2", "-fPIC", "-shared",
                    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                    "-o", so, src], check=True, capture_output=True, timeout=300)
    lib = ctypes.CDLL(so)
    lib.rr_philox.argtypes = [ctypes.c_ulonglong] * 3 + [ctypes.c_uint32, ctypes.c_void_p]
    lib.rr_philox.restype = None

    def run(seed, subsequence, block, blocks):
        out = np.zeros(4 * blocks, np.uint32)
        lib.rr_philox(seed, subsequence, 4 * block, 4 * blocks, out.ctypes.data)
        return out
    return run


def test_philox_equals_rocrand(orc, rocrand_philox):
    """rocRAND's engine: key = the seed's two 32-bit halves; block b of
    subsequence s has the counter (b low, b high, s low, s high), its four
    outputs in order.  The oracle's Philox must give the same words for every
    seed, subsequence and block, across the carry from the counter's first
    word into its second."""
    rng = np.random.default_rng(11)
    cases = [(0, 0, 0), (0xffffffffffffffff, 0xffffffffffffffff, 0),
             (0x0123456789abcdef, (7 << 32) | 5, (1 << 32) - 3)]
    cases += [(int(rng.integers(0, 2 ** 63)) * 2 + 1, int(rng.integers(0, 2 ** 63)),
               int(rng.integers(0, 2 ** 40))) for _ in range(20)]
    for seed, sub, block in cases:
        got = rocrand_philox(seed, sub, block, 6)
        key = (seed & 0xffffffff, seed >> 32)
        for j in range(6):
            b = block + j
            ctr = (b & 0xffffffff, (b >> 32) & 0xffffffff, sub & 0xffffffff, sub >> 32)
            assert tuple(int(x) for x in orc.philox(ctr, key)) == \
                tuple(int(x) for x in got[4 * j:4 * j + 4]), (seed, sub, b)


def test_uniform_grid_and_moments(orc):
    u = orc.uniforms(seed=7, solve_id=3, cfg=12345, step=9, draw=1024, count=131072)
    assert u.min() >= 0.0 and u.max() < 1.0
    k = u * 2.0 ** 53
    assert np.all(k == np.floor(k))
    assert abs(u.mean() - 0.5) < 5 * math.sqrt(1 / 12 / len(u))
    assert abs((u ** 2).mean() - 1 / 3) < 5 * math.sqrt(4 / 45 / len(u))
    # successive pairs uncorrelated
    assert abs(np.corrcoef(u[:-1], u[1:])[0, 1]) < 5 / math.sqrt(len(u))


def test_uniform_stream_is_counter_based(orc):
    # the first two uniforms of a stream come from block 0 of its counter
    seed, sid, cfg, step, draw = 0x123456789ABCDEF0, 17, 0xDEADBEEF12, 44, 3077
    u = orc.uniforms(seed, sid, cfg, step, draw, 4)
    key = (seed & 0xffffffff, (seed >> 32) ^ sid)
    for blk in range(2):
        x = orc.philox((cfg & 0xffffffff, cfg >> 32, step, (draw << 16) | blk), key)
        a = ((int(x[0]) >> 5) * 2 ** 26 + (int(x[1]) >> 6)) / 2 ** 53
        b = ((int(x[2]) >> 5) * 2 ** 26 + (int(x[3]) >> 6)) / 2 ** 53
        assert u[2 * blk] == a and u[2 * blk + 1] == b
    # a different solve id, step, draw or configuration gives another stream
    for args in [(seed, sid + 1, cfg, step, draw), (seed, sid, cfg + 1, step, draw),
                 (seed, sid, cfg, step + 1, draw), (seed, sid, cfg, step, draw + 1)]:
        assert not np.array_equal(orc.uniforms(*args, 4), u)


def _ulps(a, b):
    return abs(a - b) / math.ulp(b) if b != 0 else abs(a)


def test_det_log_against_libm(orc):
    rng = np.random.default_rng(1)
    xs = np.concatenate([rng.uniform(0, 1, 20000), np.exp(rng.uniform(-700, 700, 20000)),
                         rng.uniform(0.5, 2.0, 20000), [5e-324, 1e-310, 2.0 ** -1022, 1.0, 2.0,
                                                         1.7976931348623157e308]])
    worst = max(_ulps(orc.det_log(x), math.log(x)) for x in xs)
    assert worst <= 4.0
    assert orc.det_log(1.0) == 0.0
    assert orc.det_log(0.0) == -math.inf


def test_det_exp_against_libm(orc):
    rng = np.random.default_rng(2)
    worst = max(_ulps(orc.det_exp(x), math.exp(x)) for x in rng.uniform(-700, 700, 20000))
    assert worst <= 2.0
    assert orc.det_exp(0.0) == 1.0
