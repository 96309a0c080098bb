"""The whole method at 3x3 against the exact steady state: solves of the 3x3
workload (Jx 0.6 and 1.1, without initiator so that there is no initiator
bias) run on the GPU, whose steps are the oracle's bit for bit, and their
accumulated M_z and bond correlators compared with the exact steady states
in tests/golden/ness_3x3.json (the long-time limit of the master equation,
written by tests/golden/make_ness_3x3.py from oracle/exact.py)."""
import json
import os

import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dq():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_1802_05931_amd as m
    return m


@pytest.mark.parametrize("jx,seed", [(0.6, 1), (1.1, 2)])
def test_3x3_matches_the_exact_steady_state(dq, jx, seed):
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "ness_3x3.json")))
    ex = [s for s in g["states"] if s["Jx"] == jx][0]
    cfg = dict(Lx=3, Ly=3, Jx=jx, Jy=1.0, Jz=1.0, gamma=1.0, dt=0.005, n_a=0,
               target_walkers=100_000, initial_walkers=100, shift_init=-0.5, seed=seed,
               n_equil=4000)
    s = dq.Solve(dq.make_params(**cfg))
    s.set_graph_steps(50)
    s.step(40_000)
    o = s.observables()
    s.close()
    assert o["n_accum"] == 36_000
    print(f"  Jx {jx}: M_z {o['mz']:.5f} +- {o['se_mz']:.5f} (exact {ex['mz']:.5f}); "
          f"C_xx {o['cxx']:.5f} +- {o['se_cxx']:.5f} ({ex['cxx']:.5f}); "
          f"C_yy {o['cyy']:.5f} +- {o['se_cyy']:.5f} ({ex['cyy']:.5f}); "
          f"C_zz {o['czz']:.5f} +- {o['se_czz']:.5f} ({ex['czz']:.5f})", flush=True)
    assert 0 < o["se_mz"] < 0.01
    assert abs(o["mz"] - ex["mz"]) < 3 * o["se_mz"]
    for k in ("cxx", "cyy", "czz"):
        assert abs(o[k] - ex[k]) < 4 * o["se_" + k], k
