"""Writes ness_3x3.json: the exact steady state of the 3x3 dissipative XYZ
lattice (Jy = Jz = gamma = 1; Jx of the 3x3 workload: 0.6, 0.9, 1.1) from
oracle/exact.py's long-time integration of the master equation, as
magnetisation and bond correlators.  Calls only the oracle; takes about two
minutes."""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import exact  # noqa: E402


def main():
    out = {"lattice": [3, 3], "Jy": 1.0, "Jz": 1.0, "gamma": 1.0,
           "method": "exact.ness_evolve (RK4 on L rho, tau 0.05, relative residual < 1e-12)",
           "states": []}
    for jx in (0.6, 0.9, 1.1):
        rho, res = exact.ness_evolve(3, 3, jx, 1.0, 1.0, 1.0)
        obs = exact.observables(rho, 3, 3)
        out["states"].append(dict(Jx=jx, residual=float(res),
                                  **{k: float(v) for k, v in obs.items()}))
        print(jx, res, obs, flush=True)
    with open(os.path.join(HERE, "ness_3x3.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
