"""Writes c10_oracle_trajectory.json from the oracle alone.

The 10-atom workload's ground state X_min (the oracle's SCF to 1e-10) and
three KSA-XL-BOMD steps from it: the shadow energy and its parts, mu, the
Krylov residual and the nuclear positions.  These are the oracle's own values, a
regression anchor for its arithmetic (a later change to it shows up here and
has to be justified by the method), not an independent pin: the pins are the
closed forms, brute force and finite differences of the oracle tests.

Run from the repository root:  python tests/golden/make_golden.py
"""

import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from synth import workload  # noqa: E402
from oracle import dynamics  # noqa: E402

N_STEPS = 3


def trajectory():
    s, w = workload("c10")
    st = dynamics.Settings(T_e=w["T_e"], m=w["m"], dt=w["dt"])
    X_min = dynamics.scf(s, st)
    o = dynamics.init_state(s, st, X_min)
    out = {"workload": "c10", "T_e": w["T_e"], "m": w["m"], "dt": w["dt"],
           "X_min": X_min.tolist(), "init": {"U": o.U, "mu": o.mu, "R": o.R.tolist()}, "steps": []}
    for _ in range(N_STEPS):
        o, rep = dynamics.md_step(o, s, st)
        out["steps"].append({k: float(rep[k]) for k in ("E_tot", "KE", "U", "TS", "mu", "W0", "relres")}
                            | {"rank": int(rep["rank"]), "R": o.R.tolist()})
    return out


if __name__ == "__main__":
    data = trajectory()
    data["_about"] = ("oracle values written by tests/golden/make_golden.py (oracle/ only): "
                      "regression anchor for the oracle, not an independent pin")
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c10_oracle_trajectory.json")
    with open(path, "w") as f:
        json.dump(data, f, indent=1)
    print("wrote", path)
