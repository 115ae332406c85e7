"""Writes ``oracle_m8_q32.json``: a regression fixture of the FP64 oracle.

The paper prints no worked example with numbers that this method can be
checked against on synthetic inputs (its examples need RVE meshes and
material data that are not available), so the fixture here is not a paper
value: it stores what the oracle itself computes at six macro points of the
256-point workload (m = 8 ROM modes, Q = 32 ECM points, seeded generators):
the Newton-converged homogenised stress and condensed tangent (Sec. 3.2.3)
and the Updated-Lagrangian output (eq. biotstress, App. A) at the converged
state.  ``tests/test_oracle_fixture.py`` checks that the oracle still
reproduces them, so that any change to the oracle's arithmetic shows up and
has to name its reason.  Only ``oracle`` and ``hrom_inputs`` are called.

  python tests/golden/make_oracle_fixture.py
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from hrom_inputs import THETA_REF, make_cluster, make_macro_points  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_m8_q32.json")
M, Q, N, SEED = 8, 32, 6, 9100


def compute():
    cl = make_cluster(M, Q, SEED)
    F, _, _ = make_macro_points(N, SEED + 1, amp=0.05)
    conv = oracle.newton(cl, THETA_REF, F, tol=1e-13)
    pe = oracle.point_eval(cl, THETA_REF, F, conv["a"])
    sig, dsdD, st = oracle.cauchy(F, pe["Palg_r"], pe["Cr"])
    assert not conv["status"].any() and not st.any()
    return {"m": M, "Q": Q, "N": N, "seed": SEED, "theta": THETA_REF.tolist(),
            "Pbar": conv["Pbar"].tolist(), "Cbar": conv["Cbar"].reshape(N, 81).tolist(),
            "sigma": sig.tolist(), "dsdD": dsdD.reshape(N, 81).tolist(),
            "iters": conv["iters"].tolist()}


if __name__ == "__main__":
    oracle.build(force=False)
    with open(OUT, "w") as f:
        json.dump(compute(), f, indent=1)
    print("wrote", OUT)
