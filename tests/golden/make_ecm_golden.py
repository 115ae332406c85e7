"""Write the stored oracle result of the empirical-cubature selection used by
tests/test_gpu_ecm.py: the Box 1 greedy (Sec. 3.3) of the oracle on its own
training matrix and SVD basis, for seeded candidates and snapshots large
enough that the selection passes 256 points.  Calls only the oracle and the
seeded input generators.  Run: python tests/golden/make_ecm_golden.py"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as orc  # noqa: E402
from hrom_inputs import THETA_REF, make_cluster, make_snapshots  # noqa: E402

CASE = dict(m=16, M=2048, p=20, mt=300, seed=9416)


def main():
    c = CASE
    cl = make_cluster(c["m"], c["M"], c["seed"])
    Fr, a = make_snapshots(c["p"], c["m"], c["seed"] + 1)
    f = orc.ecm_integrand(cl, THETA_REF, Fr, a)
    xf, _ = orc.ecm_training_matrix(f, cl.w)
    lam, s = orc.ecm_basis(xf, c["mt"] - 1)
    z, w, info = orc.ecm_greedy(lam, float(cl.w.sum()), c["mt"])
    out = dict(case=c, sigma=[float(v) for v in s],
               picked=[int(k) for k in info["picked"]],
               nnls=[int(u) for u in info["nnls"]],
               dropped=[len(d) for d in info["dropped"]],
               gap=[float(g) for g in info["gap"]],
               z=[int(k) for k in z], w=[float(v) for v in w])
    path = os.path.join(HERE, "ecm_m16_M2048_p20_mt300.json")
    with open(path, "w") as fh:
        json.dump(out, fh)
    print("wrote", path, len(out["picked"]), "iterations")


if __name__ == "__main__":
    main()
