"""Write oracle results for workloads too large to solve inside a GPU test.

Calls only the oracle and the input generator.  Usage:
    python tests/golden/make_golden.py global200
Each file stores a digest of the generated inputs so a test can tell when the
generator no longer reproduces them.
"""
import hashlib
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import Params  # noqa: E402
from oracle.gn import solve_problem  # noqa: E402
from synth import make_problem  # noqa: E402


def input_digest(prob):
    h = hashlib.sha256()
    for a in (prob.depth, prob.intensity, prob.corr_i, prob.corr_j, prob.corr_p, prob.corr_q, prob.init_poses):
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def global200():
    prob = make_problem(1)
    prm = Params(num_gn=prob.n_gn, num_pcg=prob.n_pcg)
    res = solve_problem(prob, prm, linear="pcg")
    s = res["setup"]
    # trajectory X_0..X_n and the per-iteration increments (reduced, free frames in order)
    from oracle.se3 import exp_se3
    traj = [prob.init_poses.copy()]
    X = prob.init_poses.copy()
    for st in res["steps"]:
        for n, f in enumerate(s.free):
            X[f] = X[f] @ exp_se3(st["dx"][6 * n:6 * n + 6])
        traj.append(X.copy())
    np.savez_compressed(
        os.path.join(HERE, "global200_oracle.npz"),
        digest=np.array(input_digest(prob)),
        poses=res["poses"], pairs=s.pairs, edges=s.edges, free=s.free,
        traj=np.array(traj), steps=np.array([st["dx"] for st in res["steps"]]),
        energy=np.array([res["energy"][k] for k in ("total", "sparse", "geo", "photo")]),
        counts=np.array([res["energy"][k] for k in ("n_sparse", "n_geo", "n_photo")]),
        trace=np.array([[t[k] for k in ("total", "sparse", "geo", "photo")] for t in res["trace"]]),
        seconds=np.array(res["seconds"]))
    print("global200: oracle solve took", round(res["seconds"], 1), "s")


if __name__ == "__main__":
    for name in sys.argv[1:] or ["global200"]:
        globals()[name]()
