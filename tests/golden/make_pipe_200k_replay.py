"""Writes pipe_200k_fp64_replay.json: the oracle's FP64 nested solve of the
2e5-node pipe Newton step (the benchmark pipe, default solver options), as its
iteration schedule (every Krylov call's iteration count, in start order), the
norms of the velocity and pressure blocks of x, and x at seeded sample indices.
The GPU replays the schedule and is compared on these samples.

Calls only the oracle and the input generators:
    python tests/golden/make_pipe_200k_replay.py      (about 3 minutes)
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from ns_inputs import build  # noqa: E402
from oracle import amg, krylov  # noqa: E402
from oracle import discretization as dz  # noqa: E402

N_SAMPLE_V, N_SAMPLE_P = 2000, 1000


def main():
    case = build("pipe_200k")
    S = dz.assemble(case)
    ns = krylov.NestedSolver(S, amg.node_adjacency(case.n_nodes, case.tets), krylov.SolveOpts())
    x, info = ns.solve(S.rhs)
    n3 = 3 * case.n_nodes
    rng = np.random.default_rng(20)
    iv = np.sort(rng.choice(n3, N_SAMPLE_V, replace=False))
    ip = np.sort(rng.choice(case.n_nodes, N_SAMPLE_P, replace=False)) + n3
    out = {
        "case": "pipe_200k", "options": "oracle defaults (krylov.SolveOpts())",
        "outer": int(info["outer"]), "true_rel_res": float(info["true_rel_res"]),
        "schedule": [int(k) for k in info["schedule"]],
        "norm_v": float(np.linalg.norm(x[:n3])), "norm_p": float(np.linalg.norm(x[n3:])),
        "norm_rhs": float(np.linalg.norm(S.rhs)),
        "idx": [int(i) for i in np.concatenate([iv, ip])],
        "x": [float(v) for v in x[np.concatenate([iv, ip])]],
    }
    with open(os.path.join(HERE, "pipe_200k_fp64_replay.json"), "w") as f:
        json.dump(out, f, indent=0)
    print("outer", out["outer"], "calls", len(out["schedule"]), "res", out["true_rel_res"])


if __name__ == "__main__":
    main()
