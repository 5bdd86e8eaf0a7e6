"""Write oracle_small.json: oracle eigenvalues and projection norms for small
seeded inputs.  Calls only oracle/ and workloads/."""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
import oracle  # noqa: E402
from workloads import batched_cones, single_cone  # noqa: E402


def main():
    out = {"source": "oracle/ (FP64 Jacobi + clip) on workloads/ seeded inputs", "cases": []}
    cone, _ = single_cone()
    cases = [("single_cone_n50", cone.X)]
    for i, c in enumerate(batched_cones(count=3, n_min=16, n_max=48)):
        cases.append((f"batched_cone_{i}_n{c.n}", c.X))
    for name, X in cases:
        Pi, lam = oracle.project(X)
        out["cases"].append({
            "name": name, "n": int(X.shape[0]),
            "lam": [float(v) for v in lam],
            "pi_fro": float(np.linalg.norm(Pi)),
            "pi_trace": float(np.trace(Pi)),
        })
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_small.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
