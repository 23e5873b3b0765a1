"""Write tests/golden/lipschitz.json: L = ||A||_2^2 of each fixed workload's operator, by the
FP64 oracle's power method (50 iterations from the all-ones image; converged to ~1e-15 at
these sizes).  The step size gamma = 1/L is then the same double on the oracle and the GPU.

Calls only the oracle.  Run: python tests/golden/make_lipschitz.py [names...]
(A is block-diagonal over slices, so a volume's L is that of one slice.)
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_2602_09527_amd import workloads  # noqa: E402

OUT = os.path.join(HERE, "lipschitz.json")


def main(names):
    data = json.load(open(OUT)) if os.path.exists(OUT) else {}
    for w in workloads.ALL.values():
        if names and w.name not in names:
            continue
        g = oracle.Geometry(w.nx, w.ny, w.n_angles, w.n_bins, n_subsets=w.n_subsets, nz=1)
        L = oracle.lipschitz(g, 50)
        data[w.key] = {"L": L, "workload": w.name, "iters": 50,
                       "how": "oracle.lipschitz (power method, FP64) on one slice"}
        print(w.name, w.key, repr(L), flush=True)
        json.dump(data, open(OUT, "w"), indent=1, sort_keys=True)


if __name__ == "__main__":
    main(set(sys.argv[1:]))
