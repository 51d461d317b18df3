"""Writes oracle_re.json: restoration errors of the float64 oracle's plain
RTG-GMRES solves (algorithm of Sec. 4.4, discrepancy-principle mu, RE of
Sec. 5.5) on the workloads whose oracle solve takes too long to repeat in
every test or benchmark run:

* video: the 256x256x64 video workload, problem 0, X0 = 0, m = 80;
* uneven: five problems of the 256-problem uneven batch (seed 0, m = 40):
  the three with the fewest elements and the two with the most.

The observation C is formed by the oracle (eq. (59) noise scaling) from the
seeded canonical inputs.  Only oracle/ and the input generator are used.

Usage: python tests/golden/make_oracle_re.py   (about 3 minutes on 8 cores)
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from paper_2603_00839_amd import synth  # noqa: E402
from oracle.operator import Operator, make_observation  # noqa: E402
from oracle.sketch import Sketch  # noqa: E402
from oracle.gmres import rtg_gmres  # noqa: E402
from oracle.metrics import relative_error  # noqa: E402

UNEVEN_COUNT = 256


def uneven_sample():
    """Indices of the three smallest and the two largest problems of the
    uneven batch (ties broken by index)."""
    sizes = []
    for p in range(UNEVEN_COUNT):
        I1, I2, J = synth.cfg4_problem(0, p).dims
        sizes.append((I1 * I2 * J, p))
    sizes.sort()
    return [p for _, p in sizes[:3]] + [p for _, p in sizes[-2:]]


def solve(p, m):
    op = Operator(p.a1_band, p.a2_band, p.b_band)
    sk = Sketch(p.om1, p.om2, p.om3)
    C, delta, _ = make_observation(op, p.x_true, p.noise_dir, p.nu)
    C = C.astype(np.float32)
    t0 = time.time()
    r = rtg_gmres(op, sk, C, m, delta=delta, eta=1.01)
    return {"re": relative_error(p.x_true, r.X), "mu": r.mu, "flags": int(r.flags), "m_eff": int(r.m_eff),
            "dims": list(p.dims), "nu": p.nu, "seconds": round(time.time() - t0, 2)}


def main():
    out = {"citation": "float64 oracle, plain RTG-GMRES (Sec. 4.4) from X0 = 0 with the discrepancy-principle mu "
                       "(eta 1.01, delta the noise norm), RE of Sec. 5.5; written by tests/golden/make_oracle_re.py",
           "video": {}, "uneven": {}}
    for p_idx in uneven_sample():
        r = solve(synth.cfg4_problem(0, p_idx), 40)
        print("uneven", p_idx, r, flush=True)
        out["uneven"][str(p_idx)] = r
    r = solve(synth.cfg3(0), 80)
    print("video 0", r, flush=True)
    out["video"]["0"] = r
    with open(os.path.join(HERE, "oracle_re.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
