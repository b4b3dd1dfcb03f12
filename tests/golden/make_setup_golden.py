"""Write setup_sweeps.json: the oracle's adaptive setup on seeded inputs.

Paper Sec. 2 (adaptive setup): sweep 0 is a Krylov solver on A x = 0 from
random starts; every later sweep applies the multigrid built so far to the
same problem from each vector and keeps what it fails to remove.  This script
calls only the oracle and the seeded input generators; the GPU test reads the
file and compares the library's setup with it.

Usage: python tests/golden/make_setup_golden.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from inputs import prepare_gauge, random_starts  # noqa: E402
from oracle import dwf  # noqa: E402
from oracle import setup as osu  # noqa: E402

# 4^4 x 8, m_f = 0.01, eps = 0.3 (gauge seed 11), 2^4 blocks, starts seed 21.
# The coarse CGNE runs exactly 16 iterations (a tolerance never met), so the
# two sides' V-cycles are the same map whatever their stopping-test cadence.
CASES = [
    dict(name="c1_nvec8_sweeps3", nvec=8, sweeps=3, sweep0_iters=100, sweep_iters=4),
    dict(name="c1_nvec16_sweeps2", nvec=16, sweeps=2, sweep0_iters=60, sweep_iters=2),
]
COMMON = dict(L=(4, 4, 4, 4), Ls=8, M5=1.8, mf=0.01, eps=0.3, gauge_seed=11, start_seed=21, block=(2, 2, 2, 2),
              nu_pre=4, nu_post=4, coarse_tol=1e-30, coarse_maxiter=16)


def main():
    c = COMMON
    U = prepare_gauge(c["L"], c["eps"], c["gauge_seed"])
    A = dwf.DWF(U, c["M5"], c["mf"])
    out = {"common": {k: list(v) if isinstance(v, tuple) else v for k, v in c.items()}, "cases": []}
    for case in CASES:
        nh = case["nvec"] // 2
        V0 = random_starts(c["L"], c["Ls"], nh, c["start_seed"])
        prm = osu.MGParams(block=c["block"], nvec=case["nvec"], sweeps=case["sweeps"],
                           sweep0_iters=case["sweep0_iters"], sweep_iters=case["sweep_iters"],
                           nu_pre=c["nu_pre"], nu_post=c["nu_post"], smoother="mr_normal", coarse_solver="cgne",
                           coarse_tol=c["coarse_tol"], coarse_maxiter=c["coarse_maxiter"])
        mg = osu.adaptive_setup(A, V0, prm)
        per_vec = [float(np.linalg.norm(A(v)) / np.linalg.norm(v)) for v in mg.V]
        out["cases"].append(dict(case, null_residuals=[float(x) for x in mg.null_residuals],
                                 final_per_vector=per_vec))
        print(case["name"], mg.null_residuals, flush=True)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "setup_sweeps.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
