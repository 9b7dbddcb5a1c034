"""Writes grf64_bench_oracle.json: the FP64 oracle's FGMRES iteration count and final
residual on grf64 (64^3 cells, 1,348,163 unknowns) in the benchmarked configuration
(l1-Jacobi smoothing, BILU(0) on 16 x 16 x 16-cell subdomains with two sweeps, FGMRES(100)
with delayed re-orthogonalisation, rtol 1e-8).  Calls only the oracle and the input
generator; takes about 20 minutes on one core.  Run from the repository root:
python tests/golden/make_grf64_oracle.py
"""
import json
import os
import sys
import time

for _v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
    os.environ[_v] = "1"
HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from synth import workload                       # noqa: E402
from synth.jacobian import box_partition         # noqa: E402
from oracle import Options, solve                # noqa: E402

CONFIG = dict(workload="grf64", smoother="l1jac", ml_kind="bilu0", ml_sweeps=2, ml_part=(16, 16, 16),
              restart=100, rtol=1e-8, orth="dcgs2")


def main():
    t0 = time.perf_counter()
    s, b = workload(CONFIG["workload"])
    s.ml_part = box_partition(*s.meta["grid"], *CONFIG["ml_part"])
    opts = Options(smoother=CONFIG["smoother"], ml_kind=CONFIG["ml_kind"], ml_sweeps=CONFIG["ml_sweeps"],
                   restart=CONFIG["restart"], orth=CONFIG["orth"])
    out = solve(s, b, rtol=CONFIG["rtol"], opts=opts)
    rec = dict(config=CONFIG, iterations=int(out["iterations"]), restarts=int(out["restarts"]),
               status=int(out["status"]), rel_residual=float(out["rel_residual"]),
               history_every_10=[float(h) for h in out["history"][9::10]],
               seconds=round(time.perf_counter() - t0, 1))
    with open(os.path.join(HERE, "grf64_bench_oracle.json"), "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
