"""Write the FP64 oracle's IRLS solution for one seeded workload.

Calls only the oracle and the seeded input generator.  Output:
  tests/golden/oracle_<workload>_seed<seed>.npy   x_ref rounded to complex64
  tests/golden/oracle_<workload>_seed<seed>.json  norm of the FP64 x_ref,
      solver parameters and the oracle's wall time on this host.
Usage: python tests/golden/make_oracle_reference.py sg256 0
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import smsm_inputs as si  # noqa: E402
from oracle import smsm_oracle as o  # noqa: E402


def main(workload: str, seed: int):
    g = si.WORKLOADS[workload]
    case = si.make_case(g, seed, si.WORKLOAD_IDS[workload])
    _, y = o.simulate(case, g.n_slices, g.snr)
    y = y.astype(np.complex64).astype(np.complex128)       # what the GPU receives
    p = o.SolveParams(lam=g.lam, r=g.filt, n_irls=g.n_irls, n_cg=g.n_cg)
    t0 = time.time()
    x = o.solve(y, case["coils"], case["masks"], case["shifts"], p)
    dt = time.time() - t0
    stem = os.path.join(HERE, f"oracle_{workload}_seed{seed}")
    np.save(stem + ".npy", x.astype(np.complex64))
    meta = {"workload": workload, "seed": seed, "norm_fp64": float(np.linalg.norm(x.ravel())),
            "params": p.__dict__, "oracle_seconds": dt, "host_cpus": os.cpu_count()}
    with open(stem + ".json", "w") as f:
        json.dump(meta, f, indent=1)
    print(json.dumps(meta))


if __name__ == "__main__":
    main(sys.argv[1], int(sys.argv[2]) if len(sys.argv) > 2 else 0)
