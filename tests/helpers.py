"""Shared test helpers: seeded cases and tolerances."""
import numpy as np

import smsm_inputs as si
from oracle import smsm_oracle as o


def case_for(workload: str, seed: int = 0):
    """Generated ingredients + oracle-simulated data y (rounded to complex64)."""
    g = si.WORKLOADS[workload]
    case = si.make_case(g, seed, si.WORKLOAD_IDS[workload])
    x_true, y = o.simulate(case, g.n_slices, g.snr)
    return g, case, x_true, y.astype(np.complex64)


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def oracle_params(g, **kw):
    return o.SolveParams(lam=kw.get("lam", g.lam), r=g.filt, n_irls=kw.get("n_irls", g.n_irls),
                         n_cg=kw.get("n_cg", g.n_cg))
