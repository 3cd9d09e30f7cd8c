"""Batches of slice groups under one graph (smsm_batch_*): every solve of a
batch equals the plain solve of its plan bit for bit, on every replay, with
eager work between the replays, and the oracle's solve to 1e-10; a plan that
appears several times (several inputs of one slice group) runs its solves in
order."""
import numpy as np
import pytest

import smsm_inputs as si
from oracle import smsm_oracle as o

pytestmark = pytest.mark.gpu

# uneven geometries: fast column pass <16, 2>, generic column pass at 2 shots, one slice at 8 shots
GEOMS = [
    si.Geometry(n=64, n_slices=2, n_shots=4, n_coils=8, filt=5, lam=1e-3, n_irls=3, n_cg=4, phase_order=2, snr=30.0),
    si.Geometry(n=32, n_slices=2, n_shots=2, n_coils=4, filt=3, lam=1e-3, n_irls=3, n_cg=4, phase_order=2, snr=30.0),
    si.Geometry(n=64, n_slices=1, n_shots=8, n_coils=4, filt=2, lam=1e-3, n_irls=2, n_cg=3, phase_order=2, snr=30.0),
]


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1901_01893_amd  # noqa: F401  (fails loudly if the library is missing)
    return torch, torch.device("cuda:0")


ORACLE_TOL = 1e-10


def make_plan(torch, dev, g, seed):
    from paper_1901_01893_amd import smsm
    case = si.make_case(g, seed, 200 + seed)
    _, y = o.simulate(case, g.n_slices, g.snr)
    coils = torch.from_numpy(case["coils"]).to(dev)
    plan = smsm.Plan(g.n, g.n, g.n_slices, g.n_shots, g.n_coils, g.filt, coils, case["masks"], case["shifts"],
                     smsm.make_params(lam=g.lam, n_irls=g.n_irls, n_cg=g.n_cg, flags=smsm.SMSM_FLAG_X_C128))
    plan.case, plan.g = case, g
    return plan, torch.from_numpy(y.astype(np.complex64)).to(dev)


def oracle_of(plan, y):
    """The oracle's solve of the plan's geometry for the device input y."""
    g, case = plan.g, plan.case
    return o.solve(y.cpu().numpy().astype(np.complex128), case["coils"], case["masks"], case["shifts"],
                   o.SolveParams(lam=g.lam, r=g.filt, n_irls=g.n_irls, n_cg=g.n_cg))


def test_batch_matches_plain_solves_bitwise(torch_dev):
    torch, dev = torch_dev
    from paper_1901_01893_amd import smsm
    plans, ys, refs = [], [], []
    try:
        for k, g in enumerate(GEOMS):
            plan, y = make_plan(torch, dev, g, k)
            plans.append(plan)
            ys.append(y)
            refs.append(plan.solve(y).clone())
        torch.cuda.synchronize()
        oracles = [oracle_of(pl, y) for pl, y in zip(plans, ys)]
        xs = [torch.zeros_like(r) for r in refs]
        batch = smsm.Batch(plans, ys, xs, n_streams=2)
        try:
            for rep in range(3):
                print(f"[batch] replay {rep}", flush=True)
                for x in xs:
                    x.zero_()
                batch.launch()
                torch.cuda.synchronize()
                for k in range(len(plans)):
                    assert torch.equal(xs[k], refs[k]), (rep, k)
                    err = o.nrmse(xs[k].cpu().numpy(), oracles[k])
                    print(f"[batch] replay {rep} entry {k}: NRMSE vs oracle {err:.2e}", flush=True)
                    assert err < ORACLE_TOL, (rep, k, err)
                # eager work between the replays: a plain solve on one of the plans
                j = rep % len(plans)
                assert torch.equal(plans[j].solve(ys[j]), refs[j])
                torch.cuda.synchronize()
        finally:
            batch.close()
    finally:
        for plan in plans:
            plan.close()


def test_batch_runs_a_repeated_plan_in_order(torch_dev):
    # two inputs of one slice group (one plan) and a second group: the repeated
    # plan's solves share its scratch, so they run in order on one stream
    torch, dev = torch_dev
    from paper_1901_01893_amd import smsm
    plan_a, y_a = make_plan(torch, dev, GEOMS[1], 5)
    plan_b, y_b = make_plan(torch, dev, GEOMS[0], 6)
    try:
        y_a2 = (0.5 * y_a).contiguous()
        refs = [plan_a.solve(y_a).clone(), plan_b.solve(y_b).clone(), plan_a.solve(y_a2).clone()]
        torch.cuda.synchronize()
        oracles = [oracle_of(plan_a, y_a), oracle_of(plan_b, y_b), oracle_of(plan_a, y_a2)]
        xs = [torch.zeros_like(r) for r in refs]
        batch = smsm.Batch([plan_a, plan_b, plan_a], [y_a, y_b, y_a2], xs, n_streams=2)
        try:
            assert batch.n_streams == 2
            for rep in range(2):
                for x in xs:
                    x.zero_()
                batch.launch()
                torch.cuda.synchronize()
                for k in range(3):
                    assert torch.equal(xs[k], refs[k]), (rep, k)
                    assert o.nrmse(xs[k].cpu().numpy(), oracles[k]) < ORACLE_TOL, (rep, k)
        finally:
            batch.close()
    finally:
        plan_a.close()
        plan_b.close()


def test_autotuned_batch_matches_plain_solves(torch_dev):
    # n_streams = 0: the library times the candidate stream counts and keeps the fastest
    torch, dev = torch_dev
    from paper_1901_01893_amd import smsm
    plans, ys, refs = [], [], []
    try:
        for k, g in enumerate(GEOMS[:2]):
            plan, y = make_plan(torch, dev, g, 10 + k)
            plans.append(plan)
            ys.append(y)
            refs.append(plan.solve(y).clone())
        torch.cuda.synchronize()
        xs = [torch.zeros_like(r) for r in refs]
        batch = smsm.Batch(plans, ys, xs, n_streams=0)
        try:
            assert batch.n_streams in (1, 2)
            for x in xs:
                x.zero_()
            batch.launch()
            torch.cuda.synchronize()
            for k in range(len(plans)):
                assert torch.equal(xs[k], refs[k]), k
                assert o.nrmse(xs[k].cpu().numpy(), oracle_of(plans[k], ys[k])) < ORACLE_TOL, k
        finally:
            batch.close()
    finally:
        for plan in plans:
            plan.close()


def test_batch_of_many_directions_spans_several_graphs(torch_dev):
    # seven inputs of one slice group and two of another: the first plan has
    # more entries than one captured segment holds (five), so the batch runs
    # as two graphs in order; every output equals its plain solve bit for bit
    torch, dev = torch_dev
    from paper_1901_01893_amd import smsm
    plan_a, y_a = make_plan(torch, dev, GEOMS[1], 20)
    plan_b, y_b = make_plan(torch, dev, GEOMS[1], 21)
    try:
        ys = [(0.5 + 0.1 * k) * y_a for k in range(7)] + [y_b, 0.7 * y_b]
        plans = [plan_a] * 7 + [plan_b] * 2
        refs = [pl.solve(y).clone() for pl, y in zip(plans, ys)]
        torch.cuda.synchronize()
        xs = [torch.zeros_like(r) for r in refs]
        batch = smsm.Batch(plans, ys, xs, n_streams=2)
        try:
            for rep in range(2):
                for x in xs:
                    x.zero_()
                batch.launch()
                torch.cuda.synchronize()
                for k in range(len(plans)):
                    assert torch.equal(xs[k], refs[k]), (rep, k)
            assert o.nrmse(xs[6].cpu().numpy(), oracle_of(plan_a, ys[6])) < ORACLE_TOL
        finally:
            batch.close()
    finally:
        plan_a.close()
        plan_b.close()


def test_autotuned_launch_shapes_keep_oracle_parity(torch_dev):
    # smsm_plan_autotune on each benched kind of plan: the chosen shapes are
    # valid, the row shape alone leaves solves bit for bit the same, and the
    # tuned solves still match the oracle; a batch captured afterwards equals
    # the tuned plain solves bit for bit
    torch, dev = torch_dev
    from paper_1901_01893_amd import smsm
    plans, ys, refs = [], [], []
    try:
        for k, g in enumerate(GEOMS):
            plan, y = make_plan(torch, dev, g, 30 + k)
            x0 = plan.solve(y).clone()
            trw, xw = plan.autotune(5)
            print(f"[autotune] {g.n}x{g.n} Ns{g.n_shots}: rows per workgroup {trw}, columns per wave {xw}", flush=True)
            assert trw >= 1 and xw in (1, 2, 4)
            x1 = plan.solve(y)
            assert plan.status() == smsm.SMSM_OK
            err = o.nrmse(x1.cpu().numpy(), oracle_of(plan, y))
            assert err < ORACLE_TOL, (k, err)
            assert o.nrmse(x1.cpu().numpy(), x0.cpu().numpy()) < 1e-12
            plans.append(plan)
            ys.append(y)
            refs.append(x1.clone())
        xs = [torch.zeros_like(r) for r in refs]
        batch = smsm.Batch(plans, ys, xs, n_streams=2)
        try:
            batch.launch()
            torch.cuda.synchronize()
            for k in range(len(plans)):
                assert torch.equal(xs[k], refs[k]), k
        finally:
            batch.close()
    finally:
        for plan in plans:
            plan.close()

