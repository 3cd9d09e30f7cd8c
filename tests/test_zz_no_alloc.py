"""smsm_solve_noalloc: the IRLS solve run in the library's static device
scratch, called through the C ABI, against smsm_solve on the same inputs
(bit for bit: same kernels in the same order), on two calls in a row with the
second geometry smaller than the first; the FP64 oracle as well; geometries
whose workspace exceeds the scratch are rejected."""
import ctypes

import numpy as np
import pytest

import smsm_inputs as si
from oracle import smsm_oracle as o

pytestmark = pytest.mark.gpu

# first call: the 64 x 64 workload; second call: a smaller slice group
CASES = [
    (si.WORKLOADS["small"], 31, 1),
    (si.Geometry(n=32, n_slices=2, n_shots=2, n_coils=4, filt=3, lam=1e-3, n_irls=3, n_cg=4, phase_order=2,
                 snr=30.0), 32, 301),
]


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1901_01893_amd  # noqa: F401  (fails loudly if the library is missing)
    return torch, torch.device("cuda:0")


def noalloc(plan, y, x, torch):
    """smsm_solve_noalloc through the C ABI on the current stream."""
    from paper_1901_01893_amd import smsm
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return smsm.lib().smsm_solve_noalloc(plan._h, ctypes.c_void_p(y.data_ptr()), ctypes.c_void_p(x.data_ptr()), st)


def test_noalloc_solve_equals_solve_on_two_calls(torch_dev):
    torch, dev = torch_dev
    from paper_1901_01893_amd import smsm
    for k, (g, seed, wid) in enumerate(CASES):
        print(f"[noalloc] call {k}: n={g.n} L={g.n_slices} Ns={g.n_shots} Nc={g.n_coils} r={g.filt}", flush=True)
        case = si.make_case(g, seed, wid)
        _, y = o.simulate(case, g.n_slices, g.snr)
        y = y.astype(np.complex64)
        yd = torch.from_numpy(y).to(dev)
        p = smsm.make_params(lam=g.lam, n_irls=g.n_irls, n_cg=g.n_cg, flags=smsm.SMSM_FLAG_X_C128)
        coils = torch.from_numpy(case["coils"]).to(dev)
        with smsm.Plan(g.n, g.n, g.n_slices, g.n_shots, g.n_coils, g.filt, coils, case["masks"], case["shifts"],
                       p) as plan:
            assert plan.workspace_bytes() <= smsm.NOALLOC_SCRATCH_BYTES
            ref = plan.solve(yd).clone()
            x = torch.empty_like(ref)
            assert noalloc(plan, yd, x, torch) == smsm.SMSM_OK
            assert plan.status() == smsm.SMSM_OK
            assert torch.equal(x, ref), k
            # a repeat of the call allocates nothing (the first may map the module's globals)
            x2 = torch.empty_like(ref)
            torch.cuda.synchronize()
            free0 = torch.cuda.mem_get_info()[0]
            assert noalloc(plan, yd, x2, torch) == smsm.SMSM_OK
            torch.cuda.synchronize()
            assert torch.cuda.mem_get_info()[0] == free0
            assert torch.equal(x2, ref), k
            err = o.nrmse(x.cpu().numpy(), o.solve(y.astype(np.complex128), case["coils"], case["masks"],
                                                   case["shifts"], o.SolveParams(lam=g.lam, r=g.filt,
                                                                                 n_irls=g.n_irls, n_cg=g.n_cg)))
            print(f"[noalloc] call {k}: equal to smsm_solve, NRMSE vs oracle {err:.2e}", flush=True)
            assert err < 1e-11
            # the plan's own workspace was left alone: a plain solve still agrees
            assert torch.equal(plan.solve(yd), ref)


def test_noalloc_without_a_bound_workspace(torch_dev):
    torch, dev = torch_dev
    from paper_1901_01893_amd import smsm
    g, seed, wid = CASES[1]
    case = si.make_case(g, seed + 1, wid)
    _, y = o.simulate(case, g.n_slices, g.snr)
    yd = torch.from_numpy(y.astype(np.complex64)).to(dev)
    p = smsm.make_params(lam=g.lam, n_irls=g.n_irls, n_cg=g.n_cg, flags=smsm.SMSM_FLAG_X_C128)
    coils = torch.from_numpy(case["coils"]).to(dev)
    with smsm.Plan(g.n, g.n, g.n_slices, g.n_shots, g.n_coils, g.filt, coils, case["masks"], case["shifts"], p,
                   workspace=None) as plan:
        x = torch.empty(plan.shape_x, dtype=torch.complex128, device=dev)
        assert noalloc(plan, yd, x, torch) == smsm.SMSM_OK
        torch.cuda.synchronize()
        plan.set_workspace(torch.empty(plan.workspace_bytes(), dtype=torch.uint8, device=dev))
        assert torch.equal(x, plan.solve(yd))


def test_noalloc_rejects_a_workspace_above_the_scratch(torch_dev):
    torch, dev = torch_dev
    from paper_1901_01893_amd import smsm
    g = si.WORKLOADS["sg256"]
    case = si.make_case(g, 0, si.WORKLOAD_IDS["sg256"])
    coils = torch.from_numpy(case["coils"]).to(dev)
    with smsm.Plan(g.n, g.n, g.n_slices, g.n_shots, g.n_coils, g.filt, coils, case["masks"], case["shifts"],
                   smsm.make_params(lam=g.lam, n_irls=1, n_cg=1), workspace=None) as plan:
        assert plan.workspace_bytes() > smsm.NOALLOC_SCRATCH_BYTES
        y = torch.zeros(plan.shape_y, dtype=torch.complex64, device=dev)
        x = torch.empty(plan.shape_x, dtype=torch.complex64, device=dev)
        assert noalloc(plan, y, x, torch) == smsm.SMSM_E_SCRATCH
