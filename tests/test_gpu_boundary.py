"""The boundary on the GPU: the caller-owned workspace (smsm_workspace_bytes,
smsm_set_workspace) and every flat name of the binding, each called once."""
import numpy as np
import pytest

import smsm_inputs as si
from oracle import smsm_oracle as o
from tests.helpers import case_for, oracle_params

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1901_01893_amd  # noqa: F401  (fails loudly if the library is missing)
    return torch, torch.device("cuda:0")


def to_dev(torch, dev, a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def test_solve_in_a_caller_owned_workspace(torch_dev):
    torch, dev = torch_dev
    from paper_1901_01893_amd import smsm
    g, case, _, y = case_for("small", 11)
    p = smsm.make_params(lam=g.lam, n_irls=g.n_irls, n_cg=g.n_cg, flags=smsm.SMSM_FLAG_X_C128)
    coils = to_dev(torch, dev, case["coils"])
    plan = smsm.Plan(g.n, g.n, g.n_slices, g.n_shots, g.n_coils, g.filt, coils, case["masks"], case["shifts"], p,
                     workspace=None)
    try:
        yd = to_dev(torch, dev, y)
        nbytes = plan.workspace_bytes()
        print(f"[workspace] plan {plan.device_bytes()} B, workspace {nbytes} B", flush=True)
        assert nbytes > 0 and nbytes % 256 == 0
        with pytest.raises(smsm.SmsmError) as e:          # no workspace bound yet
            plan.solve(yd)
        assert e.value.status == smsm.SMSM_E_INVALID
        short = torch.empty(nbytes - 256, dtype=torch.uint8, device=dev)
        with pytest.raises(smsm.SmsmError):
            plan.set_workspace(short)
        big = torch.empty(nbytes + 512, dtype=torch.uint8, device=dev)
        with pytest.raises(smsm.SmsmError):
            plan.set_workspace(big[1:])                    # not 256-byte aligned
        ws1 = torch.full((nbytes,), 0x7f, dtype=torch.uint8, device=dev)   # arbitrary prior contents
        plan.set_workspace(ws1)
        out = torch.empty(plan.shape_x, dtype=torch.complex128, device=dev)
        plan.solve(yd, out)                                # first launches load code, spill space
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        plan.solve(yd, out)
        torch.cuda.synchronize()
        assert torch.cuda.mem_get_info()[0] == free0       # nothing allocated on the solve path
        x1 = out.cpu().numpy()
        assert plan.status() == smsm.SMSM_OK
        ref = o.solve(y.astype(np.complex128), case["coils"], case["masks"], case["shifts"], oracle_params(g))
        err = o.nrmse(x1, ref)
        print(f"[workspace] NRMSE vs oracle {err:.2e}", flush=True)
        assert err < 1e-11
        ws2 = torch.zeros(nbytes, dtype=torch.uint8, device=dev)
        plan.set_workspace(ws2)
        x2 = plan.solve(yd).cpu().numpy()
        assert np.array_equal(x1, x2)                       # another workspace: bitwise the same
        plan.set_workspace(None)
        with pytest.raises(smsm.SmsmError):
            plan.solve(yd)
    finally:
        plan.close()


def test_every_flat_binding_once(torch_dev):
    """Each flat name of the binding (the C ABI's names) runs once on a small plan."""
    torch, dev = torch_dev
    from paper_1901_01893_amd import smsm
    g, case, _, y = case_for("small", 12)
    coils = to_dev(torch, dev, case["coils"])
    p = smsm.make_params(lam=g.lam, n_irls=2, n_cg=2, flags=smsm.SMSM_FLAG_X_C128)
    called = set()

    def call(name, *a, **k):
        called.add(name)
        return getattr(smsm, name)(*a, **k)

    plan = call("smsm_plan_create", g.n, g.n, g.n_slices, g.n_shots, g.n_coils, g.filt, coils, case["masks"],
                case["shifts"], p, workspace=None)
    ws = torch.empty(call("smsm_workspace_bytes", plan), dtype=torch.uint8, device=dev)
    call("smsm_set_workspace", plan, ws)
    assert call("smsm_plan_device_bytes", plan) > 0
    call("smsm_plan_set_params", plan, p)
    trw, xw = call("smsm_plan_autotune", plan, 3)
    assert trw >= 1 and xw in (1, 2, 4)
    yd = to_dev(torch, dev, y)
    x = call("smsm_solve", plan, yd)
    assert call("smsm_plan_status", plan) == smsm.SMSM_OK
    assert torch.equal(call("smsm_solve_noalloc", plan, yd, torch.empty_like(x)), x)
    assert call("smsm_status_string", smsm.SMSM_E_NUMERIC)
    ya = call("smsm_apply_A", plan, x)
    assert ya.shape == plan.shape_y
    call("smsm_apply_AH", plan, yd)
    call("smsm_apply_AHA", plan, x)
    G = call("smsm_gram", plan, x)
    lm = call("smsm_lambda_max", plan, G).cpu().numpy()
    W = call("smsm_weights", plan, G, 0.01 * lm)
    call("smsm_set_weights", plan, W)
    call("smsm_apply_reg", plan, x)
    call("smsm_apply_normal", plan, x)
    img = call("smsm_images_sos", plan, x)
    assert img.shape == (g.n_slices, g.n, g.n)
    call("smsm_kernel_timer_start", plan, "col_normal", 4, 1)
    call("smsm_launch_kernel", plan, "col_normal", 2)
    ms, n = call("smsm_kernel_timer_read", plan)
    assert n == 2 and ms > 0
    call("smsm_kernel_timer_start", plan, "col_normal", 0, 1)
    f, b = call("smsm_kernel_cost", plan, "col_normal")
    assert f > 0 and b > 0
    xb = torch.empty_like(x)
    batch = call("smsm_batch_create", [plan], [yd], [xb], 1)
    assert call("smsm_batch_streams", batch) == 1
    call("smsm_batch_launch", batch)
    torch.cuda.synchronize()
    assert torch.equal(xb, call("smsm_solve", plan, yd))
    call("smsm_batch_destroy", batch)
    net = call("smsm_learned_create", plan, si.cnn_init(3, 2 * g.n_shots, width=8), 8, 1, 2, 0.05)
    flat = call("smsm_learned_get_params", net)
    assert flat.size == call("smsm_learned_param_count", net)
    call("smsm_learned_set_params", net, flat)
    call("smsm_learned_set_bf16", net, False)
    inp = torch.randn(net.shape_c, dtype=torch.float32, device=dev)
    out = call("smsm_learned_cnn_forward", net, inp)
    call("smsm_learned_cnn_backward", net, inp, torch.ones_like(out))
    xl = call("smsm_learned_solve", net, yd)
    call("smsm_learned_gradients", net, yd, xl)
    call("smsm_learned_train_step", net, yd, xl, 1e-4)
    assert call("smsm_learned_residual", net, xl, yd) >= 0.0
    xf, fell, r_l, r_p = call("smsm_learned_solve_fallback", net, yd, 1.5)
    assert r_l > 0 and r_p > 0 and fell == (r_l > 1.5 * r_p)
    call("smsm_learned_destroy", net)
    solver = call("smsm_al_create", plan, 1e-3, 1e-4, 2, 2)
    assert call("smsm_al_device_bytes", solver) > 0
    assert call("smsm_al_dual_stride", solver) >= solver.n_anchor
    xa = call("smsm_al_solve", solver, yd)
    assert xa.shape == plan.shape_x
    assert call("smsm_al_dual", solver).shape == solver.shape_dual
    call("smsm_al_destroy", solver)
    call("smsm_plan_destroy", plan)
    assert called == set(smsm.ABI_SYMBOLS), set(smsm.ABI_SYMBOLS) - called
