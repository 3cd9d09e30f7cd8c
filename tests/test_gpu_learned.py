"""GPU parity of the learned unrolled solver (smsm_learned_*) against the FP64
oracle in oracle/learned_oracle.py, and what training the network gains.

The network runs in FP32 (weights and accumulation), so its outputs and
gradients are held to FP32-sized relative errors; the data-consistency
solves run in FP64."""
import numpy as np
import pytest

import smsm_inputs as si
from oracle import learned_oracle as lo
from oracle import smsm_oracle as o
from tests.helpers import rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1901_01893_amd  # noqa: F401  (fails loudly if the library is missing)
    return torch, torch.device("cuda:0")


def make_case(g, seed, wid):
    case = si.make_case(g, seed, wid)
    x_true, y = o.simulate(case, g.n_slices, g.snr)
    return case, x_true, y.astype(np.complex64)


def plan_for(torch, dev, g, case, params=None):
    from paper_1901_01893_amd import smsm
    coils = torch.from_numpy(case["coils"]).to(dev)
    if params is None:
        params = smsm.make_params(lam=g.lam, n_irls=g.n_irls, n_cg=g.n_cg, flags=smsm.SMSM_FLAG_X_C128)
    return smsm.Plan(g.n, g.n, g.n_slices, g.n_shots, g.n_coils, g.filt, coils, case["masks"], case["shifts"],
                     params)


def oracle_aha(case):
    coils = case["coils"].astype(np.complex128)
    masks = case["masks"].astype(np.float64)
    theta = o.caipi_phase(case["coils"].shape[-2], case["shifts"])
    return lambda v: o.adjoint(o.forward(v, coils, masks, theta), coils, masks, theta), (coils, masks, theta)


def f64_params(params):
    return [(w.astype(np.float64), b.astype(np.float64)) for w, b in params]


# 32 x 32 is the smallest matrix with 4 shots (folded length n / Ns >= 8)
G32 = si.Geometry(n=32, n_slices=2, n_shots=4, n_coils=4, filt=3, lam=1e-3, n_irls=4, n_cg=6, phase_order=2,
                  snr=30.0)


def test_cnn_forward_backward_match_oracle(torch_dev):
    """Width 64 (the configured network) on a 32 x 32 slice group."""
    torch, dev = torch_dev
    from paper_1901_01893_amd import smsm
    case, _, _ = make_case(G32, 0, 90)
    params = si.cnn_init(3, 8, width=64, out_scale=1.0)
    print("[learned] cnn fwd/bwd width 64, 32x32, L=2, Ns=4", flush=True)
    with plan_for(torch, dev, G32, case) as plan, smsm.Learned(plan, params, width=64) as net:
        rng = np.random.default_rng(5)
        inp = rng.standard_normal(net.shape_c).astype(np.float32)
        gout = rng.standard_normal(net.shape_c).astype(np.float32)
        out = net.cnn_forward(torch.from_numpy(inp).to(dev)).cpu().numpy()
        gin, grads = net.cnn_backward(torch.from_numpy(inp).to(dev), torch.from_numpy(gout).to(dev))
        p64 = f64_params(params)
        ref, acts = lo.cnn_forward(inp.astype(np.float64), p64)
        assert rel(out, ref) < 1e-5
        rgin, rgrads = lo.cnn_backward(acts, p64, gout.astype(np.float64))
        assert rel(gin.cpu().numpy(), rgin) < 1e-5
        got = smsm.unflatten_params(grads, 8, 64)
        for k in range(5):
            assert rel(got[k][0], rgrads[k][0]) < 1e-5, k
            assert rel(got[k][1], rgrads[k][1]) < 1e-5, k


def test_unrolled_solve_and_residual_match_oracle(torch_dev):
    torch, dev = torch_dev
    from paper_1901_01893_amd import smsm
    case, _, y = make_case(G32, 1, 91)
    params = si.cnn_init(4, 8, width=16, out_scale=0.5)
    aha, (coils, masks, theta) = oracle_aha(case)
    b = o.adjoint(y.astype(np.complex128), coils, masks, theta)
    ref, _ = lo.unrolled_forward(b, aha, f64_params(params), mu=0.5, n_unroll=5, n_cg=10)
    print("[learned] unrolled solve width 16, 32x32, 5 x 10 CG", flush=True)
    with plan_for(torch, dev, G32, case) as plan, \
            smsm.Learned(plan, params, width=16, n_unroll=5, n_cg=10, mu=0.5) as net:
        yd = torch.from_numpy(y).to(dev)
        x = net.solve(yd)
        got = x.cpu().numpy()
        err = o.nrmse(got, ref)
        print(f"[learned] NRMSE vs oracle = {err:.3e}", flush=True)
        assert err < 1e-5
        res = net.residual(x, yd)
        ref_res = np.linalg.norm((o.forward(got, coils, masks, theta) - y.astype(np.complex128)).ravel())
        assert abs(res - ref_res) < 1e-10 * ref_res


def test_unrolled_gradients_match_oracle(torch_dev):
    torch, dev = torch_dev
    from paper_1901_01893_amd import smsm
    case, x_true, y = make_case(G32, 2, 92)
    params = si.cnn_init(5, 8, width=16, out_scale=0.5)
    aha, (coils, masks, theta) = oracle_aha(case)
    b = o.adjoint(y.astype(np.complex128), coils, masks, theta)
    target = x_true
    loss_ref, grads_ref = lo.unrolled_loss_and_grads(b, aha, f64_params(params), 0.8, 3, 8, target)
    print("[learned] gradients width 16, 32x32, 3 x 8 CG", flush=True)
    with plan_for(torch, dev, G32, case) as plan, \
            smsm.Learned(plan, params, width=16, n_unroll=3, n_cg=8, mu=0.8) as net:
        loss, grads = net.gradients(torch.from_numpy(y).to(dev), torch.from_numpy(target).to(dev))
        assert abs(loss - loss_ref) < 1e-5 * loss_ref
        got = smsm.unflatten_params(grads, 8, 16)
        for k in range(5):
            assert rel(got[k][0], grads_ref[k][0]) < 1e-4, k
            assert rel(got[k][1], grads_ref[k][1]) < 1e-4, k
        # the parameters did not move
        assert np.array_equal(net.get_params(), smsm.flatten_params(params))


def test_training_gains_over_the_iterations_without_the_network(torch_dev):
    """Train the width-64 network on the GPU (own forward, backward and Adam
    kernels) against the plain solver's reconstructions of 32 seeded
    instances of the small workload (64 x 64, MB = 2, 4 shots, 8 coils), then
    compare on 4 held-out seeds with the same unrolled data-consistency
    iterations run without the network (C = 0)."""
    torch, dev = torch_dev
    from paper_1901_01893_amd import smsm
    g = si.WORKLOADS["small"]
    n_train, n_eval, steps, mu, lr = 32, 4, 600, 0.05, 1e-3
    case0 = si.make_case(g, 0, 40)
    coils = torch.from_numpy(case0["coils"]).to(dev)
    with smsm.Plan(g.n, g.n, g.n_slices, g.n_shots, g.n_coils, g.filt, coils, case0["masks"], case0["shifts"],
                   smsm.make_params(lam=g.lam, n_irls=g.n_irls, n_cg=g.n_cg,
                                    flags=smsm.SMSM_FLAG_X_C128)) as plan:
        data = []
        for s in range(n_train + n_eval):
            case = si.make_case(g, s, 40)
            assert np.array_equal(case["coils"], case0["coils"])     # one coil set per workload
            _, y = o.simulate(case, g.n_slices, g.snr)
            yd = torch.from_numpy(y.astype(np.complex64)).to(dev)
            data.append((yd, plan.solve(yd)))
        params = si.cnn_init(1, 2 * g.n_shots, width=64, out_scale=0.1)
        zero = [(np.zeros_like(w), np.zeros_like(b)) for w, b in params]
        with smsm.Learned(plan, params, width=64, n_unroll=5, n_cg=10, mu=mu) as net, \
                smsm.Learned(plan, zero, width=64, n_unroll=5, n_cg=10, mu=mu) as net0:
            def held_out(n):
                return float(np.mean([float(torch.linalg.vector_norm(n.solve(yd) - xt) /
                                            torch.linalg.vector_norm(xt)) for yd, xt in data[n_train:]]))
            e_dc = held_out(net0)
            losses = [net.train_step(*data[k % n_train], lr) for k in range(steps)]
            e_tr = held_out(net)
            first, last = np.mean(losses[:50]), np.mean(losses[-50:])
            print(f"[learned] training loss {first:.3e} -> {last:.3e}; held-out error vs plain solver: "
                  f"without the network {e_dc:.4f}, trained {e_tr:.4f}", flush=True)
            assert last < 0.5 * first
            assert e_tr < 0.95 * e_dc
            # the fallback test of a caller: the data-consistency residual of the
            # learned output against the plain solver's
            yd, xt = data[n_train]
            r_l, r_p = net.residual(net.solve(yd), yd), net.residual(xt, yd)
            print(f"[learned] residual learned / plain = {r_l / r_p:.3f}", flush=True)
            assert np.isfinite(r_l) and r_p > 0


def test_zero_data_gives_exactly_zero(torch_dev):
    """y = 0: A^H y = 0 and the data scale s = 0, so the prior's term s C(.)
    vanishes and x = 0 solves every data-consistency step exactly."""
    torch, dev = torch_dev
    from paper_1901_01893_amd import smsm
    case, _, y = make_case(G32, 3, 93)
    params = [(w, np.full_like(b, 0.1)) for w, b in si.cnn_init(6, 8, width=16)]
    with plan_for(torch, dev, G32, case) as plan, smsm.Learned(plan, params, width=16, n_unroll=2, n_cg=4) as net:
        x = net.solve(torch.zeros(plan.shape_y, dtype=torch.complex64, device=dev)).cpu().numpy()
    assert np.all(x == 0)


def test_cnn_two_shots_matches_oracle(torch_dev):
    """Two shots (4 channels in and out): the 4-channel convolution instances
    and the per-channel-pair weight-gradient kernel of the first and last
    layers."""
    torch, dev = torch_dev
    from paper_1901_01893_amd import smsm
    g = si.Geometry(n=32, n_slices=2, n_shots=2, n_coils=4, filt=3, lam=1e-3, n_irls=2, n_cg=3, phase_order=2,
                    snr=30.0)
    case, _, _ = make_case(g, 4, 94)
    params = si.cnn_init(7, 4, width=16, out_scale=1.0)
    with plan_for(torch, dev, g, case) as plan, smsm.Learned(plan, params, width=16) as net:
        rng = np.random.default_rng(8)
        inp = rng.standard_normal(net.shape_c).astype(np.float32)
        gout = rng.standard_normal(net.shape_c).astype(np.float32)
        out = net.cnn_forward(torch.from_numpy(inp).to(dev)).cpu().numpy()
        gin, grads = net.cnn_backward(torch.from_numpy(inp).to(dev), torch.from_numpy(gout).to(dev))
        p64 = f64_params(params)
        ref, acts = lo.cnn_forward(inp.astype(np.float64), p64)
        assert rel(out, ref) < 1e-5
        rgin, rgrads = lo.cnn_backward(acts, p64, gout.astype(np.float64))
        assert rel(gin.cpu().numpy(), rgin) < 1e-5
        got = smsm.unflatten_params(grads, 4, 16)
        for k in range(5):
            assert rel(got[k][0], rgrads[k][0]) < 1e-5, k
            assert rel(got[k][1], rgrads[k][1]) < 1e-5, k


def test_bf16_weights_match_oracle(torch_dev):
    """BF16 weights (rounded to nearest even), FP32 accumulation: network
    outputs and gradients, and the unrolled gradients, against the oracle
    run on the same rounded weights."""
    torch, dev = torch_dev
    from paper_1901_01893_amd import smsm
    case, x_true, y = make_case(G32, 5, 95)
    params = si.cnn_init(9, 8, width=64, out_scale=1.0)
    pb = lo.bf16_params(params)
    with plan_for(torch, dev, G32, case) as plan, smsm.Learned(plan, params, width=64, n_unroll=3, n_cg=8,
                                                              mu=0.8) as net:
        net.set_bf16(True)
        rng = np.random.default_rng(9)
        inp = rng.standard_normal(net.shape_c).astype(np.float32)
        gout = rng.standard_normal(net.shape_c).astype(np.float32)
        out = net.cnn_forward(torch.from_numpy(inp).to(dev)).cpu().numpy()
        gin, grads = net.cnn_backward(torch.from_numpy(inp).to(dev), torch.from_numpy(gout).to(dev))
        ref, acts = lo.cnn_forward(inp.astype(np.float64), pb)
        assert rel(out, ref) < 1e-5
        assert rel(out, lo.cnn_forward(inp.astype(np.float64), f64_params(params))[0]) > 1e-4   # rounding is real
        rgin, rgrads = lo.cnn_backward(acts, pb, gout.astype(np.float64))
        assert rel(gin.cpu().numpy(), rgin) < 1e-5
        got = smsm.unflatten_params(grads, 8, 64)
        for k in range(5):
            assert rel(got[k][0], rgrads[k][0]) < 1e-5, k
        aha, (coils, masks, theta) = oracle_aha(case)
        b = o.adjoint(y.astype(np.complex128), coils, masks, theta)
        loss_ref, grads_ref = lo.unrolled_loss_and_grads(b, aha, pb, 0.8, 3, 8, x_true)
        loss, grads = net.gradients(torch.from_numpy(y).to(dev), torch.from_numpy(x_true).to(dev))
        assert abs(loss - loss_ref) < 1e-5 * loss_ref
        got = smsm.unflatten_params(grads, 8, 64)
        for k in range(5):
            assert rel(got[k][0], grads_ref[k][0]) < 1e-4, k
            assert rel(got[k][1], grads_ref[k][1]) < 1e-4, k


def test_bf16_network_is_exact_on_bf16_values(torch_dev):
    """The BF16 network on a network whose activations and gradients are
    all short dyadic numbers (each output channel reads one input channel at
    one tap with weight +-1; integer inputs and output gradients): every
    rounding is forced, so output, input gradient and parameter gradients
    equal the oracle's bit for bit."""
    torch, dev = torch_dev
    from paper_1901_01893_amd import smsm
    from tests.test_oracle_learned_pins import bf16_exact_network
    case, _, _ = make_case(G32, 7, 98)
    params = [(w.astype(np.float32), b.astype(np.float32)) for w, b in bf16_exact_network(31)]
    with plan_for(torch, dev, G32, case) as plan, smsm.Learned(plan, params, width=8, n_unroll=1, n_cg=1,
                                                              mu=0.5) as net:
        net.set_bf16(2)
        rng = np.random.default_rng(13)
        inp = rng.integers(-4, 5, size=net.shape_c).astype(np.float32)
        gout = rng.integers(-3, 4, size=net.shape_c).astype(np.float32)
        out = net.cnn_forward(torch.from_numpy(inp).to(dev)).cpu().numpy()
        gin, grads = net.cnn_backward(torch.from_numpy(inp).to(dev), torch.from_numpy(gout).to(dev))
        p64 = f64_params(params)
        ref, acts = lo.cnn_forward(inp.astype(np.float64), p64, act_bf16=True)
        rgin, rgrads = lo.cnn_backward(acts, p64, gout.astype(np.float64), act_bf16=True)
        assert np.array_equal(out, ref)
        assert np.array_equal(gin.cpu().numpy(), rgin)
        got = smsm.unflatten_params(grads, 8, 8)
        for k in range(5):
            assert np.array_equal(got[k][0], rgrads[k][0]) and np.array_equal(got[k][1], rgrads[k][1]), k


def test_bf16_network_weight_gradients_are_fp32_accurate(torch_dev):
    """The forced-rounding network with FP32 output gradients that are not
    BF16 values: every layer's weight and bias gradients come from the same
    BF16 activations and the same gradients on both sides (each backward-data
    sum has one term), so the matrix-core weight gradients (the FP32 gradient
    in three BF16 parts, exact products, FP32 sums) must match the FP64 oracle
    to FP32 accumulation accuracy (a part dropped from the split would be off
    by 2^-9 or 2^-17); the input gradient stays exact."""
    torch, dev = torch_dev
    from paper_1901_01893_amd import smsm
    from tests.test_oracle_learned_pins import bf16_exact_network
    case, _, _ = make_case(G32, 7, 98)
    params = [(w.astype(np.float32), b.astype(np.float32)) for w, b in bf16_exact_network(32)]
    with plan_for(torch, dev, G32, case) as plan, smsm.Learned(plan, params, width=8, n_unroll=1, n_cg=1,
                                                              mu=0.5) as net:
        net.set_bf16(2)
        rng = np.random.default_rng(14)
        inp = rng.integers(-4, 5, size=net.shape_c).astype(np.float32)
        gout = rng.standard_normal(net.shape_c).astype(np.float32)
        gin, grads = net.cnn_backward(torch.from_numpy(inp).to(dev), torch.from_numpy(gout).to(dev))
        p64 = f64_params(params)
        _, acts = lo.cnn_forward(inp.astype(np.float64), p64, act_bf16=True)
        rgin, rgrads = lo.cnn_backward(acts, p64, gout.astype(np.float64), act_bf16=True)
        assert np.array_equal(gin.cpu().numpy(), rgin)
        got = smsm.unflatten_params(grads, 8, 8)
        errs = [(rel(got[k][0], rgrads[k][0]), rel(got[k][1], rgrads[k][1])) for k in range(5)]
        print(f"[bf16 wgrad] per-layer relative errors (weights, biases): {errs}", flush=True)
        for k in range(5):
            assert errs[k][0] < 2e-5 and errs[k][1] < 2e-5, (k, errs[k])


# The BF16 network rounds every hidden activation to BF16: the GPU forms it by
# FP32 accumulation in the matrix cores' order, the oracle in FP64, so a
# fraction of about sqrt(K) 2^-24 / 2^-8 (4e-4 at K = 576 terms) of the
# activations round to the neighbouring BF16 value, each moving by 2^-8;
# through four hidden layers that is ~2e-4 in norm (measured 2.2e-4).  The
# backward pass rounds the gradient entering each of its five convolutions
# as well and passes the differing ReLU masks on, about ten times that
# (measured 2.6e-3).  Both sides' roundings are correct roundings of nearly
# equal values; the exact test above fixes the structure bit for bit.
BF16NET_TOL = 5e-4
BF16NET_GRAD_TOL = 5e-3
# Unrolled through three data-consistency iterations the first layer's
# weight gradient gathers every flip upstream (measured 1.5e-2).
BF16NET_UNROLL_TOL = 5e-2


def test_bf16_network_matches_oracle(torch_dev):
    """The BF16 network (every convolution input rounded to BF16, one BF16
    product per term on the matrix cores): outputs and gradients of the
    width-64 network, and the unrolled loss and gradients, against the
    oracle's BF16 network on the same rounded weights (tolerances above)."""
    torch, dev = torch_dev
    from paper_1901_01893_amd import smsm
    case, x_true, y = make_case(G32, 6, 97)
    params = si.cnn_init(10, 8, width=64, out_scale=1.0)
    pb = lo.bf16_params(params)
    with plan_for(torch, dev, G32, case) as plan, smsm.Learned(plan, params, width=64, n_unroll=3, n_cg=8,
                                                              mu=0.8) as net:
        net.set_bf16(2)
        rng = np.random.default_rng(10)
        inp = rng.standard_normal(net.shape_c).astype(np.float32)
        gout = rng.standard_normal(net.shape_c).astype(np.float32)
        out = net.cnn_forward(torch.from_numpy(inp).to(dev)).cpu().numpy()
        gin, grads = net.cnn_backward(torch.from_numpy(inp).to(dev), torch.from_numpy(gout).to(dev))
        ref, acts = lo.cnn_forward(inp.astype(np.float64), pb, act_bf16=True)
        rgin, rgrads = lo.cnn_backward(acts, pb, gout.astype(np.float64), act_bf16=True)
        print(f"[bf16 network] out {rel(out, ref):.2e} gin {rel(gin.cpu().numpy(), rgin):.2e}", flush=True)
        assert rel(out, ref) < BF16NET_TOL
        assert rel(out, lo.cnn_forward(inp.astype(np.float64), pb)[0]) > 4 * BF16NET_TOL   # the rounding is real
        assert rel(gin.cpu().numpy(), rgin) < BF16NET_GRAD_TOL
        got = smsm.unflatten_params(grads, 8, 64)
        for k in range(5):
            assert rel(got[k][0], rgrads[k][0]) < BF16NET_GRAD_TOL, k
            assert rel(got[k][1], rgrads[k][1]) < BF16NET_GRAD_TOL, k
        aha, (coils, masks, theta) = oracle_aha(case)
        b = o.adjoint(y.astype(np.complex128), coils, masks, theta)
        loss_ref, grads_ref = lo.unrolled_loss_and_grads(b, aha, pb, 0.8, 3, 8, x_true, act_bf16=True)
        loss, grads = net.gradients(torch.from_numpy(y).to(dev), torch.from_numpy(x_true).to(dev))
        print(f"[bf16 network] loss {abs(loss - loss_ref) / loss_ref:.2e}", flush=True)
        assert abs(loss - loss_ref) < BF16NET_TOL * loss_ref
        got = smsm.unflatten_params(grads, 8, 64)
        errs = [(rel(got[k][0], grads_ref[k][0]), rel(got[k][1], grads_ref[k][1])) for k in range(5)]
        print("[bf16 network] unrolled gradients " + " ".join(f"{a:.1e}/{b:.1e}" for a, b in errs), flush=True)
        for k, (ew, eb) in enumerate(errs):
            assert ew < BF16NET_UNROLL_TOL and eb < BF16NET_UNROLL_TOL, k


@pytest.mark.parametrize("bf16", [0, 1, 2])
def test_cnn_wide_images_match_oracle(torch_dev, bf16):
    """256-wide images (the workload's width: the weight-gradient kernel's
    two-row chunks and 258-wide halo staging, four 64-column tiles of the
    matrix-core convolution), one slice, 8-channel layers: outputs, input
    gradient and parameter gradients against the oracle, FP32 and BF16 weights."""
    torch, dev = torch_dev
    from paper_1901_01893_amd import smsm
    g = si.Geometry(n=256, n_slices=1, n_shots=4, n_coils=2, filt=3, lam=1e-3, n_irls=1, n_cg=1, phase_order=2,
                    snr=30.0)
    case = si.make_case(g, 1, 96)
    params = si.cnn_init(11, 8, width=8, out_scale=1.0)
    ref_params = lo.bf16_params(params) if bf16 else f64_params(params)
    act_bf16 = bf16 == 2
    with plan_for(torch, dev, g, case) as plan, smsm.Learned(plan, params, width=8, n_unroll=1, n_cg=1,
                                                             mu=0.5) as net:
        net.set_bf16(bf16)
        rng = np.random.default_rng(12)
        inp = rng.standard_normal(net.shape_c).astype(np.float32)
        gout = rng.standard_normal(net.shape_c).astype(np.float32)
        out = net.cnn_forward(torch.from_numpy(inp).to(dev)).cpu().numpy()
        gin, grads = net.cnn_backward(torch.from_numpy(inp).to(dev), torch.from_numpy(gout).to(dev))
        ref, acts = lo.cnn_forward(inp.astype(np.float64), ref_params, act_bf16)
        rgin, rgrads = lo.cnn_backward(acts, ref_params, gout.astype(np.float64), act_bf16)
        print(f"[cnn 256 wide bf16={bf16}] out {rel(out, ref):.2e} gin {rel(gin.cpu().numpy(), rgin):.2e}",
              flush=True)
        tol = BF16NET_GRAD_TOL if act_bf16 else 1e-5
        assert rel(out, ref) < (BF16NET_TOL if act_bf16 else 1e-5)
        assert rel(gin.cpu().numpy(), rgin) < tol
        got = smsm.unflatten_params(grads, 8, 8)
        for k in range(5):
            assert rel(got[k][0], rgrads[k][0]) < tol, k
            assert rel(got[k][1], rgrads[k][1]) < tol, k


def test_fallback_to_the_plain_solver_both_branches(torch_dev):
    """smsm_learned_solve_fallback: with a ratio no residual can meet the
    output is the plain IRLS solve (bit for bit), with one every residual
    meets it is the learned solve; the residuals are those of the outputs."""
    torch, dev = torch_dev
    from paper_1901_01893_amd import smsm
    case, _, y = make_case(G32, 8, 99)
    yd = torch.from_numpy(y).to(dev)
    with plan_for(torch, dev, G32, case) as plan, smsm.Learned(plan, si.cnn_init(4, 8, width=8), width=8,
                                                              n_unroll=2, n_cg=4, mu=0.5) as net:
        x_plain = plan.solve(yd)                   # complex128 output (the plan's flag)
        x_learned = net.solve(yd)
        torch.cuda.synchronize()
        x, fell, r_l, r_p = net.solve_fallback(yd, ratio=1e-9)
        assert fell and torch.equal(x, x_plain)
        assert abs(r_l - net.residual(x_learned, yd)) <= 1e-12 * r_l
        assert abs(r_p - net.residual(x_plain, yd)) <= 1e-12 * r_p
        x, fell, r_l2, _ = net.solve_fallback(yd, ratio=1e9)
        assert not fell and torch.equal(x, x_learned) and r_l2 == r_l
        # a caller's reference residual replaces the plain solve's
        x, fell, _, r_ref = net.solve_fallback(yd, ratio=1.5, res_ref=0.5 * r_l)
        assert fell and r_ref == 0.5 * r_l and torch.equal(x, x_plain)
