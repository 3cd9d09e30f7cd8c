"""Throughput of the SMS-MUSSELS IRLS solve on one MI355X.

One step = one complete IRLS solve of one slice group (A^H y, Gram, weights,
n_irls x (n_cg + 1) normal-operator applications with CG updates) on the
realistic workload: 256x256, MB=3 slices, 4 interleaved shots, 32 coils,
7x7 Hankel filter, lambda = 1e-3, 15 IRLS x 15 CG.  Inputs are synthetic
(seeded phantom, shot phases and coil maps), resident in HBM before timing.

Prints one JSON line.  Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_VALU_TFLOPS = 78.6   # 256 CU x 64 lanes x 2 (FMA) x 2.4 GHz
HBM_TBS = 8.0
COPY_BYTES = 256 << 20    # calibration copy: 256 MiB read + 256 MiB written


def centred_fft2(u):
    """Input synthesis only: k-space of the synthetic truth images."""
    ax = (-2, -1)
    return np.fft.fftshift(np.fft.fft2(np.fft.ifftshift(u, axes=ax), norm="ortho"), axes=ax)


def synth_inputs(torch, dev, plan, g, case, n_draws=1):
    """y = A x_true + noise, with A applied by the library itself.  The first
    draw uses the case's noise; further draws (distinct noise realisations of
    the same acquisition, seeded) give the timed loop distinct inputs."""
    m = case["rho"].astype(np.float64)[:, None] * case["phase"].astype(np.complex128)
    x_true = torch.from_numpy(centred_fft2(m)).to(dev)
    clean = plan.apply_A(x_true)
    torch.cuda.synchronize()
    mask = torch.from_numpy(case["masks"].astype(np.float64)).to(dev)[:, None, :, None]
    acquired = mask.expand_as(clean.real) > 0
    rms = torch.sqrt(torch.mean(torch.abs(clean[acquired]) ** 2)).item()
    ys = []
    for d in range(n_draws):
        if d == 0:
            noise = torch.from_numpy(case["noise"].astype(np.complex128)).to(dev)
        else:
            rng = np.random.default_rng([9000, d])
            shape = tuple(clean.shape)
            noise = torch.from_numpy((rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / np.sqrt(2)).to(dev)
        ys.append((clean + mask * (rms / g.snr) * noise).to(torch.complex64).contiguous())
    return ys


# Batched form: ten uneven slice groups (32 coils, 15 x 15 iterations) of
# matrix sizes {192, 224, 256}, shots {2, 4, 8}, MB {2, 3}; (n, MB, shots,
# filter).  8 shots take a filter of at most 5 x 5.
BATCH_GEOMS = ((256, 3, 4, 7), (256, 2, 2, 7), (256, 3, 2, 7), (256, 2, 8, 5),
               (224, 3, 4, 7), (224, 2, 2, 7), (224, 2, 8, 5),
               (192, 3, 4, 7), (192, 2, 8, 5), (192, 3, 2, 7))


def direction_truth(g, case, d, wid):
    """Host half of one diffusion direction of a slice group: its truth
    k-space (smsm_inputs.direction_case without noise)."""
    import smsm_inputs as si
    dc = si.direction_case(g, case, d, wid, noise=False)
    return centred_fft2(dc["rho"].astype(np.float64)[:, None] * dc["phase"].astype(np.complex128))


def direction_input(torch, dev, plan, g, case, x_true, d, wid):
    """y = A x_true + noise of one direction: A applied by the library, the
    complex Gaussian noise (SNR of the geometry) drawn on the device from a
    generator seeded by (wid, d)."""
    clean = plan.apply_A(torch.from_numpy(x_true).to(dev))
    mask = torch.from_numpy(case["masks"].astype(np.float64)).to(dev)[:, None, :, None]
    rms = torch.sqrt(torch.mean(torch.abs(clean[mask.expand_as(clean.real) > 0]) ** 2))
    gen = torch.Generator(device=dev)
    gen.manual_seed(7919 * wid + d)
    noise = torch.randn(tuple(clean.shape), dtype=torch.complex128, device=dev, generator=gen)
    return (clean + mask * (rms / g.snr) * noise).to(torch.complex64).contiguous()


def batched_measurement(torch, dev, n_streams, reps, directions=30):
    """Slice-groups/s of a batch, every group of BATCH_GEOMS with `directions`
    inputs (diffusion directions: shot phases reseeded, U(0.3, 1) attenuation,
    fresh noise; one plan per group, shared by its directions), as plain
    sequential solves and as one graph on n_streams streams; n_streams = 0
    lets the library's autotuners choose each plan's launch shapes and the
    stream count (on one direction per group), and the full batch is captured
    with that count.  The graph's outputs must
    equal the plain ones bit for bit."""
    from concurrent.futures import ThreadPoolExecutor
    import smsm_inputs as si
    from paper_1901_01893_amd import smsm
    autotuned = n_streams == 0
    plans, entries, shapes = [], [], []
    try:
        with ThreadPoolExecutor(8) as pool:
            for k, (n, L, Ns, r) in enumerate(BATCH_GEOMS):
                g = si.Geometry(n=n, n_slices=L, n_shots=Ns, n_coils=32, filt=r, lam=1e-3, n_irls=15, n_cg=15,
                                phase_order=3, snr=20.0)
                case = si.make_case(g, k, 30, noise=False)
                plan = smsm.Plan(n, n, L, Ns, 32, r, torch.from_numpy(case["coils"]).to(dev), case["masks"],
                                 case["shifts"], smsm.make_params(lam=g.lam, n_irls=g.n_irls, n_cg=g.n_cg))
                plans.append(plan)
                shapes.append(plan.autotune(10) if autotuned else None)
                truths = pool.map(lambda d: direction_truth(g, case, d, 30 + k), range(directions))
                for d, xt in enumerate(truths):
                    entries.append((plan, direction_input(torch, dev, plan, g, case, xt, d, 30 + k)))
        torch.cuda.synchronize()
        print(f"[bench] batched: {len(entries)} inputs of {len(plans)} slice groups ready", file=sys.stderr,
              flush=True)
        # directions interleaved across groups: (g0 d0, g1 d0, ..., g0 d1, ...)
        order = [entries[k * directions + d] for d in range(directions) for k in range(len(plans))]
        ys = [y for _, y in order]
        xs_plain = [torch.empty(pl.shape_x, dtype=torch.complex64, device=dev) for pl, _ in order]
        xs_graph = [torch.empty_like(x) for x in xs_plain]
        if autotuned:
            m = len(plans)
            probe = smsm.Batch([pl for pl, _ in order[:m]], ys[:m], xs_graph[:m], n_streams=0)
            n_streams = probe.n_streams
            probe.close()
        batch = smsm.Batch([pl for pl, _ in order], ys, xs_graph, n_streams=n_streams)
        try:
            def plain():
                for (plan, y), x in zip(order, xs_plain):
                    plan.solve(y, x)

            def timed(fn):
                fn()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(reps):
                    fn()
                torch.cuda.synchronize()
                return (time.perf_counter() - t0) / reps
            per_group = []
            for k in range(len(plans)):              # one solve of each group alone
                pl, y = order[k]
                pl.solve(y, xs_plain[k])
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                pl.solve(y, xs_plain[k])
                torch.cuda.synchronize()
                per_group.append(round((time.perf_counter() - t0) * 1e3, 2))
            t_plain = timed(plain)
            print(f"[bench] batched: plain {t_plain:.2f} s per pass", file=sys.stderr, flush=True)
            t_graph = timed(batch.launch)
            equal = all(torch.equal(a, b) for a, b in zip(xs_plain, xs_graph))
        finally:
            batch.close()
    finally:
        for plan in plans:
            plan.close()
    n = len(order)
    return {"groups": [f"{a}x{a} MB{b} Ns{c} r{d}" for a, b, c, d in BATCH_GEOMS], "coils": 32,
            "directions_per_group": directions,
            "inputs": "per direction: shot phases reseeded, magnitude x U(0.3, 1), fresh noise",
            "solves": n, "iterations": "15 IRLS x 15 CG", "streams": n_streams,
            "streams_chosen_by": "autotuner (one direction per group)" if autotuned else "caller",
            "launch_shapes": ([{"rows_per_workgroup": a, "columns_per_wave": b} for a, b in shapes]
                              if autotuned else "defaults"),
            "reps": reps,
            "ms_per_solve_by_group": per_group,
            "plain_slice_groups_per_s": round(n / t_plain, 3), "graph_slice_groups_per_s": round(n / t_graph, 3),
            "speedup": round(t_plain / t_graph, 3), "outputs_bitwise_equal_to_plain": equal}


def with_flags(smsm, params, extra):
    p = smsm.Params.from_buffer_copy(params)
    p.flags = params.flags | extra
    return p


MIXED_SEEDS = 30000          # instances of the mixed-precision comparison: 30000, 30001, ...
STORED_SEEDS = (0, 1000, 1001, 1002, 1003)   # stored FP64 oracle solutions of the 256x256 workload


MIXED_FORMS = {
    "reg_f32": ("SMSM_FLAG_REG_F32", "regulariser tables (image-domain Hankel kernel, band row and corner tables) "
                                     "stored complex64, widened on load; all arithmetic FP64"),
    "gram_bf16": ("SMSM_FLAG_GRAM_BF16", "Gram of Eq. 8-9 as a GEMM over the patch anchors on the BF16 matrix cores "
                                         "(three BF16 parts per real component, six part products, FP32 sums over "
                                         "2048 anchors, FP64 across); everything else FP64"),
    "gram_bf16+reg_f32": ("SMSM_FLAG_GRAM_BF16 | SMSM_FLAG_REG_F32", "both of the above"),
}


def mixed_measurement(torch, dev, plan, g, workload, ys, x, reps=10, n_inst=64):
    """The mixed-precision forms on the same plan (created able to take the
    GEMM-form Gram): slice-groups/s of each over `reps` solves after two
    warm-up solves; the NRMSE of each form's solution against the FP64
    form's (both complex128) on each of n_inst seeded instances of the
    workload; and, on the stored FP64 oracle solutions of the workload, the
    NRMSE of every form against the oracle."""
    import smsm_inputs as si
    from oracle import smsm_oracle as o
    from paper_1901_01893_amd import smsm
    base = smsm.Params.from_buffer_copy(plan.params)
    flags = {name: sum(getattr(smsm, f) for f in spec.split(" | ")) for name, (spec, _) in MIXED_FORMS.items()}
    f64 = with_flags(smsm, base, smsm.SMSM_FLAG_X_C128)
    nrmse = lambda a, b: float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b))
    res = {}
    try:
        for name, fl in flags.items():
            plan.set_params(with_flags(smsm, base, fl))
            for k in range(2):
                plan.solve(ys[k % len(ys)], x)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for k in range(reps):
                plan.solve(ys[k % len(ys)], x)
            torch.cuda.synchronize()
            t = (time.perf_counter() - t0) / reps
            res[name] = {"flags": MIXED_FORMS[name][0], "form": MIXED_FORMS[name][1],
                         "slice_groups_per_s": round(1.0 / t, 3), "ms_per_solve": round(t * 1e3, 3), "per": []}
        wid = si.WORKLOAD_IDS[workload]
        coils = si.make_case(g, 0, wid)["coils"]
        xa = torch.empty(plan.shape_x, dtype=torch.complex128, device=dev)
        xb = torch.empty_like(xa)
        for y in instances(torch, dev, plan, g, wid, list(range(MIXED_SEEDS, MIXED_SEEDS + n_inst)), coils):
            plan.set_params(f64)
            plan.solve(y, xa)
            for name, fl in flags.items():
                plan.set_params(with_flags(smsm, f64, fl))
                plan.solve(y, xb)
                res[name]["per"].append(nrmse(xb, xa))
        stored = []
        for seed in STORED_SEEDS:
            path = os.path.join(ROOT, "tests", "golden", f"oracle_{workload}_seed{seed}.npy")
            if not os.path.exists(path):
                continue
            _, y_or = o.simulate(si.make_case(g, seed, wid), g.n_slices, g.snr)
            yd = torch.from_numpy(y_or.astype(np.complex64)).to(dev)
            ref = torch.from_numpy(np.load(path).astype(np.complex128)).to(dev)
            plan.set_params(f64)
            plan.solve(yd, xa)
            row = {"seed": seed, "fp64": nrmse(xa, ref)}
            for name, fl in flags.items():
                plan.set_params(with_flags(smsm, f64, fl))
                plan.solve(yd, xb)
                row[name] = nrmse(xb, ref)
            stored.append(row)
    finally:
        plan.set_params(base)
    for r in res.values():
        per = r.pop("per")
        r["per_instance_nrmse_vs_fp64_form"] = {"seeds": f"{MIXED_SEEDS}..{MIXED_SEEDS + n_inst - 1}",
                                                "max": max(per), "mean": float(np.mean(per)),
                                                "all": [float(f"{e:.3e}") for e in per]}
    return {"instances": n_inst, "forms": res, "vs_stored_oracle": stored}


def host_truth(g, wid, seed, coils):
    """Host half of a seeded instance: the truth k-space x_true = F(rho phi)
    of the seeded phantoms and shot phases (smsm_inputs) and the masks."""
    import smsm_inputs as si
    case = si.make_case(g, seed, wid, noise=False, coils=coils)
    m = case["rho"].astype(np.float64)[:, None] * case["phase"].astype(np.complex128)
    return centred_fft2(m), case["masks"]


def device_instance(torch, dev, plan, g, wid, seed, truth):
    """One seeded instance of the workload, y resident on the device, from
    its host half `truth` (host_truth): clean data by the library's own A and
    complex Gaussian noise of the same distribution drawn on the device from
    a generator seeded by the seed (drawing 8.4 M complex normals on the host
    would take longer than the solve).  Returns y (complex64)."""
    x_true, masks = truth
    clean = plan.apply_A(torch.from_numpy(x_true).to(dev))
    mask = torch.from_numpy(masks.astype(np.float64)).to(dev)[:, None, :, None]
    acquired = mask.expand_as(clean.real) > 0
    rms = torch.sqrt(torch.mean(torch.abs(clean[acquired]) ** 2))
    gen = torch.Generator(device=dev)
    gen.manual_seed(1_000_003 * wid + seed)
    noise = torch.randn(tuple(clean.shape), dtype=torch.complex128, device=dev, generator=gen)
    return (clean + mask * (rms / g.snr) * noise).to(torch.complex64).contiguous()


def instances(torch, dev, plan, g, wid, seeds, coils, workers=6):
    """device_instance over `seeds` in order, the host halves of the next
    instances prepared by a thread pool while the device works."""
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(workers) as pool:
        futs = [pool.submit(host_truth, g, wid, sd, coils) for sd in seeds[:2 * workers]]
        for k, sd in enumerate(seeds):
            if k + 2 * workers < len(seeds):
                futs.append(pool.submit(host_truth, g, wid, seeds[k + 2 * workers], coils))
            yield device_instance(torch, dev, plan, g, wid, sd, futs[k].result())
            futs[k] = None


LEARNED_TRAIN_SEEDS = 10000   # training instances 10000, 10001, ...
LEARNED_EVAL_SEEDS = 20000    # held-out instances 20000, 20001, ...
FALLBACK_RATIO = 1.5


def learned_measurement(torch, dev, plan, g, workload, n_train=2000, n_eval=200, mu=0.05, lr=3e-4, bf16=2):
    """The learned form on the timed workload: the width-64 BF16 network (5
    unrolled iterations of 10 data-consistency CG steps) trained on the GPU
    with one Adam step per seeded instance (n_train instances, streamed:
    each is generated, solved by the plain solver for its target and trained
    on once), then evaluated on n_eval held-out instances against the plain
    solver, against the same iterations without the network, and with the
    plain solver as fallback when its residual exceeds FALLBACK_RATIO x the
    plain solver's; on the stored FP64 oracle solutions of the workload
    (complex64) the plain and learned solutions are compared with the oracle."""
    import smsm_inputs as si
    from oracle import smsm_oracle as o
    from paper_1901_01893_amd import smsm
    wid = si.WORKLOAD_IDS[workload]
    coils = si.make_case(g, 0, wid)["coils"]
    params = si.cnn_init(1, 2 * g.n_shots, width=64, out_scale=0.1)
    zero = [(np.zeros_like(w), np.zeros_like(b)) for w, b in params]
    xp = torch.empty(plan.shape_x, dtype=torch.complex64, device=dev)
    rel = lambda a, b: float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b))
    with smsm.Learned(plan, params, width=64, n_unroll=5, n_cg=10, mu=mu) as net, \
            smsm.Learned(plan, zero, width=64, n_unroll=5, n_cg=10, mu=mu) as net0:
        net.set_bf16(bf16)
        net0.set_bf16(bf16)
        losses, t_step = [], 0.0
        t0 = time.perf_counter()
        for k, y in enumerate(instances(torch, dev, plan, g, wid,
                                        list(range(LEARNED_TRAIN_SEEDS, LEARNED_TRAIN_SEEDS + n_train)), coils)):
            plan.solve(y, xp)
            xt = xp.to(torch.complex128)
            torch.cuda.synchronize()
            ts = time.perf_counter()
            losses.append(net.train_step(y, xt, lr))
            t_step += time.perf_counter() - ts
            if k % 500 == 0:
                print(f"[bench] learned: trained on {k + 1} of {n_train} instances", file=sys.stderr, flush=True)
        t_train_total = time.perf_counter() - t0
        e_net, e_dc, e_fb, ratios, n_fb = [], [], [], [], 0
        for y in instances(torch, dev, plan, g, wid, list(range(LEARNED_EVAL_SEEDS, LEARNED_EVAL_SEEDS + n_eval)),
                           coils):
            plan.solve(y, xp)
            xpl = xp.to(torch.complex128)
            x, fell, r_l, r_p = net.solve_fallback(y, FALLBACK_RATIO)
            xl = net.solve(y)
            e_net.append(rel(xl, xpl))
            e_dc.append(rel(net0.solve(y), xpl))
            e_fb.append(rel(x, xpl))
            ratios.append(r_l / r_p)
            n_fb += int(fell)
        # against the FP64 oracle on its stored solutions of this workload
        oracle_cmp = []
        for seed in STORED_SEEDS:
            path = os.path.join(ROOT, "tests", "golden", f"oracle_{workload}_seed{seed}.npy")
            if not os.path.exists(path):
                continue
            case = si.make_case(g, seed, wid)
            _, y_or = o.simulate(case, g.n_slices, g.snr)
            yd = torch.from_numpy(y_or.astype(np.complex64)).to(dev)
            ref = torch.from_numpy(np.load(path).astype(np.complex128)).to(dev)
            plan.solve(yd, xp)
            x, fell, _, _ = net.solve_fallback(yd, FALLBACK_RATIO)
            oracle_cmp.append({"seed": seed, "plain": rel(xp.to(torch.complex128), ref),
                               "learned": rel(net.solve(yd), ref), "learned_with_fallback": rel(x, ref),
                               "fell_back": bool(fell)})
        y = device_instance(torch, dev, plan, g, wid, LEARNED_EVAL_SEEDS,
                            host_truth(g, wid, LEARNED_EVAL_SEEDS, coils))
        xo = net.solve(y)
        torch.cuda.synchronize()
        reps = 10
        t0 = time.perf_counter()
        for _ in range(reps):
            net.solve(y, xo)
        torch.cuda.synchronize()
        t_solve = (time.perf_counter() - t0) / reps
    mode = {0: "FP32 weights", 1: "BF16 weights, exact products",
            2: "BF16 network (BF16 weights and convolution inputs)"}[bf16]
    return {"network": "5 x (residual k-space CNN 2Ns-64-64-64-64-2Ns, 3x3, ReLU, "
                       f"{mode}, FP32 accumulation on the matrix cores + 10 FP64 CG data-consistency steps, mu={mu})",
            "training": f"one Adam step (lr {lr}) on each of {n_train} seeded instances (seeds "
                        f"{LEARNED_TRAIN_SEEDS}..), targets from the plain solver",
            "train_instances": n_train, "train_ms_per_step": round(t_step / max(n_train, 1) * 1e3, 2),
            "train_total_s": round(t_train_total, 1),
            "loss_first_last100": [round(float(np.mean(losses[:100])), 4), round(float(np.mean(losses[-100:])), 4)],
            "slice_groups_per_s": round(1.0 / t_solve, 3), "ms_per_solve": round(t_solve * 1e3, 3),
            "eval_instances": n_eval,
            "heldout_rel_error_vs_plain": round(float(np.mean(e_net)), 4),
            "heldout_rel_error_vs_plain_without_network": round(float(np.mean(e_dc)), 4),
            "heldout_rel_error_vs_plain_with_fallback": round(float(np.mean(e_fb)), 4),
            "residual_ratio_vs_plain": {"mean": round(float(np.mean(ratios)), 3),
                                        "max": round(float(np.max(ratios)), 3)},
            "fallback_ratio": FALLBACK_RATIO, "fallback_rate": round(n_fb / max(n_eval, 1), 4),
            "vs_stored_oracle": oracle_cmp}


# AL penalty per workload: tau = lambda / beta keeps about a quarter of the
# singular values of H(A^H y) above the threshold (0.4 .. 43 at 64 x 64,
# 0.9 .. 241 at 256 x 256)
AL_BETA = {"small": 1e-4, "sg256": 2e-5}
AL_OUTER, AL_CG = 30, 5


def al_measurement(torch, dev, plan, g, workload, case, reps=3):
    """The augmented-Lagrangian solve of Eq. 10 (smsm_al_*) on the timed
    workload: AL_OUTER outer iterations of AL_CG CG steps at the workload's
    lambda, slice-groups/s over `reps` solves after one warm-up; the objective
    of Eq. 10 (evaluated by the oracle on the host) at its result and at the
    IRLS solve's of the same input; and its parity with the oracle's AL on the
    small workload (10 outer iterations of 5 CG steps)."""
    import smsm_inputs as si
    from oracle import al_oracle as al
    from oracle import smsm_oracle as o
    from paper_1901_01893_amd import smsm
    lam, beta = g.lam, AL_BETA[workload]
    _, y_or = o.simulate(case, g.n_slices, g.snr)
    y_or = y_or.astype(np.complex64)
    yd = torch.from_numpy(y_or).to(dev)
    with smsm.AL(plan, lam, beta, AL_OUTER, AL_CG) as s:
        x = s.solve(yd)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            s.solve(yd, x)
        torch.cuda.synchronize()
        t = (time.perf_counter() - t0) / reps
        status = plan.status()
        state_mb = s.device_bytes() / 1e6
        x_al = x.cpu().numpy()
    base = smsm.Params.from_buffer_copy(plan.params)
    try:
        plan.set_params(with_flags(smsm, base, smsm.SMSM_FLAG_X_C128))
        x_irls = plan.solve(yd).cpu().numpy()
    finally:
        plan.set_params(base)
    theta = o.caipi_phase(g.n, case["shifts"])
    y64 = y_or.astype(np.complex128)
    j_al = o.objective(x_al, y64, case["coils"], case["masks"], theta, lam, g.filt)
    j_irls = o.objective(x_irls, y64, case["coils"], case["masks"], theta, lam, g.filt)
    # parity with the oracle's AL on the small workload
    gs = si.WORKLOADS["small"]
    cs = si.make_case(gs, 3, 300)
    _, ys = o.simulate(cs, gs.n_slices, gs.snr)
    ys = ys.astype(np.complex64)
    with smsm.Plan(gs.n, gs.n, gs.n_slices, gs.n_shots, gs.n_coils, gs.filt, torch.from_numpy(cs["coils"]).to(dev),
                   cs["masks"], cs["shifts"], smsm.make_params(lam=gs.lam, n_irls=1, n_cg=1)) as ps, \
            smsm.AL(ps, gs.lam, AL_BETA["small"], 10, 5) as ss:
        xs = ss.solve(torch.from_numpy(ys).to(dev)).cpu().numpy()
    xr = al.solve_al(ys.astype(np.complex128), cs["coils"], cs["masks"], cs["shifts"],
                     al.ALParams(lam=gs.lam, r=gs.filt, beta=AL_BETA["small"], n_outer=10, n_cg=5))
    return {"form": "augmented Lagrangian (split Z = H(x), scaled duals, singular-value thresholding at "
                    "lambda / beta from the K x K Gram by Newton-Schulz matrix functions on the FP64 matrix "
                    "cores), FP64",
            "lambda": lam, "beta": beta, "outer_iterations": AL_OUTER, "cg_per_outer": AL_CG,
            "slice_groups_per_s": round(1.0 / t, 3), "ms_per_solve": round(t * 1e3, 2),
            "ms_per_outer_iteration": round(t * 1e3 / AL_OUTER, 3), "state_mb": round(state_mb, 1),
            "status": smsm.status_string(status),
            "objective_eq10": {"al": j_al, "irls": j_irls, "al_over_irls": j_al / j_irls},
            "rel_diff_al_vs_irls": float(np.linalg.norm(x_al - x_irls) / np.linalg.norm(x_irls)),
            "nrmse_vs_oracle_al_small": o.nrmse(xs, xr)}


def time_kernel(torch, plan, name, reps):
    stream = torch.cuda.current_stream()
    plan.launch_kernel(name, 2)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    plan.launch_kernel(name, reps)
    e1.record(stream)
    e1.synchronize()
    return e0.elapsed_time(e1) / reps * 1e-3   # seconds per launch


COL_SOURCES = ("smsm_col_fast.h", "smsm_wavefft.h", "smsm_device.h")
N_DRAWS = 8   # distinct noise realisations cycled through the timed solves
TIMER_STRIDE = 17   # one timed column pass in this many, inside the timed solves (prime, so the
                    # samples walk through every position of the 16 passes of an IRLS step)


def measured_traffic():
    """HBM bytes per launch of the column kernel from the committed counter
    summary, or None when the kernel sources changed since it was taken."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", "col_normal_sg256_hbm_counters.md")
    if not os.path.exists(path):
        return None
    m = re.search(r"machine-readable: (\{.*\})", open(path).read())
    if not m:
        return None
    rec = json.loads(m.group(1))
    h = hashlib.sha256()
    for f in COL_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_1901_01893_amd", "csrc", f), "rb").read())
    return rec["traffic_bytes"] if h.hexdigest()[:16] == rec["source_sha256_16"] else None


def survey_matvec_counts(g):
    """Algorithmic work of one SENSE normal-operator application (one launch
    of the column pass: one matvec): bytes = p in and out (complex64) plus the
    coil maps (complex64) = 62.9 MB at 256^2, 3 slices, 4 shots, 32 coils;
    flops = 1.31 GFLOP for the mask-pruned transforms at that size (the
    hot-path scope's per-matvec figures; no other size is quoted there)."""
    nb = g.n_slices * g.n_shots * g.n * g.n * 8.0
    bytes_ = 2 * nb + g.n_slices * g.n_coils * g.n * g.n * 8.0
    sg256 = (g.n, g.n_slices, g.n_shots, g.n_coils) == (256, 3, 4, 32)
    return (1.31e9 if sg256 else None), bytes_


def column_pass_roofline(g, f_lib, b_lib, t, launches, traffic):
    """The dominant kernel (one launch per CG matvec) against the FP64 vector
    peak (the kernel computes in FP64; an FP64 FMA issues at the FP32 rate on
    this chip, packed FP32 is not used) with the hot-path scope's per-matvec
    flops, the HBM fraction of its per-matvec bytes, and the library's own
    counts of everything the kernel does (vector updates, the Hankel term,
    complex128 operands) beside them."""
    f_alg, b_alg = survey_matvec_counts(g)
    f_use = f_alg if f_alg is not None else f_lib
    vec = g.n_slices * g.n_shots * g.n * g.n * 16.0
    out = {"bound": "alu", "achieved": round(f_use / t / 1e12, 3), "peak": FP64_VALU_TFLOPS, "unit": "TFLOP/s",
           "frac": round(f_use / t / 1e12 / FP64_VALU_TFLOPS, 4),
           "traffic": None if traffic is None else round(traffic / 1e6, 2), "traffic_unit": "MB/launch",
           "kernel": "k_col_fast (per-column SENSE + Hankel pass, one launch per CG matvec)",
           "us_per_launch": round(t * 1e6, 2), "launches_timed": launches,
           "algorithmic": {"gflop": None if f_alg is None else f_alg / 1e9, "mb": round(b_alg / 1e6, 2),
                           "source": "hot-path scope, per SENSE normal-operator matvec"},
           "hbm_frac": round(b_alg / t / (HBM_TBS * 1e12), 4),
           "library_counts": {"gflop": round(f_lib / 1e9, 3), "mb": round(b_lib / 1e6, 1),
                              "flop_frac": round(f_lib / t / 1e12 / FP64_VALU_TFLOPS, 4),
                              "hbm_frac": round(b_lib / t / (HBM_TBS * 1e12), 4)}}
    if traffic is not None:
        # what the counters see beyond the algorithmic bytes: the coil maps
        # widened to complex128, the CG vectors the pass also streams (r, p, x
        # in; p, q, x out, complex128 rather than p in / q out complex64) and the
        # image-domain Hankel kernel (10 Hermitian shot pairs, complex128)
        out["traffic_vs_algorithmic"] = round(traffic / b_alg, 2)
        out["traffic_breakdown_mb"] = {
            "coil_maps_c128": round(g.n_slices * g.n_coils * g.n * g.n * 16.0 / 1e6, 1),
            "cg_vectors_c128": round(6 * vec / 1e6, 1),
            "hankel_kernel_c128": round(g.n_slices * g.n_shots * (g.n_shots + 1) / 2 * g.n * g.n * 16.0 / 1e6, 1)}
    return out


def host_cpu():
    """CPU model, physical cores and logical CPUs of the host (from /proc/cpuinfo)."""
    model, cores = "unknown", set()
    try:
        phys = core = None
        for line in open("/proc/cpuinfo"):
            k, _, v = line.partition(":")
            k, v = k.strip(), v.strip()
            if k == "model name":
                model = v
            elif k == "physical id":
                phys = v
            elif k == "core id":
                core = v
            elif not k and phys is not None:
                cores.add((phys, core))
                phys = core = None
    except OSError:
        pass
    return {"cpu_model": model, "physical_cores": len(cores) or None, "logical_cpus": os.cpu_count()}


def oracle_solve_time(g, case, y, n_irls):
    """Seconds of the oracle's own solve of `case` with n_irls IRLS iterations
    (everything else as the workload sets it)."""
    from oracle import smsm_oracle as o
    p = o.SolveParams(lam=g.lam, r=g.filt, n_irls=n_irls, n_cg=g.n_cg)
    t0 = time.perf_counter()
    o.solve(y, case["coils"], case["masks"], case["shifts"], p)
    return time.perf_counter() - t0


def oracle_setup_time(g, case, y):
    """Seconds of the part of the oracle's solve before its first IRLS
    iteration: A^H y and the Gram of each slice with its largest eigenvalue."""
    from oracle import smsm_oracle as o
    t0 = time.perf_counter()
    b = o.adjoint(y, case["coils"].astype(np.complex128), case["masks"].astype(np.float64),
                  o.caipi_phase(g.n, case["shifts"]))
    [o.lambda_max(o.gram(b[l], g.filt)) for l in range(g.n_slices)]
    return time.perf_counter() - t0


def cpu_baseline(g, case, y_oracle):
    """The FP64 oracle timed on the host on a bounded sample of the same solve:
    the oracle's solve with one IRLS iteration (T1) and its set-up alone (T0).
    Every IRLS iteration costs the same (one Gram, one eigendecomposition and
    n_cg + 1 normal-operator applications per slice group), so the full solve
    takes T0 + n_irls (T1 - T0).  The same rule is checked against a full
    oracle solve of the 64 x 64 workload on the same host."""
    import smsm_inputs as si
    from oracle import smsm_oracle as o
    try:
        from threadpoolctl import threadpool_info
        threads = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
    except Exception:  # noqa: BLE001
        threads = os.cpu_count() or 1
    t0 = oracle_setup_time(g, case, y_oracle)
    t1 = oracle_solve_time(g, case, y_oracle, 1)
    solve_s = t0 + g.n_irls * (t1 - t0)
    # the rule against a full solve of the small workload
    gs = si.WORKLOADS["small"]
    cs = si.make_case(gs, 0, si.WORKLOAD_IDS["small"])
    _, ys = o.simulate(cs, gs.n_slices, gs.snr)
    ys = ys.astype(np.complex64).astype(np.complex128)
    s0 = oracle_setup_time(gs, cs, ys)
    s1 = oracle_solve_time(gs, cs, ys, 1)
    s_full = oracle_solve_time(gs, cs, ys, gs.n_irls)
    s_rule = s0 + gs.n_irls * (s1 - s0)
    out = {"value": 1.0 / solve_s, "unit": "slice-groups/s", "cores": int(threads), "kind": "oracle",
           "sample": (f"the oracle's solve of this workload with 1 of {g.n_irls} IRLS iterations "
                      f"({t1:.1f} s) and its set-up (A^H y, Grams, lambda_max: {t0:.1f} s), scaled to "
                      f"{g.n_irls} iterations: {solve_s:.1f} s per slice group"),
           "check_small_workload": {"full_solve_s": round(s_full, 2), "rule_s": round(s_rule, 2),
                                    "ratio_full_to_rule": round(s_full / s_rule, 3)}}
    out.update(host_cpu())
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="sg256")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--kernel-reps", type=int, default=50)
    ap.add_argument("--profile-kernel", default=None,
                    help="profiling mode: one solve, a calibration copy, then REPS launches of this kernel")
    ap.add_argument("--reps", type=int, default=20)
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-form measurement")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-form measurement")
    ap.add_argument("--learned-train", type=int, default=2000, help="training instances of the learned form")
    ap.add_argument("--learned-eval", type=int, default=200, help="held-out instances of the learned form")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision-form measurement")
    ap.add_argument("--no-al", action="store_true", help="skip the augmented-Lagrangian measurement")
    ap.add_argument("--profile-learned", type=int, default=0, metavar="STEPS",
                    help="run only STEPS training steps and STEPS solves of the learned form (for a kernel trace)")
    ap.add_argument("--profile-al", type=int, default=0, metavar="SOLVES",
                    help="run only SOLVES augmented-Lagrangian solves of the workload (for a kernel trace)")
    ap.add_argument("--batch-streams", type=int, default=0, help="0: the library's autotuner picks the count")
    ap.add_argument("--batch-directions", type=int, default=30, help="diffusion directions per slice group")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); "
              "independent slice groups would shard across GPUs with no exchange.", file=sys.stderr)
        sys.exit(2)

    import torch
    import smsm_inputs as si
    from paper_1901_01893_amd import smsm

    dev = torch.device("cuda:0")
    g = si.WORKLOADS[args.workload]
    case = si.make_case(g, 0, si.WORKLOAD_IDS[args.workload])
    coils = torch.from_numpy(case["coils"]).to(dev)
    params = smsm.make_params(lam=g.lam, n_irls=g.n_irls, n_cg=g.n_cg)
    # created able to take the GEMM-form Gram (its chunk partials in the
    # workspace) for the mixed-precision forms; the timed solves run without it
    plan = smsm.Plan(g.n, g.n, g.n_slices, g.n_shots, g.n_coils, g.filt, coils, case["masks"],
                     case["shifts"], with_flags(smsm, params, smsm.SMSM_FLAG_GRAM_BF16))
    plan.set_params(params)
    ys = synth_inputs(torch, dev, plan, g, case, 1 if args.profile_kernel else N_DRAWS)
    y = ys[0]
    x = torch.empty(plan.shape_x, dtype=torch.complex64, device=dev)
    if args.profile_al:
        with smsm.AL(plan, g.lam, AL_BETA[args.workload], AL_OUTER, AL_CG) as s:
            xa = s.solve(y)
            for _ in range(args.profile_al - 1):
                s.solve(y, xa)
            torch.cuda.synchronize()
        plan.close()
        print(json.dumps({"profile_al": args.profile_al, "workload": args.workload}))
        return
    if args.profile_learned:
        import smsm_inputs as si
        net = smsm.Learned(plan, si.cnn_init(1, 2 * g.n_shots, width=64), width=64, n_unroll=5, n_cg=10, mu=0.05)
        net.set_bf16(2)
        xt = plan.solve(y).to(torch.complex128)
        for _ in range(args.profile_learned):
            net.train_step(y, xt, 3e-4)
        for _ in range(args.profile_learned):
            net.solve(y)
        torch.cuda.synchronize()
        net.close()
        plan.close()
        print(json.dumps({"profile_learned": args.profile_learned, "workload": args.workload}))
        return
    if args.profile_kernel:
        # Kernel-level profiling: fill the plan's buffers with one solve, run a
        # plain device copy of known size (calibrates the HBM byte counters),
        # then re-launch one CG-iteration kernel.
        plan.solve(y, x)
        src = torch.ones(COPY_BYTES // 16, dtype=torch.complex128, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        plan.launch_kernel(args.profile_kernel, args.reps)
        torch.cuda.synchronize()
        f, b = plan.kernel_cost(args.profile_kernel)
        print(json.dumps({"profile_kernel": args.profile_kernel, "reps": args.reps, "copy_bytes": COPY_BYTES,
                          "algorithmic_flops": f, "algorithmic_bytes": b}))
        plan.close()
        return
    print(f"[bench] workload={args.workload} warmup={args.warmup} steps={args.steps}", file=sys.stderr,
          flush=True)
    for k in range(args.warmup):
        plan.solve(ys[k % len(ys)], x)
    torch.cuda.synchronize()
    status = plan.status()
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    # the dominant kernel is timed inside the timed solves: one column pass in
    # every TIMER_STRIDE gets a start/stop event pair on its own dispatch
    n_col = g.n_irls * (g.n_cg + 1)
    plan.kernel_timer_start("col_normal", args.steps * n_col // TIMER_STRIDE + 1, TIMER_STRIDE)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev[0].record(stream)
    for k in range(args.steps):
        plan.solve(ys[k % len(ys)], x)
        ev[k + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    col_ms, col_n = plan.kernel_timer_read()
    plan.kernel_timer_start("col_normal", 0, 1)
    per = [ev[k].elapsed_time(ev[k + 1]) for k in range(args.steps)]
    print(f"[bench] timed {args.steps} solves in {wall:.3f} s (median {np.median(per):.2f} ms)",
          file=sys.stderr, flush=True)

    # dominant kernel: per-column SENSE + Hankel pass of every CG matvec
    kern = {}
    for name in ("col_normal", "band_extract", "band_corr", "cg_update", "rows_inv", "rows_fwd"):
        t = time_kernel(torch, plan, name, args.kernel_reps)
        f, b = plan.kernel_cost(name)
        kern[name] = {"us": t * 1e6, "gflop": f / 1e9, "mb": b / 1e6,
                      "tflops": f / t / 1e12, "gbs": b / t / 1e9}
    f_col, b_col = plan.kernel_cost("col_normal")
    t_col = col_ms / col_n * 1e-3 if col_n else kern["col_normal"]["us"] * 1e-6
    roofline = column_pass_roofline(g, f_col, b_col, t_col, col_n,
                                    measured_traffic() if args.workload == "sg256" else None)

    out = {"metric": "slice-groups/sec (256^2, 32 coils, MB=3, 4 shots) @ NRMSE vs FP64 oracle",
           "value": args.steps / wall, "unit": "slice-groups/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": wall / args.steps * 1e3, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"{args.workload}: {g.n}x{g.n}, MB={g.n_slices}, {g.n_shots} shots, "
                                  f"{g.n_coils} coils, {g.filt}x{g.filt} filter, lambda={g.lam}, "
                                  f"{g.n_irls} IRLS x {g.n_cg} CG, inputs c64, arithmetic f64; "
                                  f"{N_DRAWS} seeded noise draws of one acquisition cycled over the steps",
                      "global_batch": 1},
           "roofline": roofline,
           "kernels": {k: {kk: round(vv, 3) for kk, vv in v.items()} for k, v in kern.items()},
           "solve_status": smsm.status_string(status)}
    if not args.no_batched:
        out["batched"] = batched_measurement(torch, dev, args.batch_streams, 2, args.batch_directions)
    if not args.no_mixed:
        out["mixed"] = mixed_measurement(torch, dev, plan, g, args.workload, ys, x)
    if not args.no_al and args.workload in AL_BETA:
        out["al"] = al_measurement(torch, dev, plan, g, args.workload, case)
    if not args.no_learned:
        out["learned"] = learned_measurement(torch, dev, plan, g, args.workload, n_train=args.learned_train,
                                             n_eval=args.learned_eval)

    if not args.no_cpu_baseline and args.gpus == 1:
        from oracle import smsm_oracle as o
        _, y_or = o.simulate(case, g.n_slices, g.snr)
        y_or = y_or.astype(np.complex64)
        ref_path = os.path.join(ROOT, "tests", "golden", f"oracle_{args.workload}_seed0.npy")
        if os.path.exists(ref_path):
            ref = np.load(ref_path)
            plan.solve(torch.from_numpy(y_or).to(dev), x)
            out["nrmse_vs_oracle"] = o.nrmse(x.cpu().numpy(), ref)
        out["cpu_baseline"] = cpu_baseline(g, case, y_or.astype(np.complex128))
    plan.close()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
