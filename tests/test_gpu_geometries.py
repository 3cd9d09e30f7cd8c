"""GPU parity on geometries that exercise the other kernel instances: the
generic column pass (shot counts without a register-resident instance), the
band kernel for 1, 2 and 8 shots, the vector pass with fewer than 64 ky per
row, a coil count that leaves a partial coil group, every instance of the fast
column pass (folded lengths 16, 32 and 64, two and three slices, odd coil
counts), matrix sizes 3 or 7 times a power of two (96, 112, 192, 224), and one
coil with a 1 x 1 schedule.  Each case checks the normal operator with the
oracle's weights and a short IRLS solve against the oracle's."""
import numpy as np
import pytest

import smsm_inputs as si
from oracle import smsm_oracle as o
from tests.helpers import oracle_params, rel

pytestmark = pytest.mark.gpu

OP_TOL = 1e-11
SOLVE_TOL = 1e-10     # complex128 solves (measured ~1e-14)

GEOMS = {
    # generic column pass (2 shots), band kernel <5, 2>, vector pass with 32 ky per row
    "n32_L2_Ns2_r3": (si.Geometry(n=32, n_slices=2, n_shots=2, n_coils=4, filt=3, lam=1e-3, n_irls=3, n_cg=5,
                                  phase_order=2, snr=30.0), 101),
    # generic column pass (8 shots, folded length 8), band kernel <3, 8>, one slice
    "n64_L1_Ns8_r2": (si.Geometry(n=64, n_slices=1, n_shots=8, n_coils=4, filt=2, lam=1e-3, n_irls=3, n_cg=5,
                                  phase_order=2, snr=30.0), 102),
    # generic column pass (1 shot), band kernel <7, 1>, four slices
    "n128_L4_Ns1_r4": (si.Geometry(n=128, n_slices=4, n_shots=1, n_coils=4, filt=4, lam=1e-3, n_irls=3, n_cg=4,
                                   phase_order=2, snr=30.0), 103),
    # fast column pass <32, 2>, 6 coils (a partial coil group), band kernel <7, 4>
    "n128_L2_Ns4_r4": (si.Geometry(n=128, n_slices=2, n_shots=4, n_coils=6, filt=4, lam=1e-3, n_irls=3, n_cg=4,
                                   phase_order=2, snr=30.0), 104),
    # fast column pass <64, 2> (two slices at folded length 64), 5 coils (the last
    # coil group has a clamped, zero-weighted member), band kernel <5, 4>
    "n256_L2_Ns4_r3": (si.Geometry(n=256, n_slices=2, n_shots=4, n_coils=5, filt=3, lam=1e-3, n_irls=2, n_cg=3,
                                   phase_order=2, snr=30.0), 105),
    # fast column pass <32, 3> and <16, 3> (three slices at folded lengths 32 and 16), odd coil counts
    "n128_L3_Ns4_r5": (si.Geometry(n=128, n_slices=3, n_shots=4, n_coils=7, filt=5, lam=1e-3, n_irls=2, n_cg=3,
                                   phase_order=2, snr=30.0), 107),
    "n64_L3_Ns4_r3": (si.Geometry(n=64, n_slices=3, n_shots=4, n_coils=3, filt=3, lam=1e-3, n_irls=2, n_cg=3,
                                  phase_order=2, snr=30.0), 108),
    # the batched bench's instances: band kernel <13, 2> with the fast column
    # pass at 2 shots, folded length 128 (two points per lane) at 256 ky and 64
    # at 128 ky; band kernel <9, 8> with the
    # fast column pass <16, 2, 8 shots, 1 coil group> at 128 ky (few coils, short schedules)
    "n256_L2_Ns2_r7": (si.Geometry(n=256, n_slices=2, n_shots=2, n_coils=3, filt=7, lam=1e-3, n_irls=2, n_cg=3,
                                   phase_order=3, snr=20.0), 109),
    "n128_L2_Ns2_r7": (si.Geometry(n=128, n_slices=2, n_shots=2, n_coils=3, filt=7, lam=1e-3, n_irls=2, n_cg=3,
                                   phase_order=3, snr=20.0), 110),
    "n128_L2_Ns8_r5": (si.Geometry(n=128, n_slices=2, n_shots=8, n_coils=3, filt=5, lam=1e-3, n_irls=2, n_cg=3,
                                   phase_order=3, snr=20.0), 111),
    # the other instances of the batched bench's ten groups: three slices with the
    # generic column pass at 2 and 8 shots, and the fast column pass <64, 3> with a 5 x 5 filter
    "n256_L3_Ns2_r7": (si.Geometry(n=256, n_slices=3, n_shots=2, n_coils=3, filt=7, lam=1e-3, n_irls=2, n_cg=3,
                                   phase_order=3, snr=20.0), 112),
    "n256_L3_Ns4_r5": (si.Geometry(n=256, n_slices=3, n_shots=4, n_coils=3, filt=5, lam=1e-3, n_irls=2, n_cg=3,
                                   phase_order=3, snr=20.0), 113),
    "n128_L3_Ns8_r5": (si.Geometry(n=128, n_slices=3, n_shots=8, n_coils=3, filt=5, lam=1e-3, n_irls=2, n_cg=3,
                                   phase_order=3, snr=20.0), 114),
    "n128_L3_Ns2_r7": (si.Geometry(n=128, n_slices=3, n_shots=2, n_coils=3, filt=7, lam=1e-3, n_irls=2, n_cg=3,
                                   phase_order=3, snr=20.0), 115),
    # matrix sizes with an odd factor (3 or 7 times a power of two): the generic
    # column pass with mixed-length transforms (96x96, folded length 48 at 2 shots),
    # the odd-length register-resident pass (folded lengths 28, 24, 56, 112), the
    # row, Gram and image passes for such lengths, vector-pass ky chunks of 16 and 32
    "n96_L2_Ns2_r3": (si.Geometry(n=96, n_slices=2, n_shots=2, n_coils=3, filt=3, lam=1e-3, n_irls=2, n_cg=3,
                                  phase_order=2, snr=30.0), 116),
    "n112_L2_Ns4_r3": (si.Geometry(n=112, n_slices=2, n_shots=4, n_coils=3, filt=3, lam=1e-3, n_irls=2, n_cg=3,
                                   phase_order=2, snr=30.0), 117),
    "n192_L2_Ns8_r5": (si.Geometry(n=192, n_slices=2, n_shots=8, n_coils=3, filt=5, lam=1e-3, n_irls=2, n_cg=3,
                                   phase_order=3, snr=20.0), 118),
    "n224_L2_Ns4_r7": (si.Geometry(n=224, n_slices=2, n_shots=4, n_coils=3, filt=7, lam=1e-3, n_irls=2, n_cg=3,
                                   phase_order=3, snr=20.0), 119),
    "n224_L3_Ns2_r7": (si.Geometry(n=224, n_slices=3, n_shots=2, n_coils=3, filt=7, lam=1e-3, n_irls=2, n_cg=3,
                                   phase_order=3, snr=20.0), 120),
    "n224_L2_Ns8_r5": (si.Geometry(n=224, n_slices=2, n_shots=8, n_coils=3, filt=5, lam=1e-3, n_irls=2, n_cg=3,
                                   phase_order=3, snr=20.0), 121),
    "n192_L3_Ns4_r7": (si.Geometry(n=192, n_slices=3, n_shots=4, n_coils=3, filt=7, lam=1e-3, n_irls=2, n_cg=3,
                                   phase_order=3, snr=20.0), 122),
    # eight shots at 256 ky: the fast column pass <32, 2, 8 shots, 1 coil group> for
    # the normal operator, and the generic one (forward, adjoint and regulariser
    # modes) at its largest shared-memory footprint (the coil loop's buffers and
    # the regulariser's taps share one region)
    "n256_L2_Ns8_r5": (si.Geometry(n=256, n_slices=2, n_shots=8, n_coils=3, filt=5, lam=1e-3, n_irls=2, n_cg=3,
                                   phase_order=3, snr=20.0), 123),
    # the odd-length register-resident column pass <56, 3 slices, 4 shots> (the
    # batch's 224x224 MB3 group) and <48, 2 slices, 4 shots>
    "n224_L3_Ns4_r7": (si.Geometry(n=224, n_slices=3, n_shots=4, n_coils=3, filt=7, lam=1e-3, n_irls=2, n_cg=3,
                                   phase_order=3, snr=20.0), 125),
    "n192_L2_Ns4_r5": (si.Geometry(n=192, n_slices=2, n_shots=4, n_coils=5, filt=5, lam=1e-3, n_irls=2, n_cg=3,
                                   phase_order=3, snr=20.0), 126),
    # the odd-length pass with two folded points per lane: <112, 2 slices,
    # 2 shots> (the batch's 224x224 MB2 two-shot group), <96, 3 slices> (a
    # partial second coil pass: 5 coils over 4 coil groups) and <96, 2 slices>
    "n224_L2_Ns2_r7": (si.Geometry(n=224, n_slices=2, n_shots=2, n_coils=3, filt=7, lam=1e-3, n_irls=2, n_cg=3,
                                   phase_order=3, snr=20.0), 127),
    "n192_L3_Ns2_r7": (si.Geometry(n=192, n_slices=3, n_shots=2, n_coils=5, filt=7, lam=1e-3, n_irls=2, n_cg=3,
                                   phase_order=3, snr=20.0), 128),
    "n192_L2_Ns2_r5": (si.Geometry(n=192, n_slices=2, n_shots=2, n_coils=3, filt=5, lam=1e-3, n_irls=2, n_cg=3,
                                   phase_order=3, snr=20.0), 129),
    # degenerate: one coil (three of the four coil slots of the fast column pass <16, 2>
    # clamped and zero-weighted) and the smallest schedule, 1 IRLS x 1 CG
    "n64_L2_Ns4_r3_c1": (si.Geometry(n=64, n_slices=2, n_shots=4, n_coils=1, filt=3, lam=1e-3, n_irls=1, n_cg=1,
                                     phase_order=2, snr=30.0), 106),
}


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1901_01893_amd  # noqa: F401  (fails loudly if the library is missing)
    return torch, torch.device("cuda:0")


@pytest.fixture(scope="module", params=list(GEOMS))
def geo(request, torch_dev):
    from paper_1901_01893_amd import smsm
    torch, dev = torch_dev
    g, wid = GEOMS[request.param]
    case = si.make_case(g, 0, wid)
    x_true, y = o.simulate(case, g.n_slices, g.snr)
    y = y.astype(np.complex64)
    print(f"[geometry] {request.param}", flush=True)
    coils = torch.from_numpy(case["coils"]).to(dev)
    plan = smsm.Plan(g.n, g.n, g.n_slices, g.n_shots, g.n_coils, g.filt, coils, case["masks"], case["shifts"],
                     smsm.make_params(lam=g.lam, n_irls=g.n_irls, n_cg=g.n_cg, flags=smsm.SMSM_FLAG_X_C128))
    yield dict(torch=torch, dev=dev, g=g, case=case, y=y, plan=plan, name=request.param)
    plan.close()


def to_dev(torch, dev, a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def test_normal_operator_with_oracle_weights(geo):
    torch, dev, g, case = geo["torch"], geo["dev"], geo["g"], geo["case"]
    theta = o.caipi_phase(g.n, case["shifts"])
    coils = case["coils"].astype(np.complex128)
    masks = case["masks"].astype(np.float64)
    x0 = o.adjoint(geo["y"].astype(np.complex128), coils, masks, theta)
    Ws = [o.irls_weight(o.gram(x0[l], g.filt), 0.05 * o.lambda_max(o.gram(x0[l], g.filt)))
          for l in range(g.n_slices)]
    geo["plan"].set_weights(to_dev(torch, dev, np.stack(Ws)))
    rng = np.random.default_rng(7)
    v = rng.standard_normal((g.n_slices, g.n_shots, g.n, g.n)) + 1j * rng.standard_normal(
        (g.n_slices, g.n_shots, g.n, g.n))
    vd = to_dev(torch, dev, v)
    got = geo["plan"].apply_AHA(vd).cpu().numpy()
    assert rel(got, o.adjoint(o.forward(v, coils, masks, theta), coils, masks, theta)) < OP_TOL
    got = geo["plan"].apply_reg(vd).cpu().numpy()
    assert rel(got, o.regulariser(v, Ws, g.lam, g.filt)) < OP_TOL
    got = geo["plan"].apply_normal(vd).cpu().numpy()
    assert rel(got, o.normal_op(v, coils, masks, theta, Ws, g.lam, g.filt)) < OP_TOL


def test_solve_matches_oracle(geo):
    from paper_1901_01893_amd import smsm
    g, case = geo["g"], geo["case"]
    ref = o.solve(geo["y"].astype(np.complex128), case["coils"], case["masks"], case["shifts"], oracle_params(g))
    x = geo["plan"].solve(to_dev(geo["torch"], geo["dev"], geo["y"])).cpu().numpy()
    assert geo["plan"].status() == smsm.SMSM_OK
    err = o.nrmse(x, ref)
    print(f"[solve {geo['name']}] NRMSE vs oracle = {err:.3e}", flush=True)
    assert err < SOLVE_TOL


def test_images_sos_matches_oracle(geo):
    # root-sum-of-squares images of random k-space (every n2 and shot count of the geometries)
    torch, dev, g = geo["torch"], geo["dev"], geo["g"]
    rng = np.random.default_rng(11)
    x = rng.standard_normal((g.n_slices, g.n_shots, g.n, g.n)) + 1j * rng.standard_normal(
        (g.n_slices, g.n_shots, g.n, g.n))
    got = geo["plan"].images_sos(to_dev(torch, dev, x)).cpu().numpy()
    assert got.shape == (g.n_slices, g.n, g.n)
    assert rel(got, o.sos_images(x)) < 1e-12
