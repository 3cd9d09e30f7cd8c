"""GPU parity of the augmented-Lagrangian solve (smsm_al_*) against the FP64
oracle of it (oracle/al_oracle.py): the thresholding step alone, whole solves
on several geometries (iterate and scaled duals), and the optimality
certificate of Eq. 10 evaluated by the oracle on the GPU's own result.

The GPU forms the singular-value thresholding from the K x K Gram with
Newton-Schulz iterations where the oracle takes an SVD of the P x K matrix;
both are exact to rounding (the Gram squares the condition number, which the
cases here keep far from the threshold), so the bars are rounding-sized: the
operator chains agree to ~1e-13, and ten outer iterations compound that to
well under 1e-10."""
import numpy as np
import pytest

import smsm_inputs as si
from oracle import al_oracle as al
from oracle import smsm_oracle as o
from tests.helpers import case_for, rel

pytestmark = pytest.mark.gpu

SOLVE_TOL = 1e-9    # whole AL solves (iterate and duals), NRMSE against the oracle


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1901_01893_amd  # noqa: F401  (fails loudly if the library is missing)
    return torch, torch.device("cuda:0")


def make_plan(torch, dev, g, case):
    from paper_1901_01893_amd import smsm
    coils = torch.from_numpy(np.ascontiguousarray(case["coils"], np.complex64)).to(dev)
    return smsm.Plan(g.n, g.n, g.n_slices, g.n_shots, g.n_coils, g.filt, coils, case["masks"], case["shifts"],
                     smsm.make_params(lam=g.lam, n_irls=1, n_cg=1, flags=smsm.SMSM_FLAG_X_C128))


def gpu_duals(solver, n_anchor):
    """[L][K][stride] -> the oracle's layout, a list of P x K matrices."""
    u = solver.dual().cpu().numpy()[:, :, :n_anchor]
    assert not np.any(solver.dual().cpu().numpy()[:, :, n_anchor:])    # zero beyond the anchors
    return [u[l].T for l in range(u.shape[0])]


def oracle_al(g, case, y, lam, beta, n_outer, n_cg):
    hist = []
    x = al.solve_al(y.astype(np.complex128), case["coils"], case["masks"], case["shifts"],
                    al.ALParams(lam=lam, r=g.filt, beta=beta, n_outer=n_outer, n_cg=n_cg), history=hist)
    return x, hist[-1]["U"]


def test_one_threshold_step_matches_the_svd(torch_dev):
    """No CG steps and one outer iteration: x = A^H y, and the duals are
    M - SVT(M) for M = H(A^H y), the thresholding alone against the oracle's
    SVD, at three thresholds (about a quarter, nine tenths and one twentieth
    of the singular values above tau)."""
    torch, dev = torch_dev
    from paper_1901_01893_amd import smsm
    g, case, _, y = case_for("small", 100)
    with make_plan(torch, dev, g, case) as plan:
        yd = torch.from_numpy(y).to(dev)
        for beta in (1e-4, 1e-3, 3e-5):
            with smsm.AL(plan, lam=1e-3, beta=beta, n_outer=1, n_cg=0) as s:
                x = s.solve(yd).cpu().numpy()
                u = gpu_duals(s, s.n_anchor)
                assert plan.status() == smsm.SMSM_OK
            xr, ur = oracle_al(g, case, y, 1e-3, beta, 1, 0)
            e_x = rel(x, xr)
            e_u = max(rel(u[l], ur[l]) for l in range(g.n_slices))
            print(f"[al threshold beta={beta}] x {e_x:.2e}, duals {e_u:.2e}", flush=True)
            assert e_x < 1e-12 and e_u < 1e-11


AL_GEOMS = {
    # the small workload: 64 x 64, MB2, 4 shots, 8 coils, 5 x 5 (K = 100, one column block of 64 and a ragged one)
    "small_r5": si.WORKLOADS["small"],
    # 7 x 7 filter, three slices: K = 196, four column blocks, the last holding 4 columns
    "n64_L3_Ns4_r7": si.Geometry(n=64, n_slices=3, n_shots=4, n_coils=8, filt=7, lam=1e-3, n_irls=1, n_cg=1,
                                 phase_order=2, snr=30.0),
    # two shots at 32 x 32: K = 50 (one ragged block), 784 anchors
    "n32_L2_Ns2_r5": si.Geometry(n=32, n_slices=2, n_shots=2, n_coils=4, filt=5, lam=1e-3, n_irls=1, n_cg=1,
                                 phase_order=2, snr=30.0),
}


@pytest.mark.parametrize("name", sorted(AL_GEOMS))
def test_al_solve_matches_oracle(torch_dev, name):
    torch, dev = torch_dev
    from paper_1901_01893_amd import smsm
    g = AL_GEOMS[name]
    case = si.make_case(g, 3, 300)
    _, y = o.simulate(case, g.n_slices, g.snr)
    y = y.astype(np.complex64)
    lam, beta, n_outer, n_cg = 1e-3, 1e-4, 10, 5
    with make_plan(torch, dev, g, case) as plan, smsm.AL(plan, lam, beta, n_outer, n_cg) as s:
        print(f"[al {name}] state {s.device_bytes() / 1e6:.1f} MB", flush=True)
        x = s.solve(torch.from_numpy(y).to(dev)).cpu().numpy()
        u = gpu_duals(s, s.n_anchor)
        assert plan.status() == smsm.SMSM_OK
    xr, ur = oracle_al(g, case, y, lam, beta, n_outer, n_cg)
    e_x = rel(x, xr)
    e_u = max(rel(u[l], ur[l]) for l in range(g.n_slices))
    print(f"[al {name}] NRMSE x {e_x:.2e}, duals {e_u:.2e}", flush=True)
    assert e_x < SOLVE_TOL and e_u < SOLVE_TOL


# the 256 x 256 slice group (32 coils, MB3, 4 shots, 7 x 7): tau = lam / beta = 50
# keeps about a quarter of the singular values of H(A^H y) (0.9 .. 241)
SG256_LAM, SG256_BETA = 1e-3, 2e-5


def test_al_solve_sg256_matches_oracle(torch_dev):
    """The 256 x 256 slice group, two outer iterations of three CG steps
    (the oracle takes about 20 s on the host): iterate and duals."""
    torch, dev = torch_dev
    from paper_1901_01893_amd import smsm
    g, case, _, y = case_for("sg256", 0)
    with make_plan(torch, dev, g, case) as plan, smsm.AL(plan, SG256_LAM, SG256_BETA, 2, 3) as s:
        x = s.solve(torch.from_numpy(y).to(dev)).cpu().numpy()
        u = gpu_duals(s, s.n_anchor)
        assert plan.status() == smsm.SMSM_OK
    xr, ur = oracle_al(g, case, y, SG256_LAM, SG256_BETA, 2, 3)
    e_x = rel(x, xr)
    e_u = max(rel(u[l], ur[l]) for l in range(g.n_slices))
    print(f"[al sg256] NRMSE x {e_x:.2e}, duals {e_u:.2e}", flush=True)
    assert e_x < SOLVE_TOL and e_u < SOLVE_TOL


def test_al_solve_is_deterministic_and_complex64_output(torch_dev):
    torch, dev = torch_dev
    from paper_1901_01893_amd import smsm
    g, case, _, y = case_for("small", 101)
    yd = torch.from_numpy(y).to(dev)
    with make_plan(torch, dev, g, case) as plan, smsm.AL(plan, 1e-3, 1e-4, 3, 4) as s, \
            smsm.AL(plan, 1e-3, 1e-4, 3, 4, c128=False) as s64:
        a = s.solve(yd)
        b = s.solve(yd)
        c = s64.solve(yd)
        torch.cuda.synchronize()
        assert torch.equal(a, b)
        assert c.dtype == torch.complex64 and torch.equal(c, a.to(torch.complex64))


def certificate_case(torch, dev):
    """A low-rank 16 x 16 slice group (two slices, two shots, four random
    coils, 3 x 3 filter) with noise, thresholded hard enough that the
    minimiser's Hankel matrices are rank-deficient."""
    rng = np.random.default_rng(41)
    n, L, Ns, Nc, r = 16, 2, 2, 4, 3
    crand = lambda *s: rng.standard_normal(s) + 1j * rng.standard_normal(s)
    coils = crand(L, Nc, n, n)
    coils /= np.sqrt(np.sum(np.abs(coils) ** 2, axis=1, keepdims=True))
    masks = o.interleaved_masks(n, Ns)
    shifts = np.arange(L) / L
    theta = o.caipi_phase(n, shifts)
    xt = crand(L, 1, n, n) * crand(1, Ns, 1, 1)
    y = o.forward(xt, coils, masks, theta) + 0.1 * masks[:, None, :, None] * crand(Ns, Nc, n, n)
    g = si.Geometry(n=n, n_slices=L, n_shots=Ns, n_coils=Nc, filt=r, lam=1.0, n_irls=1, n_cg=1,
                    phase_order=2, snr=30.0)
    case = {"coils": coils.astype(np.complex64), "masks": masks, "shifts": shifts}
    return g, case, y.astype(np.complex64)


def test_al_result_is_certified_optimal_for_eq10(torch_dev):
    """After 400 outer iterations the GPU's iterate and duals meet the
    optimality conditions of Eq. 10 as the oracle evaluates them: the
    stationarity of A^H(Ax - y) + (lam/2) sum H^H(Y) with Y = beta U / lam,
    ||Y||_2 <= 1 and Re<Y, H x> = ||H x||_* (which prove global optimality by
    convexity), and the minimiser has thresholded singular values."""
    torch, dev = torch_dev
    from paper_1901_01893_amd import smsm
    g, case, y = certificate_case(torch, dev)
    lam, beta = 3.0, 3.0
    with make_plan(torch, dev, g, case) as plan, smsm.AL(plan, lam, beta, 400, 20) as s:
        x = s.solve(torch.from_numpy(y).to(dev)).cpu().numpy()
        u = gpu_duals(s, s.n_anchor)
        assert plan.status() == smsm.SMSM_OK
    Y = [beta * ul / lam for ul in u]
    k = al.kkt_residuals(x, Y, y.astype(np.complex128), case["coils"].astype(np.complex128), case["masks"],
                         case["shifts"], lam, g.filt)
    print(f"[al certificate] {k}", flush=True)
    assert k["stationarity"] < 1e-8 and k["dual_norm"] < 1 + 1e-9 and k["alignment"] < 1e-8, k
    s_l = [np.linalg.svd(o.hankel(x[l], g.filt), compute_uv=False) for l in range(g.n_slices)]
    assert any(np.sum(sv > 1e-8 * sv[0]) < sv.size for sv in s_l)   # rank-deficient minimiser
