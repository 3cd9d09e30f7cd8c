"""The seeded input generators (CPU): deterministic, and a diffusion direction
changes only what a direction changes."""
import numpy as np

import smsm_inputs as si

G = si.Geometry(n=64, n_slices=2, n_shots=4, n_coils=8, filt=5, lam=1e-3, n_irls=2, n_cg=2, phase_order=2,
                snr=30.0)


def test_make_case_is_deterministic():
    a, b = si.make_case(G, 3, 7), si.make_case(G, 3, 7)
    for k in a:
        assert np.array_equal(a[k], b[k]), k
    assert not np.array_equal(a["noise"], si.make_case(G, 4, 7)["noise"])


def test_direction_case():
    case = si.make_case(G, 0, 1)
    dirs = [si.direction_case(G, case, d, 1) for d in range(12)]
    for k in ("coils", "masks", "shifts"):
        assert all(np.array_equal(d[k], case[k]) for d in dirs), k
    atts = np.array([d["attenuation"] for d in dirs])
    assert np.all((atts >= 0.3) & (atts <= 1.0)) and np.ptp(atts) > 0.2
    for d in dirs:
        # magnitude = the case's phantom times the direction's attenuation (float32 rounding)
        assert np.allclose(d["rho"], case["rho"] * d["attenuation"], rtol=1e-6, atol=1e-7)
        assert np.allclose(np.abs(d["phase"]), 1.0, atol=1e-6)      # unit-modulus shot phases
        assert not np.array_equal(d["phase"], case["phase"])
    again = si.direction_case(G, case, 5, 1)
    assert np.array_equal(again["phase"], dirs[5]["phase"]) and again["attenuation"] == dirs[5]["attenuation"]


def test_cnn_init_shapes_and_scale():
    params = si.cnn_init(2, 8, width=64, out_scale=0.1)
    chans = [8, 64, 64, 64, 64, 8]
    for k, (w, b) in enumerate(params):
        assert w.shape == (chans[k + 1], chans[k], 3, 3) and b.shape == (chans[k + 1],)
        assert w.dtype == np.float32 and np.all(b == 0)
    # He scale on the hidden layers: std ~ sqrt(2 / (9 c_in))
    assert abs(params[1][0].std() / np.sqrt(2 / (9 * 64)) - 1) < 0.05
    assert np.array_equal(si.cnn_init(2, 8)[0][0], params[0][0])
