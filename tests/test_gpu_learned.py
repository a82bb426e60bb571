"""Learned apodization end to end on the GPU: trained on minimum-variance targets by the
library's own kernels, it must move its weights towards MV's and narrow the point-spread
function relative to plain delay-and-sum (the method without the network)."""
import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def setup():
    import paper_1711_06127_amd as u
    from paper_1711_06127_amd import learned as L
    u.lib()
    g = synth.config_multiline_2d()
    dg = u.DeviceGeometry(g)
    rfs = []
    for f in range(4):
        pos, amp, _ = synth.phantom.phantom_2d(g, 300 + f)
        rfs.append(synth.rfsim.simulate_frame(g, pos, amp, 300 + f, device="cuda"))
    rf = torch.stack(rfs).contiguous()
    model = L.LearnedApodization(g.n_el, seed=0)
    hist = model.train(rf, dg, steps=400, batch=4096, lr=2e-3, log_every=50)
    torch.cuda.synchronize()
    return u, L, g, dg, model, hist


def test_training_reduces_loss(setup):
    u, L, g, dg, model, hist = setup
    losses = [l for _, l in hist]
    assert all(np.isfinite(losses))
    # the untrained network gives uniform weights: training must beat that loss clearly
    assert losses[-1] < 0.85 * losses[0]


def test_weights_move_towards_mv(setup):
    u, L, g, dg, model, hist = setup
    pos, amp, _ = synth.phantom.phantom_2d(g, 777)
    rf = synth.rfsim.simulate_frame(g, pos, amp, 777, device="cuda").contiguous()
    gen = torch.Generator(device="cuda")
    gen.manual_seed(5)
    pix = L.random_pixels(gen, 8192, 1, g.n_lines, g.n_depth, g.n_depth // 8)
    x = u.delay_gather(rf, dg, pix)
    w_mv, _ = u.mv_weights(x, L.SUBAPERTURE, L.LOADING)
    w_net = model.weights(x)
    err_net = (w_net - w_mv).norm().item()
    err_uniform = (torch.full_like(w_mv, 1.0 / g.n_el) - w_mv).norm().item()
    assert err_net < err_uniform


def test_learned_narrows_psf_against_das(setup):
    """-6 dB widths on lines a twentieth of a wavelength apart through the 8 points of a
    held-out frame."""
    u, L, g, dg, model, hist = setup
    rf, cyst, lj = L.eval_phantom(g, 90901)
    w = {m: L.psf_widths_fine(rf, g, m, model, lj) for m in ("das", "learned")}
    assert np.all(np.isfinite(w["das"])) and np.all(w["das"] > 0)
    assert np.mean(w["learned"]) < np.mean(w["das"])


def test_evaluation_runs_and_reports(setup):
    u, L, g, dg, model, hist = setup
    res = L.evaluate(model, g, dg, n_frames=2)
    for m in ("das", "mv", "learned"):
        assert np.isfinite(res[m]["cnr_mean"]) and res[m]["psf_width_mm_mean"] > 0
    # minimum variance narrows the point-spread function of delay and sum
    assert res["mv"]["psf_width_mm_mean"] < res["das"]["psf_width_mm_mean"]
    assert isinstance(res["learned_vs_mv"]["pass"], bool)
    assert res["timing"]["mv_ms_per_frame"] > 0 and res["timing"]["learned_ms_per_frame"] > 0


def test_fallback_on_non_finite_weights(setup):
    u, L, g, dg, model, hist = setup
    x = torch.randn(100, g.n_el, device="cuda")
    wts = torch.full_like(x, 1.0 / g.n_el)
    wts[7, 3] = float("nan")
    wts[50, 0] = float("inf")
    fb = torch.arange(100, dtype=torch.float32, device="cuda")
    y = u.beamform_weighted(x, wts, fb)
    ref = (x * (1.0 / g.n_el)).sum(1)
    assert y[7].item() == 7.0 and y[50].item() == 50.0
    ok = torch.ones(100, dtype=torch.bool, device="cuda")
    ok[7] = ok[50] = False
    assert torch.allclose(y[ok], ref[ok], rtol=1e-5, atol=1e-5)
