"""Plane-wave imaging on the GPU: infinite-focus transmits (and diverging waves from a virtual
source behind the array) in the binary32 delay rule (index map bit-exact), beamforming of every
line for every steered wave, and coherent compounding, against the CPU oracle."""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

TOL = 1e-4


@pytest.fixture(scope="module")
def usbf():
    import paper_1711_06127_amd as u
    u.lib()
    return u


def rel(a, b):
    return float(np.abs(np.asarray(a, np.float64) - b).max() / max(np.abs(b).max(), 1e-300))


def sim(g, seed, n_frames=1):
    frames = []
    for f in range(n_frames):
        pos, amp, _ = synth.phantom.phantom_2d(g, seed + f)
        frames.append(synth.rfsim.simulate_frame(g, pos, amp, seed + f, device="cuda"))
    return torch.stack(frames).contiguous()


FOCI = [pytest.param(np.inf, id="plane"), pytest.param(-20e-3, id="diverging")]


@pytest.mark.parametrize("focus", FOCI)
def test_planewave_delay_index_map_bit_exact(usbf, focus):
    g = synth.config_planewave_2d(n_samples=2048, lines=64, focus=focus, max_angle_deg=10.0 if np.isinf(focus) else 20.0)
    dg = usbf.DeviceGeometry(g)
    i0, fl, phi = usbf.delay_index_map(dg)
    torch.cuda.synchronize()
    oi0, ophi, oact, oval = oracle.tof32(g)
    assert np.array_equal(i0.cpu().numpy(), oi0.reshape(i0.shape))
    ofl = (oact.astype(np.uint8) | (oval.astype(np.uint8) << 1)).reshape(i0.shape)
    assert np.array_equal(fl.cpu().numpy(), ofl)
    assert np.array_equal(phi.cpu().numpy().view(np.uint32), ophi.reshape(i0.shape).view(np.uint32))


@pytest.mark.parametrize("focus", FOCI)
def test_planewave_beamform_and_compound_match_oracle(usbf, focus):
    g = synth.config_planewave_2d(n_samples=1024, lines=64, scan_n=(128, 128), focus=focus)
    rf = sim(g, 610, n_frames=3)
    dg = usbf.DeviceGeometry(g)
    lines = usbf.beamform(rf, dg)
    comp = usbf.compound(lines, g.n_angles)
    torch.cuda.synchronize()
    ref = oracle.das(g, rf.cpu().numpy())
    assert rel(lines.cpu().numpy(), ref) <= TOL
    ref_c = ref.reshape(3, g.n_angles, 64, g.n_depth).mean(axis=1)
    assert comp.shape == (3, 64, g.n_depth)
    assert rel(comp.cpu().numpy(), ref_c) <= TOL
    # and through detection to the image
    env = usbf.envelope(comp)
    img = usbf.log_scan_convert(env, dg, 50.0)
    ref_img = oracle.bmode_2d(ref_c[1], g.scan, 50.0)
    assert np.abs(img.cpu().numpy()[1] - ref_img).max() <= TOL


def test_planewave_full_size_sampled(usbf):
    """The benchmark's plane-wave frame (11 angles x 256 lines x 2048 depths, 128 elements)
    in its launch, sampled pixels against the oracle."""
    g = synth.config_planewave_2d()
    rf = sim(g, 620, n_frames=2)
    dg = usbf.DeviceGeometry(g)
    y = usbf.beamform(rf, dg).cpu().numpy()
    rng = np.random.default_rng(2)
    m = 4000
    pix = np.stack([rng.integers(0, 2, m), rng.integers(0, g.n_lines, m), rng.integers(0, g.n_depth, m)], 1)
    ref = oracle.das(g, rf.cpu().numpy(), pix)
    assert rel(y[pix[:, 0], pix[:, 1], pix[:, 2]], ref) <= TOL


def test_compound_is_the_mean(usbf):
    x = torch.randn(4, 7 * 33, 130, device="cuda")
    got = usbf.compound(x, 7)
    ref = x.view(4, 7, 33, 130).double().mean(dim=1).float()
    assert torch.allclose(got, ref, rtol=1e-6, atol=1e-6)
