"""Several apodization sets in one delay-and-sum pass (two differently parameterised beamformers
on the same input, Sec. 2): every set must equal the single-set beamformer run with its own
f-number and window, and the CPU oracle with those parameters."""
import copy

import numpy as np
import pytest
import torch

import oracle
import synth
from synth.geometry import HANN, RECT

pytestmark = pytest.mark.gpu

TOL = 1e-4


@pytest.fixture(scope="module")
def usbf():
    import paper_1711_06127_amd as u
    u.lib()
    return u


def rel(a, b):
    return float(np.abs(np.asarray(a, np.float64) - b).max() / max(np.abs(b).max(), 1e-300))


def with_params(g, f_number, window):
    g2 = copy.copy(g)
    g2.f_number = float(np.float32(f_number))
    g2.window = window
    return g2


def sim(g, seed, n_frames):
    frames = []
    for f in range(n_frames):
        pos, amp, _ = synth.phantom.phantom_2d(g, seed + f)
        frames.append(synth.rfsim.simulate_frame(g, pos, amp, seed + f, device="cuda"))
    return torch.stack(frames).contiguous()


def check_sets(usbf, g, rf, sets, full_oracle=True):
    dg = usbf.DeviceGeometry(g)
    fns = [s[0] for s in sets]
    wins = [s[1] for s in sets]
    out = usbf.beamform_sets(rf, dg, fns, wins)
    torch.cuda.synchronize()
    assert out.shape == (len(sets), rf.shape[0], g.n_lines, g.n_depth)
    got = out.cpu().numpy()
    rf_h = rf.cpu().numpy()
    for k, (fn, win) in enumerate(sets):
        gk = with_params(g, fn, win)
        single = usbf.beamform(rf, usbf.DeviceGeometry(gk)).cpu().numpy()
        # same binary32 rule and summation order as the single-set call
        assert rel(got[k], single) <= 1e-6, (k, fn, win)
        if full_oracle:
            assert rel(got[k], oracle.das(gk, rf_h)) <= TOL, (k, fn, win)
    return got


def test_two_sets_multiline(usbf):
    g = synth.linear_2d("ml16", n_el=128, n_tx=16, lines_per_tx=4, line_pitch=0.15e-3, n_samples=1024)
    rf = sim(g, 700, 3)  # 3 frames: a block of 2 and a block of 1
    got = check_sets(usbf, g, rf, [(1.0, HANN), (2.0, RECT)])
    # the sets differ: a wider aperture is not the same image
    assert rel(got[0], got[1]) > 1e-2


def test_four_sets_single_line_tiles(usbf):
    g = synth.linear_2d("s32", n_el=64, n_tx=32, lines_per_tx=1, line_pitch=0.3e-3, n_samples=1024)
    rf = sim(g, 710, 2)
    check_sets(usbf, g, rf, [(1.0, HANN), (1.5, HANN), (2.5, RECT), (0.7, HANN)])


def test_one_set_is_the_plain_beamformer(usbf):
    g = synth.linear_2d("ml8", n_el=128, n_tx=8, lines_per_tx=4, line_pitch=0.15e-3, n_samples=1024)
    rf = sim(g, 720, 2)
    dg = usbf.DeviceGeometry(with_params(g, 1.3, HANN))
    a = usbf.beamform_sets(rf, dg, [1.3], [HANN])[0]
    b = usbf.beamform(rf, dg)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_two_sets_volume_subset(usbf):
    from tests.test_gpu_parity import sub_geometry_3d
    g = sub_geometry_3d(n_lines=12, seed=3)
    rng = np.random.default_rng(1)
    rf = torch.as_tensor(rng.integers(-3000, 3000, size=(1, g.n_tx, g.n_el, g.n_samples), dtype=np.int16)).cuda()
    check_sets(usbf, g, rf, [(1.0, HANN), (1.8, RECT)])


def test_two_sets_full_multiline_batch_sampled(usbf):
    """The multi-line workload (32 frames, 128 elements, 4 lines per transmit) with two sets,
    sampled pixels of every set against the oracle."""
    g = synth.config_multiline_2d()
    rf = sim(g, 730, 4)[torch.arange(32) % 4].contiguous()
    dg = usbf.DeviceGeometry(g)
    sets = [(1.0, HANN), (1.75, RECT)]
    out = usbf.beamform_sets(rf, dg, [s[0] for s in sets], [s[1] for s in sets])
    torch.cuda.synchronize()
    rng = np.random.default_rng(8)
    m = 3000
    pix = np.stack([rng.integers(0, 32, m), rng.integers(0, g.n_lines, m), rng.integers(0, g.n_depth, m)], 1)
    rf_h = rf[:4].cpu().numpy()
    for k, (fn, win) in enumerate(sets):
        y = out[k].cpu().numpy()[pix[:, 0], pix[:, 1], pix[:, 2]]
        ref = oracle.das(with_params(g, fn, win), rf_h, np.stack([pix[:, 0] % 4, pix[:, 1], pix[:, 2]], 1))
        assert rel(y, ref) <= TOL, k
