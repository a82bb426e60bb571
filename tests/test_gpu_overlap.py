"""The overlapping multi-line layout on the GPU (255 lines from 128 transmits, Sec. 3.3,
Table 1): the beams of every transmit's line slots (unused slots give zeros), their weighted
combination into the output lines and the image, against the CPU oracle."""
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


def sim(g, seed, n_frames):
    frames = []
    for f in range(n_frames):
        pos, amp, _ = synth.phantom.phantom_2d(g, seed + f)
        frames.append(synth.rfsim.simulate_frame(g, pos, amp, seed + f, device="cuda"))
    return torch.stack(frames).contiguous()


def tables(g):
    return (torch.as_tensor(g.combine_src, device="cuda"), torch.as_tensor(g.combine_w, device="cuda"))


def test_overlap_beams_combination_and_image(usbf):
    g = synth.config_overlap_2d(n_el=32, n_samples=1024, scan_n=(128, 128))
    rf = sim(g, 800, 3)
    dg = usbf.DeviceGeometry(g)
    y = usbf.beamform(rf, dg)
    src, w = tables(g)
    out = usbf.combine_lines(y, src, w)
    torch.cuda.synchronize()
    ref = oracle.das(g, rf.cpu().numpy())
    yh = y.cpu().numpy()
    assert rel(yh, ref) <= TOL
    assert np.all(yh[:, g.line_tx < 0] == 0.0)
    ref_out = oracle.combine_lines(ref, g.combine_src, g.combine_w)
    assert out.shape == (3, g.n_out_lines, g.n_depth)
    assert rel(out.cpu().numpy(), ref_out) <= TOL
    env = usbf.envelope(out)
    img = usbf.log_scan_convert(env, dg, 50.0)
    ref_img = oracle.bmode_2d(ref_out[2], g.scan, 50.0)
    assert np.abs(img.cpu().numpy()[2] - ref_img).max() <= TOL


def test_overlap_full_size_sampled(usbf):
    """The full layout (128 transmits, 512 line slots, 4096 samples) in its launch, sampled
    pixels of the beams against the oracle."""
    g = synth.config_overlap_2d()
    rf = sim(g, 810, 2)
    dg = usbf.DeviceGeometry(g)
    y = usbf.beamform(rf, dg).cpu().numpy()
    rng = np.random.default_rng(4)
    m = 4000
    pix = np.stack([rng.integers(0, 2, m), rng.integers(0, g.n_lines, m), rng.integers(0, g.n_depth, m)], 1)
    ref = oracle.das(g, rf.cpu().numpy(), pix)
    assert rel(y[pix[:, 0], pix[:, 1], pix[:, 2]], ref) <= TOL


def test_combine_lines_general(usbf):
    """Random sources and weights, including sources that are not lines of the input."""
    gen = torch.Generator().manual_seed(3)
    x = torch.randn(3, 20, 333, generator=gen).cuda()
    src = torch.randint(-1, 22, (17, 5), generator=gen, dtype=torch.int32)  # 20, 21: not lines
    w = torch.randn(17, 5, generator=gen)
    got = usbf.combine_lines(x, src.cuda(), w.cuda()).cpu().double()
    xd = x.cpu().double()
    ref = torch.zeros(3, 17, 333, dtype=torch.float64)
    for o in range(17):
        for k in range(5):
            s = int(src[o, k])
            if 0 <= s < 20:
                ref[:, o] += float(w[o, k]) * xd[:, s]
    assert torch.allclose(got, ref, rtol=1e-5, atol=1e-5)
