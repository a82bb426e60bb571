"""usbf_bmode_noalloc (the B-mode pipeline on the library's own per-GPU scratch buffer) against
usbf_bmode with a caller workspace, through the C ABI: two calls in a row, the second with a
smaller input, so a stale first call's contents in the shared buffer would show."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def usbf():
    import paper_1711_06127_amd as u
    u.lib()
    return u


def sim(g, seed, n_frames):
    frames = []
    for f in range(n_frames):
        pos, amp, _ = synth.phantom.phantom_2d(g, seed + f)
        frames.append(synth.rfsim.simulate_frame(g, pos, amp, seed + f, device="cuda"))
    return torch.stack(frames).contiguous()


def noalloc(u, rf, dg, dr):
    img = torch.full((rf.shape[0], *dg.scan_shape), float("nan"), device=rf.device)
    st = u.lib().usbf_bmode_noalloc(u._ptr(rf), rf.shape[0], ctypes.byref(dg.geom), ctypes.byref(dg.rx),
                                    ctypes.byref(dg.scan), dr, u._ptr(img), u._stream(rf.device))
    u._check(st)
    return img


def test_noalloc_matches_workspace_entry_point_twice(usbf):
    runs = [(synth.config_multiline_2d(), 3, 7100), (synth.config_small_2d(), 1, 7200)]
    for g, F, seed in runs:
        print(f"noalloc: {g.n_el} elements, {g.n_lines} lines x {g.n_depth} depths, {F} frame(s)", flush=True)
        rf = sim(g, seed, F)
        dg = usbf.DeviceGeometry(g)
        got = noalloc(usbf, rf, dg, 50.0)
        ref = usbf.bmode(rf, dg, 50.0)
        torch.cuda.synchronize()
        assert torch.isfinite(got).all()
        assert (got - ref).abs().max().item() <= 1e-6
        # and the image itself against the float64 oracle (first frame)
        ref64 = oracle.bmode_2d(oracle.das(g, rf[:1].cpu().numpy())[0], g.scan, 50.0)
        assert np.abs(got[0].cpu().numpy() - ref64).max() <= 1e-4


def test_noalloc_rejects_requests_beyond_its_scratch(usbf):
    g = synth.config_multiline_2d()
    dg = usbf.DeviceGeometry(g)
    F = 16  # 16 frames of 256 x 2048 lines need 32 MiB + row maxima: one byte too many
    need = usbf.lib().usbf_workspace_bytes(usbf.OP_BMODE, F, g.n_lines, g.n_depth)
    assert need > (32 << 20)
    rf = torch.zeros((F, g.n_tx, g.n_el, g.n_samples), dtype=torch.int16, device="cuda")
    img = torch.zeros((F, *dg.scan_shape), device="cuda")
    st = usbf.lib().usbf_bmode_noalloc(usbf._ptr(rf), F, ctypes.byref(dg.geom), ctypes.byref(dg.rx),
                                       ctypes.byref(dg.scan), 50.0, usbf._ptr(img), usbf._stream(rf.device))
    assert st == usbf.EUNSUPPORTED
    assert (img == 0).all()
