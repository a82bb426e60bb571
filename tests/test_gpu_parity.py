"""GPU library vs CPU oracle: index maps bit-exact, values within 1e-4 of float64.

Accuracy measure for beamformed lines and envelopes: max |gpu - oracle| / max |oracle| per
frame; for log-compressed and scan-converted images: max |gpu - oracle| on the [0, 1] scale.
"""
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


def rel_err(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def sim(g, seed, n_frames=1, device="cuda", **kw):
    frames = []
    for f in range(n_frames):
        pos, amp, _ = synth.phantom.phantom_2d(g, seed + f, **kw)
        frames.append(synth.rfsim.simulate_frame(g, pos, amp, seed + f, device=device))
    return torch.stack(frames).contiguous()


def sub_geometry_3d(n_lines=48, seed=0):
    """Subset of the 3D workload's lines (and their transmits), all 1024 elements."""
    g = synth.config_volume_3d()
    rng = np.random.default_rng(seed)
    sel = np.sort(rng.choice(g.n_lines, n_lines, replace=False))
    g.line_origin = np.ascontiguousarray(g.line_origin[sel])
    g.line_dir = np.ascontiguousarray(g.line_dir[sel])
    g.tx_origin = np.ascontiguousarray(g.tx_origin[sel])
    g.tx_dir = np.ascontiguousarray(g.tx_dir[sel])
    g.tx_focus = np.ascontiguousarray(g.tx_focus[sel])
    g.line_tx = np.arange(n_lines, dtype=np.int32)
    g.scan = None
    return g


# ------------------------------------------------------------------ delay index map

@pytest.mark.parametrize("cfg", ["small", "multiline", "volume_subset"])
def test_delay_index_map_bit_exact(usbf, cfg):
    g = {"small": synth.config_small_2d, "multiline": synth.config_multiline_2d,
         "volume_subset": sub_geometry_3d}[cfg]()
    dg = usbf.DeviceGeometry(g)
    i0, fl, phi = usbf.delay_index_map(dg)
    torch.cuda.synchronize()
    oi0, ophi, oact, oval = oracle.tof32(g)
    oi0 = oi0.reshape(g.n_lines, g.n_depth, g.n_el)
    assert np.array_equal(i0.cpu().numpy(), oi0)
    ofl = (oact.astype(np.uint8) | (oval.astype(np.uint8) << 1)).reshape(i0.shape)
    assert np.array_equal(fl.cpu().numpy(), ofl)
    assert np.array_equal(phi.cpu().numpy().view(np.uint32), ophi.reshape(i0.shape).view(np.uint32))


# ------------------------------------------------------------------ beamforming

def test_beamform_small_frame_matches_oracle(usbf):
    g = synth.config_small_2d()
    rf = sim(g, 1000)
    dg = usbf.DeviceGeometry(g)
    y = usbf.beamform(rf, dg)
    torch.cuda.synchronize()
    ref = oracle.das(g, rf.cpu().numpy())
    assert rel_err(y.cpu().numpy(), ref) <= TOL


@pytest.mark.parametrize("n_frames", [1, 3, 5, 29, 33])
def test_beamform_multiline_frames(usbf, n_frames):
    """Frame blocking (1, 2, 4 ... 32 frames per pass plus a ragged remainder) on the multi-line
    geometry; sampled pixels of every frame against the oracle."""
    g = synth.config_multiline_2d()
    base = sim(g, 2000, n_frames=min(n_frames, 3))
    rf = base[torch.arange(n_frames) % base.shape[0]].clone()
    rf[3:] = torch.roll(rf[3:], shifts=1, dims=-1)       # frames beyond the first three differ too
    dg = usbf.DeviceGeometry(g)
    y = usbf.beamform(rf, dg).cpu().numpy()
    rng = np.random.default_rng(n_frames)
    m = 4000
    pix = np.stack([rng.integers(0, n_frames, m), rng.integers(0, g.n_lines, m), rng.integers(0, g.n_depth, m)], 1)
    ref = oracle.das(g, rf.cpu().numpy(), pix)
    got = y[pix[:, 0], pix[:, 1], pix[:, 2]]
    assert rel_err(got, ref) <= TOL


def test_beamform_32_frame_launch_first_and_last_frames_whole(usbf):
    """The benchmark's launch -- 32 multi-line frames in one block -- with the first and the last
    frame compared element by element (256 x 2048 lines each) against the oracle."""
    g = synth.config_multiline_2d()
    base = sim(g, 2600, n_frames=2)
    rf = base[torch.arange(32) % 2].clone()
    rf[2:] = torch.roll(rf[2:], shifts=5, dims=-1)
    rf[31] = torch.flip(rf[31], dims=[-1])  # the last frame unlike every other
    dg = usbf.DeviceGeometry(g)
    y = usbf.beamform(rf, dg).cpu().numpy()
    ref = oracle.das(g, rf[[0, 31]].cpu().numpy())
    for k, f in enumerate((0, 31)):
        assert rel_err(y[f], ref[k]) <= TOL, f


def test_beamform_small_geometry_frame_blocks(usbf):
    """One line per transmit with 37 frames (blocks of 32 + 4 + 1) against the oracle on
    sampled pixels of every frame."""
    g = synth.config_small_2d()
    base = sim(g, 2500, n_frames=2)
    rf = base[torch.arange(37) % 2].clone()
    rf[2:] = torch.roll(rf[2:], shifts=3, dims=-1)
    dg = usbf.DeviceGeometry(g)
    y = usbf.beamform(rf, dg).cpu().numpy()
    rng = np.random.default_rng(37)
    m = 4000
    pix = np.stack([rng.integers(0, 37, m), rng.integers(0, g.n_lines, m), rng.integers(0, g.n_depth, m)], 1)
    ref = oracle.das(g, rf.cpu().numpy(), pix)
    assert rel_err(y[pix[:, 0], pix[:, 1], pix[:, 2]], ref) <= TOL


def test_beamform_volume_subset(usbf):
    """3D matrix probe, steered lines, separable Hann: a subset of lines with all 1024 elements."""
    g = sub_geometry_3d(n_lines=24, seed=3)
    rng = np.random.default_rng(0)
    rf = torch.as_tensor(rng.integers(-3000, 3000, size=(1, g.n_tx, g.n_el, g.n_samples), dtype=np.int16)).cuda()
    dg = usbf.DeviceGeometry(g)
    y = usbf.beamform(rf, dg)
    torch.cuda.synchronize()
    ref = oracle.das(g, rf.cpu().numpy())
    assert rel_err(y.cpu().numpy(), ref) <= TOL


def test_beamform_full_volume_sampled(usbf):
    """The whole 3D workload (1024 steered lines, 1024 elements, 2000 samples) in the launch the
    benchmark times, checked against the oracle on sampled voxels of every line block."""
    g = synth.config_volume_3d()
    gen = torch.Generator(device="cuda")
    gen.manual_seed(11)
    rf = torch.randint(-3000, 3000, (1, g.n_tx, g.n_el, g.n_samples), dtype=torch.int16, device="cuda", generator=gen)
    dg = usbf.DeviceGeometry(g)
    y = usbf.beamform(rf, dg).cpu().numpy()
    rng = np.random.default_rng(11)
    m = 3000
    pix = np.stack([np.zeros(m, np.int64), rng.integers(0, g.n_lines, m), rng.integers(0, g.n_depth, m)], 1)
    ref = oracle.das(g, rf.cpu().numpy(), pix)
    assert rel_err(y[pix[:, 0], pix[:, 1], pix[:, 2]], ref) <= TOL


def test_beamform_full_volume_depth_rows_every_line(usbf):
    """The whole 3D workload in the benchmark's launch: eight depth rows (both ends, the
    quarter points, a row inside each of the first and last depth tiles) of every one of the
    1024 lines, element by element against the oracle."""
    g = synth.config_volume_3d()
    gen = torch.Generator(device="cuda")
    gen.manual_seed(12)
    rf = torch.randint(-3000, 3000, (1, g.n_tx, g.n_el, g.n_samples), dtype=torch.int16, device="cuda", generator=gen)
    dg = usbf.DeviceGeometry(g)
    y = usbf.beamform(rf, dg).cpu().numpy()[0]
    rows = np.array([0, 1, 200, 250, 500, 750, 900, g.n_depth - 1])
    pix = np.stack([np.zeros(g.n_lines * rows.size, np.int64), np.repeat(np.arange(g.n_lines), rows.size),
                    np.tile(rows, g.n_lines)], 1)
    ref = oracle.das(g, rf.cpu().numpy(), pix)
    assert rel_err(y[pix[:, 1], pix[:, 2]], ref) <= TOL


def test_beamform_edge_cases(usbf):
    """Ragged depth count, a transmit index out of range (zero line), a depth grid starting at
    sample 0 (empty aperture except the element under the line), rectangular window, t0 != 0."""
    g = synth.config_tiny(n_el=7, n_tx=3, lines_per_tx=3, n_samples=300, window=synth.RECT)
    g.n_depth = 137
    g.t0 = float(np.float32(3.0e-7))
    g.line_tx = g.line_tx.copy()
    g.line_tx[4] = 99
    rng = np.random.default_rng(7)
    rf = torch.as_tensor(rng.integers(-30000, 30000, size=(2, g.n_tx, g.n_el, g.n_samples), dtype=np.int16)).cuda()
    dg = usbf.DeviceGeometry(g)
    y = usbf.beamform(rf, dg).cpu().numpy()
    assert np.all(y[:, 4] == 0.0)
    ref = oracle.das(g, rf.cpu().numpy())  # the oracle also gives zeros for that line
    assert rel_err(y, ref) <= TOL


@pytest.mark.parametrize("n_samples,depth_step,n_frames", [(301, 1, 5), (600, 3, 5), (2048, 16, 2)])
def test_beamform_unusual_grids(usbf, n_samples, depth_step, n_frames):
    """A record length that is not a multiple of 4 (element-by-element staging loads), an odd
    depth step (unsplit windows), a depth step so large that the staged windows are capped (taps
    outside them read global memory), a ragged last group of lines (19 lines, 4 per transmit)
    and frame blocks of 4 + 1."""
    g = synth.linear_2d("odd", n_el=16, n_tx=5, lines_per_tx=4, line_pitch=0.15e-3, n_samples=n_samples,
                        depth_step=depth_step, scan_n=(16, 16))
    g.line_origin, g.line_dir, g.line_tx = g.line_origin[:19], g.line_dir[:19], g.line_tx[:19]
    assert usbf.lines_per_tx_hint(g.line_tx) == 4
    rng = np.random.default_rng(n_samples)
    rf = torch.as_tensor(rng.integers(-30000, 30000, size=(n_frames, g.n_tx, g.n_el, g.n_samples),
                                      dtype=np.int16)).cuda()
    y = usbf.beamform(rf, usbf.DeviceGeometry(g)).cpu().numpy()
    assert y.shape == (n_frames, 19, g.n_depth)
    assert rel_err(y, oracle.das(g, rf.cpu().numpy())) <= TOL


@pytest.mark.parametrize("nx,ny,window,n_frames", [(2, 12, synth.HANN, 1), (5, 6, synth.HANN, 3),
                                                   (8, 6, synth.RECT, 2)])
def test_beamform_one_line_tiles_on_matrix_arrays(usbf, nx, ny, window, n_frames):
    """Tiles of one line (one transmit per line) on matrix arrays whose rows are 2, 5 or 8
    elements wide: element chunks that span three or more rows, chunks that lie on one row
    (their Hann y factor applied to the chunk's sum), a rectangular window; a ragged last
    depth tile; blocks of one and of several frames."""
    g = synth.matrix_3d("rows", n_side=4, n_samples=600, n_lines_side=5, window=window)
    g.el_pos = synth.geometry.matrix_array(nx, ny, 0.3e-3)
    g.scan = None
    assert usbf.lines_per_tx_hint(g.line_tx) == 1
    rng = np.random.default_rng(100 * nx + ny)
    rf = torch.as_tensor(rng.integers(-3000, 3000, size=(n_frames, g.n_tx, g.n_el, g.n_samples),
                                      dtype=np.int16)).cuda()
    y = usbf.beamform(rf, usbf.DeviceGeometry(g)).cpu().numpy()
    assert rel_err(y, oracle.das(g, rf.cpu().numpy())) <= TOL


@pytest.mark.parametrize("n_samples,depth_step,n_frames", [(301, 1, 3), (600, 3, 2), (2048, 16, 1)])
def test_beamform_one_line_tiles_unusual_grids(usbf, n_samples, depth_step, n_frames):
    """Tiles of one line with a record length that is not a multiple of 4, an odd depth step,
    and a depth step so large that the staged windows are capped (the lanes with taps outside
    them re-derive those taps and read global memory)."""
    g = synth.linear_2d("odd1", n_el=16, n_tx=12, lines_per_tx=1, line_pitch=0.3e-3, n_samples=n_samples,
                        depth_step=depth_step, scan_n=(16, 16))
    assert usbf.lines_per_tx_hint(g.line_tx) == 1
    rng = np.random.default_rng(n_samples + 7)
    rf = torch.as_tensor(rng.integers(-30000, 30000, size=(n_frames, g.n_tx, g.n_el, g.n_samples),
                                      dtype=np.int16)).cuda()
    y = usbf.beamform(rf, usbf.DeviceGeometry(g)).cpu().numpy()
    assert rel_err(y, oracle.das(g, rf.cpu().numpy())) <= TOL


def test_beamform_deterministic(usbf):
    g = synth.config_small_2d()
    rf = sim(g, 1234)
    dg = usbf.DeviceGeometry(g)
    a = usbf.beamform(rf, dg).clone()
    b = usbf.beamform(rf, dg)
    assert torch.equal(a, b)


# ------------------------------------------------------------------ envelope, log, scan

@pytest.mark.parametrize("n", [8, 60, 256, 512, 1000, 1024, 1536, 2048, 1408, 1664, 1792, 950, 850, 1922])
def test_envelope_matches_oracle(usbf, n):
    rng = np.random.default_rng(n)
    x = rng.standard_normal((37, n)).astype(np.float32)
    env, rm = usbf.envelope(torch.as_tensor(x).cuda(), row_max=True)
    ref = oracle.envelope(x.astype(np.float64))
    assert rel_err(env.cpu().numpy(), ref) <= TOL
    assert np.array_equal(rm.cpu().numpy(), env.cpu().numpy().max(1))


@pytest.mark.parametrize("n", [256, 2048, 1000])
def test_envelope_in_place(usbf, n):
    """The pipeline detects in place (output buffer = input buffer); enough rows that every
    workgroup of the resident grid prefetches a next row while it writes the current one."""
    rng = np.random.default_rng(n + 1)
    x = rng.standard_normal((4096, n)).astype(np.float32)
    buf = torch.as_tensor(x).cuda()
    sep = usbf.envelope(buf.clone())
    env, rm = usbf.envelope(buf, out=buf, row_max=True)
    assert env.data_ptr() == buf.data_ptr()
    assert torch.equal(env, sep)
    assert rel_err(env.cpu().numpy(), oracle.envelope(x.astype(np.float64))) <= TOL
    assert np.array_equal(rm.cpu().numpy(), env.cpu().numpy().max(1))


def test_envelope_in_place(usbf):
    x = torch.randn(16, 1024, device="cuda")
    ref = usbf.envelope(x.clone())
    usbf.envelope(x, out=x)
    assert torch.equal(x, ref)


def test_log_compress_matches_oracle(usbf):
    rng = np.random.default_rng(3)
    env = rng.rayleigh(1.0, (3, 4096)).astype(np.float32)
    env[1] *= 1e-3
    env[2, :10] = 0.0
    got = usbf.log_compress(torch.as_tensor(env).cuda(), 50.0).cpu().numpy()
    for f in range(3):
        assert np.abs(got[f] - oracle.log_compress(env[f].astype(np.float64), 50.0)).max() <= TOL
    got2 = usbf.log_compress(torch.as_tensor(env).cuda(), 40.0, ref=2.5).cpu().numpy()
    assert np.abs(got2 - oracle.log_compress(env.astype(np.float64), 40.0, ref=2.5)).max() <= TOL


@pytest.mark.parametrize("cfg", ["small", "multiline", "volume"])
def test_scan_index_map_bit_exact(usbf, cfg):
    g = {"small": synth.config_small_2d, "multiline": synth.config_multiline_2d,
         "volume": synth.config_volume_3d}[cfg]()
    dg = usbf.DeviceGeometry(g)
    base = usbf.scan_index_map(dg).cpu().numpy()
    s = g.scan
    if s.kind == 1:
        iu, iv, jd, ok, *_ = oracle.scan_index_3d(s)
        want = np.where(ok, (iv * s.n_u + iu) * s.n_depth + jd, -1)
    else:
        iu, jd, ok, *_ = oracle.scan_index_2d(s)
        want = np.where(ok, iu * s.n_depth + jd, -1)
    assert np.array_equal(base, want)


def test_sector_scan_index_and_values(usbf):
    """2D sector (kind 2): lines fanning out from the origin, u = x/z."""
    tan_u = np.tan(np.radians(np.linspace(-35, 35, 96))).astype(np.float32)
    s = synth.geometry.ScanGrid(kind=2, nx=300, ny=1, nz=260, x0=-0.05, hx=1e-4 / 0.3 * 1.0, y0=0, hy=0,
                                z0=0.0, hz=2e-4, line_u=tan_u, line_v=np.zeros(1, np.float32), r0=1e-3,
                                dr=float(np.float32(5e-5)), n_depth=1000)
    s.hx = float(np.float32(1e-1 / 299))
    g = synth.config_small_2d()
    dg = usbf.DeviceGeometry(g)
    dg.set_scan(s)
    base = usbf.scan_index_map(dg).cpu().numpy()
    iu, jd, ok, *_ = oracle.scan_index_2d(s)
    assert ok.sum() > 1000
    assert np.array_equal(base, np.where(ok, iu * s.n_depth + jd, -1))
    lines = np.random.default_rng(1).standard_normal((1, 96, 1000)).astype(np.float32)
    got = usbf.scan_convert(torch.as_tensor(lines).cuda(), dg).cpu().numpy()[0]
    ref = oracle.scan_convert_2d(lines[0].astype(np.float64), s)
    assert np.abs(got - ref).max() <= TOL * np.abs(ref).max()


def test_scan_convert_3d_matches_oracle(usbf):
    g = synth.config_volume_3d()
    s = g.scan
    dg = usbf.DeviceGeometry(g)
    rng = np.random.default_rng(5)
    lines = rng.random((1, g.n_lines, g.n_depth)).astype(np.float32)
    got = usbf.scan_convert(torch.as_tensor(lines).cuda(), dg).cpu().numpy()[0]
    zs = [0, 1, 17, 64, 100, 127]
    ref = oracle.scan_convert_3d(lines[0].astype(np.float64), s, z_slices=zs)
    assert np.abs(got[zs] - ref).max() <= TOL


def test_log_scan_fused_equals_sequence(usbf):
    g = synth.config_small_2d()
    dg = usbf.DeviceGeometry(g)
    env = torch.rand(2, g.n_lines, g.n_depth, device="cuda") ** 4
    seq = usbf.scan_convert(usbf.log_compress(env, 50.0), dg)
    fused = usbf.log_scan_convert(env, dg, 50.0)
    assert (seq - fused).abs().max().item() <= 1e-6


# ------------------------------------------------------------------ whole pipeline

def test_bmode_small_frame_end_to_end(usbf):
    g = synth.config_small_2d()
    rf = sim(g, 1000)
    dg = usbf.DeviceGeometry(g)
    img = usbf.bmode(rf, dg, 50.0).cpu().numpy()[0]
    ref = oracle.bmode_2d(oracle.das(g, rf.cpu().numpy())[0], g.scan, 50.0)
    assert np.abs(img - ref).max() <= TOL


def test_bmode_multiline_frames_end_to_end(usbf):
    g = synth.config_multiline_2d()
    rf = sim(g, 2100, n_frames=2)
    dg = usbf.DeviceGeometry(g)
    img = usbf.bmode(rf, dg, 50.0).cpu().numpy()
    bf = oracle.das(g, rf.cpu().numpy())
    for f in range(2):
        ref = oracle.bmode_2d(bf[f], g.scan, 50.0)
        assert np.abs(img[f] - ref).max() <= TOL


def test_point_targets_peak_on_their_pixels(usbf):
    """Noiseless point targets on the pixel grid: the GPU envelope peaks on each target pixel
    within its neighbourhood."""
    g = synth.config_small_2d()
    pp, pa, lj = synth.phantom.points_2d(g)
    rf = synth.rfsim.simulate_frame(g, pp, pa, 0, noise=False, device="cuda").unsqueeze(0).contiguous()
    dg = usbf.DeviceGeometry(g)
    env = usbf.envelope(usbf.beamform(rf, dg))[0].cpu().numpy()
    for (l, j) in lj:
        win = env[max(l - 2, 0):l + 3, j - 20:j + 21]
        ll, jj = np.unravel_index(np.argmax(win), win.shape)
        assert (ll + max(l - 2, 0), jj + j - 20) == (l, j)


# ------------------------------------------------------------------ delay-gather and minimum variance

def test_delay_gather_matches_oracle(usbf):
    g = synth.config_multiline_2d()
    rf = sim(g, 3000, n_frames=2)
    dg = usbf.DeviceGeometry(g)
    rng = np.random.default_rng(0)
    m = 3000
    pix = np.stack([rng.integers(0, 2, m), rng.integers(0, g.n_lines, m), rng.integers(0, g.n_depth, m)], 1)
    pix[:5] = [[0, 0, 0], [1, 255, 2047], [0, 128, 1], [1, 3, 1024], [0, 77, 2046]]
    x = usbf.delay_gather(rf, dg, torch.as_tensor(pix, dtype=torch.int32).cuda()).cpu().numpy()
    ref = oracle.delay_gather(g, rf.cpu().numpy(), pix)
    assert np.abs(x - ref).max() <= TOL * np.abs(ref).max()


def test_delay_gather_out_of_range_pixels_give_zeros(usbf):
    g = synth.config_small_2d()
    rf = sim(g, 3100)
    dg = usbf.DeviceGeometry(g)
    pix = torch.tensor([[0, 5, 100], [1, 5, 100], [0, 64, 0], [0, 0, 1024], [-1, 0, 0]], dtype=torch.int32).cuda()
    x = usbf.delay_gather(rf, dg, pix).cpu().numpy()
    assert np.abs(x[0]).max() > 0 and np.all(x[1:] == 0)


def test_mv_weights_match_oracle(usbf):
    """Binary32 covariance, binary64 Cholesky, binary32 expansion and sum: weights within 1e-2
    (relative 2-norm; the loaded matrix has condition number <= 1 + L/loading = 3201) and
    outputs within 1e-3 of the float64 oracle on the same binary32 inputs."""
    from oracle import mv
    g = synth.config_multiline_2d()
    rf = sim(g, 3200)
    dg = usbf.DeviceGeometry(g)
    rng = np.random.default_rng(1)
    m = 2000
    pix = np.stack([np.zeros(m, int), rng.integers(0, g.n_lines, m), rng.integers(200, g.n_depth, m)], 1)
    # both sides solve for the same binary32 samples: the oracle's gather, rounded
    x32 = oracle.delay_gather(g, rf.cpu().numpy(), pix).astype(np.float32)
    wf, y = usbf.mv_weights(torch.as_tensor(x32).cuda(), 32, 1e-2)
    wf_ref, y_ref, _ = mv.mv_weights(x32.astype(np.float64), 32, 1e-2)
    wf = wf.cpu().numpy()
    rel = np.linalg.norm(wf - wf_ref, axis=1) / np.linalg.norm(wf_ref, axis=1)
    assert np.median(rel) < 1e-3 and rel.max() < 1e-2
    assert np.abs(y.cpu().numpy() - y_ref).max() <= 1e-3 * np.abs(y_ref).max()
    np.testing.assert_allclose(wf.sum(1), 1.0, atol=1e-5)


def test_mv_closed_forms_on_gpu(usbf):
    """Coherent data -> uniform subaperture weights; a nulled interferer (cf. the oracle pins)."""
    M = 128
    x = torch.full((3, M), 2.5, device="cuda")
    wf, y = usbf.mv_weights(x, 32, 1e-2)
    np.testing.assert_allclose(y.cpu().numpy(), 2.5, rtol=1e-5)
    K = 97
    count = np.array([min(e, 31) - max(0, e - K + 1) + 1 for e in range(M)])
    np.testing.assert_allclose(wf.cpu().numpy(), np.broadcast_to(count / (K * 32), (3, M)), atol=1e-6)


def test_mv_weights_averaged_match_oracle(usbf):
    """Covariance averaged over 5 neighbouring depths (clamped at the line ends) of gathered
    samples, against the float64 oracle on the same binary32 inputs, at the tolerances of the
    single-depth estimator; one depth equals the single-depth entry point bit for bit."""
    from oracle import mv
    g = synth.config_multiline_2d()
    rf = sim(g, 3300)
    dg = usbf.DeviceGeometry(g)
    rng = np.random.default_rng(2)
    m = 1500
    pix = np.stack([np.zeros(m, int), rng.integers(0, g.n_lines, m), rng.integers(0, g.n_depth, m)], 1)
    pix[:3, 2] = [0, 1, g.n_depth - 1]  # the clamped ends of a line
    x = usbf.delay_gather(rf, dg, torch.as_tensor(pix, dtype=torch.int32).cuda(), n_avg=5)
    assert x.shape == (m, 5, g.n_el)
    # the library's neighbour rows against the oracle's gather at the clamped depths
    nb = np.repeat(pix[:, None, :], 5, axis=1)
    nb[:, :, 2] = np.clip(nb[:, :, 2] + np.arange(-2, 3)[None, :], 0, g.n_depth - 1)
    ref_x = oracle.delay_gather(g, rf.cpu().numpy(), nb.reshape(-1, 3)).reshape(m, 5, g.n_el)
    assert rel_err(x.cpu().numpy(), ref_x) <= TOL
    # both sides solve for the same binary32 samples: the oracle's gather, rounded
    x32 = ref_x.astype(np.float32)
    wf, y = usbf.mv_weights_averaged(torch.as_tensor(x32).cuda(), 32, 1e-2)
    wf_ref, y_ref, _ = mv.mv_weights_averaged(x32.astype(np.float64), 32, 1e-2)
    wf = wf.cpu().numpy()
    rel = np.linalg.norm(wf - wf_ref, axis=1) / np.linalg.norm(wf_ref, axis=1)
    assert np.median(rel) < 1e-3 and rel.max() < 1e-2
    assert np.abs(y.cpu().numpy() - y_ref).max() <= 1e-3 * np.abs(y_ref).max()
    np.testing.assert_allclose(wf.sum(1), 1.0, atol=1e-5)
    # the middle row is the pixel itself, and one row is the single-depth estimator exactly
    x1 = usbf.delay_gather(rf, dg, torch.as_tensor(pix, dtype=torch.int32).cuda())
    assert torch.equal(x[:, 2].contiguous(), x1)
    a, ya = usbf.mv_weights_averaged(x1.view(m, 1, g.n_el).contiguous(), 32, 1e-2)
    b, yb = usbf.mv_weights(x1, 32, 1e-2)
    assert torch.equal(a, b) and torch.equal(ya, yb)
