"""The C-ABI library loads, exports every declared entry point, and rejects bad arguments with
the documented status codes before touching the GPU (runs without a GPU)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "usbf.h")


@pytest.fixture(scope="module")
def u():
    import paper_1711_06127_amd as u
    if not os.path.exists(u.LIB_PATH):
        pytest.skip("libusbf.so not built")
    u.lib()
    return u


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(usbf_[a-z0-9_]+)\s*\(", src)))


def test_every_declared_symbol_is_exported(u):
    names = declared_functions()
    assert len(names) >= 12
    L = ctypes.CDLL(u.LIB_PATH)
    for n in names:
        assert hasattr(L, n), n
    assert set(names) <= set(u.exported_symbols()) | {"usbf_version"}


def test_status_strings(u):
    L = u.lib()
    assert L.usbf_status_string(0) == b"ok"
    assert L.usbf_status_string(-1) == b"invalid argument"
    assert L.usbf_status_string(-4) == b"workspace too small"
    assert b"gfx950" in L.usbf_version()


FAKE = 0x10000  # never dereferenced: every call below fails validation first


def geom(u, n_el=4, n_tx=2, n_lines=3, dims=1):
    return u.CGeometry(n_el, FAKE, n_tx, FAKE, FAKE, FAKE, n_lines, FAKE, FAKE, FAKE, dims, 0)


def rx(u, **kw):
    d = dict(c=1540.0, fs=40e6, t0=0.0, n_samples=64, depth_start=0, depth_step=2, n_depth=32,
             f_number=1.0, window=1)
    d.update(kw)
    return u.CRx(**d)


@pytest.mark.parametrize("change,status", [
    (dict(c=0.0), -1), (dict(c=float("nan")), -1), (dict(fs=-1.0), -1), (dict(f_number=0.0), -1),
    (dict(n_samples=1), -1), (dict(depth_step=0), -1), (dict(n_depth=0), -1), (dict(window=7), -1),
    (dict(depth_start=-1), -1), (dict(depth_step=1 << 20, n_depth=100), -3),
])
def test_beamform_rejects_bad_receive_parameters(u, change, status):
    g, r = geom(u), rx(u, **change)
    assert u.lib().usbf_beamform(FAKE, 1, ctypes.byref(g), ctypes.byref(r), FAKE, None) == status
    assert len(u.lib().usbf_last_error_detail()) > 0


def test_beamform_rejects_bad_geometry_and_sizes(u):
    L = u.lib()
    r = rx(u)
    assert L.usbf_beamform(FAKE, 1, ctypes.byref(geom(u, n_el=0)), ctypes.byref(r), FAKE, None) == -2
    assert L.usbf_beamform(FAKE, 1, ctypes.byref(geom(u, n_el=2000)), ctypes.byref(r), FAKE, None) == -3
    assert L.usbf_beamform(FAKE, 1, ctypes.byref(geom(u, dims=3)), ctypes.byref(r), FAKE, None) == -1
    assert L.usbf_beamform(FAKE, 0, ctypes.byref(geom(u)), ctypes.byref(r), FAKE, None) == -1
    assert L.usbf_beamform(None, 1, ctypes.byref(geom(u)), ctypes.byref(r), FAKE, None) == -1
    assert L.usbf_beamform(FAKE, 1, None, ctypes.byref(r), FAKE, None) == -1
    g = geom(u)
    g.line_tx = None
    assert L.usbf_beamform(FAKE, 1, ctypes.byref(g), ctypes.byref(r), FAKE, None) == -1


def test_beamform_sets_rejects(u):
    """Every call fails validation before anything is enqueued (FAKE pointers)."""
    L = u.lib()
    g, r = geom(u), rx(u)

    def call(n, fns, wins, rf=FAKE, frames=1):
        fa = (ctypes.c_float * max(1, len(fns)))(*fns) if fns is not None else None
        wa = (ctypes.c_int32 * max(1, len(wins)))(*wins) if wins is not None else None
        return L.usbf_beamform_sets(rf, frames, ctypes.byref(g), ctypes.byref(r), n, fa, wa, FAKE, None)

    assert call(3, [1.0, 1.5, 2.0], [1, 1, 1]) == -3             # 1, 2 or 4 sets
    assert call(8, [1.0] * 8, [1] * 8) == -3
    assert call(0, [1.0], [1]) == -3
    assert call(2, [1.0, 0.0], [1, 1]) == -1                     # f-number must be > 0
    assert call(2, [1.0, float("inf")], [1, 1]) == -1
    assert call(2, [1.0, 2.0], [1, 7]) == -1                     # unknown window
    assert call(2, None, [1, 1]) == -1
    assert call(2, [1.0, 2.0], None) == -1
    assert call(2, [1.0, 2.0], [1, 1], rf=None) == -1
    assert call(2, [1.0, 2.0], [1, 1], frames=0) == -1


def test_combine_lines_rejects(u):
    L = u.lib()
    assert L.usbf_combine_lines(None, 1, 4, 10, FAKE, FAKE, 2, 3, FAKE, None) == -1
    assert L.usbf_combine_lines(FAKE, 0, 4, 10, FAKE, FAKE, 2, 3, FAKE + (1 << 20), None) == -1
    assert L.usbf_combine_lines(FAKE, 1, 4, 0, FAKE, FAKE, 2, 3, FAKE + (1 << 20), None) == -1
    assert L.usbf_combine_lines(FAKE, 1, 4, 10, FAKE, FAKE, 0, 3, FAKE + (1 << 20), None) == -3
    assert L.usbf_combine_lines(FAKE, 1, 4, 10, FAKE, FAKE, 65, 3, FAKE + (1 << 20), None) == -3
    assert L.usbf_combine_lines(FAKE, 1, 4, 10, FAKE, FAKE, 2, 0, FAKE + (1 << 20), None) == -1
    # out inside the input
    assert L.usbf_combine_lines(FAKE, 1, 4, 10, FAKE, FAKE, 2, 3, FAKE + 8, None) == -1


def test_mv_rejects(u):
    L = u.lib()
    assert L.usbf_mv_weights(None, 4, 128, 32, 1e-2, FAKE, FAKE, None) == -1
    assert L.usbf_mv_weights(FAKE, 4, 128, 16, 1e-2, FAKE, FAKE, None) == -3       # subaperture 32 only
    assert L.usbf_mv_weights(FAKE, 4, 300, 32, 1e-2, FAKE, FAKE, None) == -3
    assert L.usbf_mv_weights(FAKE, 4, 128, 32, 0.0, FAKE, FAKE, None) == -1
    assert L.usbf_mv_weights_averaged(FAKE, 4, 2, 128, 32, 1e-2, FAKE, FAKE, None) == -1   # even
    assert L.usbf_mv_weights_averaged(FAKE, 4, 0, 128, 32, 1e-2, FAKE, FAKE, None) == -1
    assert L.usbf_mv_weights_averaged(FAKE, 4, 257, 128, 32, 1e-2, FAKE, FAKE, None) == -1
    assert L.usbf_mv_weights_averaged(FAKE, 4, 5, 128, 32, 1e-2, None, None, None) == -1
    assert L.usbf_mv_weights_complex(None, 4, 128, 32, 1e-2, FAKE, FAKE, None) == -1
    assert L.usbf_mv_weights_complex(FAKE, 4, 128, 16, 1e-2, FAKE, FAKE, None) == -3
    assert L.usbf_mv_weights_complex(FAKE, 4, 16, 32, 1e-2, FAKE, FAKE, None) == -3     # fewer elements than L
    assert L.usbf_mv_weights_complex(FAKE, 0, 128, 32, 1e-2, FAKE, FAKE, None) == -1


def test_analytic_and_complex_gather_reject(u):
    L = u.lib()
    assert L.usbf_analytic_channels(None, 4, 1024, FAKE, None) == -1
    assert L.usbf_analytic_channels(FAKE, 0, 1024, FAKE, None) == -1
    assert L.usbf_analytic_channels(FAKE, 4, 4, FAKE, None) == -3
    assert L.usbf_analytic_channels(FAKE, 4, 8192, FAKE, None) == -3          # longer than 4096
    assert L.usbf_analytic_channels(FAKE, 4, 37 * 64, FAKE, None) == -3       # prime factor 37
    assert L.usbf_analytic_channels(FAKE, 4, 1024, FAKE + 4, None) == -1      # za not 8-byte aligned
    g, r = geom(u), rx(u)
    assert L.usbf_delay_gather_complex(None, 1, ctypes.byref(g), ctypes.byref(r), FAKE, 4, FAKE, None) == -1
    assert L.usbf_delay_gather_complex(FAKE, 1, ctypes.byref(g), ctypes.byref(r), FAKE, 0, FAKE, None) == -1
    assert L.usbf_delay_gather_complex(FAKE, 1, ctypes.byref(g), ctypes.byref(rx(u, c=-1.0)), FAKE, 4, FAKE,
                                       None) == -1


def test_bmode_noalloc_rejects_requests_beyond_its_scratch(u):
    L = u.lib()
    g, r = geom(u, n_lines=4), rx(u, n_samples=4096, depth_step=2, n_depth=2048)
    s = scan(u, n_depth=2048)
    assert L.usbf_workspace_bytes(3, 1100, 4, 2048) > (32 << 20)
    assert L.usbf_bmode_noalloc(FAKE, 1100, ctypes.byref(g), ctypes.byref(r), ctypes.byref(s), 50.0, FAKE,
                                None) == -3
    assert L.usbf_bmode_noalloc(FAKE, 1, ctypes.byref(g), ctypes.byref(r), ctypes.byref(s), -1.0, FAKE, None) == -1


def test_envelope_and_log_reject(u):
    L = u.lib()
    assert L.usbf_envelope(FAKE, 4, 4, FAKE, None, None) == -3            # too short
    assert L.usbf_envelope(FAKE, 4, 37 * 8, FAKE, None, None) == -3       # prime factor 37 > 31
    assert L.usbf_envelope(FAKE, 4, 8192, FAKE, None, None) == -3          # too long
    assert L.usbf_envelope(None, 4, 64, FAKE, None, None) == -1
    assert L.usbf_envelope(FAKE, 0, 64, FAKE, None, None) == -1
    assert L.usbf_log_compress(FAKE, 2, 100, 0.0, 1.0, FAKE, None, 0, None) == -1
    assert L.usbf_log_compress(FAKE, 2, 100, 50.0, 0.0, FAKE, None, 0, None) == -4   # needs workspace
    assert L.usbf_log_compress(FAKE, 2, 100, 50.0, 0.0, FAKE, FAKE, 4, None) == -4   # too small
    assert L.usbf_log_compress(FAKE, 0, 100, 50.0, 1.0, FAKE, None, 0, None) == -1


def scan(u, **kw):
    d = dict(kind=0, nx=8, ny=1, nz=8, x0=0.0, hx=1.0, y0=0.0, hy=0.0, z0=0.0, hz=1.0, line_u=FAKE,
             line_v=FAKE, n_u=4, n_v=1, r0=0.0, dr=1.0, n_depth=16, fill=0.0)
    d.update(kw)
    return u.CScan(**d)


@pytest.mark.parametrize("change,status", [
    (dict(kind=3), -1), (dict(line_u=None), -1), (dict(nx=0), -1), (dict(n_u=1), -2),
    (dict(kind=1, n_v=1), -2), (dict(kind=1, line_v=None), -1), (dict(dr=0.0), -1), (dict(n_depth=1), -2),
])
def test_scan_rejects(u, change, status):
    s = scan(u, **change)
    assert u.lib().usbf_scan_convert(FAKE, 1, ctypes.byref(s), FAKE, None) == status
    assert u.lib().usbf_scan_index_map(ctypes.byref(s), FAKE, None) == status


def test_bmode_rejects_inconsistent_shapes(u):
    L = u.lib()
    g, r = geom(u, n_lines=4), rx(u)
    s = scan(u, n_depth=32)
    ws = u.lib().usbf_workspace_bytes(3, 1, 4, 32)
    assert ws > 0
    s_bad = scan(u, n_depth=31)
    assert L.usbf_bmode(FAKE, 1, ctypes.byref(g), ctypes.byref(r), ctypes.byref(s_bad), 50.0, FAKE, FAKE, ws,
                        None) == -2
    g5 = geom(u, n_lines=5)
    assert L.usbf_bmode(FAKE, 1, ctypes.byref(g5), ctypes.byref(r), ctypes.byref(s), 50.0, FAKE, FAKE, ws,
                        None) == -2
    assert L.usbf_bmode(FAKE, 1, ctypes.byref(g), ctypes.byref(r), ctypes.byref(s), 50.0, FAKE, FAKE, ws - 1,
                        None) == -4
    r7 = rx(u, n_depth=37 * 2, n_samples=200)
    s7 = scan(u, n_depth=74)
    ws7 = u.lib().usbf_workspace_bytes(3, 1, 4, 74)
    assert L.usbf_bmode(FAKE, 1, ctypes.byref(g), ctypes.byref(r7), ctypes.byref(s7), 50.0, FAKE, FAKE, ws7,
                        None) == -3


def test_workspace_sizes(u):
    L = u.lib()
    assert L.usbf_workspace_bytes(1, 32, 0, 0) >= 32 * 4
    b = L.usbf_workspace_bytes(3, 32, 256, 2048)
    assert b >= 32 * 256 * 2048 * 4 + 32 * 256 * 4 + 32 * 4
    assert L.usbf_workspace_bytes(99, 1, 1, 1) == 0


def test_batch_plan_rejects(u):
    """Batch validation runs before any device call: every case fails with its status on a
    machine without a GPU."""
    L = u.lib()
    plan = ctypes.c_void_p()
    good = u.CBatchItem(FAKE, geom(u, n_lines=4), rx(u), scan(u, n_depth=32), 50.0, FAKE, FAKE, FAKE)
    arr = (u.CBatchItem * 2)(good, good)
    assert L.usbf_batch_plan_create(arr, 0, None, ctypes.byref(plan), None) == -1
    assert L.usbf_batch_plan_create(None, 1, None, ctypes.byref(plan), None) == -1
    assert L.usbf_batch_plan_create(arr, 1, None, None, None) == -1
    bad = (u.CBatchItem * 2)(good, u.CBatchItem(FAKE, geom(u, n_lines=5), rx(u), scan(u, n_depth=32), 50.0,
                                                 FAKE, FAKE, FAKE))
    assert L.usbf_batch_plan_create(bad, 2, None, ctypes.byref(plan), None) == -2      # scan lines != n_lines
    bad[1] = u.CBatchItem(FAKE, geom(u, n_lines=4), rx(u), scan(u, n_depth=31), 50.0, FAKE, FAKE, FAKE)
    assert L.usbf_batch_plan_create(bad, 2, None, ctypes.byref(plan), None) == -2      # depth counts differ
    bad[1] = u.CBatchItem(FAKE, geom(u, n_lines=4), rx(u), scan(u, n_depth=32), 0.0, FAKE, FAKE, FAKE)
    assert L.usbf_batch_plan_create(bad, 2, None, ctypes.byref(plan), None) == -1      # dynamic range
    bad[1] = u.CBatchItem(None, geom(u, n_lines=4), rx(u), scan(u, n_depth=32), 50.0, FAKE, FAKE, FAKE)
    assert L.usbf_batch_plan_create(bad, 2, None, ctypes.byref(plan), None) == -1      # null rf
    bad[1] = u.CBatchItem(FAKE, geom(u, n_lines=4), rx(u, n_depth=74, n_samples=200), scan(u, n_depth=74), 50.0,
                          FAKE, FAKE, FAKE)
    assert L.usbf_batch_plan_create(bad, 2, None, ctypes.byref(plan), None) == -3      # envelope length
    assert L.usbf_batch_run(None, None) == -1
    assert L.usbf_batch_plan_destroy(None) == 0
    sh = u.CBatchShape()
    assert L.usbf_batch_plan_shape(None, ctypes.byref(sh)) == -1
    for bad_shape in [(0, 1, 4, 1), (9, 1, 4, 1), (2, 2, 4, 1), (2, 1, 2, 1), (2, 1, 4, 0), (2, 1, 4, 9)]:
        sh = u.CBatchShape(*bad_shape)
        assert L.usbf_batch_plan_create_shaped(arr, 1, ctypes.byref(sh), ctypes.byref(plan), None) == -1, bad_shape
    assert L.usbf_batch_plan_create_shaped(arr, 1, None, ctypes.byref(plan), None) == -1
    assert L.usbf_autotune(arr, 1, None, None) == -1


def test_envelope_iq_rejects(u):
    L = u.lib()
    f = (ctypes.c_float * 4)(5e6, 4e6, 6e6, 7e6)
    assert L.usbf_envelope_iq(None, 4, 2048, 40e6, f, 3, 2e6, 63, FAKE, None, None) == -1
    assert L.usbf_envelope_iq(FAKE, 4, 2048, 40e6, f, 3, 2e6, 63, FAKE, None, None) == -1  # in place
    assert L.usbf_envelope_iq(FAKE, 0, 2048, 40e6, f, 3, 2e6, 63, FAKE + 64, None, None) == -1
    assert L.usbf_envelope_iq(FAKE, 4, 4, 40e6, f, 3, 2e6, 63, FAKE + 64, None, None) == -3
    assert L.usbf_envelope_iq(FAKE, 4, 9000, 40e6, f, 3, 2e6, 63, FAKE + 64, None, None) == -3
    assert L.usbf_envelope_iq(FAKE, 4, 2048, 40e6, f, 5, 2e6, 63, FAKE + 64, None, None) == -3
    assert L.usbf_envelope_iq(FAKE, 4, 2048, 40e6, f, 3, 2e6, 64, FAKE + 64, None, None) == -3
    assert L.usbf_envelope_iq(FAKE, 4, 2048, 40e6, f, 3, 2e6, 129, FAKE + 64, None, None) == -3
    assert L.usbf_envelope_iq(FAKE, 4, 2048, 40e6, f, 3, 0.0, 63, FAKE + 64, None, None) == -1
    bad = (ctypes.c_float * 3)(5e6, 25e6, 6e6)
    assert L.usbf_envelope_iq(FAKE, 4, 2048, 40e6, bad, 3, 2e6, 63, FAKE + 64, None, None) == -1


def test_compound_rejects(u):
    L = u.lib()
    assert L.usbf_compound(None, 1, 2, 100, FAKE, None) == -1
    assert L.usbf_compound(FAKE, 0, 2, 100, FAKE + 4096, None) == -1
    assert L.usbf_compound(FAKE, 1, 0, 100, FAKE + 4096, None) == -1
    assert L.usbf_compound(FAKE, 1, 2, 100, FAKE + 400, None) == -1   # out inside the input


def test_lines_per_tx_hint(u):
    """Tiles of G lines share one staging of a transmit's channel data when every line of the
    group that has a transmit has the group's first line's transmit."""
    import numpy as np
    import synth
    h = u.lines_per_tx_hint
    assert h(synth.config_multiline_2d().line_tx) == 4
    assert h(synth.config_small_2d().line_tx) == 1
    assert h(synth.config_planewave_2d(lines=64, n_samples=256).line_tx) == 64
    assert h(synth.config_overlap_2d(n_el=16, n_samples=256).line_tx) == 4
    assert h(np.array([0, 1, 1, 1, 1])) == 1
    assert h(np.array([0, 0, 1, 1, 2, 2, 3])) == 2
    assert h(np.array([-1, -1, -1, -1, 0, 0, 0, 0])) == 4
    assert h(np.array([0, -1, 0, -1, 1, 1, 1, -1])) == 4
    assert h(np.array([-1, 0, 0, 0, 1, 1, 1, 1])) == 1


def test_delay_gather_rejects(u):
    L = u.lib()
    g, r = geom(u), rx(u)
    bg, br = ctypes.byref(g), ctypes.byref(r)
    assert L.usbf_delay_gather(None, 1, bg, br, FAKE, 4, FAKE, None) == -1
    assert L.usbf_delay_gather(FAKE, 0, bg, br, FAKE, 4, FAKE, None) == -1
    assert L.usbf_delay_gather(FAKE, 1, bg, br, FAKE, 0, FAKE, None) == -1
    assert L.usbf_delay_gather_depths(FAKE, 1, bg, br, FAKE, 4, 4, FAKE, None) == -1     # even
    assert L.usbf_delay_gather_depths(FAKE, 1, bg, br, FAKE, 4, 0, FAKE, None) == -1
    assert L.usbf_delay_gather_depths(FAKE, 1, bg, br, FAKE, 4, 257, FAKE, None) == -1
    assert L.usbf_delay_gather_depths(FAKE, 1, bg, br, None, 4, 5, FAKE, None) == -1
    assert L.usbf_delay_gather_depths(FAKE, 1, bg, br, FAKE, 4, 5, None, None) == -1
