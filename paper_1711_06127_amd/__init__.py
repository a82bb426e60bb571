"""Python binding of libusbf, the MI355X receive-pipeline library (include/usbf.h).

Argument marshalling only: every step runs in the library's HIP kernels.  PyTorch supplies
device memory and the current stream.  There is no CPU fallback: when libusbf.so is not
built, or no GPU is present, every call raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libusbf.so")

OK, EINVAL, ESHAPE, EUNSUPPORTED, EWORKSPACE, EDEVICE = 0, -1, -2, -3, -4, -5
WINDOW_RECT, WINDOW_HANN = 0, 1
OP_LOG_COMPRESS, OP_LOG_SCAN, OP_BMODE, OP_MV, OP_APODNET = 1, 2, 3, 4, 5

P = ctypes.c_void_p
I32, I64, F32 = ctypes.c_int32, ctypes.c_int64, ctypes.c_float


class UsbfError(RuntimeError):
    def __init__(self, status: int, detail: str):
        super().__init__(f"usbf status {status}: {detail}")
        self.status = status


class CGeometry(ctypes.Structure):
    _fields_ = [("n_el", I32), ("el_pos", P), ("n_tx", I32), ("tx_origin", P), ("tx_dir", P),
                ("tx_focus", P), ("n_lines", I32), ("line_origin", P), ("line_dir", P),
                ("line_tx", P), ("array_dims", I32), ("lines_per_tx", I32)]


class CRx(ctypes.Structure):
    _fields_ = [("c", F32), ("fs", F32), ("t0", F32), ("n_samples", I32), ("depth_start", I32),
                ("depth_step", I32), ("n_depth", I32), ("f_number", F32), ("window", I32)]


class CScan(ctypes.Structure):
    _fields_ = [("kind", I32), ("nx", I32), ("ny", I32), ("nz", I32), ("x0", F32), ("hx", F32),
                ("y0", F32), ("hy", F32), ("z0", F32), ("hz", F32), ("line_u", P), ("line_v", P),
                ("n_u", I32), ("n_v", I32), ("r0", F32), ("dr", F32), ("n_depth", I32), ("fill", F32)]


class CBatchItem(ctypes.Structure):
    _fields_ = [("rf", P), ("geom", CGeometry), ("rx", CRx), ("scan", CScan), ("dyn_range_db", F32),
                ("lines", P), ("row_max", P), ("image", P)]


class CBatchShape(ctypes.Structure):
    _fields_ = [("groups_per_cu", I32), ("cost_order", I32), ("multi_line_tile", I32), ("chunk_div", I32)]


# name -> (restype, argtypes)
_SIGS = {
    "usbf_beamform": (I32, [P, I32, P, P, P, P]),
    "usbf_beamform_sets": (I32, [P, I32, P, P, I32, P, P, P, P]),
    "usbf_envelope": (I32, [P, I64, I32, P, P, P]),
    "usbf_envelope_iq": (I32, [P, I64, I32, F32, P, I32, F32, I32, P, P, P]),
    "usbf_compound": (I32, [P, I32, I32, I64, P, P]),
    "usbf_combine_lines": (I32, [P, I32, I32, I64, P, P, I32, I32, P, P]),
    "usbf_log_compress": (I32, [P, I32, I64, F32, F32, P, P, ctypes.c_size_t, P]),
    "usbf_scan_convert": (I32, [P, I32, P, P, P]),
    "usbf_log_scan_convert": (I32, [P, P, I32, P, F32, F32, P, P, ctypes.c_size_t, P]),
    "usbf_bmode": (I32, [P, I32, P, P, P, F32, P, P, ctypes.c_size_t, P]),
    "usbf_bmode_noalloc": (I32, [P, I32, P, P, P, F32, P, P]),
    "usbf_workspace_bytes": (ctypes.c_size_t, [I32, I64, I64, I64]),
    "usbf_delay_index_map": (I32, [P, P, P, P, P, P]),
    "usbf_scan_index_map": (I32, [P, P, P]),
    "usbf_delay_gather": (I32, [P, I32, P, P, P, I32, P, P]),
    "usbf_delay_gather_depths": (I32, [P, I32, P, P, P, I32, I32, P, P]),
    "usbf_mv_weights": (I32, [P, I32, I32, I32, F32, P, P, P]),
    "usbf_mv_weights_averaged": (I32, [P, I32, I32, I32, I32, F32, P, P, P]),
    "usbf_analytic_channels": (I32, [P, I64, I32, P, P]),
    "usbf_delay_gather_complex": (I32, [P, I32, P, P, P, I32, P, P]),
    "usbf_mv_weights_complex": (I32, [P, I32, I32, I32, F32, P, P, P]),
    "usbf_apodnet_state_bytes": (ctypes.c_size_t, []),
    "usbf_apodnet_num_params": (I32, []),
    "usbf_apodnet_init": (I32, [P, P, P]),
    "usbf_apodnet_forward": (I32, [P, P, I32, I32, P, P, ctypes.c_size_t, P]),
    "usbf_apodnet_train_step": (I32, [P, P, P, I32, I32, F32, P, P, ctypes.c_size_t, P]),
    "usbf_apodnet_gradients": (I32, [P, P, P, I32, I32, P, P, ctypes.c_size_t, P]),
    "usbf_apodnet_apply": (I32, [P, P, I32, I32, P, P, P, P]),
    "usbf_beamform_weighted": (I32, [P, P, P, I32, I32, P, P]),
    "usbf_batch_plan_create": (I32, [P, I32, ctypes.c_char_p, P, P]),
    "usbf_batch_run": (I32, [P, P]),
    "usbf_batch_plan_destroy": (I32, [P]),
    "usbf_batch_plan_create_shaped": (I32, [P, I32, P, P, P]),
    "usbf_batch_plan_shape": (I32, [P, P]),
    "usbf_autotune": (I32, [P, I32, ctypes.c_char_p, P]),
    "usbf_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "usbf_last_error_detail": (ctypes.c_char_p, []),
    "usbf_version": (ctypes.c_char_p, []),
}

_lib = None


def lib():
    """The loaded libusbf.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with python paper_1711_06127_amd/build.py "
                               "(or __graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def exported_symbols():
    return list(_SIGS)


def _check(status: int):
    if status != OK:
        detail = lib().usbf_last_error_detail().decode()
        raise UsbfError(int(status), f"{lib().usbf_status_string(status).decode()}: {detail}")


def _stream(dev: torch.device):
    return ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def _need_cuda(t: torch.Tensor, name: str, dtype=None):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def lines_per_tx_hint(line_tx) -> int:
    """Length of the runs of consecutive lines that share a transmit when all runs have the same
    length; else the largest G in (8, 4, 2) such that in every aligned group of G lines each line
    that has a transmit (index >= 0) has the transmit of the group's first line (lines without
    one are zeros and share anything); else 1."""
    lt = np.asarray(line_tx)
    if lt.size:
        change = np.flatnonzero(lt[1:] != lt[:-1])
        run = int(change[0]) + 1 if change.size else int(lt.size)
        if run > 1 and lt.size % run == 0 and np.all(lt.reshape(-1, run) == lt.reshape(-1, run)[:, :1]):
            return run
    for G in (8, 4, 2):
        n = (lt.size // G) * G
        if not n:
            continue
        t = lt[:n].reshape(-1, G)
        if np.all((t < 0) | (t == t[:, :1])) and np.all((t[:, 0] >= 0) | np.all(t < 0, axis=1)):
            return G
    return 1


class DeviceGeometry:
    """Probe/scanline geometry, receive parameters and (optionally) a scan grid, uploaded to
    the device once and reused by every call.  `g` is any object with the attributes of
    synth.geometry.Geometry (el_pos, tx_origin, ..., scan)."""

    def __init__(self, g, device="cuda"):
        dev = torch.device(device)
        f32 = lambda a: torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32), device=dev)
        self.device = dev
        self.n_el, self.n_tx, self.n_lines = int(g.el_pos.shape[0]), int(g.tx_origin.shape[0]), int(g.line_origin.shape[0])
        self.n_samples, self.n_depth = int(g.n_samples), int(g.n_depth)
        self.el_pos, self.tx_origin, self.tx_dir = f32(g.el_pos), f32(g.tx_origin), f32(g.tx_dir)
        self.tx_focus, self.line_origin, self.line_dir = f32(g.tx_focus), f32(g.line_origin), f32(g.line_dir)
        self.line_tx = torch.as_tensor(np.ascontiguousarray(g.line_tx, dtype=np.int32), device=dev)
        self.geom = CGeometry(self.n_el, self.el_pos.data_ptr(), self.n_tx, self.tx_origin.data_ptr(),
                              self.tx_dir.data_ptr(), self.tx_focus.data_ptr(), self.n_lines,
                              self.line_origin.data_ptr(), self.line_dir.data_ptr(), self.line_tx.data_ptr(),
                              int(g.array_dims), lines_per_tx_hint(g.line_tx))
        self.rx = CRx(g.c, g.fs, g.t0, g.n_samples, g.depth_start, g.depth_step, g.n_depth, g.f_number,
                      int(g.window))
        self.scan = None
        s = getattr(g, "scan", None)
        if s is not None:
            self.set_scan(s)

    def set_scan(self, s):
        dev = self.device
        self.line_u = torch.as_tensor(np.ascontiguousarray(s.line_u, dtype=np.float32), device=dev)
        self.line_v = torch.as_tensor(np.ascontiguousarray(s.line_v, dtype=np.float32), device=dev)
        self.scan = CScan(s.kind, s.nx, s.ny, s.nz, s.x0, s.hx, s.y0, s.hy, s.z0, s.hz,
                          self.line_u.data_ptr(), self.line_v.data_ptr(), s.n_u, s.n_v, s.r0, s.dr,
                          s.n_depth, s.fill)
        self.scan_shape = tuple(s.out_shape)


def workspace_bytes(op: int, n_frames: int, n_lines: int = 0, n_depth: int = 0) -> int:
    return int(lib().usbf_workspace_bytes(op, n_frames, n_lines, n_depth))


def _ws(nbytes: int, dev):
    return torch.empty(max(nbytes, 1), dtype=torch.uint8, device=dev)


def beamform(rf: torch.Tensor, dg: DeviceGeometry, out: torch.Tensor | None = None) -> torch.Tensor:
    """Delay-and-sum.  rf int16 [F, n_tx, n_el, S] (or [n_tx, n_el, S]) -> float32 [F, n_lines, n_depth]."""
    _need_cuda(rf, "rf", torch.int16)
    if rf.dim() == 3:
        rf = rf.unsqueeze(0)
    F = rf.shape[0]
    if tuple(rf.shape[1:]) != (dg.n_tx, dg.n_el, dg.n_samples):
        raise ValueError(f"rf shape {tuple(rf.shape)} does not match geometry")
    if out is None:
        out = torch.empty((F, dg.n_lines, dg.n_depth), dtype=torch.float32, device=rf.device)
    _check(lib().usbf_beamform(_ptr(rf), F, ctypes.byref(dg.geom), ctypes.byref(dg.rx), _ptr(out), _stream(rf.device)))
    return out


def beamform_sets(rf: torch.Tensor, dg: DeviceGeometry, f_numbers, windows, out: torch.Tensor | None = None):
    """Delay-and-sum with several apodizations (f-number, window) in one pass over the channel
    data.  rf int16 [F, n_tx, n_el, S] -> float32 [n_sets, F, n_lines, n_depth]."""
    _need_cuda(rf, "rf", torch.int16)
    if rf.dim() == 3:
        rf = rf.unsqueeze(0)
    F = rf.shape[0]
    if tuple(rf.shape[1:]) != (dg.n_tx, dg.n_el, dg.n_samples):
        raise ValueError(f"rf shape {tuple(rf.shape)} does not match geometry")
    n = len(f_numbers)
    if len(windows) != n:
        raise ValueError("one window per f-number")
    fn = (ctypes.c_float * n)(*[float(v) for v in f_numbers])
    wn = (ctypes.c_int32 * n)(*[int(v) for v in windows])
    if out is None:
        out = torch.empty((n, F, dg.n_lines, dg.n_depth), dtype=torch.float32, device=rf.device)
    _check(lib().usbf_beamform_sets(_ptr(rf), F, ctypes.byref(dg.geom), ctypes.byref(dg.rx), n, fn, wn, _ptr(out),
                                    _stream(rf.device)))
    return out


def envelope(x: torch.Tensor, out: torch.Tensor | None = None, row_max=False):
    """Analytic-signal magnitude along the last axis.  Returns env, or (env, per-row maxima)
    when row_max is True or a preallocated float32 tensor of x.shape[:-1]."""
    _need_cuda(x, "x", torch.float32)
    n = x.shape[-1]
    rows = x.numel() // n
    if out is None:
        out = torch.empty_like(x)
    if isinstance(row_max, torch.Tensor):
        _need_cuda(row_max, "row_max", torch.float32)
        rm = row_max
    else:
        rm = torch.empty(x.shape[:-1], dtype=torch.float32, device=x.device) if row_max else None
    _check(lib().usbf_envelope(_ptr(x), rows, n, _ptr(out), _ptr(rm), _stream(x.device)))
    return (out, rm) if rm is not None else out


def envelope_iq(x: torch.Tensor, fs: float, freqs, bandwidth: float, n_taps: int = 63,
                out: torch.Tensor | None = None, row_max=False):
    """IQ-demodulation envelope with frequency compounding along the last axis (centre
    frequencies `freqs` in Hz).  Returns env, or (env, per-row maxima) when row_max is True or a
    preallocated float32 tensor of x.shape[:-1]."""
    _need_cuda(x, "x", torch.float32)
    n = x.shape[-1]
    rows = x.numel() // n
    if out is None:
        out = torch.empty_like(x)
    if isinstance(row_max, torch.Tensor):
        _need_cuda(row_max, "row_max", torch.float32)
        rm = row_max
    else:
        rm = torch.empty(x.shape[:-1], dtype=torch.float32, device=x.device) if row_max else None
    f = (ctypes.c_float * len(freqs))(*[float(v) for v in freqs])
    _check(lib().usbf_envelope_iq(_ptr(x), rows, n, float(fs), f, len(freqs), float(bandwidth), int(n_taps),
                                  _ptr(out), _ptr(rm), _stream(x.device)))
    return (out, rm) if rm is not None else out


def compound(x: torch.Tensor, n_groups: int, out: torch.Tensor | None = None) -> torch.Tensor:
    """Coherent compounding: x [F, n_groups * L, ...] (per-transmit beamformed lines, transmit
    major) -> mean over the transmits, [F, L, ...]."""
    _need_cuda(x, "x", torch.float32)
    F = x.shape[0]
    per = x.numel() // F
    if per % n_groups:
        raise ValueError("lines are not a multiple of n_groups")
    if out is None:
        out = torch.empty((F, x.shape[1] // n_groups, *x.shape[2:]), dtype=torch.float32, device=x.device)
    _check(lib().usbf_compound(_ptr(x), F, n_groups, per // n_groups, _ptr(out), _stream(x.device)))
    return out


def combine_lines(x: torch.Tensor, src: torch.Tensor, w: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
    """Weighted combination of beamformed lines: x [F, n_in, D], src int32 / w float32
    [n_out, K] (device) -> out [F, n_out, D], out[f, o] = sum_k w[o, k] x[f, src[o, k]]
    (sources outside [0, n_in) add nothing)."""
    _need_cuda(x, "x", torch.float32)
    _need_cuda(src, "src", torch.int32)
    _need_cuda(w, "w", torch.float32)
    if src.shape != w.shape or src.dim() != 2:
        raise ValueError("src and w must both be [n_out, K]")
    F, n_in = x.shape[0], x.shape[1]
    length = x.numel() // (F * n_in)
    n_out, k = src.shape
    if out is None:
        out = torch.empty((F, n_out, *x.shape[2:]), dtype=torch.float32, device=x.device)
    _check(lib().usbf_combine_lines(_ptr(x), F, n_in, length, _ptr(src), _ptr(w), k, n_out, _ptr(out),
                                    _stream(x.device)))
    return out


def log_compress(env: torch.Tensor, dyn_range_db: float = 50.0, ref: float | None = None,
                 out: torch.Tensor | None = None) -> torch.Tensor:
    """Per-frame log compression to [0, 1]; env [F, ...]; ref None -> each frame's maximum."""
    _need_cuda(env, "env", torch.float32)
    F = env.shape[0]
    if out is None:
        out = torch.empty_like(env)
    ws = _ws(workspace_bytes(OP_LOG_COMPRESS, F), env.device)
    _check(lib().usbf_log_compress(_ptr(env), F, env.numel() // F, dyn_range_db, 0.0 if ref is None else ref,
                                   _ptr(out), _ptr(ws), ws.numel(), _stream(env.device)))
    return out


def scan_convert(lines: torch.Tensor, dg: DeviceGeometry, out: torch.Tensor | None = None) -> torch.Tensor:
    """Bilinear/trilinear scan conversion; lines [F, n_lines, n_depth] -> [F, *grid]."""
    _need_cuda(lines, "lines", torch.float32)
    F = lines.shape[0]
    if out is None:
        out = torch.empty((F, *dg.scan_shape), dtype=torch.float32, device=lines.device)
    _check(lib().usbf_scan_convert(_ptr(lines), F, ctypes.byref(dg.scan), _ptr(out), _stream(lines.device)))
    return out


def log_scan_convert(env: torch.Tensor, dg: DeviceGeometry, dyn_range_db: float = 50.0, ref: float | None = None,
                     row_max: torch.Tensor | None = None, out: torch.Tensor | None = None) -> torch.Tensor:
    _need_cuda(env, "env", torch.float32)
    F = env.shape[0]
    if out is None:
        out = torch.empty((F, *dg.scan_shape), dtype=torch.float32, device=env.device)
    ws = _ws(workspace_bytes(OP_LOG_SCAN, F), env.device)
    _check(lib().usbf_log_scan_convert(_ptr(env), _ptr(row_max), F, ctypes.byref(dg.scan), dyn_range_db,
                                       0.0 if ref is None else ref, _ptr(out), _ptr(ws), ws.numel(),
                                       _stream(env.device)))
    return out


class BmodeWorkspace:
    """Reusable workspace for bmode() (keeps allocation out of timed loops)."""

    def __init__(self, dg: DeviceGeometry, n_frames: int):
        self.nbytes = workspace_bytes(OP_BMODE, n_frames, dg.n_lines, dg.n_depth)
        self.buf = _ws(self.nbytes, dg.device)
        self.n_frames = n_frames

    def lines(self, dg: DeviceGeometry) -> torch.Tensor:
        n = self.n_frames * dg.n_lines * dg.n_depth
        return self.buf[: 4 * n].view(torch.float32).view(self.n_frames, dg.n_lines, dg.n_depth)


def bmode(rf: torch.Tensor, dg: DeviceGeometry, dyn_range_db: float = 50.0, out: torch.Tensor | None = None,
          ws: BmodeWorkspace | None = None) -> torch.Tensor:
    """Channel data -> display image: beamform, envelope, log compression, scan conversion."""
    _need_cuda(rf, "rf", torch.int16)
    if rf.dim() == 3:
        rf = rf.unsqueeze(0)
    F = rf.shape[0]
    if out is None:
        out = torch.empty((F, *dg.scan_shape), dtype=torch.float32, device=rf.device)
    if ws is None or ws.n_frames != F:
        ws = BmodeWorkspace(dg, F)
    _check(lib().usbf_bmode(_ptr(rf), F, ctypes.byref(dg.geom), ctypes.byref(dg.rx), ctypes.byref(dg.scan),
                            dyn_range_db, _ptr(out), _ptr(ws.buf), ws.nbytes, _stream(rf.device)))
    return out


def delay_index_map(dg: DeviceGeometry, with_phi: bool = True):
    """(i0 int32, flags uint8, phi float32) each [n_lines, n_depth, n_el]."""
    shape = (dg.n_lines, dg.n_depth, dg.n_el)
    i0 = torch.empty(shape, dtype=torch.int32, device=dg.device)
    fl = torch.empty(shape, dtype=torch.uint8, device=dg.device)
    phi = torch.empty(shape, dtype=torch.float32, device=dg.device) if with_phi else None
    _check(lib().usbf_delay_index_map(ctypes.byref(dg.geom), ctypes.byref(dg.rx), _ptr(i0), _ptr(fl), _ptr(phi),
                                      _stream(dg.device)))
    return i0, fl, phi


def scan_index_map(dg: DeviceGeometry) -> torch.Tensor:
    base = torch.empty(dg.scan_shape, dtype=torch.int32, device=dg.device)
    _check(lib().usbf_scan_index_map(ctypes.byref(dg.scan), _ptr(base), _stream(dg.device)))
    return base


def delay_gather(rf: torch.Tensor, dg: DeviceGeometry, pix: torch.Tensor, out: torch.Tensor | None = None,
                 n_avg: int = 1):
    """Delayed channel samples for pixels pix int32 [n_pix, 3] (frame, line, depth): x [n_pix, n_el],
    or with n_avg > 1 (odd) x [n_pix, n_avg, n_el], the samples at the n_avg depths centred on
    each pixel (clamped to the line by the library)."""
    _need_cuda(rf, "rf", torch.int16)
    if rf.dim() == 3:
        rf = rf.unsqueeze(0)
    _need_cuda(pix, "pix", torch.int32)
    n = pix.shape[0]
    shape = (n, dg.n_el) if n_avg == 1 else (n, n_avg, dg.n_el)
    if out is None:
        out = torch.empty(shape, dtype=torch.float32, device=rf.device)
    _need_cuda(out, "out", torch.float32)
    if tuple(out.shape) != shape:
        raise ValueError(f"out must be {shape}")
    if n_avg == 1:
        _check(lib().usbf_delay_gather(_ptr(rf), rf.shape[0], ctypes.byref(dg.geom), ctypes.byref(dg.rx), _ptr(pix),
                                       n, _ptr(out), _stream(rf.device)))
    else:
        _check(lib().usbf_delay_gather_depths(_ptr(rf), rf.shape[0], ctypes.byref(dg.geom), ctypes.byref(dg.rx),
                                              _ptr(pix), n, n_avg, _ptr(out), _stream(rf.device)))
    return out


def mv_weights(x: torch.Tensor, subap: int = 32, loading: float = 1e-2, want_weights: bool = True):
    """Minimum-variance weights (w_full [n_pix, n_el] or None, y [n_pix]) of delayed samples x."""
    _need_cuda(x, "x", torch.float32)
    n, m = x.shape
    wf = torch.empty_like(x) if want_weights else None
    y = torch.empty(n, dtype=torch.float32, device=x.device)
    _check(lib().usbf_mv_weights(_ptr(x), n, m, subap, loading, _ptr(wf), _ptr(y), _stream(x.device)))
    return wf, y


def mv_weights_averaged(x: torch.Tensor, subap: int = 32, loading: float = 1e-2, want_weights: bool = True):
    """Minimum variance with the covariance averaged over depths: x [n_pix, n_avg, n_el]
    (n_avg odd; the pixel's own samples in the middle row) -> (w_full or None, y)."""
    _need_cuda(x, "x", torch.float32)
    n, t, m = x.shape
    wf = torch.empty((n, m), dtype=torch.float32, device=x.device) if want_weights else None
    y = torch.empty(n, dtype=torch.float32, device=x.device)
    _check(lib().usbf_mv_weights_averaged(_ptr(x), n, t, m, subap, loading, _ptr(wf), _ptr(y), _stream(x.device)))
    return wf, y


def analytic_channels(rf: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
    """Analytic signal of every channel trace (last axis) of int16 rf: complex64 of rf's shape."""
    _need_cuda(rf, "rf", torch.int16)
    n = rf.shape[-1]
    rows = rf.numel() // n
    if out is None:
        out = torch.empty(rf.shape, dtype=torch.complex64, device=rf.device)
    _need_cuda(out, "out", torch.complex64)
    if tuple(out.shape) != tuple(rf.shape):
        raise ValueError(f"out must be {tuple(rf.shape)}")
    _check(lib().usbf_analytic_channels(_ptr(rf), rows, n, _ptr(out), _stream(rf.device)))
    return out


def delay_gather_complex(za: torch.Tensor, dg: DeviceGeometry, pix: torch.Tensor) -> torch.Tensor:
    """Delayed complex samples z [n_pix, n_el] (complex64) of analytic channel data za
    complex64 [n_frames, n_tx, n_el, n_samples] at pixels pix int32 [n_pix, 3]."""
    _need_cuda(za, "za", torch.complex64)
    if za.dim() == 3:
        za = za.unsqueeze(0)
    _need_cuda(pix, "pix", torch.int32)
    n = pix.shape[0]
    out = torch.empty((n, dg.n_el), dtype=torch.complex64, device=za.device)
    _check(lib().usbf_delay_gather_complex(_ptr(za), za.shape[0], ctypes.byref(dg.geom), ctypes.byref(dg.rx),
                                           _ptr(pix), n, _ptr(out), _stream(za.device)))
    return out


def mv_weights_complex(z: torch.Tensor, subap: int = 32, loading: float = 1e-2, want_weights: bool = True):
    """Minimum variance on complex delayed samples z complex64 [n_pix, n_el]:
    (w_full complex64 [n_pix, n_el] or None, y complex64 [n_pix]), y = w_full^H z."""
    _need_cuda(z, "z", torch.complex64)
    n, m = z.shape
    wf = torch.empty_like(z) if want_weights else None
    y = torch.empty(n, dtype=torch.complex64, device=z.device)
    _check(lib().usbf_mv_weights_complex(_ptr(z), n, m, subap, loading, _ptr(wf), _ptr(y), _stream(z.device)))
    return wf, y


OP_APODNET_TRAIN = 6

# flattened parameter layout of the apodization network
NET_LAYOUT = [("W1", (32, 1, 5)), ("b1", (32,)), ("W2", (32, 32, 5)), ("b2", (32,)),
              ("W3", (32, 32, 5)), ("b3", (32,)), ("W4", (1, 32, 5)), ("b4", (1,))]


def flatten_params(params: dict) -> np.ndarray:
    return np.concatenate([np.asarray(params[k], np.float32).reshape(-1) for k, _ in NET_LAYOUT])


def unflatten_params(flat) -> dict:
    flat = np.asarray(flat, np.float32)
    out, o = {}, 0
    for k, shp in NET_LAYOUT:
        n = int(np.prod(shp))
        out[k] = flat[o:o + n].reshape(shp)
        o += n
    return out


class ApodNet:
    """Device state of the learned-apodization network (parameters, Adam moments, packed
    weights) and a reusable workspace."""

    def __init__(self, params: dict, device="cuda"):
        self.device = torch.device(device)
        self.state = torch.zeros(int(lib().usbf_apodnet_state_bytes()), dtype=torch.uint8, device=self.device)
        flat = torch.as_tensor(flatten_params(params), device=self.device)
        _check(lib().usbf_apodnet_init(_ptr(self.state), _ptr(flat), _stream(self.device)))
        torch.cuda.current_stream(self.device).synchronize()
        self._ws = None

    def params(self) -> dict:
        n = int(lib().usbf_apodnet_num_params())
        flat = self.state[: 4 * n].view(torch.float32).cpu().numpy()
        return unflatten_params(flat)

    def _workspace(self, n_pix, n_el, train):
        need = workspace_bytes(OP_APODNET_TRAIN if train else OP_APODNET, n_pix, n_el, 0)
        if self._ws is None or self._ws.numel() < need:
            self._ws = _ws(need, self.device)
        return self._ws

    def forward(self, x: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        _need_cuda(x, "x", torch.float32)
        n, m = x.shape
        if out is None:
            out = torch.empty_like(x)
        ws = self._workspace(n, m, False)
        _check(lib().usbf_apodnet_forward(_ptr(self.state), _ptr(x), n, m, _ptr(out), _ptr(ws), ws.numel(),
                                          _stream(x.device)))
        return out

    def apply(self, x: torch.Tensor, fallback: torch.Tensor | None = None, out: torch.Tensor | None = None,
              w_out: torch.Tensor | None = None) -> torch.Tensor:
        """Network weights and the weighted sum in one pass: y [n_pix] (fallback[p] where a weight
        is not finite); the weights go to w_out if given."""
        _need_cuda(x, "x", torch.float32)
        n, m = x.shape
        if out is None:
            out = torch.empty(n, dtype=torch.float32, device=x.device)
        _check(lib().usbf_apodnet_apply(_ptr(self.state), _ptr(x), n, m, _ptr(fallback), _ptr(w_out), _ptr(out),
                                        _stream(x.device)))
        return out

    def train_step(self, x: torch.Tensor, target: torch.Tensor, lr: float = 1e-3,
                   loss: torch.Tensor | None = None):
        _need_cuda(x, "x", torch.float32)
        _need_cuda(target, "target", torch.float32)
        n, m = x.shape
        ws = self._workspace(n, m, True)
        _check(lib().usbf_apodnet_train_step(_ptr(self.state), _ptr(x), _ptr(target), n, m, lr, _ptr(loss),
                                             _ptr(ws), ws.numel(), _stream(x.device)))
        return loss

    def gradients(self, x: torch.Tensor, target: torch.Tensor) -> torch.Tensor:
        n, m = x.shape
        grad = torch.empty(int(lib().usbf_apodnet_num_params()), dtype=torch.float32, device=x.device)
        ws = self._workspace(n, m, True)
        _check(lib().usbf_apodnet_gradients(_ptr(self.state), _ptr(x), _ptr(target), n, m, _ptr(grad), _ptr(ws),
                                            ws.numel(), _stream(x.device)))
        return grad


def beamform_weighted(x: torch.Tensor, w: torch.Tensor, fallback: torch.Tensor | None = None) -> torch.Tensor:
    _need_cuda(x, "x", torch.float32)
    _need_cuda(w, "w", torch.float32)
    n, m = x.shape
    y = torch.empty(n, dtype=torch.float32, device=x.device)
    _check(lib().usbf_beamform_weighted(_ptr(x), _ptr(w), _ptr(fallback), n, m, _ptr(y), _stream(x.device)))
    return y


class BatchPlan:
    """A batch of acquisitions of different geometries taken through the whole B-mode pipeline by
    one persistent delay-and-sum launch plus per-item epilogues, captured once as a HIP graph.

    items: list of (rf int16 [n_tx, n_el, n_samples], DeviceGeometry).  The plan owns the line,
    row-maximum and image buffers (``lines[i]``, ``images[i]``); write new channel data into the
    rf tensors in place and call ``run()``.
    """

    def __init__(self, items, dyn_range_db: float = 50.0, tune_cache: str | None = None, autotune: bool = False,
                 shape: dict | None = None):
        self._plan = None
        self.rf, self.dgs, self.lines, self.row_max, self.images = [], [], [], [], []
        arr = (CBatchItem * len(items))()
        for k, (rf, dg) in enumerate(items):
            _need_cuda(rf, "rf", torch.int16)
            if rf.dim() == 4:
                if rf.shape[0] != 1:
                    raise ValueError("batch items hold one frame each")
                rf = rf[0]
            lines = torch.empty((dg.n_lines, dg.n_depth), dtype=torch.float32, device=rf.device)
            rmax = torch.empty((dg.n_lines,), dtype=torch.float32, device=rf.device)
            img = torch.empty(dg.scan_shape, dtype=torch.float32, device=rf.device)
            self.rf.append(rf)
            self.dgs.append(dg)
            self.lines.append(lines)
            self.row_max.append(rmax)
            self.images.append(img)
            arr[k] = CBatchItem(_ptr(rf), dg.geom, dg.rx, dg.scan, dyn_range_db, _ptr(lines), _ptr(rmax), _ptr(img))
        self._items = arr
        self.device = items[0][0].device
        cache = tune_cache.encode() if tune_cache else None
        if autotune:
            if not tune_cache:
                raise ValueError("autotune needs a tune_cache path")
            _check(lib().usbf_autotune(arr, len(items), cache, _stream(self.device)))
        plan = ctypes.c_void_p()
        if shape is not None:
            cs = CBatchShape(**shape)
            _check(lib().usbf_batch_plan_create_shaped(arr, len(items), ctypes.byref(cs), ctypes.byref(plan),
                                                       _stream(self.device)))
        else:
            _check(lib().usbf_batch_plan_create(arr, len(items), cache, ctypes.byref(plan), _stream(self.device)))
        self._plan = plan

    def shape(self) -> dict:
        cs = CBatchShape()
        _check(lib().usbf_batch_plan_shape(self._plan, ctypes.byref(cs)))
        return {k: getattr(cs, k) for k, _ in CBatchShape._fields_}

    def run(self):
        _check(lib().usbf_batch_run(self._plan, _stream(self.device)))
        return self.images

    def close(self):
        if self._plan is not None and _lib is not None:
            _lib.usbf_batch_plan_destroy(self._plan)
        self._plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
