"""CPU oracle of the receive pipeline -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import this
package; the GPU library never does, and this package never imports the library.

Stages, in the paper's order (Sec. 1, pipeline list; Sec. 2, method list):
  receive beamforming (delay and sum)  -> das_oracle.c via ctypes, float64
  envelope detection                    -> envelope(), float64 (analytic-signal magnitude)
  log compression                       -> log_compress(), float64
  scan conversion                       -> scan_convert_2d() / scan_convert_3d(), float64 values,
                                           binary32 index decisions (scan_index_2d/3d)
and the adaptive-apodization additions in oracle.mv and oracle.apodnet.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "das_oracle.c")


def build(force: bool = True) -> str:
    """Compile the C part of the oracle with gcc (float64 arithmetic, no FMA contraction)."""
    if force or not os.path.exists(_LIB_PATH):
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
               "-std=c11", "-D_DEFAULT_SOURCE", "-o", _LIB_PATH + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


class _OG(ctypes.Structure):
    _fields_ = [
        ("n_el", ctypes.c_int32), ("el_pos", ctypes.c_void_p),
        ("n_tx", ctypes.c_int32), ("tx_origin", ctypes.c_void_p), ("tx_dir", ctypes.c_void_p),
        ("tx_focus", ctypes.c_void_p),
        ("n_lines", ctypes.c_int32), ("line_origin", ctypes.c_void_p), ("line_dir", ctypes.c_void_p),
        ("line_tx", ctypes.c_void_p),
        ("array_dims", ctypes.c_int32),
        ("c", ctypes.c_float), ("fs", ctypes.c_float), ("t0", ctypes.c_float),
        ("n_samples", ctypes.c_int32), ("depth_start", ctypes.c_int32), ("depth_step", ctypes.c_int32),
        ("n_depth", ctypes.c_int32),
        ("f_number", ctypes.c_float), ("window", ctypes.c_int32),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        L = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        L.oracle_tof32.argtypes = [ctypes.POINTER(_OG), ctypes.c_int64, P, P, P, P]
        L.oracle_tau64.argtypes = [ctypes.POINTER(_OG), ctypes.c_int64, P, P]
        L.oracle_das.argtypes = [ctypes.POINTER(_OG), P, ctypes.c_int32, ctypes.c_int64, P, P]
        L.oracle_delay_gather.argtypes = [ctypes.POINTER(_OG), P, ctypes.c_int64, P, P]
        L.oracle_num_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def num_threads() -> int:
    return int(lib().oracle_num_threads())


class _GeomHandle:
    """Keeps the contiguous arrays alive while C holds pointers into them."""

    def __init__(self, g):
        self.keep = [np.ascontiguousarray(a) for a in (
            np.asarray(g.el_pos, np.float32), np.asarray(g.tx_origin, np.float32),
            np.asarray(g.tx_dir, np.float32), np.asarray(g.tx_focus, np.float32),
            np.asarray(g.line_origin, np.float32), np.asarray(g.line_dir, np.float32),
            np.asarray(g.line_tx, np.int32))]
        k = self.keep
        self.s = _OG(g.n_el, k[0].ctypes.data, g.n_tx, k[1].ctypes.data, k[2].ctypes.data, k[3].ctypes.data,
                     g.n_lines, k[4].ctypes.data, k[5].ctypes.data, k[6].ctypes.data, g.array_dims,
                     g.c, g.fs, g.t0, g.n_samples, g.depth_start, g.depth_step, g.n_depth,
                     g.f_number, g.window)


def _pix_arg(pix, ncol):
    if pix is None:
        return None, None
    a = np.ascontiguousarray(np.asarray(pix, dtype=np.int32).reshape(-1, ncol))
    return a, a.ctypes.data


def tof32(g, pix=None):
    """Binary32 delay decisions: (i0 int32, phi float32, active bool, valid bool), each [n_pix][n_el].
    pix: [n][2] (line, depth index) or None for every pixel (line-major)."""
    h = _GeomHandle(g)
    a, p = _pix_arg(pix, 2)
    n = a.shape[0] if a is not None else g.n_lines * g.n_depth
    i0 = np.empty((n, g.n_el), np.int32)
    phi = np.empty((n, g.n_el), np.float32)
    fl = np.empty((n, g.n_el), np.uint8)
    lib().oracle_tof32(ctypes.byref(h.s), n, p, i0.ctypes.data, phi.ctypes.data, fl.ctypes.data)
    return i0, phi, (fl & 1).astype(bool), (fl & 2).astype(bool)


def tau64(g, pix=None):
    """Float64 two-way delays in samples, [n_pix][n_el]."""
    h = _GeomHandle(g)
    a, p = _pix_arg(pix, 2)
    n = a.shape[0] if a is not None else g.n_lines * g.n_depth
    out = np.empty((n, g.n_el), np.float64)
    lib().oracle_tau64(ctypes.byref(h.s), n, p, out.ctypes.data)
    return out


def das(g, rf, pix=None):
    """Delay-and-sum, float64.  rf: int16 [n_frames][n_tx][n_el][S] (or 3D for one frame).
    pix: [n][3] (frame, line, depth index) or None -> array [n_frames][n_lines][n_depth]."""
    rf = np.ascontiguousarray(np.asarray(rf, dtype=np.int16))
    if rf.ndim == 3:
        rf = rf[None]
    assert rf.shape[1:] == (g.n_tx, g.n_el, g.n_samples), rf.shape
    h = _GeomHandle(g)
    a, p = _pix_arg(pix, 3)
    if a is not None:
        assert a[:, 0].max(initial=0) < rf.shape[0]
    n = a.shape[0] if a is not None else rf.shape[0] * g.n_lines * g.n_depth
    out = np.empty(n, np.float64)
    lib().oracle_das(ctypes.byref(h.s), rf.ctypes.data, rf.shape[0], n, p, out.ctypes.data)
    if a is None:
        return out.reshape(rf.shape[0], g.n_lines, g.n_depth)
    return out


def delay_gather(g, rf, pix):
    """Delayed channel samples x[n][n_el] (float64), no summation, every element."""
    rf = np.ascontiguousarray(np.asarray(rf, dtype=np.int16))
    if rf.ndim == 3:
        rf = rf[None]
    h = _GeomHandle(g)
    a, p = _pix_arg(pix, 3)
    out = np.empty((a.shape[0], g.n_el), np.float64)
    lib().oracle_delay_gather(ctypes.byref(h.s), rf.ctypes.data, a.shape[0], p, out.ctypes.data)
    return out


def combine_lines(y, src, w) -> np.ndarray:
    """Output lines as weighted sums of beamformed lines, float64: out[..., m, :] =
    sum_k w[m, k] y[..., src[m, k], :] over the sources that are lines of y (overlapping
    multi-line layouts interpolate a line between two transmits from both beams of it,
    Sec. 3.3, Table 1; coherent compounding is the case of equal weights)."""
    y = np.asarray(y, np.float64)
    n_in = y.shape[-2]
    out = np.zeros(y.shape[:-2] + (len(src), y.shape[-1]))
    for m in range(len(src)):
        for s, wk in zip(src[m], w[m]):
            if 0 <= int(s) < n_in:
                out[..., m, :] += float(wk) * y[..., int(s), :]
    return out


# ---------------------------------------------------------------- envelope detection

def analytic_filter(n: int) -> np.ndarray:
    """Frequency-domain weights that keep DC (and Nyquist for even n), double the positive
    frequencies and remove the negative ones."""
    H = np.zeros(n)
    H[0] = 1.0
    if n % 2 == 0:
        H[n // 2] = 1.0
        H[1:n // 2] = 2.0
    else:
        H[1:(n + 1) // 2] = 2.0
    return H


def envelope(y: np.ndarray) -> np.ndarray:
    """Magnitude of the analytic signal of each row (last axis, circular, length n), float64."""
    y = np.asarray(y, dtype=np.float64)
    n = y.shape[-1]
    Y = np.fft.fft(y, axis=-1)
    return np.abs(np.fft.ifft(Y * analytic_filter(n), axis=-1))


# ---------------------------------------------------------------- log compression

def log_compress(env: np.ndarray, dyn_range_db: float = 50.0, ref: float | None = None) -> np.ndarray:
    """Map env to [0, 1]: 1 at the reference level, 0 at dyn_range_db below it and under."""
    env = np.asarray(env, dtype=np.float64)
    if ref is None:
        ref = float(env.max())
    out = np.zeros_like(env)
    pos = env > 0
    if ref > 0:
        out[pos] = 1.0 + (20.0 / dyn_range_db) * np.log10(env[pos] / ref)
    return np.clip(out, 0.0, 1.0)


# ---------------------------------------------------------------- scan conversion

def _last_le(table: np.ndarray, x: np.ndarray) -> np.ndarray:
    """Largest i with table[i] <= x (exact binary32 comparisons), -1 if none."""
    return np.searchsorted(table, x, side="right").astype(np.int64) - 1


def scan_index_2d(s):
    """Binary32 index decisions of the 2D scan converter.  Returns (line_idx, depth_idx, inside,
    x32, z32) for the grid [nz][nx].  Parallel lines at x = line_u (kind 0) or, for kind 2,
    a sector whose lines have tangents line_u (u = x/z, depth = |(x, z)|)."""
    f32 = np.float32
    i = np.arange(s.nx, dtype=f32)
    k = np.arange(s.nz, dtype=f32)
    x = (f32(s.x0) + i * f32(s.hx)).astype(f32)
    z = (f32(s.z0) + k * f32(s.hz)).astype(f32)
    X = np.broadcast_to(x[None, :], (s.nz, s.nx)).astype(f32)
    Z = np.broadcast_to(z[:, None], (s.nz, s.nx)).astype(f32)
    u_tab = np.asarray(s.line_u, dtype=f32)
    if s.kind == 0:
        U = X
        R = Z
        ok = np.ones_like(X, dtype=bool)
    else:
        ok = Z > 0
        Zs = np.where(ok, Z, f32(1))
        U = (X / Zs).astype(f32)
        R = np.sqrt((X * X + Z * Z).astype(f32)).astype(f32)
    q = ((R - f32(s.r0)) / f32(s.dr)).astype(f32)
    nu = u_tab.shape[0]
    iu = _last_le(u_tab, U)
    ok &= (U >= u_tab[0]) & (U <= u_tab[-1])
    ok &= (q >= f32(0)) & (q <= f32(s.n_depth - 1))
    iu = np.clip(iu, 0, nu - 2)
    jd = np.clip(np.floor(q).astype(np.int64), 0, s.n_depth - 2)
    return iu, jd, ok, U, q


def scan_convert_2d(lines: np.ndarray, s) -> np.ndarray:
    """Bilinear scan conversion of [n_u][n_depth] line data (float64 values) to [nz][nx]."""
    lines = np.asarray(lines, dtype=np.float64)
    iu, jd, ok, U, q = scan_index_2d(s)
    u_tab = np.asarray(s.line_u, dtype=np.float64)
    u64 = U.astype(np.float64)
    fu = (u64 - u_tab[iu]) / (u_tab[iu + 1] - u_tab[iu])
    fd = q.astype(np.float64) - jd
    v00 = lines[iu, jd]
    v01 = lines[iu, jd + 1]
    v10 = lines[iu + 1, jd]
    v11 = lines[iu + 1, jd + 1]
    out = (1 - fu) * ((1 - fd) * v00 + fd * v01) + fu * ((1 - fd) * v10 + fd * v11)
    return np.where(ok, out, s.fill)


def scan_index_3d(s, z_slices=None):
    """Binary32 index decisions of the 3D scan converter (tangent space u = x/z, v = y/z,
    range r = |(x, y, z)|).  Returns (iu, iv, jd, inside, U, V, q) over [nz][ny][nx]."""
    f32 = np.float32
    ks = np.arange(s.nz) if z_slices is None else np.asarray(z_slices)
    x = (f32(s.x0) + np.arange(s.nx, dtype=f32) * f32(s.hx)).astype(f32)
    y = (f32(s.y0) + np.arange(s.ny, dtype=f32) * f32(s.hy)).astype(f32)
    z = (f32(s.z0) + ks.astype(f32) * f32(s.hz)).astype(f32)
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    ok = Z > 0
    Zs = np.where(ok, Z, f32(1)).astype(f32)
    U = (X / Zs).astype(f32)
    V = (Y / Zs).astype(f32)
    R = np.sqrt(((X * X + Y * Y).astype(f32) + Z * Z).astype(f32)).astype(f32)
    q = ((R - f32(s.r0)) / f32(s.dr)).astype(f32)
    ut = np.asarray(s.line_u, dtype=f32)
    vt = np.asarray(s.line_v, dtype=f32)
    ok &= (U >= ut[0]) & (U <= ut[-1]) & (V >= vt[0]) & (V <= vt[-1])
    ok &= (q >= f32(0)) & (q <= f32(s.n_depth - 1))
    iu = np.clip(_last_le(ut, U), 0, ut.shape[0] - 2)
    iv = np.clip(_last_le(vt, V), 0, vt.shape[0] - 2)
    jd = np.clip(np.floor(q).astype(np.int64), 0, s.n_depth - 2)
    return iu, iv, jd, ok, U, V, q


def scan_convert_3d(lines: np.ndarray, s, z_slices=None) -> np.ndarray:
    """Trilinear scan conversion of [n_v*n_u][n_depth] line data to [nz][ny][nx] (float64)."""
    lines = np.asarray(lines, dtype=np.float64)
    iu, iv, jd, ok, U, V, q = scan_index_3d(s, z_slices)
    ut = np.asarray(s.line_u, dtype=np.float64)
    vt = np.asarray(s.line_v, dtype=np.float64)
    fu = (U.astype(np.float64) - ut[iu]) / (ut[iu + 1] - ut[iu])
    fv = (V.astype(np.float64) - vt[iv]) / (vt[iv + 1] - vt[iv])
    fd = q.astype(np.float64) - jd
    nu = ut.shape[0]
    out = np.zeros(U.shape)
    for dv in (0, 1):
        for du in (0, 1):
            wl = (fv if dv else 1 - fv) * (fu if du else 1 - fu)
            ln = (iv + dv) * nu + (iu + du)
            out += wl * ((1 - fd) * lines[ln, jd] + fd * lines[ln, jd + 1])
    return np.where(ok, out, s.fill)


def bmode_2d(beamformed: np.ndarray, s, dyn_range_db: float = 50.0) -> np.ndarray:
    """Envelope -> log compression (frame maximum as reference) -> scan conversion, one frame."""
    env = envelope(beamformed)
    return scan_convert_2d(log_compress(env, dyn_range_db), s)


def bmode_3d(beamformed: np.ndarray, s, dyn_range_db: float = 50.0, z_slices=None) -> np.ndarray:
    env = envelope(beamformed)
    return scan_convert_3d(log_compress(env, dyn_range_db), s, z_slices)
