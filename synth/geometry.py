"""Probe, transmit, scanline and output-grid layouts for the synthetic workloads.

Input generation only: this module builds binary32 arrays describing where the
elements, transmit beams, receive lines and output pixels are.  It contains no
beamforming, envelope, compression or interpolation arithmetic; both the CPU
oracle and the GPU library receive the same arrays.

The paper's evaluation hardware (a 128-element, 0.3 mm pitch linear array and a
32x32 matrix probe, Sec. 3 and its run-time Table 1) motivates the layouts; the
exact numbers are those of the config_* functions below.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

RECT = 0
HANN = 1


@dataclasses.dataclass
class ScanGrid:
    """Cartesian output grid and the line tables the scan converter searches.

    kind 0 (2D): pixel (i, k) sits at x = x0 + i*hx, z = z0 + k*hz; line_u holds
    the sorted x positions of the n_u receive lines.
    kind 1 (3D): voxel (i, j, k) sits at x0 + i*hx, y0 + j*hy, z0 + k*hz;
    line_u / line_v hold the sorted tangents of the steering angles.
    Line data are samples at depth r0 + n*dr, n = 0 .. n_depth-1.
    """

    kind: int
    nx: int
    ny: int
    nz: int
    x0: float
    hx: float
    y0: float
    hy: float
    z0: float
    hz: float
    line_u: np.ndarray
    line_v: np.ndarray
    r0: float
    dr: float
    n_depth: int
    fill: float = 0.0

    @property
    def n_u(self) -> int:
        return int(self.line_u.shape[0])

    @property
    def n_v(self) -> int:
        return int(self.line_v.shape[0])

    @property
    def out_shape(self):
        if self.kind != 1:
            return (self.nz, self.nx)
        return (self.nz, self.ny, self.nx)


@dataclasses.dataclass
class Geometry:
    """Everything one beamforming call needs besides the channel data."""

    name: str
    el_pos: np.ndarray        # [n_el][3] f32
    tx_origin: np.ndarray     # [n_tx][3] f32
    tx_dir: np.ndarray        # [n_tx][3] f32
    tx_focus: np.ndarray      # [n_tx]    f32
    line_origin: np.ndarray   # [n_lines][3] f32
    line_dir: np.ndarray      # [n_lines][3] f32
    line_tx: np.ndarray       # [n_lines] i32
    array_dims: int           # 1 linear array, 2 matrix array
    c: float
    fs: float
    t0: float
    n_samples: int
    depth_start: int
    depth_step: int
    n_depth: int
    f_number: float
    window: int
    f0: float
    scan: ScanGrid | None = None

    @property
    def n_el(self) -> int:
        return int(self.el_pos.shape[0])

    @property
    def n_tx(self) -> int:
        return int(self.tx_origin.shape[0])

    @property
    def n_lines(self) -> int:
        return int(self.line_origin.shape[0])

    def rf_shape(self, n_frames: int = 1):
        return (n_frames, self.n_tx, self.n_el, self.n_samples)

    def depth_of(self, j):
        """Nominal (float64) depth of output sample j along its line."""
        return (self.depth_start + self.depth_step * np.asarray(j, dtype=np.float64)) * (
            float(np.float32(self.c)) / (2.0 * float(np.float32(self.fs))))


def _f32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float32))


def linear_array(n_el: int, pitch: float) -> np.ndarray:
    x = (np.arange(n_el, dtype=np.float64) - (n_el - 1) / 2.0) * pitch
    return _f32(np.stack([x, np.zeros(n_el), np.zeros(n_el)], axis=1))


def matrix_array(nx: int, ny: int, pitch: float) -> np.ndarray:
    ix = np.arange(nx, dtype=np.float64) - (nx - 1) / 2.0
    iy = np.arange(ny, dtype=np.float64) - (ny - 1) / 2.0
    X, Y = np.meshgrid(ix * pitch, iy * pitch, indexing="xy")   # element e = iy*nx + ix
    return _f32(np.stack([X.ravel(), Y.ravel(), np.zeros(nx * ny)], axis=1))


def scan_grid_2d(line_x: np.ndarray, r0: float, dr: float, n_depth: int, nx: int, nz: int) -> ScanGrid:
    """Pixel centres span [first line, last line] x [first depth, last depth]."""
    line_x = _f32(line_x)
    x_first, x_last = float(line_x[0]), float(line_x[-1])
    r_last = r0 + dr * (n_depth - 1)
    return ScanGrid(kind=0, nx=nx, ny=1, nz=nz,
                    x0=float(np.float32(x_first)), hx=float(np.float32((x_last - x_first) / (nx - 1))),
                    y0=0.0, hy=0.0,
                    z0=float(np.float32(r0)), hz=float(np.float32((r_last - r0) / (nz - 1))),
                    line_u=line_x, line_v=_f32(np.zeros(1)),
                    r0=float(np.float32(r0)), dr=float(np.float32(dr)), n_depth=n_depth)


def scan_grid_3d(tan_u: np.ndarray, tan_v: np.ndarray, r0: float, dr: float, n_depth: int,
                 n: int, half_angle_deg: float) -> ScanGrid:
    r_max = r0 + dr * (n_depth - 1)
    half = r_max * math.sin(math.radians(half_angle_deg))
    return ScanGrid(kind=1, nx=n, ny=n, nz=n,
                    x0=float(np.float32(-half)), hx=float(np.float32(2 * half / (n - 1))),
                    y0=float(np.float32(-half)), hy=float(np.float32(2 * half / (n - 1))),
                    z0=float(np.float32(r_max / n)), hz=float(np.float32(r_max / n)),
                    line_u=_f32(tan_u), line_v=_f32(tan_v),
                    r0=float(np.float32(r0)), dr=float(np.float32(dr)), n_depth=n_depth)


def linear_2d(name: str, n_el: int, n_tx: int, lines_per_tx: int, line_pitch: float,
              n_samples: int, *, pitch=0.3e-3, f0=5e6, fs=40e6, c=1540.0, focus=30e-3,
              f_number=1.0, window=HANN, depth_step=2, scan_n=(256, 256)) -> Geometry:
    """Linear array with vertical scanlines; transmit t fires along the mean of its lines."""
    el = linear_array(n_el, pitch)
    n_lines = n_tx * lines_per_tx
    lx = (np.arange(n_lines, dtype=np.float64) - (n_lines - 1) / 2.0) * line_pitch
    line_origin = _f32(np.stack([lx, np.zeros(n_lines), np.zeros(n_lines)], axis=1))
    line_dir = _f32(np.tile([0.0, 0.0, 1.0], (n_lines, 1)))
    line_tx = np.ascontiguousarray(np.arange(n_lines, dtype=np.int32) // lines_per_tx)
    tx_x = lx.reshape(n_tx, lines_per_tx).mean(axis=1)
    if lines_per_tx == 1:
        tx_origin = line_origin.copy()
    else:
        tx_origin = _f32(np.stack([tx_x, np.zeros(n_tx), np.zeros(n_tx)], axis=1))
    tx_dir = _f32(np.tile([0.0, 0.0, 1.0], (n_tx, 1)))
    tx_focus = _f32(np.full(n_tx, focus))
    n_depth = n_samples // depth_step
    g = Geometry(name=name, el_pos=el, tx_origin=tx_origin, tx_dir=tx_dir, tx_focus=tx_focus,
                 line_origin=line_origin, line_dir=line_dir, line_tx=line_tx, array_dims=1,
                 c=float(np.float32(c)), fs=float(np.float32(fs)), t0=0.0, n_samples=n_samples,
                 depth_start=0, depth_step=depth_step, n_depth=n_depth,
                 f_number=float(np.float32(f_number)), window=window, f0=f0)
    h = float(np.float32(c)) / (2.0 * float(np.float32(fs)))
    g.scan = scan_grid_2d(lx, 0.0, depth_step * h, n_depth, nx=scan_n[0], nz=scan_n[1])
    return g


def matrix_3d(name: str, n_side: int, n_samples: int, *, n_lines_side=32, half_angle_deg=30.0,
              pitch=0.3e-3, f0=3.5e6, fs=20e6, c=1540.0, focus=30e-3, f_number=1.0,
              window=HANN, depth_step=2, scan_n=128) -> Geometry:
    """Matrix array, steered lines from the array centre, one focused transmit per line."""
    el = matrix_array(n_side, n_side, pitch)
    theta = np.radians(-half_angle_deg + np.arange(n_lines_side) * (2 * half_angle_deg) / (n_lines_side - 1))
    tan_t = np.tan(theta).astype(np.float32)
    TX, TY = np.meshgrid(tan_t, tan_t, indexing="xy")        # line = iy*n + ix
    n_lines = n_lines_side * n_lines_side
    line_dir = _f32(np.stack([TX.ravel(), TY.ravel(), np.ones(n_lines, dtype=np.float32)], axis=1))
    line_origin = _f32(np.zeros((n_lines, 3)))
    n_depth = n_samples // depth_step
    g = Geometry(name=name, el_pos=el, tx_origin=line_origin.copy(), tx_dir=line_dir.copy(),
                 tx_focus=_f32(np.full(n_lines, focus)), line_origin=line_origin, line_dir=line_dir,
                 line_tx=np.arange(n_lines, dtype=np.int32), array_dims=2,
                 c=float(np.float32(c)), fs=float(np.float32(fs)), t0=0.0, n_samples=n_samples,
                 depth_start=0, depth_step=depth_step, n_depth=n_depth,
                 f_number=float(np.float32(f_number)), window=window, f0=f0)
    h = float(np.float32(c)) / (2.0 * float(np.float32(fs)))
    g.scan = scan_grid_3d(tan_t, tan_t, 0.0, depth_step * h, n_depth, scan_n, half_angle_deg)
    return g


# ---- the five workloads -------------------------------------------------------------------

def config_small_2d() -> Geometry:
    """64-element linear array, 64 focused transmits with one line each, 2048 samples,
    output 64 x 1024 lines and a 256 x 256 image."""
    return linear_2d("linear64_64tx_2048", n_el=64, n_tx=64, lines_per_tx=1, line_pitch=0.3e-3,
                     n_samples=2048, scan_n=(256, 256))


def config_multiline_2d() -> Geometry:
    """128-element linear array, 256 lines from 64 transmits (4 receive lines each),
    4096 samples, output 256 x 2048 lines and a 512 x 512 image per frame."""
    return linear_2d("linear128_64tx_x4_4096", n_el=128, n_tx=64, lines_per_tx=4, line_pitch=0.15e-3,
                     n_samples=4096, scan_n=(512, 512))


def config_volume_3d() -> Geometry:
    """32 x 32 matrix array, 32 x 32 steered lines over +-30 deg, 2000 samples,
    output 32 x 32 x 1000 beamformed volume and a 128^3 scan-converted volume."""
    return matrix_3d("matrix32x32_1024tx_2000", n_side=32, n_samples=2000)


def config_tiny(n_el=4, n_tx=2, lines_per_tx=3, n_samples=32, depth_step=2, window=HANN,
                f_number=1.0, pitch=0.3e-3) -> Geometry:
    """Very small linear case for brute-force checks."""
    g = linear_2d("tiny", n_el=n_el, n_tx=n_tx, lines_per_tx=lines_per_tx, line_pitch=pitch / 2,
                  n_samples=n_samples, pitch=pitch, window=window, f_number=f_number,
                  depth_step=depth_step, scan_n=(8, 8))
    return g


def stream_mix(seed: int = 0, n_items: int = 100, frac_2d: float = 0.7) -> list:
    """An uneven acquisition stream in a seeded random order: round(frac_2d * n_items)
    linear-array frames and the rest matrix-array volumes.

    Linear: n_el uniform in {64, 128, 192}, n_samples uniform in {2048, 2304, ..., 4096},
    n_el / 2 transmits with 4 receive lines each (lines at half the element pitch), 5 MHz,
    40 MHz sampling, 512 x 512 image.  Matrix: 16 x 16 or 32 x 32 elements with equal
    probability, n_samples uniform in {1000, 1100, ..., 2000}, 32 x 32 steered lines with one
    transmit each, 3.5 MHz, 20 MHz sampling, 128^3 volume."""
    rng = np.random.default_rng(seed)
    n2 = int(round(frac_2d * n_items))
    kinds = rng.permutation(np.array([2] * n2 + [3] * (n_items - n2)))
    out = []
    for k in kinds:
        if k == 2:
            n_el = int(rng.choice([64, 128, 192]))
            n_s = int(rng.choice(np.arange(2048, 4097, 256)))
            out.append(linear_2d(f"linear{n_el}_{n_el // 2}tx_x4_{n_s}", n_el=n_el, n_tx=n_el // 2, lines_per_tx=4,
                                 line_pitch=0.15e-3, n_samples=n_s, scan_n=(512, 512)))
        else:
            side = int(rng.choice([16, 32]))
            n_s = int(rng.choice(np.arange(1000, 2001, 100)))
            out.append(matrix_3d(f"matrix{side}x{side}_1024tx_{n_s}", n_side=side, n_samples=n_s))
    return out


def config_planewave_2d(n_el: int = 128, n_angles: int = 11, max_angle_deg: float = 10.0, n_samples: int = 4096,
                        lines: int = 256, scan_n=(512, 512), focus: float = np.inf) -> Geometry:
    """Plane-wave imaging with the linear array: n_angles plane waves steered over
    +-max_angle_deg from the array centre (infinite focus); every one of the `lines` receive
    lines (half the element pitch apart) is beamformed for every angle, so the geometry holds
    n_angles x lines lines, angle-major (line a * lines + l belongs to transmit a); the scan
    grid is that of the `lines` compounded lines.  A negative `focus` gives diverging waves
    instead: each transmit spreads from a virtual source |focus| behind the array centre,
    along the steering direction."""
    el = linear_array(n_el, 0.3e-3)
    lx = (np.arange(lines, dtype=np.float64) - (lines - 1) / 2.0) * 0.15e-3
    theta = np.radians(np.linspace(-max_angle_deg, max_angle_deg, n_angles))
    line_origin = _f32(np.tile(np.stack([lx, np.zeros(lines), np.zeros(lines)], axis=1), (n_angles, 1)))
    line_dir = _f32(np.tile([0.0, 0.0, 1.0], (n_angles * lines, 1)))
    line_tx = np.ascontiguousarray(np.repeat(np.arange(n_angles, dtype=np.int32), lines))
    tx_origin = _f32(np.zeros((n_angles, 3)))
    tx_dir = _f32(np.stack([np.sin(theta), np.zeros(n_angles), np.cos(theta)], axis=1))
    tx_focus = np.full(n_angles, focus, dtype=np.float32)
    depth_step = 2
    n_depth = n_samples // depth_step
    c, fs = 1540.0, 40e6
    kind = "planewave" if np.isinf(focus) else "divergingwave"
    g = Geometry(name=f"{kind}{n_el}_{n_angles}angles_{n_samples}", el_pos=el, tx_origin=tx_origin,
                 tx_dir=tx_dir, tx_focus=tx_focus, line_origin=line_origin, line_dir=line_dir, line_tx=line_tx,
                 array_dims=1, c=float(np.float32(c)), fs=float(np.float32(fs)), t0=0.0, n_samples=n_samples,
                 depth_start=0, depth_step=depth_step, n_depth=n_depth, f_number=1.0, window=HANN, f0=5e6)
    h = float(np.float32(c)) / (2.0 * float(np.float32(fs)))
    g.scan = scan_grid_2d(lx, 0.0, depth_step * h, n_depth, nx=scan_n[0], nz=scan_n[1])
    g.n_angles = n_angles
    return g


def config_overlap_2d(n_el: int = 128, n_samples: int = 4096, pitch: float = 0.3e-3, focus: float = 30e-3,
                      scan_n=(512, 512)) -> Geometry:
    """128 transmits, 255 lines: the overlapping multi-line layout.  Transmit t is focused along
    element t's axis; the 2 n_el - 1 output lines lie at half pitch from the first element to the
    last.  Line 2t (on transmit t's axis) is transmit t's beam; line 2t + 1 (half way to the next
    transmit) is the mean of the beams of transmits t and t + 1 (linear interpolation between
    the two nearest transmits).  The geometry holds the beams to form: four line slots per
    transmit -- lines 2t, 2t - 1, 2t + 1 and an unused slot (transmit -1, a line of zeros), so
    that every tile of four slots shares one transmit's channel data -- and `combine_src` /
    `combine_w` ([2 n_el - 1][2]) say which beams make each output line, with which weight
    (a source of -1 contributes nothing)."""
    x_t = (np.arange(n_el, dtype=np.float64) - (n_el - 1) / 2.0) * pitch
    n_out = 2 * n_el - 1
    x_m = x_t[0] + np.arange(n_out) * (pitch / 2.0)
    slots = np.full((n_el, 4), -1, dtype=np.int64)  # output line of each slot, -1 unused
    for t in range(n_el):
        for k, m in enumerate((2 * t, 2 * t - 1, 2 * t + 1)):
            if 0 <= m < n_out:
                slots[t, k] = m
    n_lines = 4 * n_el
    lx = np.where(slots.ravel() >= 0, x_m[np.clip(slots.ravel(), 0, n_out - 1)], np.repeat(x_t, 4))
    line_origin = _f32(np.stack([lx, np.zeros(n_lines), np.zeros(n_lines)], axis=1))
    line_dir = _f32(np.tile([0.0, 0.0, 1.0], (n_lines, 1)))
    line_tx = np.where(slots.ravel() >= 0, np.repeat(np.arange(n_el), 4), -1).astype(np.int32)
    src = np.full((n_out, 2), -1, dtype=np.int32)
    w = np.zeros((n_out, 2), dtype=np.float32)
    for m in range(n_out):
        t = m // 2
        if m % 2 == 0:
            src[m, 0], w[m, 0] = 4 * t, 1.0
        else:
            src[m] = (4 * t + 2, 4 * (t + 1) + 1)
            w[m] = (0.5, 0.5)
    depth_step = 2
    n_depth = n_samples // depth_step
    c, fs = 1540.0, 40e6
    g = Geometry(name=f"overlap{n_el}tx_{n_out}lines_{n_samples}", el_pos=linear_array(n_el, pitch),
                 tx_origin=_f32(np.stack([x_t, np.zeros(n_el), np.zeros(n_el)], axis=1)),
                 tx_dir=_f32(np.tile([0.0, 0.0, 1.0], (n_el, 1))), tx_focus=_f32(np.full(n_el, focus)),
                 line_origin=line_origin, line_dir=line_dir, line_tx=np.ascontiguousarray(line_tx), array_dims=1,
                 c=float(np.float32(c)), fs=float(np.float32(fs)), t0=0.0, n_samples=n_samples,
                 depth_start=0, depth_step=depth_step, n_depth=n_depth, f_number=1.0, window=HANN, f0=5e6)
    h = float(np.float32(c)) / (2.0 * float(np.float32(fs)))
    g.scan = scan_grid_2d(x_m, 0.0, depth_step * h, n_depth, nx=scan_n[0], nz=scan_n[1])
    g.combine_src, g.combine_w = src, w
    g.n_out_lines = n_out
    g.out_line_x = x_m
    return g
