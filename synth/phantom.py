"""Seeded scatterer phantoms (input generation only).

Point targets plus uniformly scattered speckle with Gaussian amplitudes, and
optional anechoic cysts, for the 2D linear and 3D matrix workloads.  The paper
images a wire target for its point-spread-function study (Sec. 3.2); here
point targets are placed on the beamformer's own pixel grid so that a correct
beamformer peaks exactly on them.
"""
from __future__ import annotations

import numpy as np

from .geometry import Geometry


def rng_for(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def pixel_position(g: Geometry, line: int, j: int) -> np.ndarray:
    """Nominal float64 position of output sample j on line `line` (origin + depth * unit dir)."""
    o = g.line_origin[line].astype(np.float64)
    d = g.line_dir[line].astype(np.float64)
    d = d / np.linalg.norm(d)
    return o + g.depth_of(j) * d


def points_2d(g: Geometry, amplitude: float = 10.0):
    """4 x 5 grid of point targets: x at (+-0.1, +-0.3) of the line span, z at 0.15..0.75 of
    the deepest output sample, each moved onto the nearest (line, depth) pixel."""
    lx = g.line_origin[:, 0].astype(np.float64)
    width = lx[-1] - lx[0]
    z_max = float(g.depth_of(g.n_depth - 1))
    pos, lj = [], []
    for fx in (-0.3, -0.1, 0.1, 0.3):
        for fz in (0.15, 0.3, 0.45, 0.6, 0.75):
            line = int(np.argmin(np.abs(lx - fx * width)))
            j = int(round(fz * z_max / float(g.depth_of(1) - g.depth_of(0))))
            pos.append(pixel_position(g, line, j))
            lj.append((line, j))
    return np.array(pos), np.full(len(pos), amplitude), lj


def points_3d(g: Geometry, amplitude: float = 10.0, ranges=(25e-3, 50e-3)):
    """5 x 5 angular grid of lines x 2 ranges, on pixel positions."""
    n_side = int(round(np.sqrt(g.n_lines)))
    idx = np.linspace(0, n_side - 1, 7)[1:-1].round().astype(int)
    step = float(g.depth_of(1) - g.depth_of(0))
    pos, lj = [], []
    for rr in ranges:
        j = int(round(rr / step))
        for iy in idx:
            for ix in idx:
                line = int(iy * n_side + ix)
                pos.append(pixel_position(g, line, j))
                lj.append((line, j))
    return np.array(pos), np.full(len(pos), amplitude), lj


def speckle_2d(g: Geometry, rng: np.random.Generator, n: int, z_min: float = 1e-3,
               cysts=()):
    lx = g.line_origin[:, 0].astype(np.float64)
    half = 0.5 * (lx[-1] - lx[0])
    z_max = float(g.depth_of(g.n_depth - 1))
    x = rng.uniform(-half, half, n)
    z = rng.uniform(z_min, z_max, n)
    a = rng.standard_normal(n)
    keep = np.ones(n, dtype=bool)
    for (cx, cz, cr) in cysts:
        keep &= (x - cx) ** 2 + (z - cz) ** 2 > cr * cr
    pos = np.stack([x, np.zeros(n), z], axis=1)[keep]
    return pos, a[keep]


def phantom_2d(g: Geometry, seed: int, n_points: bool = True, n_speckle: int = 5000, cysts=(),
               extra_points=()):
    """The small and multi-line 2D workloads' phantom: 20 points + speckle, seeded."""
    rng = rng_for(seed)
    sp, sa = speckle_2d(g, rng, n_speckle, cysts=cysts)
    parts_p, parts_a = [sp], [sa]
    lj = []
    if n_points:
        pp, pa, lj = points_2d(g)
        parts_p.append(pp)
        parts_a.append(pa)
    for (x, z, a) in extra_points:
        parts_p.append(np.array([[x, 0.0, z]]))
        parts_a.append(np.array([a]))
    return np.concatenate(parts_p), np.concatenate(parts_a), lj


def phantom_3d_points(g: Geometry):
    pp, pa, lj = points_3d(g)
    return pp, pa, lj
