"""Host-side check of the delay-and-sum staging loads (no GPU): every channel-data load the
tile issues stays inside the element's record, including for record lengths that are not a
multiple of 4, where the kernel loads sample by sample.

The tile stages, for each element in the aperture, the window [lo, hi] of samples its taps can
reach (lo from the tile's first depth, hi from its last, both by the binary32 delay rule),
starting at lo rounded down to a multiple of 4, in quads of 4 samples.  Windows reach past the
end of the record for deep pixels at the edge of the aperture.  The model below takes the
windows from the oracle's binary32 index map and applies the kernel's clamping rule: a quad
with no sample inside the record loads from the record's start (and masks the data), and the
samples of a partly inside quad are clamped to the record's last sample."""
import numpy as np
import pytest

import oracle
import synth


def windows(g, G, TD):
    """(element, lo4, hi) of every staged window, per tile of G lines x TD depths."""
    out = []
    span = (g.depth_step * TD + 32 + 3) & ~3
    lt = np.asarray(g.line_tx)
    ex = np.asarray(g.el_pos, np.float32)[:, 0]
    lx = np.asarray(g.line_origin, np.float32)[:, 0]
    for l0 in range(0, g.n_lines, G):
        lines = [l for l in range(l0, min(l0 + G, g.n_lines)) if lt[l] == lt[l0] and 0 <= lt[l] < g.n_tx]
        for j0 in range(0, g.n_depth, TD):
            j1 = min(g.n_depth, j0 + TD) - 1
            pix = [(l, j) for l in lines for j in (j0, j1)]
            if not pix:
                continue
            i0 = oracle.tof32(g, pix)[0].reshape(len(lines), 2, g.n_el)
            r1 = np.float32(g.depth_start + g.depth_step * j1) * np.float32(g.c / (2 * g.fs))
            for e in range(g.n_el):
                act = [k for k, l in enumerate(lines)
                       if np.float32(2 * g.f_number) * abs(np.float32(ex[e] - lx[l])) <= r1]
                if not act:
                    continue
                lo = min(i0[k, 0, e] for k in act)
                hi = max(i0[k, 1, e] for k in act) + 1
                lo4 = 4 * (lo // 4)
                if hi - lo4 + 1 > span:
                    lo4 = 4 * -((-(hi + 1 - span)) // 4)
                out.append((e, lo4, hi, span))
    return out


def load_offsets(e, lo4, hi, span, S, clamp_quads):
    """Sample offsets (within the transmit's block) of one window's element-by-element loads."""
    offs = []
    for q in range(span // 4):
        i = lo4 + 4 * q
        if i > hi:
            break
        inside = [0 <= i + s < S for s in range(4)]
        ic = (i if any(inside) else 0) if clamp_quads else max(i, 0)
        for s in range(4):
            offs.append(e * S + ic + (s if ic + s < S else 0))
    return offs


@pytest.mark.parametrize("n_samples,depth_step,G", [(301, 1, 4), (600, 3, 4), (250, 2, 1), (250, 2, 4)])
def test_staging_loads_stay_in_the_record(n_samples, depth_step, G):
    g = synth.linear_2d("odd", n_el=16, n_tx=5, lines_per_tx=4, line_pitch=0.15e-3, n_samples=n_samples,
                        depth_step=depth_step, scan_n=(16, 16))
    S = g.n_samples
    reach_past = False
    for (e, lo4, hi, span) in windows(g, G, 256 // G):
        offs = load_offsets(e, lo4, hi, span, S, clamp_quads=True)
        assert all(e * S <= o < (e + 1) * S for o in offs), (e, lo4, hi)
        # without clamping whole quads, windows past the end of the record would be read past it
        old = load_offsets(e, lo4, hi, span, S, clamp_quads=False)
        reach_past |= max(old) >= (e + 1) * S
    assert reach_past, "the configuration should exercise windows that reach past the record"
