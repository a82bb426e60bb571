"""Learned adaptive apodization on top of the delay-and-sum path.

A small 1D convolutional network (4 layers, 32 channels, kernel 5) maps the delayed channel
samples of one pixel to one weight per element.  It is trained to reproduce minimum-variance
(Capon) weights, which the library computes on the GPU for the same pixels (spatial smoothing
over subapertures, diagonal loading, binary64 Cholesky); inference replaces the covariance
estimate and the solve by one network evaluation.  Plain delay-and-sum stays the fallback for
any pixel whose weights are not finite.  Every numeric step -- gathering the delayed samples,
the minimum-variance solve, the network's forward and backward passes, the Adam update, the
weighted sum, envelope and compression -- runs in the library's HIP kernels; this module only
schedules them and measures the resulting images.

Image measures: contrast-to-noise ratio of anechoic cysts, |mu_in - mu_out| / sqrt(var_in +
var_out) of the envelope inside 0.75 R against the ring 1.25 R .. 1.75 R, and the lateral -6 dB
width of point-target responses, measured on an auxiliary set of lines a twentieth of a
wavelength apart through each target.

Run ``python -m paper_1711_06127_amd.learned`` on a GPU to train and compare the three
beamformers on held-out phantoms (prints one JSON line).
"""
from __future__ import annotations

import argparse
import copy
import json
import time

import numpy as np
import torch

from . import (ApodNet, DeviceGeometry, beamform, beamform_weighted, delay_gather, envelope, mv_weights)

SUBAPERTURE = 32
LOADING = 1e-2


def init_params(seed: int = 0, n_el: int = 128) -> dict:
    """He-uniform initialisation of the hidden layers; the output layer starts near zero
    (1e-3 of its He bound) and its bias at 1 / n_el, so the untrained network gives almost
    exactly uniform weights and training starts from the uniform-weight loss."""
    rng = np.random.default_rng(seed)

    def u(shape, fan_in, scale=1.0):
        b = np.sqrt(6.0 / fan_in) * scale
        return rng.uniform(-b, b, shape).astype(np.float32)

    return {"W1": u((32, 1, 5), 5), "b1": np.zeros(32, np.float32),
            "W2": u((32, 32, 5), 160), "b2": np.zeros(32, np.float32),
            "W3": u((32, 32, 5), 160), "b3": np.zeros(32, np.float32),
            "W4": u((1, 32, 5), 160, 1e-3), "b4": np.full(1, 1.0 / n_el, np.float32)}


def frame_pixels(n_lines: int, n_depth: int, frame: int = 0, device="cuda") -> torch.Tensor:
    """Every (frame, line, depth) pixel of one frame, line-major, int32 [n_lines * n_depth, 3]."""
    l = torch.arange(n_lines, dtype=torch.int32, device=device).repeat_interleave(n_depth)
    j = torch.arange(n_depth, dtype=torch.int32, device=device).repeat(n_lines)
    f = torch.full_like(l, frame)
    return torch.stack([f, l, j], dim=1).contiguous()


def random_pixels(gen: torch.Generator, n: int, n_frames: int, n_lines: int, n_depth: int, j_min: int,
                  device="cuda") -> torch.Tensor:
    f = torch.randint(0, n_frames, (n,), generator=gen, device=device, dtype=torch.int32)
    l = torch.randint(0, n_lines, (n,), generator=gen, device=device, dtype=torch.int32)
    j = torch.randint(j_min, n_depth, (n,), generator=gen, device=device, dtype=torch.int32)
    return torch.stack([f, l, j], dim=1).contiguous()


class LearnedApodization:
    """Network state plus the training loop on minimum-variance targets."""

    def __init__(self, n_el: int = 128, seed: int = 0, params: dict | None = None, device="cuda"):
        self.n_el = n_el
        self.net = ApodNet(params if params is not None else init_params(seed, n_el), device)
        self.device = torch.device(device)

    def train(self, rf: torch.Tensor, dg: DeviceGeometry, steps: int, batch: int = 4096, lr: float = 1e-3,
              seed: int = 0, j_min: int = 0, log_every: int = 0) -> list:
        """Adam steps on random pixels of the frames rf [F, n_tx, n_el, S]; the targets are
        minimum-variance weights computed for the same pixels.  Returns the loss history."""
        gen = torch.Generator(device=self.device)
        gen.manual_seed(seed)
        loss = torch.zeros(1, device=self.device)
        hist = []
        for s in range(steps):
            pix = random_pixels(gen, batch, rf.shape[0], dg.n_lines, dg.n_depth, j_min, self.device)
            x = delay_gather(rf, dg, pix)
            target, _ = mv_weights(x, SUBAPERTURE, LOADING)
            cur_lr = lr * (0.1 if s >= int(0.8 * steps) else 1.0)
            self.net.train_step(x, target, cur_lr, loss)
            if log_every and (s % log_every == 0 or s == steps - 1):
                hist.append((s, float(loss.item())))
        return hist

    def weights(self, x: torch.Tensor) -> torch.Tensor:
        return self.net.forward(x)


def beamform_lines(rf: torch.Tensor, dg: DeviceGeometry, method: str, model: LearnedApodization | None = None,
                   chunk: int = 65536) -> torch.Tensor:
    """Beamformed lines [n_lines, n_depth] of one frame rf [n_tx, n_el, S] by 'das' (the
    library's delay-and-sum), 'mv' (minimum variance) or 'learned' (network weights, with the
    delay-and-sum value as the fallback)."""
    das = beamform(rf.unsqueeze(0) if rf.dim() == 3 else rf, dg)[0]
    if method == "das":
        return das
    pix_all = frame_pixels(dg.n_lines, dg.n_depth, 0, rf.device)
    out = torch.empty(dg.n_lines * dg.n_depth, dtype=torch.float32, device=rf.device)
    fb = das.reshape(-1)
    for c0 in range(0, pix_all.shape[0], chunk):
        pix = pix_all[c0:c0 + chunk]
        x = delay_gather(rf, dg, pix)
        if method == "mv":
            _, y = mv_weights(x, SUBAPERTURE, LOADING, want_weights=False)
        elif method == "learned":
            y = model.net.apply(x, fb[c0:c0 + chunk].contiguous())
        else:
            raise ValueError(method)
        out[c0:c0 + pix.shape[0]] = y
    return out.reshape(dg.n_lines, dg.n_depth)


def frame_envelope(lines: torch.Tensor) -> np.ndarray:
    env = envelope(lines.unsqueeze(0).contiguous())[0].cpu().numpy().astype(np.float64)
    return env


def psf_widths(env: np.ndarray, line_x: np.ndarray, targets) -> np.ndarray:
    """Lateral -6 dB width (metres) of each point target (line, depth) on envelope lines
    [n_lines, n_depth]; the lateral profile takes the maximum over +-2 depth samples."""
    widths = []
    n_lines = env.shape[0]
    for (l0, j0) in targets:
        prof = env[:, max(0, j0 - 2): j0 + 3].max(axis=1)
        lo, hi = max(0, l0 - 2), min(n_lines, l0 + 3)
        lp = lo + int(np.argmax(prof[lo:hi]))
        half = 0.5 * prof[lp]
        # walk out from the peak to the first sample below half amplitude, interpolate linearly
        def cross(step):
            k = lp
            while 0 <= k + step < n_lines and prof[k + step] >= half:
                k += step
            if not 0 <= k + step < n_lines:
                return float(line_x[k])
            a, b = prof[k], prof[k + step]
            t = (a - half) / (a - b)
            return float(line_x[k] + t * (line_x[k + step] - line_x[k]))
        widths.append(abs(cross(1) - cross(-1)))
    return np.array(widths)


def cnr(env: np.ndarray, line_x: np.ndarray, depth_z: np.ndarray, cysts) -> np.ndarray:
    """Contrast-to-noise ratio of each cyst (cx, cz, r): inside 0.75 r against the ring
    1.25 r .. 1.75 r."""
    X, Z = np.meshgrid(line_x, depth_z, indexing="ij")
    out = []
    for (cx, cz, r) in cysts:
        d2 = (X - cx) ** 2 + (Z - cz) ** 2
        inside = env[d2 <= (0.75 * r) ** 2]
        ring = env[(d2 >= (1.25 * r) ** 2) & (d2 <= (1.75 * r) ** 2)]
        out.append(abs(inside.mean() - ring.mean()) / np.sqrt(inside.var() + ring.var()))
    return np.array(out)


def aux_geometry(g, xs):
    """Vertical lines from the array plane at lateral positions xs, on g's depth grid; each
    line takes the transmit whose origin is laterally nearest (the transmit that would fire
    for a line there)."""
    xs = np.asarray(xs, np.float64)
    n = xs.size
    a = copy.copy(g)
    a.line_origin = np.ascontiguousarray(np.stack([xs, np.zeros(n), np.zeros(n)], 1).astype(np.float32))
    a.line_dir = np.ascontiguousarray(np.tile(np.float32([0.0, 0.0, 1.0]), (n, 1)))
    tx_x = np.asarray(g.tx_origin[:, 0], np.float64)
    a.line_tx = np.ascontiguousarray(np.argmin(np.abs(xs[:, None] - tx_x[None, :]), axis=1).astype(np.int32))
    a.scan = None
    return a


def psf_widths_fine(rf: torch.Tensor, g, method: str, model=None, targets=(), half_width: float = 1.5e-3,
                    device="cuda") -> np.ndarray:
    """Lateral -6 dB width (metres) of each point target (line, depth) of g, measured on lines
    spaced a twentieth of the wavelength c / f0 within +-half_width of the target's line."""
    step = g.c / g.f0 / 20.0
    offs = np.arange(-round(half_width / step), round(half_width / step) + 1) * step
    x0 = np.asarray(g.line_origin[:, 0], np.float64)
    xs = np.concatenate([x0[l] + offs for (l, _) in targets])
    dg = DeviceGeometry(aux_geometry(g, xs), device)
    env = frame_envelope(beamform_lines(rf, dg, method, model))
    n, c = offs.size, offs.size // 2
    return np.array([psf_widths(env[k * n:(k + 1) * n], offs, [(c, j)])[0] for k, (_, j) in enumerate(targets)])


def _sim(g, seed, cysts=(), n_speckle=5000, device="cuda"):
    import synth  # seeded input generation (synthetic phantoms)
    pos, amp, lj = synth.phantom.phantom_2d(g, seed, n_speckle=n_speckle, cysts=cysts)
    return synth.rfsim.simulate_frame(g, pos, amp, seed, device=device).contiguous(), lj


def eval_phantom(g, seed: int, device="cuda"):
    """A held-out frame: speckle, one anechoic cyst of radius 4 mm at (0, 40 mm) and 8 point
    targets from 15 to 70 mm deep, alternately 6 mm left and right of the centre, each moved
    onto the nearest output pixel.  Returns (rf, cyst, point pixels)."""
    import synth  # seeded input generation (synthetic phantoms)
    lx = np.asarray(g.line_origin[:, 0], np.float64)
    dz = float(g.depth_of(1) - g.depth_of(0))
    cyst = (0.0, 40e-3, 4e-3)
    pts, lj = [], []
    for k, z in enumerate(np.linspace(15e-3, 70e-3, 8)):
        l = int(np.argmin(np.abs(lx - (6e-3 if k % 2 else -6e-3))))
        j = int(round(z / dz))
        p = synth.phantom.pixel_position(g, l, j)
        pts.append((float(p[0]), float(p[2]), 10.0))
        lj.append((l, j))
    pos, amp, _ = synth.phantom.phantom_2d(g, seed, n_points=False, cysts=[cyst], extra_points=pts)
    rf = synth.rfsim.simulate_frame(g, pos, amp, seed, device=device).contiguous()
    return rf, cyst, lj


def evaluate(model: LearnedApodization, g, dg: DeviceGeometry, n_frames: int = 32, seed: int = 90000) -> dict:
    """Mean CNR of the cyst and mean -6 dB width of the points over n_frames held-out frames for
    DAS, MV and the network; the network passes if its mean CNR and mean width are both within
    10 % of MV's and its mean width is narrower than DAS's.  Also the GPU time of the MV and
    network weight paths for one frame's pixels."""
    lx = g.line_origin[:, 0].astype(np.float64)
    z = np.array([g.depth_of(j) for j in range(g.n_depth)], dtype=np.float64)
    c = {m: [] for m in ("das", "mv", "learned")}
    w = {m: [] for m in ("das", "mv", "learned")}
    for f in range(n_frames):
        rf, cyst, lj = eval_phantom(g, seed + f, dg.device)
        for m in c:
            env = frame_envelope(beamform_lines(rf, dg, m, model))
            c[m].append(float(cnr(env, lx, z, [cyst])[0]))
            w[m].extend((psf_widths_fine(rf, g, m, model, lj, device=dg.device) * 1e3).tolist())
    res = {m: {"cnr_mean": float(np.mean(c[m])), "cnr_std": float(np.std(c[m])),
               "psf_width_mm_mean": float(np.mean(w[m])), "psf_width_mm_std": float(np.std(w[m]))} for m in c}
    dc = res["learned"]["cnr_mean"] / res["mv"]["cnr_mean"] - 1.0
    dw = res["learned"]["psf_width_mm_mean"] / res["mv"]["psf_width_mm_mean"] - 1.0
    res["learned_vs_mv"] = {"cnr_rel": dc, "width_rel": dw,
                            "pass": bool(abs(dc) <= 0.1 and abs(dw) <= 0.1 and
                                         res["learned"]["psf_width_mm_mean"] < res["das"]["psf_width_mm_mean"])}
    rf, _, _ = eval_phantom(g, seed, dg.device)
    res["timing"] = time_paths(model, rf, dg)
    res["eval"] = f"{n_frames} held-out frames (seeds {seed}..), 1 cyst and 8 points each"
    return res


def time_paths(model: LearnedApodization, rf: torch.Tensor, dg: DeviceGeometry, reps: int = 5) -> dict:
    """GPU time of the two adaptive paths from channel data to beamformed values for every
    pixel of one frame: delay-gather + minimum-variance weights and weighted sum (the MV
    kernel forms y = w_full^T x itself), against delay-gather + network forward + weighted sum
    in one pass (with the delay-and-sum value of the frame as the fallback, computed
    beforehand; the separate forward and weighted-sum calls are timed as well).  The
    stages both share afterwards (envelope, compression, scan conversion) are left out.  HIP
    events on the stream the kernels run on."""
    pix = frame_pixels(dg.n_lines, dg.n_depth, 0, rf.device)
    n = pix.shape[0]
    fb = beamform(rf.unsqueeze(0) if rf.dim() == 3 else rf, dg)[0].reshape(-1).contiguous()
    x = torch.empty((n, dg.n_el), dtype=torch.float32, device=rf.device)
    w = torch.empty_like(x)
    y = torch.empty(n, dtype=torch.float32, device=rf.device)

    def mv_path():
        delay_gather(rf, dg, pix, out=x)
        return mv_weights(x, SUBAPERTURE, LOADING, want_weights=False)[1]

    def learned_path():
        delay_gather(rf, dg, pix, out=x)
        return model.net.apply(x, fb, out=y)

    def learned_unfused():
        delay_gather(rf, dg, pix, out=x)
        model.net.forward(x, out=w)
        return beamform_weighted(x, w, fb)

    def gather_only():
        delay_gather(rf, dg, pix, out=x)

    out = {"pixels": int(n)}
    stream = torch.cuda.current_stream(rf.device)
    for name, fn in (("mv", mv_path), ("learned", learned_path), ("learned_unfused", learned_unfused),
                     ("gather", gather_only)):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        out[f"{name}_ms_per_frame"] = e0.elapsed_time(e1) / reps
    out["learned_speedup_vs_mv"] = out["mv_ms_per_frame"] / out["learned_ms_per_frame"]
    return out


def simulate_training_frames(g, n: int, seed0: int = 100, device="cuda", log=None) -> torch.Tensor:
    """n training frames, each with two random anechoic cysts (radius 2-5 mm) in speckle and
    the workload's 20 point targets."""
    rng = np.random.default_rng(1)
    lx = g.line_origin[:, 0].astype(np.float64)
    zmax = g.depth_of(g.n_depth - 1)
    frames = []
    for f in range(n):
        cysts = [(rng.uniform(0.8 * lx[0], 0.8 * lx[-1]), rng.uniform(0.15, 0.85) * zmax, rng.uniform(2e-3, 5e-3))
                 for _ in range(2)]
        frames.append(_sim(g, seed0 + f, cysts=cysts, device=device)[0])
        if log and (f + 1) % 16 == 0:
            log(f"simulated {f + 1} / {n} training frames")
    return torch.stack(frames).contiguous()


def main():
    import synth
    ap = argparse.ArgumentParser()
    ap.add_argument("--frames", type=str, default="16",
                    help="training-set sizes, comma separated (each trains its own network from the same start)")
    ap.add_argument("--steps", type=int, default=8000)
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--eval-frames", type=int, default=32)
    ap.add_argument("--save", default="")
    ap.add_argument("--out", default="", help="also write the result JSON to this file")
    ap.add_argument("--timing-only", action="store_true",
                    help="only time the two adaptive paths on one held-out frame (untrained network)")
    args = ap.parse_args()
    g = synth.config_multiline_2d()
    dg = DeviceGeometry(g)
    if args.timing_only:
        rf, _, _ = eval_phantom(g, 90000)
        print(json.dumps({"timing": time_paths(LearnedApodization(g.n_el, seed=0), rf, dg)}), flush=True)
        return
    sizes = [int(v) for v in args.frames.split(",")]
    t = time.perf_counter()
    import sys
    rf_all = simulate_training_frames(g, max(sizes), log=lambda m: print(m, file=sys.stderr, flush=True))
    torch.cuda.synchronize()
    t_sim = time.perf_counter() - t
    runs = []
    for n in sizes:
        model = LearnedApodization(g.n_el, seed=0)
        t = time.perf_counter()
        hist = model.train(rf_all[:n], dg, args.steps, args.batch, args.lr, log_every=max(1, args.steps // 20))
        torch.cuda.synchronize()
        t_train = time.perf_counter() - t
        res = evaluate(model, g, dg, n_frames=args.eval_frames)
        runs.append({"train_frames": n, "train_s": t_train, "final_loss": hist[-1][1], "eval": res})
        print(json.dumps(runs[-1]), flush=True)
        if args.save and n == sizes[-1]:
            np.savez(args.save, **model.net.params())
    out = {"workload": "linear 128 el, 64 tx x 4 lines, 4096 samples; MV L = 32, loading 1e-2",
           "steps": args.steps, "batch": args.batch, "lr": args.lr, "sim_s": t_sim, "runs": runs}
    if args.out:
        with open(args.out, "w") as f:
            json.dump(out, f, indent=1)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
