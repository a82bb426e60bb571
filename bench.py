"""Throughput of the receive pipeline (delay-and-sum -> envelope -> log compression -> scan
conversion) on one MI355X.

Default workload: 128-element linear array, 256 scanlines from 64 focused transmits with 4
receive lines each, 4096 int16 samples per channel at 40 MHz, 2048 output samples per line,
512 x 512 B-mode image per frame, batches of 32 frames.  One step = one batch through the whole
path.  Inputs are synthetic phantoms (20 points + 5000 speckle scatterers, 40 dB SNR) already
resident in HBM when the timed region starts.

Prints one JSON line: metric, value (pixel·channel samples per second over the timed steps),
stage times, the delay-and-sum roofline (algorithmic bytes over the event-timed launch, against
8 TB/s, with the HBM traffic counted by rocprofv3 when it matches the source) and the CPU
oracle's rate on a bounded sample.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "pixel·channel samples/s and frames(volumes)/s for DAS→B-mode; learned vs MV at stated error"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def code_tokens(text):
    """C++ source with its comments removed and whitespace collapsed: what the compiler sees
    (string and character literals are kept as they are)."""
    out, i, n = [], 0, len(text)
    while i < n:
        c = text[i]
        if text.startswith("//", i):
            j = text.find("\n", i)
            i = n if j < 0 else j
        elif text.startswith("/*", i):
            j = text.find("*/", i + 2)
            i = n if j < 0 else j + 2
            out.append(" ")
        elif c in "\"'":
            j = i + 1
            while j < n and text[j] != c:
                j += 2 if text[j] == "\\" else 1
            out.append(text[i:j + 1])
            i = j + 1
        else:
            out.append(c)
            i += 1
    return " ".join("".join(out).split())


def kernel_hash(paths):
    """Hash of the sources' code (comments and layout ignored): traffic counted for one build
    stays valid while only the comments change."""
    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(ROOT, p), encoding="utf-8") as f:
            h.update(code_tokens(f.read()).encode())
    return h.hexdigest()[:16]


CALIB_BYTES = 1 << 30
DAS_SOURCES = ["paper_1711_06127_amd/csrc/das.hip", "paper_1711_06127_amd/csrc/das.h",
               "paper_1711_06127_amd/csrc/das_tile.h", "paper_1711_06127_amd/csrc/das_g1.hip",
               "paper_1711_06127_amd/csrc/das_g2.hip", "paper_1711_06127_amd/csrc/das_g4.hip",
               "paper_1711_06127_amd/csrc/das_g8.hip", "paper_1711_06127_amd/csrc/tof.h",
               "paper_1711_06127_amd/csrc/common.h"]


def _counter_rows(path, counter):
    """(kernel name, value) per dispatch of one counter from a rocprofv3 counter_collection.csv."""
    import csv
    out = {}
    with open(path) as f:
        for r in csv.DictReader(f):
            if r["Counter_Name"] != counter:
                continue
            key = int(r["Dispatch_Id"]) if "Dispatch_Id" in r else len(out)
            name, val = r["Kernel_Name"], float(r["Counter_Value"])
            out[key] = (name, out.get(key, (name, 0.0))[1] + val)
    return [out[k] for k in sorted(out)]


def write_traffic(args):
    """HBM bytes per DAS launch, each counter scaled so that the 1 GiB copy reads and writes
    exactly 1 GiB."""
    res = {}
    for counter, path in (("FETCH_SIZE", args.traffic_from[0]), ("WRITE_SIZE", args.traffic_from[1])):
        rows = _counter_rows(path, counter)
        das = [v for n, v in rows if "das_tile_kernel" in n]
        # the calibration copy: a streaming kernel that moved about 1 GiB (the fetch counter reads
        # about half of it on this part)
        copies = [v for n, v in rows if ("copyBuffer" in n or "elementwise" in n) and v * 1024 > 0.25 * CALIB_BYTES]
        if not das or not copies:
            raise SystemExit(f"{path}: no das_tile_kernel or calibration copy dispatch for {counter}")
        scale = CALIB_BYTES / (copies[-1] * 1024.0)
        res[counter] = {"raw_kib_per_launch": sum(das) / len(das), "copy_raw_kib": copies[-1], "scale": scale,
                        "bytes_per_launch": sum(das) / len(das) * 1024.0 * scale, "launches": len(das)}
    entry = {"sources": DAS_SOURCES, "source_hash": kernel_hash(DAS_SOURCES), "units": args.frames or 32,
             "bytes_per_launch": res["FETCH_SIZE"]["bytes_per_launch"] + res["WRITE_SIZE"]["bytes_per_launch"],
             "counters": res, "command": args.traffic_command}
    path = os.path.join(ROOT, "profiles", "traffic.json")
    d = json.load(open(path)) if os.path.exists(path) else {}
    d["das"] = entry
    with open(path, "w") as f:
        json.dump(d, f, indent=1)
    print(json.dumps(entry, indent=1))


def traffic_from_profile(name, per_launch_units):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it still matches
    the kernel source; otherwise None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f).get(name)
    if not d or d.get("source_hash") != kernel_hash(d.get("sources", [])):
        return None
    if d.get("units") != per_launch_units:
        return None
    return d.get("bytes_per_launch")


WORKLOADS = {
    # name: (geometry builder, default frames per batch, description)
    "multiline": ("config_multiline_2d", 32, "linear 128 el, 64 tx x 4 receive lines, 4096 int16 samples @ 40 MHz, "
                                              "256 x 2048 lines -> 512 x 512 B-mode"),
    "small": ("config_small_2d", 64, "linear 64 el, 64 tx x 1 line, 2048 int16 samples @ 40 MHz, "
                                     "64 x 1024 lines -> 256 x 256 B-mode"),
    "volume": ("config_volume_3d", 1, "matrix 32 x 32 el, 1024 steered tx/lines over +-30 deg, 2000 int16 samples "
                                      "@ 20 MHz, 32 x 32 x 1000 lines -> 128^3 B-mode volume"),
    "planewave": ("config_planewave_2d", 16, "plane-wave imaging, linear 128 el, 11 steered plane waves (-10..10 deg), "
                                             "256 lines x 2048 depths beamformed per wave, 4096 int16 samples @ 40 MHz, "
                                             "coherent compounding -> 512 x 512 B-mode"),
    "overlap": ("config_overlap_2d", 16, "overlapping multi-line layout, linear 128 el, 128 focused tx, 255 lines "
                                         "at half pitch (lines between two transmits interpolated from both beams: "
                                         "382 beams of 2048 depths per frame), 4096 int16 samples @ 40 MHz -> "
                                         "512 x 512 B-mode"),
    "stream": ("stream_mix", 100, "uneven stream of 100 items, seeded 70/30 mix of linear frames (64/128/192 el, "
                                  "2048..4096 samples, n_el/2 transmits x 4 lines, 512^2 images) and matrix volumes "
                                  "(16x16 or 32x32 el, 1000..2000 samples, 32x32 lines, 128^3 volumes), one "
                                  "persistent graph-captured delay-and-sum launch per batch"),
}


def make_batch(g, n_frames, n_unique, device, volume=False):
    import torch
    import synth
    frames = []
    for f in range(n_unique):
        if volume:
            frames.append(synth.rfsim.simulate_volume(g, 7000 + f, device=device))
        else:
            pos, amp, _ = synth.phantom.phantom_2d(g, 5000 + f)
            frames.append(synth.rfsim.simulate_frame(g, pos, amp, 5000 + f, device=device))
    idx = torch.arange(n_frames) % n_unique
    return torch.stack(frames)[idx].contiguous()


def beams(g):
    """Beamformed lines per frame that the image uses (unused line slots excluded)."""
    import numpy as np
    return int((np.asarray(g.line_tx) >= 0).sum())


def cpu_baseline(g, rf_host, budget_s):
    """The oracle, as it stands, on a bounded sample of the same batch (whole frames)."""
    import oracle
    t0 = time.perf_counter()
    n = 0
    while True:  # whole frames, cycling through the batch, until the budget is spent
        i = n % rf_host.shape[0]
        y = oracle.das(g, rf_host[i:i + 1])
        n_angles = getattr(g, "n_angles", 0)
        if n_angles:  # coherent compounding of the plane-wave lines
            y = y.reshape(1, n_angles, g.n_lines // n_angles, g.n_depth).mean(axis=1)
        if hasattr(g, "combine_src"):  # overlapping lines: interpolation between transmits
            y = oracle.combine_lines(y, g.combine_src, g.combine_w)
        if g.scan.kind == 1:
            oracle.bmode_3d(y[0], g.scan, 50.0)
        else:
            oracle.bmode_2d(y[0], g.scan, 50.0)
        n += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    dt = time.perf_counter() - t0
    pcs = n * beams(g) * g.n_depth * g.n_el
    return {"value": pcs / dt, "unit": "pixel·channel samples/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"{n} frame(s) of the batch, cycled, through the float64 oracle (DAS"
                      f"{' + compounding' if getattr(g, 'n_angles', 0) else ''}"
                      f"{' + line interpolation' if hasattr(g, 'combine_src') else ''} + envelope + log + scan "
                      f"conversion), {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="multiline", choices=sorted(WORKLOADS))
    ap.add_argument("--frames", type=int, default=0, help="frames per batch (0: workload default)")
    ap.add_argument("--unique-frames", type=int, default=8)
    ap.add_argument("--cpu-budget", type=float, default=12.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--envelope", default="hilbert", choices=["hilbert", "iq"],
                    help="envelope detector: analytic signal (default) or IQ demodulation with three "
                         "compounded bands at 0.8, 1.0, 1.2 f0 (63 taps, bandwidth 0.4 f0)")
    ap.add_argument("--streams", type=int, default=1, choices=[1, 2, 3],
                    help="streams that consecutive batches alternate between (detection and scan "
                         "conversion of one batch overlap the next batch's delay-and-sum)")
    ap.add_argument("--unordered", action="store_true",
                    help="with several streams, let the delay-and-sum launches of consecutive batches "
                         "overlap too (their event-timed durations then include each other)")
    ap.add_argument("--apod-sets", type=int, default=1, choices=[1, 2, 4],
                    help="beamform with this many apodization sets in one pass (f-number 1.0 Hann, "
                         "1.75 rect, 1.5 Hann, 2.5 rect) and take every set through the pipeline")
    ap.add_argument("--calib-copy", action="store_true",
                    help="after the timed steps, copy a 1 GiB buffer (the reference kernel for HBM counters)")
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="no GPU: turn two rocprofv3 counter collections (FETCH_SIZE, WRITE_SIZE) of a "
                         "--calib-copy run into profiles/traffic.json")
    ap.add_argument("--traffic-command", default="", help="the profiled command, recorded with the figures")
    ap.add_argument("--no-volume", action="store_true",
                    help="skip the 3D volume measurement that the default (multi-line) run adds to its line")
    args = ap.parse_args()
    if args.traffic_from:
        return write_traffic(args)
    if args.gpus != 1:
        print(json.dumps({"error": "this library runs on one GPU; multi-GPU runs are not part of it "
                                   f"(asked for --gpus {args.gpus})"}))
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1711_06127_amd as u
    import synth

    dev = torch.device("cuda:0")
    u.lib()
    if args.workload == "stream":
        return run_stream(args, dev)
    result = measure(args, args.workload, dev)
    if args.workload == "multiline" and not args.no_volume and args.apod_sets == 1:
        # the volume rate of the 3D workload beside the headline 2D figure
        vargs = argparse.Namespace(**vars(args))
        vargs.frames, vargs.streams, vargs.unordered, vargs.envelope = 1, 1, False, "hilbert"
        vargs.steps, vargs.warmup = max(3, min(args.steps, 10)), 2
        vargs.calib_copy = False
        v = measure(vargs, "volume", dev, cpu_stages=not args.no_cpu)
        result["volume"] = {"workload": v["config"]["workload"], "volumes_per_s": v["frames_per_s"],
                            "ms_per_volume": v["ms_per_step"], "steps": v["steps"], "stage_ms": v["stage_ms"],
                            "pixel_channel_samples_per_s": v["value"], "roofline": v["roofline"],
                            "cpu_stages_s": v.get("cpu_stages_s")}
    print(json.dumps(result), flush=True)


def cpu_stage_times(g, rf_host):
    """The oracle's time per stage on the first frame (volume) of the batch: delay and sum,
    envelope, log compression, scan conversion."""
    import oracle
    t = time.perf_counter()
    y = oracle.das(g, rf_host[:1])[0]
    t_das = time.perf_counter() - t
    t = time.perf_counter()
    env = oracle.envelope(y)
    t_env = time.perf_counter() - t
    t = time.perf_counter()
    b = oracle.log_compress(env, 50.0)
    t_log = time.perf_counter() - t
    t = time.perf_counter()
    if g.scan.kind == 1:
        oracle.scan_convert_3d(b, g.scan)
    else:
        oracle.scan_convert_2d(b, g.scan)
    t_scan = time.perf_counter() - t
    return {"das": t_das, "envelope": t_env, "log_compress": t_log, "scan_convert": t_scan,
            "cores": oracle.num_threads(), "kind": "oracle"}


def measure(args, workload, dev, cpu_stages=False):
    """Times `workload` per the arguments; returns the result dict of the bench line."""
    import numpy as np
    import torch

    import paper_1711_06127_amd as u
    import synth

    builder, default_frames, desc = WORKLOADS[workload]
    g = getattr(synth, builder)()
    F = args.frames or default_frames
    t = time.perf_counter()
    rf = make_batch(g, F, min(args.unique_frames, F), dev, volume=workload == "volume")
    torch.cuda.synchronize()
    log(f"inputs: {tuple(rf.shape)} int16 ({rf.numel() * 2 / 2**30:.2f} GiB) generated in {time.perf_counter() - t:.1f} s")
    dg = u.DeviceGeometry(g, dev)
    n_sets = args.apod_sets
    set_fn, set_win = [1.0, 1.75, 1.5, 2.5][:n_sets], [1, 0, 1, 0][:n_sets]
    # with several apodization sets every set is an image of its own: S x F images per step
    FI = F * n_sets
    n_angles = getattr(g, "n_angles", 0)
    overlap = hasattr(g, "combine_src")
    if overlap:
        c_src = torch.as_tensor(g.combine_src, device=dev)
        c_w = torch.as_tensor(g.combine_w, device=dev)
    line_fs = float(g.fs) / g.depth_step
    iq_bands = [0.8 * g.f0, g.f0, 1.2 * g.f0]

    def buffers():
        b = {"lines": torch.empty((FI, g.n_lines, g.n_depth), dtype=torch.float32, device=dev)}
        # plane waves: the lines of every angle are compounded into the image lines first;
        # overlapping layouts: the output lines are interpolated from the transmits' beams
        if n_angles:
            b["det"] = torch.empty((FI, g.n_lines // n_angles, g.n_depth), dtype=torch.float32, device=dev)
        elif overlap:
            b["det"] = torch.empty((FI, g.n_out_lines, g.n_depth), dtype=torch.float32, device=dev)
        else:
            b["det"] = b["lines"]
        b["row_max"] = torch.empty(b["det"].shape[:2], dtype=torch.float32, device=dev)
        b["img"] = torch.empty((FI, *dg.scan_shape), dtype=torch.float32, device=dev)
        b["iq_env"] = torch.empty_like(b["det"]) if args.envelope == "iq" else None
        return b

    # Consecutive batches alternate between n_streams streams, each with its own buffers: the
    # delay-and-sum launches stay in order (each waits for the previous one), and a batch's
    # detection and scan conversion overlap the next batch's delay-and-sum.
    n_streams = args.streams
    streams = [torch.cuda.current_stream(dev)] + [torch.cuda.Stream(dev) for _ in range(n_streams - 1)]
    bufs = [buffers() for _ in range(n_streams)]
    das_done = [torch.cuda.Event() for _ in range(n_streams)]
    last = [None]

    def step(k, ev=None):
        si = k % n_streams
        b = bufs[si]
        with torch.cuda.stream(streams[si]):
            if last[0] is not None and not args.unordered:
                streams[si].wait_event(das_done[last[0]])
            if ev is not None:
                ev[0].record()
            if n_sets > 1:
                u.beamform_sets(rf, dg, set_fn, set_win, out=b["lines"].view(n_sets, F, *b["lines"].shape[1:]))
            else:
                u.beamform(rf, dg, out=b["lines"])
            das_done[si].record()
            last[0] = si
            if ev is not None:
                ev[1].record()
            if n_angles:
                u.compound(b["lines"], n_angles, out=b["det"])
            elif overlap:
                u.combine_lines(b["lines"], c_src, c_w, out=b["det"])
            if b["iq_env"] is not None:
                u.envelope_iq(b["det"], line_fs, iq_bands, 0.4 * g.f0, 63, out=b["iq_env"], row_max=b["row_max"])
            else:
                u.envelope(b["det"], out=b["det"], row_max=b["row_max"])
            if ev is not None:
                ev[2].record()
            u.log_scan_convert(b["iq_env"] if b["iq_env"] is not None else b["det"], dg, 50.0,
                               row_max=b["row_max"], out=b["img"])
            if ev is not None:
                ev[3].record()

    for k in range(args.warmup):
        step(k)
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(k, evs[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    das_ms = np.array([e[0].elapsed_time(e[1]) for e in evs])
    env_ms = np.array([e[1].elapsed_time(e[2]) for e in evs])
    scan_ms = np.array([e[2].elapsed_time(e[3]) for e in evs])
    step_ms = wall * 1e3 / args.steps
    img = bufs[(args.steps - 1) % n_streams]["img"]
    iq_env = bufs[0]["iq_env"]

    # the whole-pipeline entry point gives the same image (it has the analytic-signal envelope
    # and no compounding)
    same = None
    if iq_env is None and not n_angles and not overlap and n_sets == 1:
        ref = u.bmode(rf, dg, 50.0, ws=u.BmodeWorkspace(dg, F))
        torch.cuda.synchronize()
        same = bool(torch.equal(ref, img))

    pcs = FI * beams(g) * g.n_depth * g.n_el
    rf_bytes = rf.numel() * 2
    out_bytes = FI * g.n_lines * g.n_depth * 4
    das_s = float(das_ms.mean()) * 1e-3
    achieved = (rf_bytes + out_bytes) / das_s / 1e9
    result = {
        "metric": METRIC,
        "value": pcs / (step_ms * 1e-3),
        "unit": "pixel·channel samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": step_ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": desc, "frames_per_batch": F, "envelope": args.envelope, "apod_sets": n_sets,
                   "streams": n_streams, "unordered_das": bool(args.unordered and n_streams > 1),
                   "unique_frames": min(args.unique_frames, F), "dyn_range_db": 50},
        "frames_per_s": FI / (step_ms * 1e-3),
        "stage_ms": {"das": float(das_ms.mean()),
                     ("compound+envelope" if n_angles else "combine+envelope" if overlap else "envelope"):
                         float(env_ms.mean()),
                     "log_scan": float(scan_ms.mean())},
        "bmode_entry_matches": same,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic_from_profile("das", F) if n_sets == 1 else None, "kernel": "das (delay-and-sum)",
                     "algorithmic_bytes": rf_bytes + out_bytes},
    }
    if args.calib_copy:
        # a plain streaming kernel that reads and writes exactly CALIB_BYTES
        src = torch.ones(CALIB_BYTES // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
    if cpu_stages:
        result["cpu_stages_s"] = cpu_stage_times(g, rf[:1].cpu().numpy())
    elif not args.no_cpu:
        rf_h = rf.cpu().numpy()
        result["cpu_baseline"] = cpu_baseline(g, rf_h, args.cpu_budget)
    del rf
    torch.cuda.empty_cache()
    return result


def run_stream(args, dev):
    """The uneven stream through BatchPlan: one persistent delay-and-sum launch over every item,
    then each item's envelope and log/scan epilogue, all replayed from one HIP graph."""
    import tempfile

    import numpy as np
    import torch

    import paper_1711_06127_amd as u
    import synth

    n_items = args.frames or WORKLOADS["stream"][1]
    gs = synth.stream_mix(seed=0, n_items=n_items)
    t = time.perf_counter()
    # one simulated acquisition per probe at its longest record; each item takes the first
    # n_samples of it, as its own copy (separate acquisitions)
    base = {}
    for g in gs:
        key = (g.array_dims, g.n_el)
        if key in base:
            continue
        if g.array_dims == 1:
            gl = synth.linear_2d("sim", n_el=g.n_el, n_tx=g.n_tx, lines_per_tx=4, line_pitch=0.15e-3, n_samples=4096)
            base[key] = make_batch(gl, 1, 1, dev)[0]
        else:
            gm = synth.matrix_3d("sim", n_side=int(round(g.n_el ** 0.5)), n_samples=2000)
            base[key] = make_batch(gm, 1, 1, dev, volume=True)[0]
    items = [(base[(g.array_dims, g.n_el)][..., :g.n_samples].contiguous(), u.DeviceGeometry(g, dev)) for g in gs]
    base.clear()
    torch.cuda.synchronize()
    log(f"stream: {len(gs)} items, {sum(x[0].numel() for x in items) * 2 / 2**30:.2f} GiB int16, "
        f"generated in {time.perf_counter() - t:.1f} s")
    cache = os.path.join(tempfile.mkdtemp(prefix="usbf_tune_"), "tune.json")
    plan = u.BatchPlan(items, 50.0, tune_cache=cache, autotune=True)
    shape = plan.shape()
    for _ in range(args.warmup):
        plan.run()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    for _ in range(args.steps):
        plan.run()
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    step_ms = wall * 1e3 / args.steps
    graph_ms = e0.elapsed_time(e1) / args.steps
    # the per-call pipeline gives the same images
    worst = 0.0
    for (rf, dg), img in zip(items, plan.images):
        ref = u.bmode(rf.unsqueeze(0), dg, 50.0)[0]
        worst = max(worst, float((ref - img).abs().max()))
    pcs = sum(g.n_lines * g.n_depth * g.n_el for g in gs)
    rf_bytes = sum(x[0].numel() * 2 for x in items)
    out_bytes = sum(g.n_lines * g.n_depth * 4 for g in gs)
    achieved = (rf_bytes + out_bytes) / (graph_ms * 1e-3) / 1e9
    result = {
        "metric": METRIC,
        "value": pcs / (step_ms * 1e-3),
        "unit": "pixel·channel samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": step_ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": WORKLOADS["stream"][2], "items": len(gs),
                   "linear_frames": sum(g.array_dims == 1 for g in gs),
                   "matrix_volumes": sum(g.array_dims == 2 for g in gs), "dyn_range_db": 50},
        "items_per_s": len(gs) / (step_ms * 1e-3),
        "graph_ms": graph_ms,
        "autotuned_shape": shape,
        "max_abs_diff_vs_per_call": worst,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "whole graph (persistent delay-and-sum + epilogues)",
                     "algorithmic_bytes": rf_bytes + out_bytes},
    }
    if not args.no_cpu:
        import oracle
        t0 = time.perf_counter()
        done = 0
        n = 0
        for (rf, dg), g in zip(items, gs):
            if g.scan.kind == 1:
                continue  # a single volume takes minutes in the oracle
            y = oracle.das(g, rf.unsqueeze(0).cpu().numpy())
            (oracle.bmode_3d if g.scan.kind == 1 else oracle.bmode_2d)(y[0], g.scan, 50.0)
            done += g.n_lines * g.n_depth * g.n_el
            n += 1
            if time.perf_counter() - t0 >= args.cpu_budget:
                break
        dt = time.perf_counter() - t0
        result["cpu_baseline"] = {"value": done / dt, "unit": "pixel·channel samples/s",
                                  "cores": oracle.num_threads(), "kind": "oracle",
                                  "sample": f"{n} linear frame(s) of the stream through "
                                            f"the float64 oracle, {dt:.1f} s"}
    plan.close()
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
