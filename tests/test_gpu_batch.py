"""Persistent batched pipeline (one work-queue delay-and-sum launch + per-item epilogues in a
HIP graph) against the per-call library path and the oracle."""
import json

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


def sim(g, seed):
    pos, amp, _ = synth.phantom.phantom_2d(g, seed)
    return synth.rfsim.simulate_frame(g, pos, amp, seed, device="cuda").contiguous()


def random_rf(g, seed):
    rng = np.random.default_rng(seed)
    return torch.as_tensor(rng.integers(-3000, 3000, size=(g.n_tx, g.n_el, g.n_samples), dtype=np.int16)).cuda()


@pytest.fixture(scope="module")
def mixed(usbf):
    """A single-line 2D frame, a 4-line multi-line 2D frame, a full 3D volume and a second
    single-line frame: different element counts, sample counts and scan kinds."""
    gs = [synth.config_small_2d(), synth.config_multiline_2d(), synth.config_volume_3d(), synth.config_small_2d()]
    rfs = [sim(gs[0], 11), sim(gs[1], 12), random_rf(gs[2], 13), sim(gs[3], 14)]
    dgs = [usbf.DeviceGeometry(g) for g in gs]
    return gs, rfs, dgs


def test_batch_matches_per_call_pipeline(usbf, mixed):
    gs, rfs, dgs = mixed
    plan = usbf.BatchPlan(list(zip(rfs, dgs)), 50.0)
    imgs = [x.clone() for x in plan.run()]
    torch.cuda.synchronize()
    for rf, dg, img in zip(rfs, dgs, imgs):
        ref = usbf.bmode(rf.unsqueeze(0), dg, 50.0)[0]
        assert img.shape == ref.shape
        assert (img - ref).abs().max().item() <= 1e-5
    plan.close()


def test_batch_lines_match_oracle(usbf, mixed):
    gs, rfs, dgs = mixed
    plan = usbf.BatchPlan([(rfs[0], dgs[0]), (rfs[1], dgs[1])], 50.0)
    plan.run()
    torch.cuda.synchronize()
    for k in range(2):
        ref_bf = oracle.das(gs[k], rfs[k].unsqueeze(0).cpu().numpy())[0]
        ref_img = oracle.bmode_2d(ref_bf, gs[k].scan, 50.0)
        assert np.abs(plan.images[k].cpu().numpy() - ref_img).max() <= TOL
    plan.close()


def test_batch_replays_are_identical_and_follow_new_data(usbf, mixed):
    gs, rfs, dgs = mixed
    rf0 = rfs[0].clone()
    rf1 = rfs[1].clone()
    plan = usbf.BatchPlan([(rf0, dgs[0]), (rf1, dgs[1])], 45.0)
    a = [x.clone() for x in plan.run()]
    b = [x.clone() for x in plan.run()]
    torch.cuda.synchronize()
    for x, y in zip(a, b):
        assert torch.equal(x, y)
    rf0.copy_(rfs[3])  # new acquisition written in place
    plan.run()
    torch.cuda.synchronize()
    ref = usbf.bmode(rfs[3].unsqueeze(0), dgs[0], 45.0)[0]
    assert (plan.images[0] - ref).abs().max().item() <= 1e-5
    assert torch.equal(plan.images[1], b[1])
    plan.close()


def test_batch_ragged_items(usbf):
    """Items whose sample count is not a multiple of 4 (scalar loads), odd depth step, ragged
    depth tiles and a line count that is not a multiple of the 4-line tile."""
    g1 = synth.linear_2d("ragged1", n_el=7, n_tx=3, lines_per_tx=3, line_pitch=0.15e-3, n_samples=250,
                         window=synth.RECT, depth_step=2, scan_n=(40, 50))      # 125 depths
    g2 = synth.linear_2d("ragged2", n_el=12, n_tx=2, lines_per_tx=5, line_pitch=0.15e-3, n_samples=360,
                         depth_step=1, scan_n=(33, 70))                          # 360 depths
    rfs = [random_rf(g1, 1), random_rf(g2, 2)]
    dgs = [usbf.DeviceGeometry(g) for g in (g1, g2)]
    plan = usbf.BatchPlan(list(zip(rfs, dgs)), 50.0)
    plan.run()
    torch.cuda.synchronize()
    for k, g in enumerate((g1, g2)):
        ref_bf = oracle.das(g, rfs[k].unsqueeze(0).cpu().numpy())[0]
        assert np.abs(plan.lines[k].cpu().numpy() - oracle.envelope(ref_bf)).max() <= TOL * np.abs(
            oracle.envelope(ref_bf)).max()
        ref_img = oracle.bmode_2d(ref_bf, g.scan, 50.0)
        assert np.abs(plan.images[k].cpu().numpy() - ref_img).max() <= TOL
    plan.close()


def test_autotune_writes_cache_and_plan_reads_it(usbf, mixed, tmp_path):
    gs, rfs, dgs = mixed
    cache = str(tmp_path / "tune.json")
    items = [(rfs[0], dgs[0]), (rfs[1], dgs[1])]
    plan = usbf.BatchPlan(items, 50.0, tune_cache=cache, autotune=True)
    entries = json.load(open(cache))
    assert len(entries) == 1
    (key, val), = entries.items()
    assert key.startswith("gfx950")
    assert plan.shape() == {k: val[k] for k in ("groups_per_cu", "cost_order", "multi_line_tile", "chunk_div")}
    assert val["ms"] > 0
    plan.run()
    torch.cuda.synchronize()
    for rf, dg, img in zip(rfs[:2], dgs[:2], plan.images):
        ref = usbf.bmode(rf.unsqueeze(0), dg, 50.0)[0]
        assert (img - ref).abs().max().item() <= 1e-5
    plan.close()


@pytest.mark.parametrize("tile,div,gpc", [(4, 1, 1), (1, 1, 3), (4, 2, 2), (1, 2, 4)])
def test_every_launch_shape_gives_the_same_images(usbf, mixed, tile, div, gpc):
    """Tile height, element-chunk size and launch size change only the schedule: the images stay
    those of the per-call pipeline."""
    gs, rfs, dgs = mixed
    shape = {"groups_per_cu": gpc, "cost_order": 1, "multi_line_tile": tile, "chunk_div": div}
    plan = usbf.BatchPlan([(rfs[0], dgs[0]), (rfs[1], dgs[1])], 50.0, shape=shape)
    assert plan.shape() == shape
    plan.run()
    torch.cuda.synchronize()
    for rf, dg, img in zip(rfs[:2], dgs[:2], plan.images):
        ref = usbf.bmode(rf.unsqueeze(0), dg, 50.0)[0]
        assert (img - ref).abs().max().item() <= 1e-5
    plan.close()
