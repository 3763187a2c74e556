"""Device frame counters and whole-frame HIP graph replay.

The counters only move where the frame number and the Adam step come from,
so results with them must equal results with the same values passed
directly (bit-exact: the same kernels run on the same inputs).  A frame
recorded into a graph must then reproduce eager execution of the same calls,
checked on every replay with eager work and synchronisation in between.
"""
import numpy as np
import pytest
import torch

from paper_2506_05930_amd import api
from paper_2506_05930_amd.cache import FrameGraph
from tests.gpu_common import make_cache, p1080, params
from workloads import LightAnimation, box_scene, moving_light_table

pytestmark = pytest.mark.gpu

DEV = "cuda"


def t(x, dtype=None):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype).to(DEV)


@pytest.fixture(scope="module")
def scene():
    return box_scene(0, 160, 90, 64, 32, 256)


def test_counters_equal_explicit_frame_and_step(scene):
    n = scene["pos"].shape[0]
    rng = np.random.default_rng(40)
    vis = t(rng.uniform(0, 1, (n, 32)).astype(np.float16))
    pos, nrm, lights = t(scene["pos"]), t(scene["nrm"]), t(scene["lights"])
    ctr = api.new_counters(frame=7, step=3)
    outs = []
    for c in (None, ctr):
        o = [torch.empty(n, dtype=dt, device=DEV) for dt in (torch.int32, torch.float32, torch.float32, torch.float32)]
        api.nvc_sample_wrs(vis, pos, nrm, lights, 1e-3, 2, 7 if c is None else 12345, *o, ctr=c)
        pix = torch.empty(4096, dtype=torch.int32, device=DEV)
        ws = torch.empty(api.nvc_select_pixels_workspace_bytes(n), dtype=torch.uint8, device=DEV)
        api.nvc_select_pixels(2, 7 if c is None else 999, n, pix, ws, ctr=c)
        outs.append(o + [pix])
    for a, b in zip(*outs):
        assert torch.equal(a, b)
    # Adam: step 3 passed directly vs read from the counters
    g = torch.as_tensor(rng.normal(size=1001).astype(np.float32), device=DEV)
    res = []
    for c in (None, ctr):
        p = torch.ones(1001, device=DEV)
        m = torch.full((1001,), 0.1, device=DEV)
        v = torch.full((1001,), 0.2, device=DEV)
        api.nvc_adam(p, g.clone(), m, v, 3 if c is None else 1, 1e-2, 0.9, 0.99, 1e-8, ctr=c)
        res.append((p, m, v))
    for a, b in zip(*res):
        assert torch.equal(a, b)
    api.nvc_counters_advance(ctr)
    assert ctr.cpu().tolist() == [8, 4]


def _later_frame_close(vis_a, vis_b, idx_a, idx_b, f):
    """Outputs of two runs after f >= 1 training steps whose gradients differ by the order of the FP32
    atomics only.  Adam's first steps move an entry by about lr * sign(g), so an entry whose gradient is
    near zero can move by up to 2 lr between the runs; a few visibilities then differ by more than the
    output rounding.  Gated: the mean difference, the share of equal light picks, and a cap on the
    largest difference."""
    d = (vis_a.float() - vis_b.float()).abs()
    agree = (idx_a == idx_b).float().mean().item()
    print(f"  frame {f}: |dvis| max {d.max().item():.2e} mean {d.mean().item():.2e}, picks equal {agree:.5f}")
    assert d.mean().item() < 1e-4 and d.max().item() < 5e-2 and agree > 0.99, (f, d.max().item(), agree)


def _params_close(ca, cb, what, bound=2e-4):
    """Parameters and loss of two caches after the same frames.  Their gradients differ by the order of
    the FP32 atomics only, but Adam's first steps amplify that for entries with a near-zero gradient
    (a sign change moves the entry by up to 2 lr), so the bound is relative to the whole tensor: 2e-4
    after four frames.  An ordering fault between the streams (a gradient pass reading half-updated
    parameters, inference racing Adam) moves whole tensors, far beyond it."""
    for a in ("table", "w"):
        x, y = getattr(ca, a), getattr(cb, a)
        rel = ((x - y).norm() / x.norm()).item()
        moved = int(((x - y).abs() > 0.5 * ca.lr).sum().item())
        print(f"  {what} {a}: relative difference {rel:.2e}, {moved} of {x.numel()} entries apart by > lr/2")
        assert rel < bound, (what, a, rel)
    la, lb = ca.loss_buf.item(), cb.loss_buf.item()
    assert abs(la - lb) <= 1e-4 * abs(la), (what, la, lb)


def test_frame_graph_replays_match_eager(scene):
    wl = p1080()
    p = params(wl)
    batch = 4096
    base = scene["lights"]
    table_np = moving_light_table(base, 60)

    def setup():
        cache = make_cache(wl, p)
        pos_unit, pos, nrm = t(scene["pos_unit"]), t(scene["pos"]), t(scene["nrm"])
        lights, spheres = t(base), t(scene["spheres"])
        tab = t(table_np)
        fg = FrameGraph(cache, pos_unit, pos, nrm, lights, spheres, batch)
        fg.pre = LightAnimation(tab, lights, fg.ctr)
        return cache, fg, lights

    ce, fe, le = setup()
    cg, fgr, lg = setup()
    fgr.capture()
    for f in range(4):
        fe.run_eager()
        torch.cuda.synchronize()
        fgr.replay()
        torch.cuda.synchronize()
        assert torch.equal(le, lg) and torch.equal(le[0].cpu(), torch.as_tensor(table_np[f]))
        be, bg = fe.bufs, fgr.bufs
        assert torch.equal(be["train"]["pix"], bg["train"]["pix"])
        assert torch.equal(be["train"]["labels"], bg["train"]["labels"])
        if f == 0:      # same parameters: every output identical
            assert torch.equal(be["vis"], bg["vis"])
            for k in ("idx", "pmf", "wsum", "di"):
                assert torch.equal(be["sample"][k], bg["sample"][k])
        else:           # parameters differ by the order of the table-gradient atomics only
            _later_frame_close(be["vis"], bg["vis"], be["sample"]["idx"], bg["sample"]["idx"], f)
        _params_close(ce, cg, f"frame {f}")
        assert fe.ctr.cpu().tolist() == fgr.ctr.cpu().tolist() == [f + 1, f + 2]
        assert ce.step == cg.step == f + 1


def test_pipelined_frames_match_joined_frames(scene):
    """frame(join=False) leaves the training step with Adam on the second stream and never joins; four such
    frames queued without a host synchronisation equal four joined frames: the same training pixels and
    labels every frame, every output of the first frame, and afterwards what the order of the gradient
    atomics allows (as for the graph replays)."""
    wl = p1080()
    p = params(wl)
    batch = 4096
    args = [t(scene[k]) for k in ("pos_unit", "pos", "nrm", "lights", "spheres")]
    joined, piped = make_cache(wl, p), make_cache(wl, p)
    side_j, side_p = torch.cuda.Stream(), torch.cuda.Stream()
    out_j, out_p = [], []
    for f in range(4):
        out_j.append(joined.frame(*args, frame=f, batch=batch, side=side_j))
        torch.cuda.synchronize()
    for f in range(4):                                  # queued back to back
        out_p.append(piped.frame(*args, frame=f, batch=batch, side=side_p, join=False))
    piped.wait_training()
    torch.cuda.synchronize()
    assert joined.step == piped.step == 4
    for f, (bj, bp) in enumerate(zip(out_j, out_p)):
        assert torch.equal(bj["train"]["pix"], bp["train"]["pix"])
        assert torch.equal(bj["train"]["labels"], bp["train"]["labels"])
        if f == 0:
            assert torch.equal(bj["vis"], bp["vis"])
            for k in ("idx", "pmf", "wsum", "di"):
                assert torch.equal(bj["sample"][k], bp["sample"][k])
        else:
            _later_frame_close(bj["vis"], bp["vis"], bj["sample"]["idx"], bp["sample"]["idx"], f)
    _params_close(joined, piped, "after four frames")


@pytest.mark.parametrize("name", ["1080p", "paper_world", "clustered", "fused_labels"])
def test_frame_pipeline_matches_joined_frames(scene, name):
    """FramePipeline (inference + WRS, gradient pass + Adam, and the next frame's pixels, labels and routing
    plan on three streams) over four frames queued without a host synchronisation, against four joined
    frames: every output of the first frame, the later frames within what the order of the gradient
    atomics allows, the parameters and the loss.  Cases: the 1080p network; the paper's configuration
    with its world-space points (double-buffered with the pixels); the clustered cache (256 lights in 32
    k-means clusters: one ray per cluster, the two-step pick); labels computed inside the training kernel
    (the prep stream then only picks the pixels)."""
    from paper_2506_05930_amd.cache import FramePipeline
    from workloads import get_workload
    from workloads.scenes import SCENE_EXTENT
    sc = scene
    kw = {}
    if name == "paper_world":
        wl = get_workload("paper_1080p")
        batch = wl.train_batch
    elif name == "clustered":
        wl = get_workload("clustered_1080p", n_lights=256)
        sc = box_scene(0, 160, 90, 64, 256, 256)
        batch = 4096
    else:
        wl, batch = p1080(), 4096
        if name == "fused_labels":
            kw = {"fused_labels": True}
    p = params(wl)
    args = [t(sc[k]) for k in ("pos_unit", "pos", "nrm", "lights", "spheres")]
    joined, piped = make_cache(wl, p, **kw), make_cache(wl, p, **kw)
    if wl.world_batch:
        for c in (joined, piped):
            c.set_world_samples(wl.world_batch, wl.world_box, SCENE_EXTENT)
    if name == "clustered":
        off, mem = api.nvc_cluster_lights(sc["lights"], 32)
        for c in (joined, piped):
            c.set_clusters(off, mem, n_cand=8)
    keys = ("idx", "weight", "cluster") if name == "clustered" else ("idx", "pmf", "wsum", "di")
    side = torch.cuda.Stream()
    out_j = []
    for f in range(4):
        b = joined.frame(*args, frame=f, batch=batch, side=side)
        torch.cuda.synchronize()
        out_j.append({"vis": b["vis"].clone(), **{k: b["sample"][k].clone() for k in keys}})
    pipe = FramePipeline(piped, *args, batch)
    out_p = []
    for f in range(4):                                  # queued back to back
        b = pipe.run(f)
        out_p.append({"vis": b["vis"].clone(), **{k: b["sample"][k].clone() for k in keys}})
    pipe.finish()
    torch.cuda.synchronize()
    assert joined.step == piped.step == 4
    for f, (bj, bp) in enumerate(zip(out_j, out_p)):
        if f == 0:
            for k in bj:
                assert torch.equal(bj[k], bp[k]), k
        else:
            _later_frame_close(bj["vis"], bp["vis"], bj["idx"], bp["idx"], f)
    _params_close(joined, piped, "after four frames")


@pytest.mark.parametrize("name", ["1080p", "paper_world", "clustered", "fused_labels"])
def test_pipeline_graph_replays_match_joined_frames(scene, name):
    """PipelineGraph (the three-stream frame, the next frame's lights, pixels, labels and routing plan
    prepared inside the replay, two graphs alternating by pixel set) over six replays, light 0 moving on
    a circle, against six joined frames with the light placed from the host: the lights of every frame,
    the training pixels and labels of every frame bit for bit, every output of the first frame, the later
    frames within what the order of the gradient atomics allows, the parameters, the loss and the
    counters.  Replays 0-1 and 3-4 follow each other without a host synchronisation; clones of the
    outputs run between all of them."""
    from paper_2506_05930_amd.cache import PipelineGraph
    from workloads import get_workload
    from workloads.scenes import SCENE_EXTENT
    sc = scene
    kw = {}
    if name == "paper_world":
        wl = get_workload("paper_1080p")
        batch = wl.train_batch
    elif name == "clustered":
        wl = get_workload("clustered_1080p", n_lights=256)
        sc = box_scene(0, 160, 90, 64, 256, 256)
        batch = 4096
    else:
        wl, batch = p1080(), 4096
        if name == "fused_labels":
            kw = {"fused_labels": True}
    p = params(wl)
    table_np = moving_light_table(sc["lights"], 60)
    args_j = [t(sc[k]) for k in ("pos_unit", "pos", "nrm", "lights", "spheres")]
    args_g = [t(sc[k]) for k in ("pos_unit", "pos", "nrm", "lights", "spheres")]
    joined, graphed = make_cache(wl, p, **kw), make_cache(wl, p, **kw)
    if wl.world_batch:
        for c in (joined, graphed):
            c.set_world_samples(wl.world_batch, wl.world_box, SCENE_EXTENT)
    if name == "clustered":
        off, mem = api.nvc_cluster_lights(sc["lights"], 32)
        for c in (joined, graphed):
            c.set_clusters(off, mem, n_cand=8)
    keys = ("idx", "weight", "cluster") if name == "clustered" else ("idx", "pmf", "wsum", "di")
    tab = t(table_np)
    pg = PipelineGraph(graphed, *args_g, batch, make_anim=lambda lights, ctr: LightAnimation(tab, lights, ctr))
    pg.capture()
    side = torch.cuda.Stream()
    fused = name == "fused_labels"
    n_frames = 6
    out_j = []
    for f in range(n_frames):
        args_j[3][0].copy_(t(table_np[f]))
        b = joined.frame(*args_j, frame=f, batch=batch, side=side)
        torch.cuda.synchronize()
        out_j.append({"vis": b["vis"].clone(), **{k: b["sample"][k].clone() for k in keys},
                      "pix": b["train"]["pix"].clone(), "labels": b["train"]["labels"].clone(),
                      "lights": args_j[3].clone()})
    out_g = []
    for f in range(n_frames):
        pg.replay()
        s = pg.sets[f % 2]
        out_g.append({"vis": pg.bufs["vis"].clone(), **{k: pg.bufs["sample"][k].clone() for k in keys},
                      "pix": s["pix"].clone(), "labels": s["labels"].clone(), "lights": args_g[3].clone(),
                      "lights_next": pg.lights_next.clone()})
        if f not in (0, 3):
            torch.cuda.synchronize()
    torch.cuda.synchronize()
    for f, (bj, bg) in enumerate(zip(out_j, out_g)):
        assert torch.equal(bg["lights"], bj["lights"]), f
        assert torch.equal(bg["lights_next"][0].cpu(), torch.as_tensor(table_np[(f + 1) % 60])), f
        assert torch.equal(bg["pix"], bj["pix"]), f
        if not fused:
            assert torch.equal(bg["labels"], bj["labels"]), f
        if f == 0:
            for k in ("vis",) + keys:
                assert torch.equal(bj[k], bg[k]), k
        else:
            _later_frame_close(bj["vis"], bg["vis"], bj["idx"], bg["idx"], f)
    torch.cuda.synchronize()
    assert joined.step == graphed.step == n_frames
    assert pg.ctr.cpu().tolist() == [n_frames, n_frames + 1]
    assert pg.ctr_next.cpu().tolist() == [n_frames + 1, n_frames + 2]
    # six frames: what the atomics' order changes in one frame changes the gradients of the later frames
    # too, so the differences compound; an ordering fault would still be far beyond the bound
    _params_close(joined, graphed, f"after {n_frames} frames", bound=1e-3)
    pg.close()


@pytest.mark.skip(reason="LaggedPickGraph is switched off: one GPU run of this test (the clustered case) ended "
                         "in a host segmentation fault inside the graph launch, cause not found")
@pytest.mark.parametrize("name", ["1080p", "paper_world", "clustered", "fused_labels"])
def test_lagged_pick_graph_matches_joined_frames(scene, name):
    """LaggedPickGraph (the pick of frame f inside replay f + 1, beside that frame's inference; visibility
    and light buffers alternating) over six frames, light 0 moving on a circle, against six joined frames
    with the light placed from the host: every frame's lights, training pixels and labels bit for bit, the
    first frame's visibilities and pick bit for bit, the later frames' within what the order of the gradient
    atomics allows (the pick of frame f read after replay f + 1, the last one after flush()), the
    parameters and the counters.  Replays 1-2 and 4-5 follow each other without a host synchronisation."""
    from paper_2506_05930_amd.cache import LaggedPickGraph
    from workloads import get_workload
    from workloads.scenes import SCENE_EXTENT
    sc = scene
    kw = {}
    if name == "paper_world":
        wl = get_workload("paper_1080p")
        batch = wl.train_batch
    elif name == "clustered":
        wl = get_workload("clustered_1080p", n_lights=256)
        sc = box_scene(0, 160, 90, 64, 256, 256)
        batch = 4096
    else:
        wl, batch = p1080(), 4096
        if name == "fused_labels":
            kw = {"fused_labels": True}
    p = params(wl)
    table_np = moving_light_table(sc["lights"], 60)
    args_j = [t(sc[k]) for k in ("pos_unit", "pos", "nrm", "lights", "spheres")]
    args_g = [t(sc[k]) for k in ("pos_unit", "pos", "nrm", "lights", "spheres")]
    joined, graphed = make_cache(wl, p, **kw), make_cache(wl, p, **kw)
    if wl.world_batch:
        for c in (joined, graphed):
            c.set_world_samples(wl.world_batch, wl.world_box, SCENE_EXTENT)
    if name == "clustered":
        off, mem = api.nvc_cluster_lights(sc["lights"], 32)
        for c in (joined, graphed):
            c.set_clusters(off, mem, n_cand=8)
    keys = ("idx", "weight", "cluster") if name == "clustered" else ("idx", "pmf", "wsum", "di")
    tab = t(table_np)
    side = torch.cuda.Stream()
    fused = name == "fused_labels"
    n_frames = 6
    out_j = []
    for f in range(n_frames):
        args_j[3][0].copy_(t(table_np[f]))
        b = joined.frame(*args_j, frame=f, batch=batch, side=side)
        torch.cuda.synchronize()
        out_j.append({"vis": b["vis"].clone(), **{k: b["sample"][k].clone() for k in keys},
                      "pix": b["train"]["pix"].clone(), "labels": b["train"]["labels"].clone(),
                      "lights": args_j[3].clone()})
    lg = LaggedPickGraph(graphed, *args_g, batch, make_anim=lambda lights, ctr: LightAnimation(tab, lights, ctr))
    out_g = [dict() for _ in range(n_frames)]
    for f in range(n_frames):
        lg.replay()
        s = lg.sets[f % 2]
        out_g[f].update({"vis": lg.vis_of(f).clone(), "pix": s["pix"].clone(), "labels": s["labels"].clone(),
                         "lights": lg.lights_of(f).clone()})
        if f >= 1:
            out_g[f - 1].update({k: lg.bufs["sample"][k].clone() for k in keys})
        if f not in (1, 4):
            torch.cuda.synchronize()
    lg.flush()
    out_g[n_frames - 1].update({k: lg.bufs["sample"][k].clone() for k in keys})
    torch.cuda.synchronize()
    for f, (bj, bg) in enumerate(zip(out_j, out_g)):
        assert torch.equal(bg["lights"], bj["lights"]), f
        assert torch.equal(bg["pix"], bj["pix"]), f
        if not fused:
            assert torch.equal(bg["labels"], bj["labels"]), f
        if f == 0:
            for k in ("vis",) + keys:
                assert torch.equal(bj[k], bg[k]), k
        else:
            _later_frame_close(bj["vis"], bg["vis"], bj["idx"], bg["idx"], f)
    assert joined.step == graphed.step == n_frames
    assert lg.ctr.cpu().tolist() == [n_frames, n_frames + 1]
    assert lg.ctr_prev.cpu().tolist()[0] == n_frames - 1
    _params_close(joined, graphed, f"after {n_frames} frames", bound=1e-3)
    lg.close()
