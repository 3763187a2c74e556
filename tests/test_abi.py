"""The C ABI library loads, exports every entry point of include/nvc.h, and
validates arguments on the host (no GPU needed: every call here returns
before anything is launched)."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

from paper_2506_05930_amd import _lib
from paper_2506_05930_amd._lib import NvcGrid, NvcMlp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nvc.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(nvc_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    return _lib.load()


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 16
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (nvc_[a-z0-9_]+)", out))
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    assert set(names) == set(_lib.EXPORTS)


def test_version_and_status_strings(lib):
    assert lib.nvc_version() == 1
    for code in range(0, -7, -1):
        assert _lib.status_string(code) != "unknown status"
    assert _lib.status_string(-99) == "unknown status"


def g(**kw):
    d = dict(n_levels=16, n_feat=2, log2_T=19, base_res=16, growth=1.447)
    d.update(kw)
    return NvcGrid(d["n_levels"], d["n_feat"], d["log2_T"], d["base_res"], d["growth"])


def m(**kw):
    d = dict(n_in=32, width=64, n_hidden=3, n_out=32, act=0, slope=0.01, dtype=1)
    d.update(kw)
    return NvcMlp(d["n_in"], d["width"], d["n_hidden"], d["n_out"], d["act"], d["slope"], d["dtype"])


def test_grid_levels_match_published_formula(lib):
    res = (ctypes.c_int32 * 16)()
    dense = (ctypes.c_int32 * 16)()
    assert lib.nvc_grid_levels(ctypes.byref(g()), res, dense) == 0
    from oracle import hashgrid
    assert list(res) == hashgrid.level_resolutions(16, 1.447, 16)
    assert [bool(x) for x in dense] == [hashgrid.level_is_dense(r, 1 << 19) for r in res]


@pytest.mark.parametrize("bad,code", [
    (dict(n_levels=0), _lib.NVC_ERR_SHAPE), (dict(n_levels=33), _lib.NVC_ERR_SHAPE),
    (dict(n_feat=3), _lib.NVC_ERR_UNSUPPORTED), (dict(log2_T=9), _lib.NVC_ERR_SHAPE),
    (dict(log2_T=25), _lib.NVC_ERR_SHAPE), (dict(base_res=0), _lib.NVC_ERR_SHAPE),
    (dict(growth=0.5), _lib.NVC_ERR_SHAPE), (dict(growth=float("nan")), _lib.NVC_ERR_SHAPE),
])
def test_grid_validation(lib, bad, code):
    assert lib.nvc_grid_levels(ctypes.byref(g(**bad)), None, None) == code


def test_param_counts(lib):
    assert lib.nvc_mlp_param_count(ctypes.byref(m())) == 32 * 64 + 2 * 64 * 64 + 64 * 32
    assert lib.nvc_mlp_param_count(ctypes.byref(m(n_in=16, width=32, n_hidden=2, n_out=8, dtype=0))) == 1792
    assert lib.nvc_mlp_param_count(ctypes.byref(m(dtype=7))) == _lib.NVC_ERR_DTYPE
    assert lib.nvc_mlp_param_count(ctypes.byref(m(n_out=129))) == _lib.NVC_ERR_UNSUPPORTED
    assert lib.nvc_mlp_param_count(ctypes.byref(m(act=1, slope=1.5))) == _lib.NVC_ERR_SHAPE
    assert lib.nvc_mlp_param_count(ctypes.byref(m(act=1, slope=float("nan")))) == _lib.NVC_ERR_SHAPE
    assert lib.nvc_mlp_param_count(ctypes.byref(m(act=1, slope=0.01))) > 0
    assert lib.nvc_mlp_packed_bytes(ctypes.byref(m())) >= 2 * 2 * 12288


def test_calls_reject_bad_arguments_before_launching(lib):
    # P is never dereferenced: every call below must fail validation (or be a no-op)
    # before anything is launched.  Never pass it to a call that would launch.
    P = ctypes.c_void_p(16)
    N = None
    gg, mm = ctypes.byref(g()), ctypes.byref(m())
    assert lib.nvc_encode(None, P, P, 10, P, 0, N) == _lib.NVC_ERR_NULL
    assert lib.nvc_encode(gg, P, P, -1, P, 0, N) == _lib.NVC_ERR_SHAPE
    assert lib.nvc_encode(gg, P, P, 10, P, 9, N) == _lib.NVC_ERR_DTYPE
    assert lib.nvc_encode(gg, None, P, 10, P, 0, N) == _lib.NVC_ERR_NULL
    assert lib.nvc_encode(gg, None, None, 0, None, 0, N) == 0           # n == 0 is a no-op
    assert lib.nvc_infer(gg, ctypes.byref(m(n_in=30)), P, P, P, 10, P, 1, N) == _lib.NVC_ERR_SHAPE
    assert lib.nvc_infer(gg, ctypes.byref(m(width=48)), P, P, P, 10, P, 1, N) == _lib.NVC_ERR_UNSUPPORTED
    assert lib.nvc_infer(gg, mm, None, P, P, 10, P, 1, N) == _lib.NVC_ERR_NULL
    assert lib.nvc_infer(gg, mm, None, None, None, 0, None, 1, N) == 0
    assert lib.nvc_sample_wrs(P, 1, 10, 0, P, N, P, 1e-3, 0, 0, N, P, P, P, N, N, N, N) == _lib.NVC_ERR_SHAPE
    assert lib.nvc_sample_wrs(P, 1, 10, 129, P, N, P, 1e-3, 0, 0, N, P, P, P, N, N, N, N) == _lib.NVC_ERR_SHAPE
    assert lib.nvc_sample_wrs(P, 1, 10, 32, P, N, P, -1.0, 0, 0, N, P, P, P, N, N, N, N) == _lib.NVC_ERR_SHAPE
    assert lib.nvc_sample_wrs(P, 1, 10, 32, None, N, P, 1e-3, 0, 0, N, P, P, P, N, N, N, N) == _lib.NVC_ERR_NULL
    assert lib.nvc_sample_wrs(P, 5, 10, 32, P, N, P, 1e-3, 0, 0, N, P, P, P, N, N, N, N) == _lib.NVC_ERR_DTYPE
    ws = lib.nvc_select_pixels_workspace_bytes(100)
    assert ws >= 800
    assert lib.nvc_select_pixels_workspace_bytes(0) == _lib.NVC_ERR_SHAPE
    assert lib.nvc_select_pixels(0, 0, N, 0, 10, P, P, ws, N) == _lib.NVC_ERR_SHAPE
    assert lib.nvc_select_pixels(0, 0, N, 1 << 31, 10, P, P, ws, N) == _lib.NVC_ERR_SHAPE
    assert lib.nvc_select_pixels(0, 0, N, 100, 10, None, P, ws, N) == _lib.NVC_ERR_NULL
    assert lib.nvc_select_pixels(0, 0, N, 100, 10, P, P, ws - 1, N) == _lib.NVC_ERR_WORKSPACE
    assert lib.nvc_select_pixels(0, 0, N, 100, 10, P, None, ws, N) == _lib.NVC_ERR_WORKSPACE
    assert lib.nvc_shadow_labels(P, N, 10, P, 0, P, 1, P, N) == _lib.NVC_ERR_SHAPE
    assert lib.nvc_shadow_labels(P, N, 10, P, 32, None, 4, P, N) == _lib.NVC_ERR_NULL
    assert lib.nvc_shadow_labels(P, N, 10, P, 128, P, 4097, P, N) == _lib.NVC_ERR_SHAPE
    assert lib.nvc_shadow_labels(P, N, -1, P, 32, P, 16, P, N) == _lib.NVC_ERR_SHAPE
    assert lib.nvc_adam(P, P, P, P, 10, 0, N, 1e-2, 1e-2, 0, 0.9, 0.99, 1e-8, 0, N) == _lib.NVC_ERR_SHAPE
    assert lib.nvc_adam(P, P, P, P, 10, 1, N, 1e-2, 1e-2, 0, 1.0, 0.99, 1e-8, 0, N) == _lib.NVC_ERR_SHAPE
    assert lib.nvc_adam(None, P, P, P, 10, 1, N, 1e-2, 1e-2, 0, 0.9, 0.99, 1e-8, 0, N) == _lib.NVC_ERR_NULL
    assert lib.nvc_adam(P, P, P, P, 10, 0, P, 1e-2, 1e-2, 0, 0.9, 1.5, 1e-8, 0, N) == _lib.NVC_ERR_SHAPE
    assert lib.nvc_adam(P, P, P, P, 10, 1, N, 5e-2, 1e-3, -1, 0.9, 0.99, 1e-8, 0, N) == _lib.NVC_ERR_SHAPE
    assert lib.nvc_adam(P, P, P, P, 10, 1, N, 5e-2, -1e-3, 200, 0.9, 0.99, 1e-8, 0, N) == _lib.NVC_ERR_SHAPE
    assert lib.nvc_adam(P, P, P, P, 10, 1, N, 5e-2, float("nan"), 200, 0.9, 0.99, 1e-8, 0, N) == _lib.NVC_ERR_SHAPE
    assert lib.nvc_counters_advance(None, N) == _lib.NVC_ERR_NULL
    # clustered cache
    sc = lib.nvc_sample_clustered
    assert lib.nvc_shadow_labels_clustered(P, N, 10, P, 100, P, P, 0, P, 16, 0, 0, N, P, N) == _lib.NVC_ERR_SHAPE
    assert lib.nvc_shadow_labels_clustered(P, N, 10, P, 100, P, P, 129, P, 16, 0, 0, N, P, N) == _lib.NVC_ERR_SHAPE
    assert lib.nvc_shadow_labels_clustered(P, N, 10, P, 100, None, P, 32, P, 16, 0, 0, N, P, N) == _lib.NVC_ERR_NULL
    assert lib.nvc_shadow_labels_clustered(P, N, 0, P, 100, P, P, 32, P, 16, 0, 0, N, P, N) == 0
    assert sc(P, 1, 10, 32, P, N, P, 100, P, P, 1e-3, 0, 0, 0, N, P, P, N, N, N, N) == _lib.NVC_ERR_SHAPE
    assert sc(P, 1, 10, 32, P, N, P, 100, P, P, 1e-3, 65, 0, 0, N, P, P, N, N, N, N) == _lib.NVC_ERR_SHAPE
    assert sc(P, 1, 10, 32, P, N, P, 100, P, P, -1.0, 8, 0, 0, N, P, P, N, N, N, N) == _lib.NVC_ERR_SHAPE
    assert sc(P, 7, 10, 32, P, N, P, 100, P, P, 1e-3, 8, 0, 0, N, P, P, N, N, N, N) == _lib.NVC_ERR_DTYPE
    assert sc(P, 1, 10, 32, P, N, P, 100, P, P, 1e-3, 8, 0, 0, N, None, P, N, N, N, N) == _lib.NVC_ERR_NULL
    assert lib.nvc_cluster_lights(P, 10, 11, 5, P, P) == _lib.NVC_ERR_SHAPE
    assert lib.nvc_cluster_lights(P, 10, 0, 5, P, P) == _lib.NVC_ERR_SHAPE
    assert lib.nvc_cluster_lights(None, 10, 4, 5, P, P) == _lib.NVC_ERR_NULL
    box = (ctypes.c_float * 6)(0, 0, 0, 1, 1, 1)
    bad = (ctypes.c_float * 6)(0, 2, 0, 1, 1, 1)
    assert lib.nvc_world_samples(0, 0, N, 10, box, 0.0, P, P, N) == _lib.NVC_ERR_SHAPE
    assert lib.nvc_world_samples(0, 0, N, 10, bad, 10.0, P, P, N) == _lib.NVC_ERR_SHAPE
    assert lib.nvc_world_samples(0, 0, N, 10, None, 10.0, P, P, N) == _lib.NVC_ERR_NULL
    assert lib.nvc_world_samples(0, 0, N, 10, box, 10.0, None, P, N) == _lib.NVC_ERR_NULL
    assert lib.nvc_world_samples(0, 0, N, 0, box, 10.0, None, None, N) == 0


def test_host_kmeans_equals_the_oracle():
    """nvc_cluster_lights (host C++) and the oracle's k-means reach the same partition."""
    import numpy as np

    from oracle import clustered
    from paper_2506_05930_amd import api
    from workloads import box_scene
    for seed, n, k in ((0, 300, 32), (1, 4096, 32), (2, 64, 64), (3, 1000, 7)):
        lights = box_scene(seed, 8, 8, 4, n, 4)["lights"]
        off, mem = api.nvc_cluster_lights(lights, k, 20)
        ro, rm = clustered.kmeans(lights, k, 20)
        assert np.array_equal(off, ro) and np.array_equal(mem, rm), (seed, n, k)
    bad = np.ones((5, 4), np.float32)
    bad[2, 1] = np.nan
    with pytest.raises(Exception):
        api.nvc_cluster_lights(bad, 2, 5)


def test_train_step_validation(lib):
    gg, mm = ctypes.byref(g()), ctypes.byref(m())
    P = ctypes.c_void_p(16)
    N = None
    ws = lib.nvc_train_workspace_bytes(gg, mm, 1 << 18)
    assert ws > 0
    # neither or both of labels / dvis
    assert lib.nvc_train_step(gg, mm, P, P, P, N, 64, N, N, 0, 0.0, P, P, N, P, ws, N) == _lib.NVC_ERR_NULL
    assert lib.nvc_train_step(gg, mm, P, P, P, N, 64, P, P, 0, 0.0, P, P, N, P, ws, N) == _lib.NVC_ERR_SHAPE
    assert lib.nvc_train_step(gg, mm, P, P, P, N, 64, P, N, 5, 0.0, P, P, N, P, ws, N) == _lib.NVC_ERR_SHAPE
    assert lib.nvc_train_step(gg, mm, P, P, P, N, 64, P, N, 0, -1.0, P, P, N, P, ws, N) == _lib.NVC_ERR_SHAPE
    assert lib.nvc_train_step(gg, mm, P, P, P, N, 1 << 18, P, N, 0, 0.0, P, P, N, P, ws - 1, N) == \
        _lib.NVC_ERR_WORKSPACE
    assert lib.nvc_train_step(gg, mm, P, P, P, N, 64, P, N, 0, 0.0, P, P, N, None, ws, N) == _lib.NVC_ERR_WORKSPACE
    # the 128-wide network trains; a shape with no kernel is refused
    g20 = ctypes.byref(g(log2_T=20))
    assert lib.nvc_train_workspace_bytes(g20, ctypes.byref(m(width=128, n_out=128)), 1024) > 0
    assert lib.nvc_train_workspace_bytes(g20, ctypes.byref(m(width=128, n_out=128, n_hidden=2)), 1024) == \
        _lib.NVC_ERR_UNSUPPORTED


def test_routed_scatter_is_limited_to_32_bit_record_numbers(lib):
    """The routed table scatter numbers its batch * n_levels * 4 records with 32-bit offsets; a batch that
    would reach 2^32 records trains through direct atomics instead, whose workspace holds no records."""
    gg, mm = ctypes.byref(g()), ctypes.byref(m())           # 16 levels: the limit is 2^26 samples
    routed = lib.nvc_train_workspace_bytes(gg, mm, (1 << 26) - 1)
    direct = lib.nvc_train_workspace_bytes(gg, mm, 1 << 26)
    assert routed > ((1 << 26) - 1) * 16 * 4 * 20           # 20-byte records of every corner x-pair
    assert 0 < direct < routed // 1000
    # a batch the entry point refuses outright
    P = ctypes.c_void_p(16)
    assert lib.nvc_train_step(gg, mm, P, P, P, None, 1 << 31, P, None, 0, 0.0, P, P, None, P, direct, None) == \
        _lib.NVC_ERR_SHAPE


def test_python_binding_rejects_cpu_tensors():
    import torch

    from paper_2506_05930_amd import api
    grid = api.make_grid(8, 2, 14, 16, 1.5)
    with pytest.raises(ValueError):
        api.nvc_encode(grid, torch.zeros(8, 1 << 14, 2), torch.zeros(4, 3), torch.zeros(4, 16))


def test_scene_pixel_orders_are_permutations_of_one_gbuffer():
    """The G-buffer orders (tiled Morton, row-major, shuffled) hold the same pixels: each is a permutation of
    the row-major image, `pixel_xy` says where every stored pixel sits, and the positions agree."""
    from workloads import box_scene
    sc = {o: box_scene(0, 48, 20, 8, 4, 8, order=o) for o in ("rows", "morton", "shuffled")}
    ref = sc["rows"]
    for o, s in sc.items():
        xy = s["pixel_xy"].astype(np.int64)
        idx = xy[:, 1] * 48 + xy[:, 0]
        assert np.array_equal(np.sort(idx), np.arange(48 * 20)), o
        assert np.array_equal(s["pos"], ref["pos"][idx]) and np.array_equal(s["nrm"], ref["nrm"][idx]), o
    assert not np.array_equal(sc["shuffled"]["pixel_xy"], sc["morton"]["pixel_xy"])


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU; --gpus N > 1 exits with a message (before touching any GPU)."""
    import json
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    out = json.loads(r.stdout.strip().splitlines()[-1])
    assert out["n_gpus"] == 2 and "one GPU" in out["error"]


def test_graph_entry_points_validate_before_calling_hip(lib):
    P = ctypes.c_void_p(16)
    ex = ctypes.c_void_p()
    assert lib.nvc_graph_begin(None) == _lib.NVC_ERR_NULL          # the legacy default stream cannot be captured
    assert lib.nvc_graph_end(None, ctypes.byref(ex)) == _lib.NVC_ERR_NULL
    assert lib.nvc_graph_end(P, None) == _lib.NVC_ERR_NULL
    assert lib.nvc_graph_launch(None, P) == _lib.NVC_ERR_NULL
    assert lib.nvc_graph_launch(P, None) == _lib.NVC_ERR_NULL
    assert lib.nvc_graph_destroy(None) == _lib.NVC_ERR_NULL


def test_capture_ledger_names_streams_not_joined_back():
    """The host-side guard of a graph recording: every stream that received library calls must have been
    forked from the capturing stream and joined back to it after its last call (HIP refuses to end a
    capture otherwise).  Streams are plain handles here; the binding notes each call's stream."""
    from paper_2506_05930_amd import api
    origin, side, other = 1001, 1002, 1003
    ok = api.CaptureLedger(origin)
    with api.recording(ok):
        api._stream(origin)
        ok.fork(side)
        api._stream(side)
        api._stream(origin)
        ok.join(side)
    ok.check()
    # work on the side stream after its join is not joined
    late = api.CaptureLedger(origin)
    late.fork(side)
    late.use(side)
    late.join(side)
    with api.recording(late):
        api._stream(side)
    with pytest.raises(RuntimeError, match=str(side)):
        late.check()
    # a stream that was never forked from the capture
    stray = api.CaptureLedger(origin)
    with api.recording(stray):
        api._stream(other)
    with pytest.raises(RuntimeError, match=str(other)):
        stray.check()
    # recordings do not nest, and the ledger is released afterwards
    with api.recording(api.CaptureLedger(origin)):
        with pytest.raises(RuntimeError):
            with api.recording(api.CaptureLedger(origin)):
                pass
    assert api._ledger is None


def test_noalloc_pixel_selection_validates_before_launching(lib):
    P = ctypes.c_void_p(16)
    big = _lib.NVC_SELECT_PIXELS_NOALLOC_MAX_PIX
    assert lib.nvc_select_pixels_noalloc(0, 0, None, big + 1, 10, P, None) == _lib.NVC_ERR_SHAPE
    assert lib.nvc_select_pixels_noalloc(0, 0, None, 0, 10, P, None) == _lib.NVC_ERR_SHAPE
    assert lib.nvc_select_pixels_noalloc(0, 0, None, 100, -1, P, None) == _lib.NVC_ERR_SHAPE
    assert lib.nvc_select_pixels_noalloc(0, 0, None, 100, 10, None, None) == _lib.NVC_ERR_NULL
    assert lib.nvc_select_pixels_noalloc(0, 0, None, 100, 0, None, None) == 0      # empty batch: no-op
    hdr = open(HEADER).read()
    assert f"#define NVC_SELECT_PIXELS_NOALLOC_MAX_PIX (1 << {big.bit_length() - 1})" in hdr


def test_fp64_forward_validates_before_launching(lib):
    P = ctypes.c_void_p(16)
    N = None
    gg, mm = ctypes.byref(g()), ctypes.byref(m())
    f = lib.nvc_forward_f64
    assert f(None, mm, P, P, P, 10, N, 0, P, N, N, N) == _lib.NVC_ERR_NULL
    assert f(gg, ctypes.byref(m(n_in=30)), P, P, P, 10, N, 0, P, N, N, N) == _lib.NVC_ERR_SHAPE
    assert f(gg, mm, P, P, P, -1, N, 0, P, N, N, N) == _lib.NVC_ERR_SHAPE
    assert f(gg, mm, P, P, P, (1 << 20) + 1, N, 0, P, N, N, N) == _lib.NVC_ERR_SHAPE
    assert f(gg, mm, P, P, P, 10, P, 7, P, N, P, N) == _lib.NVC_ERR_SHAPE          # unknown loss
    assert f(gg, mm, None, P, P, 10, N, 0, P, N, N, N) == _lib.NVC_ERR_NULL
    assert f(gg, mm, P, P, P, 10, P, 0, P, N, None, N) == _lib.NVC_ERR_NULL        # labels without loss_out
    assert f(gg, mm, None, None, None, 0, N, 0, N, N, N, N) == 0                   # n == 0 is a no-op


def test_train_step_shadow_validates_before_launching(lib):
    """The training pass with in-kernel shadow labels: one output per light, at most 32 lights and 512
    spheres, the plain pass's workspace, required pointers; an empty batch does nothing."""
    gg, mm = ctypes.byref(g()), ctypes.byref(m())            # 32 outputs
    P = ctypes.c_void_p(16)
    N = None
    ws = lib.nvc_train_workspace_bytes(gg, mm, 1 << 18)
    f = lib.nvc_train_step_shadow

    def call(grid=gg, mlp=mm, table=P, pos_scene=P, batch=1 << 18, lights=P, nl=32, spheres=P, ns=64, loss=0,
             scale=0.0, g_table=P, wsp=P, wsb=ws):
        return f(grid, mlp, table, P, P, pos_scene, N, batch, lights, nl, spheres, ns, loss, scale, g_table, P, N,
                 N, wsp, wsb, N)

    assert call(grid=None) == _lib.NVC_ERR_NULL
    assert call(nl=31) == _lib.NVC_ERR_SHAPE                                 # one output per light
    assert call(mlp=ctypes.byref(m(n_out=48)), nl=48) == _lib.NVC_ERR_SHAPE  # more than 32 lights
    assert call(ns=-1) == _lib.NVC_ERR_SHAPE
    assert call(ns=_lib.NVC_TRAIN_SHADOW_MAX_SPHERES + 1) == _lib.NVC_ERR_SHAPE
    assert call(loss=3) == _lib.NVC_ERR_SHAPE
    assert call(scale=-1.0) == _lib.NVC_ERR_SHAPE
    assert call(batch=-1) == _lib.NVC_ERR_SHAPE
    assert call(batch=1 << 31) == _lib.NVC_ERR_SHAPE
    assert call(table=None) == _lib.NVC_ERR_NULL
    assert call(pos_scene=None) == _lib.NVC_ERR_NULL
    assert call(lights=None) == _lib.NVC_ERR_NULL
    assert call(g_table=None) == _lib.NVC_ERR_NULL
    assert call(spheres=None) == _lib.NVC_ERR_NULL                           # spheres given but no pointer
    assert call(wsp=None) == _lib.NVC_ERR_WORKSPACE
    assert call(wsb=255) == _lib.NVC_ERR_WORKSPACE
    assert call(table=None, pos_scene=None, lights=None, spheres=None, g_table=None, wsp=None, batch=0) == 0
    hdr = open(HEADER).read()
    assert f"#define NVC_TRAIN_SHADOW_MAX_LIGHTS {_lib.NVC_TRAIN_SHADOW_MAX_LIGHTS}" in hdr
    assert f"#define NVC_TRAIN_SHADOW_MAX_SPHERES {_lib.NVC_TRAIN_SHADOW_MAX_SPHERES}" in hdr


def test_train_plan_validates_before_launching(lib):
    """The routing plan computed ahead: its size is the plan part of the training workspace (0 when the
    batch trains through direct atomics); plan and planned step reject bad arguments before launching."""
    gg, mm = ctypes.byref(g()), ctypes.byref(m())
    P = ctypes.c_void_p(16)
    N = None
    b = 1 << 18
    pb = lib.nvc_train_plan_bytes(gg, mm, b)
    ws = lib.nvc_train_workspace_bytes(gg, mm, b)
    assert 0 < pb < ws
    assert lib.nvc_train_plan_bytes(gg, mm, 0) == 0
    assert lib.nvc_train_plan_bytes(gg, mm, -1) == _lib.NVC_ERR_SHAPE
    assert lib.nvc_train_plan_bytes(gg, mm, 1 << 26) == 0                  # direct atomics: no plan
    assert lib.nvc_train_plan_bytes(None, mm, b) == _lib.NVC_ERR_NULL
    f = lib.nvc_train_plan
    assert f(gg, mm, None, N, b, P, pb, N) == _lib.NVC_ERR_NULL
    assert f(gg, mm, P, N, b, None, pb, N) == _lib.NVC_ERR_WORKSPACE
    assert f(gg, mm, P, N, b, P, pb - 1, N) == _lib.NVC_ERR_WORKSPACE
    assert f(gg, mm, P, N, -3, P, pb, N) == _lib.NVC_ERR_SHAPE
    assert f(None, None, None, N, 0, None, 0, N) == _lib.NVC_ERR_NULL
    assert f(gg, mm, None, N, 0, None, 0, N) == 0                          # empty batch: nothing to do
    assert f(gg, mm, None, N, 1 << 26, None, 0, N) == 0                    # nothing to plan
    s = lib.nvc_train_step_planned

    def call(labels=P, dvis=N, loss=0, scale=0.0, plan=P, plan_bytes=pb, wsp=P, wsb=ws, batch=b, table=P):
        return s(gg, mm, table, P, P, N, batch, labels, dvis, loss, scale, P, P, N, plan, plan_bytes, wsp, wsb, N)

    assert call(labels=N) == _lib.NVC_ERR_NULL                             # neither labels nor dvis
    assert call(dvis=P) == _lib.NVC_ERR_SHAPE                              # both
    assert call(loss=4) == _lib.NVC_ERR_SHAPE
    assert call(scale=-1.0) == _lib.NVC_ERR_SHAPE
    assert call(table=None) == _lib.NVC_ERR_NULL
    assert call(wsp=None) == _lib.NVC_ERR_WORKSPACE
    assert call(plan=None) == _lib.NVC_ERR_WORKSPACE
    assert call(plan_bytes=pb - 1) == _lib.NVC_ERR_WORKSPACE
    assert call(batch=0, table=None, plan=None, wsp=None) == 0
