"""Python binding of include/nvc.h on torch tensors: argument marshalling only.

Each function has the name of the C entry point it calls, checks that tensors
live on the GPU with the expected dtype, shape and contiguity, passes their
device pointers and the current HIP stream, and raises NvcError on a
negative status.  All computation happens in the HIP kernels of libnvc.so.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import NvcGrid, NvcMlp, NVC_F32, NVC_F16, NVC_BF16

_DT_CODE = {torch.float32: NVC_F32, torch.float16: NVC_F16, torch.bfloat16: NVC_BF16}
_DT_TORCH = {v: k for k, v in _DT_CODE.items()}
DTYPES = {"f32": NVC_F32, "f16": NVC_F16, "bf16": NVC_BF16}


def dtype_code(x) -> int:
    if isinstance(x, str):
        return DTYPES[x]
    if isinstance(x, torch.dtype):
        return _DT_CODE[x]
    return int(x)


def torch_dtype(code: int) -> torch.dtype:
    return _DT_TORCH[code]


def make_grid(n_levels, n_feat, log2_T, base_res, growth) -> NvcGrid:
    return NvcGrid(int(n_levels), int(n_feat), int(log2_T), int(base_res), float(growth))


def make_mlp(n_in, width, n_hidden, n_out, act="relu", leaky_slope=0.01, dtype="f16") -> NvcMlp:
    act_code = {"relu": _lib.NVC_ACT_RELU, "leaky": _lib.NVC_ACT_LEAKY}[act] if isinstance(act, str) else int(act)
    return NvcMlp(int(n_in), int(width), int(n_hidden), int(n_out), act_code, float(leaky_slope), dtype_code(dtype))


def _stream(stream) -> int:
    if stream is None:
        h = torch.cuda.current_stream().cuda_stream
    elif isinstance(stream, torch.cuda.Stream):
        h = stream.cuda_stream
    else:
        h = int(stream)
    if _ledger is not None:
        _ledger.use(h)
    return h


class CaptureLedger:
    """Which streams a recording has forked from the capturing stream, and whether each was joined back
    after its last library call.

    While a ledger is active (`recording(ledger)`), every entry point of this module notes the stream it
    enqueues on; `fork` / `join` (below) note the event edges between streams.  HIP ends a capture only when
    every stream that received captured work has been joined back to the capturing stream; `check` raises
    before that point instead, naming the streams that were not joined or never forked.
    """

    def __init__(self, origin: int):
        self.origin = int(origin)
        self.forked: set[int] = set()
        self.pending: set[int] = set()      # forked streams with library calls after their last join
        self.stray: set[int] = set()        # streams used without a fork from the capture

    def use(self, h: int) -> None:
        h = int(h)
        if h == self.origin:
            return
        if h in self.forked:
            self.pending.add(h)
        else:
            self.stray.add(h)

    def fork(self, h: int) -> None:
        self.forked.add(int(h))

    def join(self, h: int) -> None:
        self.pending.discard(int(h))

    def check(self) -> None:
        if self.pending or self.stray:
            raise RuntimeError("graph recording: streams with work not joined back to the capturing stream: "
                               f"{sorted(self.pending)}; streams used without a fork from it: {sorted(self.stray)}")


_ledger: CaptureLedger | None = None


class recording:
    """Context manager making `ledger` the active capture ledger."""

    def __init__(self, ledger: CaptureLedger):
        self.ledger = ledger

    def __enter__(self):
        global _ledger
        if _ledger is not None:
            raise RuntimeError("a graph recording is already active")
        _ledger = self.ledger
        return self.ledger

    def __exit__(self, *exc):
        global _ledger
        _ledger = None
        return False


def _handle(stream) -> int:
    return stream.cuda_stream if isinstance(stream, torch.cuda.Stream) else int(stream)


def fork(side: torch.cuda.Stream, main: torch.cuda.Stream) -> None:
    """side waits for the work enqueued on main so far (an event edge; also inside a recording)."""
    side.wait_stream(main)
    if _ledger is not None and _handle(main) in (_ledger.origin, *_ledger.forked):
        _ledger.fork(_handle(side))


def join(main: torch.cuda.Stream, side: torch.cuda.Stream) -> None:
    """main waits for the work enqueued on side so far."""
    main.wait_stream(side)
    if _ledger is not None:
        _ledger.join(_handle(side))


def _ptr(t, name, dtype=None, shape=None, optional=False):
    if t is None:
        if optional:
            return None
        raise ValueError(f"{name} is required")
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA (HIP) tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype not in (dtype if isinstance(dtype, tuple) else (dtype,)):
        raise ValueError(f"{name} has dtype {t.dtype}, expected {dtype}")
    if shape is not None:
        if t.dim() != len(shape) or any(s is not None and a != s for a, s in zip(t.shape, shape)):
            raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {shape}")
    return t.data_ptr()


def nvc_version() -> int:
    return _lib.load().nvc_version()


def nvc_grid_levels(grid: NvcGrid):
    L = _lib.load()
    res = (ctypes.c_int32 * grid.n_levels)()
    dense = (ctypes.c_int32 * grid.n_levels)()
    _lib.check("nvc_grid_levels", L.nvc_grid_levels(ctypes.byref(grid), res, dense))
    return list(res), [bool(d) for d in dense]


def nvc_mlp_param_count(mlp: NvcMlp) -> int:
    return _lib.check("nvc_mlp_param_count", _lib.load().nvc_mlp_param_count(ctypes.byref(mlp)))


def nvc_mlp_packed_bytes(mlp: NvcMlp) -> int:
    return _lib.check("nvc_mlp_packed_bytes", _lib.load().nvc_mlp_packed_bytes(ctypes.byref(mlp)))


def nvc_train_workspace_bytes(grid: NvcGrid, mlp: NvcMlp, batch: int) -> int:
    return _lib.check("nvc_train_workspace_bytes",
                      _lib.load().nvc_train_workspace_bytes(ctypes.byref(grid), ctypes.byref(mlp), int(batch)))


def nvc_pack_mlp(mlp: NvcMlp, w: torch.Tensor, packed: torch.Tensor, stream=None) -> None:
    n = nvc_mlp_param_count(mlp)
    pw = _ptr(w, "w", torch.float32, (n,))
    if packed.numel() * packed.element_size() < nvc_mlp_packed_bytes(mlp):
        raise ValueError("packed buffer too small")
    pp = _ptr(packed, "packed")
    _lib.check("nvc_pack_mlp", _lib.load().nvc_pack_mlp(ctypes.byref(mlp), pw, pp, _stream(stream)))


def nvc_encode(grid: NvcGrid, table: torch.Tensor, pos: torch.Tensor, enc: torch.Tensor, stream=None) -> None:
    n = pos.shape[0]
    L, F = grid.n_levels, grid.n_feat
    pt = _ptr(table, "table", torch.float32, (L, 1 << grid.log2_T, F))
    pp = _ptr(pos, "pos", torch.float32, (n, 3))
    pe = _ptr(enc, "enc", (torch.float32, torch.float16, torch.bfloat16), (n, L * F))
    _lib.check("nvc_encode", _lib.load().nvc_encode(ctypes.byref(grid), pt, pp, n, pe, _DT_CODE[enc.dtype],
                                                    _stream(stream)))


def nvc_infer(grid: NvcGrid, mlp: NvcMlp, table: torch.Tensor, packed: torch.Tensor, pos: torch.Tensor,
              vis: torch.Tensor, stream=None) -> None:
    n = pos.shape[0]
    pt = _ptr(table, "table", torch.float32, (grid.n_levels, 1 << grid.log2_T, grid.n_feat))
    pk = _ptr(packed, "packed")
    pp = _ptr(pos, "pos", torch.float32, (n, 3))
    pv = _ptr(vis, "vis", (torch.float32, torch.float16, torch.bfloat16), (n, mlp.n_out))
    _lib.check("nvc_infer", _lib.load().nvc_infer(ctypes.byref(grid), ctypes.byref(mlp), pt, pk, pp, n, pv,
                                                  _DT_CODE[vis.dtype], _stream(stream)))


def _counters(ctr):
    """Device pointer of an nvc_counters block: an int32 tensor of 2 elements (frame, step), or None."""
    return _ptr(ctr, "ctr", torch.int32, (2,), optional=True)


def new_counters(frame: int = 0, step: int = 1, device="cuda") -> torch.Tensor:
    """Device counters {uint32 frame; int32 step} for nvc_sample_wrs / nvc_select_pixels / nvc_adam."""
    return torch.tensor([frame, step], dtype=torch.int32, device=device)


def nvc_counters_advance(ctr: torch.Tensor, stream=None) -> None:
    _lib.check("nvc_counters_advance", _lib.load().nvc_counters_advance(_counters(ctr), _stream(stream)))


def nvc_graph_begin(stream) -> None:
    """Start recording `stream` (a created stream, not the default one) into a HIP graph."""
    _lib.check("nvc_graph_begin", _lib.load().nvc_graph_begin(_stream(stream)))


def nvc_graph_end(stream) -> int:
    """End the recording of `stream`; returns the executable graph's handle (owned by the caller)."""
    ex = ctypes.c_void_p()
    _lib.check("nvc_graph_end", _lib.load().nvc_graph_end(_stream(stream), ctypes.byref(ex)))
    return int(ex.value)


def nvc_graph_launch(exec_handle: int, stream=None) -> None:
    _lib.check("nvc_graph_launch", _lib.load().nvc_graph_launch(ctypes.c_void_p(exec_handle), _stream(stream)))


def nvc_graph_destroy(exec_handle: int) -> None:
    _lib.check("nvc_graph_destroy", _lib.load().nvc_graph_destroy(ctypes.c_void_p(exec_handle)))


def nvc_mlp_forward(mlp: NvcMlp, packed: torch.Tensor, enc: torch.Tensor, vis: torch.Tensor, stream=None) -> None:
    n = enc.shape[0]
    pk = _ptr(packed, "packed")
    pe = _ptr(enc, "enc", (torch.float32, torch.float16, torch.bfloat16), (n, mlp.n_in))
    pv = _ptr(vis, "vis", (torch.float32, torch.float16, torch.bfloat16), (n, mlp.n_out))
    _lib.check("nvc_mlp_forward", _lib.load().nvc_mlp_forward(ctypes.byref(mlp), pk, pe, _DT_CODE[enc.dtype], n, pv,
                                                              _DT_CODE[vis.dtype], _stream(stream)))


def nvc_sample_wrs(vis: torch.Tensor, pos: torch.Tensor, nrm, lights: torch.Tensor, vis_floor: float, seed: int,
                   frame: int, idx: torch.Tensor, pmf: torch.Tensor, wsum: torch.Tensor, di=None,
                   stream=None, ctr=None, mask=None, res=None) -> None:
    """mask: uint8 [n] (0 = skip the pixel) or None; res: a 4-byte tensor [n][4] receiving nvc_reservoir
    records (int32 y, int32 M, float32 w_sum, float32 W) or None."""
    n, m = vis.shape
    pv = _ptr(vis, "vis", (torch.float32, torch.float16, torch.bfloat16))
    pp = _ptr(pos, "pos", torch.float32, (n, 3))
    pn = _ptr(nrm, "nrm", torch.float32, (n, 3), optional=True)
    pl = _ptr(lights, "lights", torch.float32, (m, 4))
    pi = _ptr(idx, "idx", torch.int32, (n,))
    pm = _ptr(pmf, "pmf", torch.float32, (n,))
    pw = _ptr(wsum, "wsum", torch.float32, (n,))
    pd = _ptr(di, "di", torch.float32, (n,), optional=True)
    pk = _ptr(mask, "mask", torch.uint8, (n,), optional=True)
    pr = _ptr(res, "res", (torch.int32, torch.float32), (n, 4), optional=True)
    _lib.check("nvc_sample_wrs", _lib.load().nvc_sample_wrs(pv, _DT_CODE[vis.dtype], n, m, pp, pn, pl,
                                                            float(vis_floor), int(seed) & (2 ** 64 - 1),
                                                            int(frame) & 0xFFFFFFFF, _counters(ctr), pi, pm, pw,
                                                            pd, pk, pr, _stream(stream)))


def nvc_select_pixels_workspace_bytes(n_pix: int) -> int:
    return _lib.check("nvc_select_pixels_workspace_bytes", _lib.load().nvc_select_pixels_workspace_bytes(int(n_pix)))


def nvc_select_pixels(seed: int, frame: int, n_pix: int, pix: torch.Tensor, workspace: torch.Tensor,
                      stream=None, ctr=None) -> None:
    pp = _ptr(pix, "pix", torch.int32)
    pw = _ptr(workspace, "workspace")
    _lib.check("nvc_select_pixels", _lib.load().nvc_select_pixels(int(seed) & (2 ** 64 - 1),
                                                                  int(frame) & 0xFFFFFFFF, _counters(ctr), int(n_pix),
                                                                  pix.numel(), pp, pw,
                                                                  workspace.numel() * workspace.element_size(),
                                                                  _stream(stream)))


def nvc_select_pixels_noalloc(seed: int, frame: int, n_pix: int, pix: torch.Tensor, stream=None, ctr=None) -> None:
    """nvc_select_pixels with the library's static workspace (no allocation; n_pix <= 2^23)."""
    pp = _ptr(pix, "pix", torch.int32)
    _lib.check("nvc_select_pixels_noalloc", _lib.load().nvc_select_pixels_noalloc(
        int(seed) & (2 ** 64 - 1), int(frame) & 0xFFFFFFFF, _counters(ctr), int(n_pix), pix.numel(), pp,
        _stream(stream)))


def nvc_shadow_labels(pos: torch.Tensor, pix, lights: torch.Tensor, spheres: torch.Tensor, labels: torch.Tensor,
                      stream=None) -> None:
    n, m = labels.shape
    pp = _ptr(pos, "pos", torch.float32, (None, 3))
    px = _ptr(pix, "pix", torch.int32, (n,), optional=True)
    if pix is None and pos.shape[0] < n:
        raise ValueError("pos has fewer rows than labels")
    pl = _ptr(lights, "lights", torch.float32, (m, 4))
    ps = _ptr(spheres, "spheres", torch.float32, (None, 4)) if spheres.numel() else None
    pb = _ptr(labels, "labels", torch.uint8)
    _lib.check("nvc_shadow_labels", _lib.load().nvc_shadow_labels(pp, px, n, pl, m, ps, spheres.shape[0], pb,
                                                                  _stream(stream)))


def nvc_world_samples(seed: int, frame: int, box, extent: float, pos_scene: torch.Tensor, pos_unit: torch.Tensor,
                      stream=None, ctr=None) -> None:
    """World-space training points uniform in box = (lo xyz, hi xyz), scene and unit-cube positions."""
    n = pos_scene.shape[0]
    ps = _ptr(pos_scene, "pos_scene", torch.float32, (n, 3))
    pu = _ptr(pos_unit, "pos_unit", torch.float32, (n, 3))
    b = (ctypes.c_float * 6)(*[float(x) for x in box])
    _lib.check("nvc_world_samples", _lib.load().nvc_world_samples(int(seed) & (2 ** 64 - 1), int(frame) & 0xFFFFFFFF,
                                                                  _counters(ctr), n, b, float(extent), ps, pu,
                                                                  _stream(stream)))


def nvc_cluster_lights(lights, k: int, iters: int = 20):
    """Host k-means of the lights (array-like [n][4] on the host) -> (offsets int32 [k+1], members int32 [n])."""
    arr = np.ascontiguousarray(np.asarray(lights.cpu() if isinstance(lights, torch.Tensor) else lights,
                                          dtype=np.float32))
    if arr.ndim != 2 or arr.shape[1] != 4:
        raise ValueError("lights must be [n][4]")
    n = arr.shape[0]
    offsets = np.zeros(k + 1, np.int32)
    members = np.zeros(n, np.int32)
    _lib.check("nvc_cluster_lights", _lib.load().nvc_cluster_lights(arr.ctypes.data, n, int(k), int(iters),
                                                                    offsets.ctypes.data, members.ctypes.data))
    return offsets, members


def nvc_shadow_labels_clustered(pos: torch.Tensor, pix, lights: torch.Tensor, offsets: torch.Tensor,
                                members: torch.Tensor, spheres: torch.Tensor, seed: int, frame: int,
                                labels: torch.Tensor, stream=None, ctr=None) -> None:
    n, k = labels.shape
    pp = _ptr(pos, "pos", torch.float32, (None, 3))
    px = _ptr(pix, "pix", torch.int32, (n,), optional=True)
    if pix is None and pos.shape[0] < n:
        raise ValueError("pos has fewer rows than labels")
    pl = _ptr(lights, "lights", torch.float32, (None, 4))
    po = _ptr(offsets, "offsets", torch.int32, (k + 1,))
    pm = _ptr(members, "members", torch.int32, (lights.shape[0],))
    ps = _ptr(spheres, "spheres", torch.float32, (None, 4)) if spheres.numel() else None
    pb = _ptr(labels, "labels", torch.uint8)
    _lib.check("nvc_shadow_labels_clustered", _lib.load().nvc_shadow_labels_clustered(
        pp, px, n, pl, lights.shape[0], po, pm, k, ps, spheres.shape[0], int(seed) & (2 ** 64 - 1),
        int(frame) & 0xFFFFFFFF, _counters(ctr), pb, _stream(stream)))


def nvc_sample_clustered(vis: torch.Tensor, pos: torch.Tensor, nrm, lights: torch.Tensor, offsets: torch.Tensor,
                         members: torch.Tensor, vis_floor: float, n_cand: int, seed: int, frame: int,
                         idx: torch.Tensor, weight: torch.Tensor, cluster=None, stream=None, ctr=None, mask=None,
                         res=None) -> None:
    n, k = vis.shape
    pv = _ptr(vis, "vis", (torch.float32, torch.float16, torch.bfloat16))
    pp = _ptr(pos, "pos", torch.float32, (n, 3))
    pn = _ptr(nrm, "nrm", torch.float32, (n, 3), optional=True)
    pl = _ptr(lights, "lights", torch.float32, (None, 4))
    po = _ptr(offsets, "offsets", torch.int32, (k + 1,))
    pm = _ptr(members, "members", torch.int32, (lights.shape[0],))
    pi = _ptr(idx, "idx", torch.int32, (n,))
    pw = _ptr(weight, "weight", torch.float32, (n,))
    pc = _ptr(cluster, "cluster", torch.int32, (n,), optional=True)
    pk = _ptr(mask, "mask", torch.uint8, (n,), optional=True)
    pr = _ptr(res, "res", (torch.int32, torch.float32), (n, 4), optional=True)
    _lib.check("nvc_sample_clustered", _lib.load().nvc_sample_clustered(
        pv, _DT_CODE[vis.dtype], n, k, pp, pn, pl, lights.shape[0], po, pm, float(vis_floor), int(n_cand),
        int(seed) & (2 ** 64 - 1), int(frame) & 0xFFFFFFFF, _counters(ctr), pi, pw, pc, pk, pr, _stream(stream)))


def nvc_train_step(grid: NvcGrid, mlp: NvcMlp, table: torch.Tensor, packed: torch.Tensor, pos: torch.Tensor, pix,
                   batch: int, labels, dvis, loss: int, grad_scale: float, g_table: torch.Tensor,
                   g_w: torch.Tensor, loss_out, workspace: torch.Tensor, stream=None) -> None:
    tshape = (grid.n_levels, 1 << grid.log2_T, grid.n_feat)
    pt = _ptr(table, "table", torch.float32, tshape)
    pk = _ptr(packed, "packed")
    pp = _ptr(pos, "pos", torch.float32, (None, 3))
    px = _ptr(pix, "pix", torch.int32, (batch,), optional=True)
    if pix is None and pos.shape[0] < batch:
        raise ValueError("pos has fewer rows than the batch")
    pl = _ptr(labels, "labels", torch.uint8, (batch, mlp.n_out), optional=True)
    pd = _ptr(dvis, "dvis", torch.float32, (batch, mlp.n_out), optional=True)
    pg = _ptr(g_table, "g_table", torch.float32, tshape)
    pw = _ptr(g_w, "g_w", torch.float32, (nvc_mlp_param_count(mlp),))
    po = _ptr(loss_out, "loss_out", torch.float32, (1,), optional=True)
    pws = _ptr(workspace, "workspace")
    wsb = workspace.numel() * workspace.element_size()
    _lib.check("nvc_train_step", _lib.load().nvc_train_step(ctypes.byref(grid), ctypes.byref(mlp), pt, pk, pp, px,
                                                            int(batch), pl, pd, int(loss), float(grad_scale), pg,
                                                            pw, po, pws, wsb, _stream(stream)))


def nvc_train_plan_bytes(grid: NvcGrid, mlp: NvcMlp, batch: int) -> int:
    return _lib.check("nvc_train_plan_bytes", _lib.load().nvc_train_plan_bytes(ctypes.byref(grid), ctypes.byref(mlp),
                                                                               int(batch)))


def nvc_train_plan(grid: NvcGrid, mlp: NvcMlp, pos: torch.Tensor, pix, batch: int, plan: torch.Tensor,
                   stream=None) -> None:
    """The routing plan of the table scatter for these samples (see nvc_train_step_planned)."""
    pp = _ptr(pos, "pos", torch.float32, (None, 3))
    px = _ptr(pix, "pix", torch.int32, (batch,), optional=True)
    if pix is None and pos.shape[0] < batch:
        raise ValueError("pos has fewer rows than the batch")
    pl = _ptr(plan, "plan")
    _lib.check("nvc_train_plan", _lib.load().nvc_train_plan(ctypes.byref(grid), ctypes.byref(mlp), pp, px, int(batch),
                                                            pl, plan.numel() * plan.element_size(), _stream(stream)))


def nvc_train_step_planned(grid: NvcGrid, mlp: NvcMlp, table: torch.Tensor, packed: torch.Tensor,
                           pos: torch.Tensor, pix, batch: int, labels, dvis, loss: int, grad_scale: float,
                           g_table: torch.Tensor, g_w: torch.Tensor, loss_out, plan: torch.Tensor,
                           workspace: torch.Tensor, stream=None) -> None:
    tshape = (grid.n_levels, 1 << grid.log2_T, grid.n_feat)
    pt = _ptr(table, "table", torch.float32, tshape)
    pk = _ptr(packed, "packed")
    pp = _ptr(pos, "pos", torch.float32, (None, 3))
    px = _ptr(pix, "pix", torch.int32, (batch,), optional=True)
    if pix is None and pos.shape[0] < batch:
        raise ValueError("pos has fewer rows than the batch")
    pl = _ptr(labels, "labels", torch.uint8, (batch, mlp.n_out), optional=True)
    pd = _ptr(dvis, "dvis", torch.float32, (batch, mlp.n_out), optional=True)
    pg = _ptr(g_table, "g_table", torch.float32, tshape)
    pw = _ptr(g_w, "g_w", torch.float32, (nvc_mlp_param_count(mlp),))
    po = _ptr(loss_out, "loss_out", torch.float32, (1,), optional=True)
    ppl = _ptr(plan, "plan")
    pws = _ptr(workspace, "workspace")
    _lib.check("nvc_train_step_planned",
               _lib.load().nvc_train_step_planned(ctypes.byref(grid), ctypes.byref(mlp), pt, pk, pp, px, int(batch), pl,
                                                  pd, int(loss), float(grad_scale), pg, pw, po, ppl,
                                                  plan.numel() * plan.element_size(), pws,
                                                  workspace.numel() * workspace.element_size(), _stream(stream)))


def nvc_train_step_shadow(grid: NvcGrid, mlp: NvcMlp, table: torch.Tensor, packed: torch.Tensor, pos: torch.Tensor,
                          pos_scene: torch.Tensor, pix, batch: int, lights: torch.Tensor, spheres: torch.Tensor,
                          loss: int, grad_scale: float, g_table: torch.Tensor, g_w: torch.Tensor, loss_out,
                          labels_out, workspace: torch.Tensor, stream=None) -> None:
    """Labelled training gradients with the shadow labels computed inside the training kernel
    (pos_scene: the scene-space positions, indexed like pos; labels_out [batch][m] uint8 or None)."""
    tshape = (grid.n_levels, 1 << grid.log2_T, grid.n_feat)
    pt = _ptr(table, "table", torch.float32, tshape)
    pk = _ptr(packed, "packed")
    pp = _ptr(pos, "pos", torch.float32, (None, 3))
    ps = _ptr(pos_scene, "pos_scene", torch.float32, (pos.shape[0], 3))
    px = _ptr(pix, "pix", torch.int32, (batch,), optional=True)
    if pix is None and pos.shape[0] < batch:
        raise ValueError("pos has fewer rows than the batch")
    m = lights.shape[0]
    pl = _ptr(lights, "lights", torch.float32, (m, 4))
    n_s = spheres.shape[0]
    psp = _ptr(spheres, "spheres", torch.float32, (n_s, 4))
    pg = _ptr(g_table, "g_table", torch.float32, tshape)
    pw = _ptr(g_w, "g_w", torch.float32, (nvc_mlp_param_count(mlp),))
    po = _ptr(loss_out, "loss_out", torch.float32, (1,), optional=True)
    plo = _ptr(labels_out, "labels_out", torch.uint8, (batch, m), optional=True)
    pws = _ptr(workspace, "workspace")
    wsb = workspace.numel() * workspace.element_size()
    _lib.check("nvc_train_step_shadow",
               _lib.load().nvc_train_step_shadow(ctypes.byref(grid), ctypes.byref(mlp), pt, pk, pp, ps, px,
                                                 int(batch), pl, int(m), psp, int(n_s), int(loss),
                                                 float(grad_scale), pg, pw, po, plo, pws, wsb, _stream(stream)))


def nvc_adam(p: torch.Tensor, g: torch.Tensor, m: torch.Tensor, v: torch.Tensor, step: int, lr: float,
             beta1: float, beta2: float, eps: float, zero_grad: bool = False, stream=None, ctr=None,
             lr_end: float | None = None, lr_decay_steps: int = 0) -> None:
    """lr_end / lr_decay_steps: the rate falls linearly from lr to lr_end over lr_decay_steps steps (0: constant)."""
    n = p.numel()
    ptrs = [_ptr(t, name, torch.float32) for t, name in ((p, "p"), (g, "g"), (m, "m"), (v, "v"))]
    if any(t.numel() != n for t in (g, m, v)):
        raise ValueError("p, g, m, v must have the same number of elements")
    _lib.check("nvc_adam", _lib.load().nvc_adam(*ptrs, n, int(step), _counters(ctr), float(lr),
                                                float(lr if lr_end is None else lr_end), int(lr_decay_steps),
                                                float(beta1), float(beta2), float(eps), int(bool(zero_grad)),
                                                _stream(stream)))


def nvc_forward_f64(grid: NvcGrid, mlp: NvcMlp, table: torch.Tensor, w: torch.Tensor, pos: torch.Tensor,
                    labels=None, loss: int = 0, z=None, masks=None, loss_out=None, stream=None) -> None:
    """FP64 forward pass (gradient checks): logits z [n][n_out], branch masks [n][n_hidden][ceil(width/8)],
    per-point losses and their mean in loss_out [n + 1] (with labels)."""
    n = pos.shape[0]
    pt = _ptr(table, "table", torch.float64, (grid.n_levels, 1 << grid.log2_T, grid.n_feat))
    pw = _ptr(w, "w", torch.float64, (nvc_mlp_param_count(mlp),))
    pp = _ptr(pos, "pos", torch.float32, (n, 3))
    pl = _ptr(labels, "labels", torch.uint8, (n, mlp.n_out), optional=True)
    pz = _ptr(z, "z", torch.float64, (n, mlp.n_out), optional=True)
    pm = _ptr(masks, "masks", torch.uint8, (n, mlp.n_hidden, (mlp.width + 7) // 8), optional=True)
    po = _ptr(loss_out, "loss_out", torch.float64, (n + 1,), optional=labels is None)
    _lib.check("nvc_forward_f64", _lib.load().nvc_forward_f64(ctypes.byref(grid), ctypes.byref(mlp), pt, pw, pp, int(n),
                                                              pl, int(loss), pz, pm, po, _stream(stream)))
