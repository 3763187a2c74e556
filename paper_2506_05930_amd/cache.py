"""The neural visibility cache as a stateful object, and its autograd wrapper.

`NVCache` owns the device tensors of one cache (hash table, FP32 master
weights, packed low-precision weights, Adam moments, gradient buffers,
training workspace) and strings the C-ABI calls together:

  infer    encoding + MLP -> visibility per light        (Sec. 3.1 steps 1-2)
  sample   WRS light pick + neural DI                    (Sec. 3.1 step 3, Sec. 3.2)
  train    pixel pick, shadow labels, gradients, Adam    (Sec. 3.4)
  frame    one frame: sample on every pixel, then train  (Sec. 4, passes 2-4)

torch is used for device memory and the stream only; every step runs in
libnvc.so.  `NVCFunction` exposes inference to torch autograd with the
library's own backward (the training kernel in upstream-gradient mode).
`FrameGraph` records one whole frame into a HIP graph once and replays it;
the frame number and the Adam step then come from device counters.
"""
from __future__ import annotations

import numpy as np
import torch

from . import api
from ._lib import NVC_LOSS_BCE, NVC_LOSS_L2


class NVCache:
    def __init__(self, grid_cfg, mlp_cfg, table, weights, device="cuda", seed: int = 2, lr: float = 1e-2,
                 beta1: float = 0.9, beta2: float = 0.99, eps: float = 1e-8, loss: str = "bce",
                 vis_floor: float = 1e-3, max_batch: int = 0, lr_end: float | None = None, lr_decay_steps: int = 0,
                 fused_labels: bool = False):
        self.grid = api.make_grid(grid_cfg.n_levels, grid_cfg.n_feat, grid_cfg.log2_T, grid_cfg.base_res,
                                  grid_cfg.growth)
        self.mlp = api.make_mlp(mlp_cfg.n_in, mlp_cfg.width, mlp_cfg.n_hidden, mlp_cfg.n_out, mlp_cfg.act,
                                mlp_cfg.leaky_slope, mlp_cfg.dtype)
        self.device = torch.device(device)
        self.vis_dtype = api.torch_dtype(self.mlp.dtype)
        self.seed = int(seed)
        self.lr, self.beta1, self.beta2, self.eps = lr, beta1, beta2, eps
        self.lr_end, self.lr_decay_steps = lr_end, lr_decay_steps     # linear decay of Sec. 3.4 (0: constant)
        self.loss = {"bce": NVC_LOSS_BCE, "l2": NVC_LOSS_L2}[loss]
        self.vis_floor = vis_floor
        # training pixels labelled inside the training kernel (nvc_train_step_shadow) instead of by the
        # separate label kernel; same labels and gradients
        self.fused_labels = bool(fused_labels)
        self.table = torch.as_tensor(np.ascontiguousarray(table), dtype=torch.float32).to(self.device)
        flat = np.concatenate([np.asarray(w, np.float32).reshape(-1) for w in weights]) \
            if isinstance(weights, (list, tuple)) else np.asarray(weights, np.float32)
        self.w = torch.as_tensor(flat, dtype=torch.float32).to(self.device).contiguous()
        if self.w.numel() != api.nvc_mlp_param_count(self.mlp):
            raise ValueError("weight count does not match the network shape")
        self.packed = torch.empty(api.nvc_mlp_packed_bytes(self.mlp), dtype=torch.uint8, device=self.device)
        self.m_table = torch.zeros_like(self.table)
        self.v_table = torch.zeros_like(self.table)
        self.g_table = torch.zeros_like(self.table)
        self.m_w = torch.zeros_like(self.w)
        self.v_w = torch.zeros_like(self.w)
        self.g_w = torch.zeros_like(self.w)
        self.loss_buf = torch.zeros(1, dtype=torch.float32, device=self.device)
        self.step = 0
        self.workspace = None
        self._ws_batch = 0
        if max_batch:
            self._ensure_workspace(max_batch)
        self.pack()

    # ------------------------------------------------------------ plumbing
    def _ensure_workspace(self, batch: int):
        need = api.nvc_train_workspace_bytes(self.grid, self.mlp, batch)
        if self.workspace is None or self.workspace.numel() < need:
            self.workspace = torch.empty(max(need, 256), dtype=torch.uint8, device=self.device)
        self._ws_batch = max(self._ws_batch, batch)

    def pixel_workspace(self, n_pix: int) -> torch.Tensor:
        need = api.nvc_select_pixels_workspace_bytes(n_pix)
        if getattr(self, "_pix_ws", None) is None or self._pix_ws.numel() < need:
            self._pix_ws = torch.empty(need, dtype=torch.uint8, device=self.device)
        return self._pix_ws

    def pack(self, stream=None):
        api.nvc_pack_mlp(self.mlp, self.w, self.packed, stream)

    def set_clusters(self, offsets, members, n_cand: int = 8):
        """Clustered cache (Sec. 3.6): output j is the visibility of cluster j of the lights (CSR offsets
        [k+1], members [n_lights], e.g. from api.nvc_cluster_lights).  sample() then takes the two-step pick
        with n_cand RIS candidates and the training labels shoot one ray per cluster."""
        if len(offsets) != self.mlp.n_out + 1:
            raise ValueError("one cluster per network output expected")
        self.cl_offsets = torch.as_tensor(np.asarray(offsets, np.int32)).to(self.device)
        self.cl_members = torch.as_tensor(np.asarray(members, np.int32)).to(self.device)
        self.n_cand = int(n_cand)

    def set_world_samples(self, n_world: int, box, extent: float):
        """Add n_world world-space training points per step, uniform in box = (lo xyz, hi xyz) of the scene
        (Sec. 3.4: the paper trains on 4096 world-space and 4096 screen-space samples); extent maps scene
        positions to the unit cube (x / extent).  The two halves' gradients are added; with equal halves
        that is twice the mean over the whole batch, a factor Adam does not see (up to eps)."""
        self.world = (int(n_world), tuple(float(x) for x in box), float(extent))

    @property
    def clustered(self) -> bool:
        return getattr(self, "cl_offsets", None) is not None

    # ------------------------------------------------------------ inference and sampling
    def infer(self, pos_unit: torch.Tensor, vis: torch.Tensor | None = None, dtype=None, stream=None) -> torch.Tensor:
        if vis is None:
            vis = torch.empty((pos_unit.shape[0], self.mlp.n_out), dtype=dtype or self.vis_dtype, device=self.device)
        api.nvc_infer(self.grid, self.mlp, self.table, self.packed, pos_unit, vis, stream)
        return vis

    def encode(self, pos_unit: torch.Tensor, dtype=torch.float32, stream=None) -> torch.Tensor:
        enc = torch.empty((pos_unit.shape[0], self.grid.n_levels * self.grid.n_feat), dtype=dtype,
                          device=self.device)
        api.nvc_encode(self.grid, self.table, pos_unit, enc, stream)
        return enc

    def sample(self, vis, pos, nrm, lights, frame: int, out: dict | None = None, with_di: bool = True,
               stream=None, ctr=None) -> dict:
        n = vis.shape[0]
        if self.clustered:
            if out is None:
                out = {"idx": torch.empty(n, dtype=torch.int32, device=self.device),
                       "weight": torch.empty(n, dtype=torch.float32, device=self.device),
                       "cluster": torch.empty(n, dtype=torch.int32, device=self.device)}
            api.nvc_sample_clustered(vis, pos, nrm, lights, self.cl_offsets, self.cl_members, self.vis_floor,
                                     self.n_cand, self.seed, frame, out["idx"], out["weight"], out["cluster"], stream,
                                     ctr=ctr)
            return out
        if out is None:
            out = {"idx": torch.empty(n, dtype=torch.int32, device=self.device),
                   "pmf": torch.empty(n, dtype=torch.float32, device=self.device),
                   "wsum": torch.empty(n, dtype=torch.float32, device=self.device),
                   "di": torch.empty(n, dtype=torch.float32, device=self.device) if with_di else None}
        api.nvc_sample_wrs(vis, pos, nrm, lights, self.vis_floor, self.seed, frame, out["idx"], out["pmf"],
                           out["wsum"], out.get("di"), stream, ctr=ctr)
        return out

    # ------------------------------------------------------------ training
    def gradients(self, pos_unit, labels=None, dvis=None, pix=None, batch: int | None = None,
                  grad_scale: float = 0.0, stream=None, plan=None):
        """Accumulate the gradients of one batch into g_table / g_w (and the loss into loss_buf).  plan: the
        routing plan of these samples from plan() (computed ahead), else the pass computes its own."""
        if batch is None:
            batch = pix.shape[0] if pix is not None else pos_unit.shape[0]
        self._ensure_workspace(batch)
        loss_out = self.loss_buf if labels is not None else None
        if plan is not None:
            api.nvc_train_step_planned(self.grid, self.mlp, self.table, self.packed, pos_unit, pix, batch, labels,
                                       dvis, self.loss, grad_scale, self.g_table, self.g_w, loss_out, plan,
                                       self.workspace, stream)
            return
        api.nvc_train_step(self.grid, self.mlp, self.table, self.packed, pos_unit, pix, batch, labels, dvis,
                           self.loss, grad_scale, self.g_table, self.g_w, loss_out, self.workspace, stream)

    def new_plan(self, batch: int) -> torch.Tensor:
        """A buffer for the routing plan of a batch of this size."""
        return torch.empty(max(api.nvc_train_plan_bytes(self.grid, self.mlp, batch), 256), dtype=torch.uint8,
                           device=self.device)

    def plan(self, pos_unit, pix, batch: int, plan: torch.Tensor, stream=None) -> torch.Tensor:
        """The routing plan of the table scatter for these samples, for gradients(plan=...): it depends on
        the positions only, so it can be computed ahead of the gradient pass on another stream."""
        api.nvc_train_plan(self.grid, self.mlp, pos_unit, pix, batch, plan, stream)
        return plan

    def gradients_shadow(self, pos_unit, pos_scene, lights, spheres, pix=None, batch: int | None = None,
                         grad_scale: float = 0.0, labels_out=None, stream=None):
        """gradients() with the shadow labels of pos_scene (indexed like pos_unit) computed inside the
        training kernel: one network output per light (at most 32 lights, 512 spheres); labels_out
        (uint8 [batch][m]) receives them if given."""
        if batch is None:
            batch = pix.shape[0] if pix is not None else pos_unit.shape[0]
        self._ensure_workspace(batch)
        api.nvc_train_step_shadow(self.grid, self.mlp, self.table, self.packed, pos_unit, pos_scene, pix, batch,
                                  lights, spheres, self.loss, grad_scale, self.g_table, self.g_w, self.loss_buf,
                                  labels_out, self.workspace, stream)

    def adam(self, stream=None, ctr=None):
        """One Adam step on table and weights (gradients cleared), then repack the weights.

        With device counters `ctr` the step is ctr[1] when the kernels run (the
        host mirror `self.step` is then advanced by the caller)."""
        if ctr is None:
            self.step += 1
        for p, g, m, v in ((self.table, self.g_table, self.m_table, self.v_table), (self.w, self.g_w, self.m_w, self.v_w)):
            api.nvc_adam(p, g, m, v, self.step, self.lr, self.beta1, self.beta2, self.eps, True, stream, ctr=ctr,
                         lr_end=self.lr_end, lr_decay_steps=self.lr_decay_steps)
        self.pack(stream)

    def train_gradients(self, pos_unit, pos_scene, lights, spheres, frame: int, batch: int,
                        bufs: dict | None = None, stream=None, ctr=None) -> dict:
        """Pick `batch` pixels, label them with shadow rays, one gradient pass (no parameter update)."""
        if bufs is None:
            bufs = {"pix": torch.empty(batch, dtype=torch.int32, device=self.device),
                    "labels": torch.empty((batch, self.mlp.n_out), dtype=torch.uint8, device=self.device)}
        api.nvc_select_pixels(self.seed, frame, pos_unit.shape[0], bufs["pix"], self.pixel_workspace(pos_unit.shape[0]),
                              stream, ctr=ctr)
        if self.clustered:
            api.nvc_shadow_labels_clustered(pos_scene, bufs["pix"], lights, self.cl_offsets, self.cl_members, spheres,
                                            self.seed, frame, bufs["labels"], stream, ctr=ctr)
            self.gradients(pos_unit, labels=bufs["labels"], pix=bufs["pix"], batch=batch, stream=stream)
        elif self.fused_labels:
            self.gradients_shadow(pos_unit, pos_scene, lights, spheres, pix=bufs["pix"], batch=batch,
                                  labels_out=bufs["labels"], stream=stream)
        else:
            api.nvc_shadow_labels(pos_scene, bufs["pix"], lights, spheres, bufs["labels"], stream)
            self.gradients(pos_unit, labels=bufs["labels"], pix=bufs["pix"], batch=batch, stream=stream)
        if getattr(self, "world", None) is not None and self.world[0] > 0:
            nw, box, extent = self.world
            if "wpos" not in bufs:
                bufs["wpos"] = torch.empty((nw, 3), dtype=torch.float32, device=self.device)
                bufs["wunit"] = torch.empty((nw, 3), dtype=torch.float32, device=self.device)
                bufs["wlabels"] = torch.empty((nw, self.mlp.n_out), dtype=torch.uint8, device=self.device)
            api.nvc_world_samples(self.seed, frame, box, extent, bufs["wpos"], bufs["wunit"], stream, ctr=ctr)
            if self.clustered:
                api.nvc_shadow_labels_clustered(bufs["wpos"], None, lights, self.cl_offsets, self.cl_members, spheres,
                                                self.seed, frame, bufs["wlabels"], stream, ctr=ctr)
            else:
                api.nvc_shadow_labels(bufs["wpos"], None, lights, spheres, bufs["wlabels"], stream)
            self.gradients(bufs["wunit"], labels=bufs["wlabels"], batch=nw, stream=stream)
        return bufs

    def train_step(self, pos_unit, pos_scene, lights, spheres, frame: int, batch: int, bufs: dict | None = None,
                   stream=None, ctr=None) -> dict:
        """Pick `batch` pixels, label them with shadow rays, one gradient pass and one Adam step."""
        bufs = self.train_gradients(pos_unit, pos_scene, lights, spheres, frame, batch, bufs, stream, ctr)
        self.adam(stream, ctr=ctr)
        return bufs

    def frame(self, pos_unit, pos_scene, nrm, lights, spheres, frame: int, batch: int, bufs: dict | None = None,
              stream=None, ctr=None, side=None, join: bool = True) -> dict:
        """Inference + WRS + neural DI on every pixel, and one training step.

        Without `side` everything runs in order on `stream`.  With a second
        stream `side`, the training pixels, labels and gradients run on it
        beside inference and WRS (they only read the parameters), and Adam
        runs on `stream` once both are done; the results are the same.

        join=False (with `side`): the whole training step, Adam included, stays
        on `side` and nothing joins at the end of the frame.  Inference waits
        for the previous such frame's Adam, and Adam for this frame's
        inference, the only two orderings between the halves; consecutive
        frames then run without a cross-stream wait on the training side.
        The parameters are still being updated on `side` when this returns:
        another stream that reads them (inference outside a frame, a
        checkpoint) first calls wait_training().
        """
        if bufs is None:
            n = pos_unit.shape[0]
            bufs = {"vis": torch.empty((n, self.mlp.n_out), dtype=self.vis_dtype, device=self.device)}
        if side is not None and not join:
            main = stream if isinstance(stream, torch.cuda.Stream) else torch.cuda.current_stream()
            self.wait_training(main)
            self.infer(pos_unit, bufs["vis"], stream=main)
            inferred = torch.cuda.Event()
            inferred.record(main)
            bufs["sample"] = self.sample(bufs["vis"], pos_scene, nrm, lights, frame, bufs.get("sample"), stream=main,
                                         ctr=ctr)
            bufs["train"] = self.train_gradients(pos_unit, pos_scene, lights, spheres, frame, batch,
                                                 bufs.get("train"), stream=side, ctr=ctr)
            side.wait_event(inferred)
            self.adam(side, ctr=ctr)
            self._trained = torch.cuda.Event()
            self._trained.record(side)
            return bufs
        if side is None:
            self.infer(pos_unit, bufs["vis"], stream=stream)
            bufs["sample"] = self.sample(bufs["vis"], pos_scene, nrm, lights, frame, bufs.get("sample"),
                                         stream=stream, ctr=ctr)
            bufs["train"] = self.train_step(pos_unit, pos_scene, lights, spheres, frame, batch, bufs.get("train"),
                                            stream=stream, ctr=ctr)
            return bufs
        main = stream if isinstance(stream, torch.cuda.Stream) else torch.cuda.current_stream()
        api.fork(side, main)
        bufs["train"] = self.train_gradients(pos_unit, pos_scene, lights, spheres, frame, batch, bufs.get("train"),
                                             stream=side, ctr=ctr)
        self.infer(pos_unit, bufs["vis"], stream=main)
        bufs["sample"] = self.sample(bufs["vis"], pos_scene, nrm, lights, frame, bufs.get("sample"), stream=main,
                                     ctr=ctr)
        api.join(main, side)
        self.adam(main, ctr=ctr)
        return bufs

    def wait_training(self, stream=None):
        """Make `stream` (default: the current one) wait for the training step left running by the last
        frame(join=False); nothing to wait for otherwise."""
        ev = getattr(self, "_trained", None)
        if ev is not None:
            (stream if isinstance(stream, torch.cuda.Stream) else torch.cuda.current_stream()).wait_event(ev)

    # ------------------------------------------------------------ checkpoint
    def state_dict(self) -> dict:
        self.wait_training()
        return {"table": self.table.detach().cpu(), "w": self.w.detach().cpu(),
                "m_table": self.m_table.cpu(), "v_table": self.v_table.cpu(), "m_w": self.m_w.cpu(),
                "v_w": self.v_w.cpu(), "step": self.step, "seed": self.seed}

    def load_state_dict(self, sd: dict):
        self.wait_training()
        for k in ("table", "w", "m_table", "v_table", "m_w", "v_w"):
            getattr(self, k).copy_(sd[k].to(self.device))
        self.step = int(sd["step"])
        self.seed = int(sd["seed"])
        self.g_table.zero_()
        self.g_w.zero_()
        self.pack()


class FramePipeline:
    """Frames of a static scene queued on three streams, each frame's training pixels and shadow labels
    prepared one frame ahead.

    Frame f is the work of NVCache.frame: inference + WRS (+ DI) of every pixel, the training pixels
    (and world-space points) with their shadow labels, the gradient pass and Adam.  The pixels and
    labels of a frame depend only on the seed, the frame number and the scene, not on the parameters,
    so they run on a third stream (`prep`) while the previous frame's gradient pass and Adam run on
    `train`; inference + WRS run on `main`.  The orderings kept between the streams:
      * inference of frame f after Adam of frame f - 1, Adam of frame f after inference of frame f;
      * the gradient pass of frame f after the labels of frame f;
      * the pixels of frame f + 2 after the gradient pass of frame f has read the pixel and label set
        that they overwrite (two sets alternate).
    The routing plan of each frame's table scatter (a function of the pixels' positions only) is
    computed on `prep` too, into the set's own plan buffer.
    Each frame computes what it computes when the frames run one after another; only the placement
    in time across the streams changes.  run(f) already queues the labels of frame f + 1, so the scene
    tensors must stay unchanged while frames are queued: call finish() before changing them, or
    before reading the parameters on another stream.  `bufs` ("vis", "sample") hold the last frame's
    outputs, ordered on `main`.  With the cache's fused labels the prep stream only picks the pixels.
    """

    def __init__(self, cache: NVCache, pos_unit, pos_scene, nrm, lights, spheres, batch: int, main=None):
        dev = cache.device
        self.cache = cache
        self.args = (pos_unit, pos_scene, nrm, lights, spheres)
        self.batch = int(batch)
        self.main = main if isinstance(main, torch.cuda.Stream) else torch.cuda.current_stream(dev)
        self.train = torch.cuda.Stream(device=dev)
        self.prep = torch.cuda.Stream(device=dev)
        n, m = pos_unit.shape[0], cache.mlp.n_out
        self.bufs = {"vis": torch.empty((n, m), dtype=cache.vis_dtype, device=dev), "sample": None}
        world = getattr(cache, "world", None)
        self.n_world = world[0] if world is not None else 0
        self.sets = []
        for _ in range(2):
            s = {"pix": torch.empty(self.batch, dtype=torch.int32, device=dev),
                 "labels": torch.empty((self.batch, m), dtype=torch.uint8, device=dev),
                 "plan": cache.new_plan(self.batch)}
            if self.n_world:
                s["wpos"] = torch.empty((self.n_world, 3), dtype=torch.float32, device=dev)
                s["wunit"] = torch.empty((self.n_world, 3), dtype=torch.float32, device=dev)
                s["wlabels"] = torch.empty((self.n_world, m), dtype=torch.uint8, device=dev)
            self.sets.append(s)
        self.labelled = [torch.cuda.Event(), torch.cuda.Event()]
        self.consumed = [torch.cuda.Event(), torch.cuda.Event()]
        self.inferred = torch.cuda.Event()
        self.trained = torch.cuda.Event()
        self.pix_ws = cache.pixel_workspace(n)
        cache._ensure_workspace(max(self.batch, self.n_world))
        self._queued = None                    # frame whose pixels and labels are queued on `prep`

    def _labels(self, pos, pix, out, frame):
        c = self.cache
        lights, spheres = self.args[3], self.args[4]
        if c.clustered:
            api.nvc_shadow_labels_clustered(pos, pix, lights, c.cl_offsets, c.cl_members, spheres, c.seed, frame,
                                            out, self.prep)
        else:
            api.nvc_shadow_labels(pos, pix, lights, spheres, out, self.prep)

    def _prepare(self, frame: int):
        c, s, k = self.cache, self.sets[frame % 2], frame % 2
        pos_unit, pos_scene = self.args[0], self.args[1]
        self.prep.wait_event(self.consumed[k])
        api.nvc_select_pixels(c.seed, frame, pos_unit.shape[0], s["pix"], self.pix_ws, self.prep)
        fused = c.fused_labels and not c.clustered
        if not fused:
            c.plan(pos_unit, s["pix"], self.batch, s["plan"], stream=self.prep)
        if not fused:
            self._labels(pos_scene, s["pix"], s["labels"], frame)
        if self.n_world:
            _, box, extent = c.world
            api.nvc_world_samples(c.seed, frame, box, extent, s["wpos"], s["wunit"], self.prep)
            if not fused:
                self._labels(s["wpos"], None, s["wlabels"], frame)
        self.labelled[k].record(self.prep)
        self._queued = frame

    def run(self, frame: int, events=None) -> dict:
        """Queue frame `frame` (and the pixels and labels of frame + 1).  events: optional three timing
        events recorded on `main` before inference, after inference and after WRS."""
        c = self.cache
        pos_unit, pos_scene, nrm, lights, spheres = self.args
        if self._queued != frame:
            self._prepare(frame)
        self.main.wait_event(self.trained)
        if events is not None:
            events[0].record(self.main)
        c.infer(pos_unit, self.bufs["vis"], stream=self.main)
        self.inferred.record(self.main)
        if events is not None:
            events[1].record(self.main)
        self.bufs["sample"] = c.sample(self.bufs["vis"], pos_scene, nrm, lights, frame, self.bufs["sample"],
                                       stream=self.main)
        if events is not None:
            events[2].record(self.main)
        k, s = frame % 2, self.sets[frame % 2]
        self.train.wait_event(self.labelled[k])
        fused = c.fused_labels and not c.clustered
        if fused:
            c.gradients_shadow(pos_unit, pos_scene, lights, spheres, pix=s["pix"], batch=self.batch,
                               stream=self.train)
            if self.n_world:
                c.gradients_shadow(s["wunit"], s["wpos"], lights, spheres, batch=self.n_world, stream=self.train)
        else:
            c.gradients(pos_unit, labels=s["labels"], pix=s["pix"], batch=self.batch, stream=self.train,
                        plan=s["plan"])
            if self.n_world:
                c.gradients(s["wunit"], labels=s["wlabels"], batch=self.n_world, stream=self.train)
        self.consumed[k].record(self.train)
        self.train.wait_event(self.inferred)
        c.adam(self.train)
        self.trained.record(self.train)
        c._trained = self.trained
        self._prepare(frame + 1)
        return self.bufs

    def finish(self):
        """`main` waits for everything queued (the labels prepared ahead included)."""
        self.main.wait_stream(self.train)
        self.main.wait_stream(self.prep)


class FrameGraph:
    """One frame of the cache recorded once into a HIP graph and replayed.

    The frame is `NVCache.frame` (inference, WRS + neural DI, training pixels,
    shadow labels, gradients, Adam, repack; the training half on a second
    stream beside inference unless `concurrent` is False) followed by a
    device-counter increment; the frame number and the Adam step are read from the counters
    `ctr` (int32 [2]) when the kernels run, so every replay is the next
    frame.  `pre(stream)`, if given, is recorded first (e.g. scene animation
    driven by `ctr`); it must not allocate device memory.  Every buffer is
    allocated before the recording; the library calls allocate nothing, issue
    no memset and never synchronise.  Recording and replay go through the
    library's nvc_graph_begin / nvc_graph_end / nvc_graph_launch.  Before the
    recording ends, the capture ledger checks that the training stream was
    joined back after its last call, and the torch allocator's counters that
    nothing was allocated while recording (such memory could be handed to
    another tensor later while the graph still writes it): either raises.
    """

    def __init__(self, cache: NVCache, pos_unit, pos_scene, nrm, lights, spheres, batch: int, pre=None,
                 frame0: int = 0, concurrent: bool = True):
        self.cache = cache
        self.side = torch.cuda.Stream(device=cache.device) if concurrent else None
        self.stream = torch.cuda.Stream(device=cache.device)      # the recorded (and replaying) stream
        self.args = (pos_unit, pos_scene, nrm, lights, spheres)
        self.batch = int(batch)
        self.pre = pre
        dev = cache.device
        self.ctr = api.new_counters(frame0, cache.step + 1, device=dev)
        n = pos_unit.shape[0]
        self.bufs = {"vis": torch.empty((n, cache.mlp.n_out), dtype=cache.vis_dtype, device=dev),
                     "sample": {"idx": torch.empty(n, dtype=torch.int32, device=dev),
                                "pmf": torch.empty(n, dtype=torch.float32, device=dev),
                                "wsum": torch.empty(n, dtype=torch.float32, device=dev),
                                "di": torch.empty(n, dtype=torch.float32, device=dev)},
                     "train": {"pix": torch.empty(self.batch, dtype=torch.int32, device=dev),
                               "labels": torch.empty((self.batch, cache.mlp.n_out), dtype=torch.uint8, device=dev)}}
        cache._ensure_workspace(self.batch)
        cache.pixel_workspace(n)
        self.exec = None

    def _body(self, stream):
        if self.pre is not None:
            self.pre(stream)
        self.cache.frame(*self.args, 0, self.batch, self.bufs, stream=stream, ctr=self.ctr, side=self.side)
        api.nvc_counters_advance(self.ctr, stream)

    def run_eager(self):
        """The same frame without the graph (the counters advance the same way)."""
        self._body(torch.cuda.current_stream())
        self.cache.step += 1

    @staticmethod
    def _allocations() -> int:
        return int(torch.cuda.memory_stats().get("allocation.all.allocated", 0))

    def capture(self):
        torch.cuda.synchronize()
        saved = self.ctr.clone()
        st = self.stream
        st.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(st):         # warm-up of the recorded torch work, then restore the state
            if self.pre is not None:
                self.pre(st)
        torch.cuda.synchronize()
        self.ctr.copy_(saved)
        torch.cuda.synchronize()
        ledger = api.CaptureLedger(st.cuda_stream)
        n_alloc = self._allocations()
        api.nvc_graph_begin(st)
        problem = None
        try:
            with torch.cuda.stream(st), api.recording(ledger):
                self._body(st)
                try:
                    ledger.check()
                except RuntimeError as e:
                    problem = e
                    if self.side is not None:          # join so that the capture can still be ended cleanly
                        api.join(st, self.side)
        except BaseException:
            try:                                       # end the capture, drop what it recorded
                api.nvc_graph_destroy(api.nvc_graph_end(st))
            except Exception:
                pass
            raise
        ex = api.nvc_graph_end(st)
        if problem is None and self._allocations() != n_alloc:
            problem = RuntimeError("graph recording: device memory was allocated while recording")
        if problem is not None:
            api.nvc_graph_destroy(ex)
            raise problem
        self.exec = ex
        torch.cuda.synchronize()
        return self

    def replay(self):
        if self.exec is None:
            self.capture()
        st = self.stream
        st.wait_stream(torch.cuda.current_stream())
        api.nvc_graph_launch(self.exec, st)
        torch.cuda.current_stream().wait_stream(st)
        self.cache.step += 1

    def close(self):
        if self.exec is not None:
            torch.cuda.synchronize()
            api.nvc_graph_destroy(self.exec)
            self.exec = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class PipelineGraph:
    """FramePipeline's frames recorded as HIP graphs and replayed, one replay per frame.

    Replay of frame f: on the recorded stream the light animation of frame f (`anim`, e.g.
    LightAnimation on `lights` and `ctr`), inference and WRS + DI; on a second stream the gradient pass
    on the pixel/label set of frame f and, once inference is done, Adam and the repack; on a third the
    animation of frame f + 1 into a second light buffer (`lights_next`, through `anim_next`) and frame
    f + 1's training pixels (and world-space points), shadow labels and routing plan into the other
    set.  Both streams fork after the animation and join back before the counter increments that end
    the graph.  The frame number and the Adam step come from device counters (`ctr`: frame f and the
    step; `ctr_next`: frame f + 1), so every replay is the next frame; two graphs, one per set,
    alternate.  The first replay computes the first frame's set beforehand.  Each frame computes what
    the frames run one after another compute (its labels with its own lights).  `make_anim(lights, ctr)`
    returns the animation of a light buffer driven by a counter block, or None for static lights.
    Recording follows FrameGraph's rules (no allocation, every forked stream joined).
    """

    def __init__(self, cache: NVCache, pos_unit, pos_scene, nrm, lights, spheres, batch: int, make_anim=None,
                 frame0: int = 0):
        dev = cache.device
        self.cache = cache
        self.args = (pos_unit, pos_scene, nrm, lights, spheres)
        self.batch = int(batch)
        self.stream = torch.cuda.Stream(device=dev)
        self.train = torch.cuda.Stream(device=dev)
        self.prep = torch.cuda.Stream(device=dev)
        self.ctr = api.new_counters(frame0, cache.step + 1, device=dev)
        self.ctr_next = api.new_counters(frame0 + 1, cache.step + 2, device=dev)
        self.frame = int(frame0)                     # host mirror of the next frame to replay
        self.lights_next = lights.clone() if make_anim is not None else lights
        self.anim = make_anim(lights, self.ctr) if make_anim is not None else None
        self.anim_next = make_anim(self.lights_next, self.ctr_next) if make_anim is not None else None
        n, m = pos_unit.shape[0], cache.mlp.n_out
        self.bufs = {"vis": torch.empty((n, m), dtype=cache.vis_dtype, device=dev), "sample": None}
        world = getattr(cache, "world", None)
        self.n_world = world[0] if world is not None else 0
        self.sets = []
        for _ in range(2):
            st = {"pix": torch.empty(self.batch, dtype=torch.int32, device=dev),
                  "labels": torch.empty((self.batch, m), dtype=torch.uint8, device=dev),
                  "plan": cache.new_plan(self.batch)}
            if self.n_world:
                st["wpos"] = torch.empty((self.n_world, 3), dtype=torch.float32, device=dev)
                st["wunit"] = torch.empty((self.n_world, 3), dtype=torch.float32, device=dev)
                st["wlabels"] = torch.empty((self.n_world, m), dtype=torch.uint8, device=dev)
            self.sets.append(st)
        if cache.clustered:
            self.bufs["sample"] = {"idx": torch.empty(n, dtype=torch.int32, device=dev),
                                   "weight": torch.empty(n, dtype=torch.float32, device=dev),
                                   "cluster": torch.empty(n, dtype=torch.int32, device=dev)}
        else:
            self.bufs["sample"] = {"idx": torch.empty(n, dtype=torch.int32, device=dev),
                                   "pmf": torch.empty(n, dtype=torch.float32, device=dev),
                                   "wsum": torch.empty(n, dtype=torch.float32, device=dev),
                                   "di": torch.empty(n, dtype=torch.float32, device=dev)}
        self.inferred = torch.cuda.Event()
        self.pix_ws = cache.pixel_workspace(n)
        cache._ensure_workspace(max(self.batch, self.n_world))
        self.exec = [None] * self.n_graphs
        self._prepared = False

    def _prepare(self, s, stream, ctr, lights):
        """Training pixels (+ world-space points), shadow labels and routing plan of the frame in `ctr`."""
        c = self.cache
        pos_unit, pos_scene = self.args[0], self.args[1]
        spheres = self.args[4]
        fused = c.fused_labels and not c.clustered
        api.nvc_select_pixels(c.seed, 0, pos_unit.shape[0], s["pix"], self.pix_ws, stream, ctr=ctr)
        if not fused:
            if c.clustered:
                api.nvc_shadow_labels_clustered(pos_scene, s["pix"], lights, c.cl_offsets, c.cl_members, spheres,
                                                c.seed, 0, s["labels"], stream, ctr=ctr)
            else:
                api.nvc_shadow_labels(pos_scene, s["pix"], lights, spheres, s["labels"], stream)
            c.plan(pos_unit, s["pix"], self.batch, s["plan"], stream=stream)
        if self.n_world:
            _, box, extent = c.world
            api.nvc_world_samples(c.seed, 0, box, extent, s["wpos"], s["wunit"], stream, ctr=ctr)
            if not fused:
                if c.clustered:
                    api.nvc_shadow_labels_clustered(s["wpos"], None, lights, c.cl_offsets, c.cl_members, spheres,
                                                    c.seed, 0, s["wlabels"], stream, ctr=ctr)
                else:
                    api.nvc_shadow_labels(s["wpos"], None, lights, spheres, s["wlabels"], stream)

    def _body(self, k: int):
        """One frame that trains on set k and prepares set 1 - k, recorded (or run) on self.stream."""
        c = self.cache
        main = self.stream
        pos_unit, pos_scene, nrm, lights, spheres = self.args
        if self.anim is not None:
            self.anim(main)
        api.fork(self.train, main)
        api.fork(self.prep, main)
        c.infer(pos_unit, self.bufs["vis"], stream=main)
        self.inferred.record(main)
        self.bufs["sample"] = c.sample(self.bufs["vis"], pos_scene, nrm, lights, 0, self.bufs["sample"],
                                       stream=main, ctr=self.ctr)
        if self.anim_next is not None:
            with torch.cuda.stream(self.prep):
                self.anim_next(self.prep)
        self._prepare(self.sets[1 - k], self.prep, self.ctr_next, self.lights_next)
        s = self.sets[k]
        fused = c.fused_labels and not c.clustered
        if fused:
            c.gradients_shadow(pos_unit, pos_scene, lights, spheres, pix=s["pix"], batch=self.batch,
                               stream=self.train)
            if self.n_world:
                c.gradients_shadow(s["wunit"], s["wpos"], lights, spheres, batch=self.n_world, stream=self.train)
        else:
            c.gradients(pos_unit, labels=s["labels"], pix=s["pix"], batch=self.batch, stream=self.train,
                        plan=s["plan"])
            if self.n_world:
                c.gradients(s["wunit"], labels=s["wlabels"], batch=self.n_world, stream=self.train)
        self.train.wait_event(self.inferred)
        c.adam(self.train, ctr=self.ctr)
        api.join(main, self.train)
        api.join(main, self.prep)
        api.nvc_counters_advance(self.ctr, main)
        api.nvc_counters_advance(self.ctr_next, main)

    def _prologue(self):
        """The first frame's set, computed eagerly before the first replay (its lights animated first)."""
        main = self.stream
        main.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(main):
            if self.anim is not None:
                self.anim(main)
            self._prepare(self.sets[self.frame % 2], main, self.ctr, self.args[3])
        torch.cuda.current_stream().wait_stream(main)
        self._prepared = True

    def _capture(self, k: int):
        torch.cuda.synchronize()
        st = self.stream
        saved = (self.ctr.clone(), self.ctr_next.clone())
        st.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(st):                # warm-up of the recorded torch work, then restore the state
            if self.anim is not None:
                self.anim(st)
                self.anim_next(st)
        torch.cuda.synchronize()
        self.ctr.copy_(saved[0])
        self.ctr_next.copy_(saved[1])
        torch.cuda.synchronize()
        ledger = api.CaptureLedger(st.cuda_stream)
        n_alloc = FrameGraph._allocations()
        api.nvc_graph_begin(st)
        problem = None
        try:
            with torch.cuda.stream(st), api.recording(ledger):
                self._body(k)
                try:
                    ledger.check()
                except RuntimeError as e:
                    problem = e
                    for side in self._side_streams():      # join so that the capture can still be ended
                        api.join(st, side)
        except BaseException:
            try:
                api.nvc_graph_destroy(api.nvc_graph_end(st))
            except Exception:
                pass
            raise
        ex = api.nvc_graph_end(st)
        if problem is None and FrameGraph._allocations() != n_alloc:
            problem = RuntimeError("graph recording: device memory was allocated while recording")
        if problem is not None:
            api.nvc_graph_destroy(ex)
            raise problem
        self.exec[k] = ex
        torch.cuda.synchronize()

    def _side_streams(self):
        return (self.train, self.prep)

    n_graphs = 2          # recorded frames: one per pixel/label set

    def capture(self):
        for k in range(self.n_graphs):
            if self.exec[k] is None:
                self._capture(k)
        return self

    def replay(self):
        """Replay the next frame (on self.stream, ordered after the current stream's work so far)."""
        self.capture()
        if not self._prepared:
            self._prologue()
        st = self.stream
        st.wait_stream(torch.cuda.current_stream())
        api.nvc_graph_launch(self.exec[self.frame % 2], st)
        torch.cuda.current_stream().wait_stream(st)
        self.cache.step += 1
        self.frame += 1

    def run_eager(self):
        """The same frame without the graph (the counters advance the same way)."""
        if not self._prepared:
            self._prologue()
        st = self.stream
        st.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(st):
            self._body(self.frame % 2)
        torch.cuda.current_stream().wait_stream(st)
        self.cache.step += 1
        self.frame += 1

    def close(self):
        if any(e is not None for e in self.exec):
            torch.cuda.synchronize()
            for k in range(self.n_graphs):
                if self.exec[k] is not None:
                    api.nvc_graph_destroy(self.exec[k])
                    self.exec[k] = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class LaggedPickGraph(PipelineGraph):
    """PipelineGraph with the light pick (WRS + DI) of frame f moved into the replay of frame f + 1, where it
    runs beside that frame's inference instead of after this frame's.

    A replay ends when all of its streams are done, so in PipelineGraph the next frame's inference also waits
    for this frame's pick; queued eagerly (FramePipeline) the two overlap.  Here replay f runs: inference of
    frame f into its own visibility buffer (two alternate); on a fourth stream the pick of frame f - 1 from the
    other buffer, with frame f - 1's lights and frame number (`ctr_prev`); the gradient pass and Adam of
    frame f; frame f + 1's pixels, routing plan and world points, then (once the pick is done, since frame
    f + 1 reuses frame f - 1's light buffer) its light animation and labels.  Two light buffers alternate
    the same way: frame f's lights are `lights_of(f)`.  After replay f the pick outputs (`bufs["sample"]`)
    are frame f - 1's; `flush()` runs the last frame's pick.  The first frame runs eagerly (there is no
    earlier pick); the frames compute what the frames run one after another compute.  (Three light buffers,
    so that the labels need not wait for the pick, measured the same.)
    """

    def __init__(self, cache: NVCache, pos_unit, pos_scene, nrm, lights, spheres, batch: int, make_anim=None,
                 frame0: int = 0):
        # Switched off: one GPU run of its test (the clustered case, after 38 other GPU tests) ended in a
        # segmentation fault on the host inside the graph launch; the same tests had passed in two runs of
        # their own file, and the cause has not been found.
        raise RuntimeError("LaggedPickGraph is disabled: a host-side fault in its graph launch is not explained")
        super().__init__(cache, pos_unit, pos_scene, nrm, lights, spheres, batch, make_anim, frame0)
        dev = cache.device
        self.pick = torch.cuda.Stream(device=dev)
        self.ctr_prev = api.new_counters(frame0 - 1, cache.step, device=dev)
        self.L = [None, None]
        self.L[frame0 % 2] = lights
        self.L[1 - frame0 % 2] = self.lights_next
        self.vis = [self.bufs["vis"], torch.empty_like(self.bufs["vis"])]
        self.anim_into = ([make_anim(self.L[j], self.ctr_next) for j in (0, 1)] if make_anim is not None
                          else [None, None])
        self.picked = torch.cuda.Event()
        self.frame0 = int(frame0)

    def lights_of(self, frame: int) -> torch.Tensor:
        return self.L[frame % 2]

    def vis_of(self, frame: int) -> torch.Tensor:
        return self.vis[frame % 2]

    def _side_streams(self):
        return (self.train, self.prep, self.pick)

    def _body(self, k: int, pick: bool = True):
        """Frame f (f % 2 == k), with the pick of frame f - 1 unless `pick` is False."""
        c = self.cache
        main = self.stream
        pos_unit, pos_scene, nrm, _, spheres = self.args
        api.fork(self.train, main)
        api.fork(self.prep, main)
        if pick:
            api.fork(self.pick, main)
        c.infer(pos_unit, self.vis[k], stream=main)
        self.inferred.record(main)
        if pick:
            self.bufs["sample"] = c.sample(self.vis[1 - k], pos_scene, nrm, self.L[1 - k], 0, self.bufs["sample"],
                                           stream=self.pick, ctr=self.ctr_prev)
            self.picked.record(self.pick)
        # frame f + 1: pixels, plan and world points first; its lights go into the buffer the pick reads
        fused = c.fused_labels and not c.clustered
        nxt = self.sets[1 - k]
        prep = self.prep
        api.nvc_select_pixels(c.seed, 0, pos_unit.shape[0], nxt["pix"], self.pix_ws, prep, ctr=self.ctr_next)
        if not fused:
            c.plan(pos_unit, nxt["pix"], self.batch, nxt["plan"], stream=prep)
        if self.n_world:
            _, box, extent = c.world
            api.nvc_world_samples(c.seed, 0, box, extent, nxt["wpos"], nxt["wunit"], prep, ctr=self.ctr_next)
        if pick:
            prep.wait_event(self.picked)
        if self.anim_into[1 - k] is not None:
            with torch.cuda.stream(prep):
                self.anim_into[1 - k](prep)
        light_n = self.L[1 - k]
        if not fused:
            if c.clustered:
                api.nvc_shadow_labels_clustered(pos_scene, nxt["pix"], light_n, c.cl_offsets, c.cl_members, spheres,
                                                c.seed, 0, nxt["labels"], prep, ctr=self.ctr_next)
            else:
                api.nvc_shadow_labels(pos_scene, nxt["pix"], light_n, spheres, nxt["labels"], prep)
            if self.n_world:
                if c.clustered:
                    api.nvc_shadow_labels_clustered(nxt["wpos"], None, light_n, c.cl_offsets, c.cl_members, spheres,
                                                    c.seed, 0, nxt["wlabels"], prep, ctr=self.ctr_next)
                else:
                    api.nvc_shadow_labels(nxt["wpos"], None, light_n, spheres, nxt["wlabels"], prep)
        s = self.sets[k]
        light_k = self.L[k]
        if fused:
            c.gradients_shadow(pos_unit, pos_scene, light_k, spheres, pix=s["pix"], batch=self.batch,
                               stream=self.train)
            if self.n_world:
                c.gradients_shadow(s["wunit"], s["wpos"], light_k, spheres, batch=self.n_world, stream=self.train)
        else:
            c.gradients(pos_unit, labels=s["labels"], pix=s["pix"], batch=self.batch, stream=self.train,
                        plan=s["plan"])
            if self.n_world:
                c.gradients(s["wunit"], labels=s["wlabels"], batch=self.n_world, stream=self.train)
        self.train.wait_event(self.inferred)
        c.adam(self.train, ctr=self.ctr)
        api.join(main, self.train)
        api.join(main, self.prep)
        if pick:
            api.join(main, self.pick)
        api.nvc_counters_advance(self.ctr, main)
        api.nvc_counters_advance(self.ctr_next, main)
        api.nvc_counters_advance(self.ctr_prev, main)

    def _prologue(self):
        """The first frame's lights and set, computed eagerly before its frame."""
        main = self.stream
        k = self.frame % 2
        main.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(main):
            if self.anim is not None:
                self.anim(main)                    # make_anim(lights, ctr): the first frame's lights
            self._prepare(self.sets[k], main, self.ctr, self.L[k])
        torch.cuda.current_stream().wait_stream(main)
        self._prepared = True

    def _run(self, graph: bool):
        st = self.stream
        k = self.frame % 2
        first = self.frame == self.frame0
        if graph:
            # recorded before the first frame runs: the warm-up of the recorded light animations writes
            # the first frame's lights and the next frame's, as the first frame itself does
            self.capture()
        if not self._prepared:
            self._prologue()
        st.wait_stream(torch.cuda.current_stream())
        if graph and not first:
            api.nvc_graph_launch(self.exec[k], st)
        else:
            with torch.cuda.stream(st):
                self._body(k, pick=not first)
        torch.cuda.current_stream().wait_stream(st)
        self.cache.step += 1
        self.frame += 1

    def replay(self):
        """The next frame (the first one eagerly), and the previous frame's pick."""
        self._run(graph=True)

    def run_eager(self):
        self._run(graph=False)

    def flush(self):
        """The pick of the last frame run (into bufs["sample"])."""
        if self.frame == self.frame0:
            return
        st = self.stream
        k = (self.frame - 1) % 2
        st.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(st):
            self.bufs["sample"] = self.cache.sample(self.vis[k], self.args[1], self.args[2], self.L[k], 0,
                                                    self.bufs["sample"], stream=st, ctr=self.ctr_prev)
        torch.cuda.current_stream().wait_stream(st)


class NVCFunction(torch.autograd.Function):
    """vis = sigmoid(MLP(encode(pos))) with gradients for the table and the FP32 master weights.

    forward packs `w` into a packed copy of its own (the cache's `packed`,
    which inference uses, is left alone) and runs nvc_infer (FP32 output);
    backward runs nvc_train_step with the upstream gradient on that same
    packed copy and the saved table, recomputing the activations, so other
    forwards, repacks or Adam steps between the two do not change the result.
    """

    @staticmethod
    def forward(ctx, pos_unit, table, w, cache: NVCache, grad_scale: float = 0.0):
        packed = torch.empty(api.nvc_mlp_packed_bytes(cache.mlp), dtype=torch.uint8, device=pos_unit.device)
        api.nvc_pack_mlp(cache.mlp, w.detach().contiguous(), packed)
        vis = torch.empty((pos_unit.shape[0], cache.mlp.n_out), dtype=torch.float32, device=pos_unit.device)
        api.nvc_infer(cache.grid, cache.mlp, table.detach().contiguous(), packed, pos_unit, vis)
        ctx.save_for_backward(pos_unit, table, w, packed)
        ctx.cache = cache
        ctx.grad_scale = grad_scale
        return vis

    @staticmethod
    def backward(ctx, dvis):
        pos_unit, table, w, packed = ctx.saved_tensors
        cache = ctx.cache
        g_table = torch.zeros_like(table)
        g_w = torch.zeros_like(w)
        cache._ensure_workspace(pos_unit.shape[0])
        api.nvc_train_step(cache.grid, cache.mlp, table.detach().contiguous(), packed, pos_unit, None,
                           pos_unit.shape[0], None, dvis.contiguous().float(), cache.loss, ctx.grad_scale,
                           g_table, g_w, None, cache.workspace)
        return None, g_table, g_w, None, None


class NVCLossFunction(torch.autograd.Function):
    """loss = the training loss of a labelled batch (Sec. 3.3-3.4) with gradients for the table and the FP32
    master weights: the library's training kernel in labelled mode.  forward runs nvc_train_step once on a
    private packed copy of `w` and keeps the gradients it returns; backward scales them by the incoming
    gradient.  labels: uint8 [n][n_out]; the loss kind is the cache's (BCE or L2)."""

    @staticmethod
    def forward(ctx, pos_unit, table, w, labels, cache: NVCache, grad_scale: float = 0.0):
        packed = torch.empty(api.nvc_mlp_packed_bytes(cache.mlp), dtype=torch.uint8, device=pos_unit.device)
        api.nvc_pack_mlp(cache.mlp, w.detach().contiguous(), packed)
        g_table = torch.zeros_like(table, dtype=torch.float32)
        g_w = torch.zeros_like(w, dtype=torch.float32)
        loss = torch.zeros(1, dtype=torch.float32, device=pos_unit.device)
        cache._ensure_workspace(pos_unit.shape[0])
        api.nvc_train_step(cache.grid, cache.mlp, table.detach().contiguous(), packed, pos_unit, None,
                           pos_unit.shape[0], labels, None, cache.loss, grad_scale, g_table, g_w, loss,
                           cache.workspace)
        ctx.save_for_backward(g_table, g_w)
        return loss[0]

    @staticmethod
    def backward(ctx, grad_out):
        g_table, g_w = ctx.saved_tensors
        return None, g_table * grad_out, g_w * grad_out, None, None, None
