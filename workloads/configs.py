"""Workload definitions: sizes, seeds and network shapes of the five synthetic workloads.

The paper measures on its own scenes (Kitchen, Sponza, ...) at 1920x1080 with
32 lights, a two-hidden-layer MLP and a ten-level hash grid (Sec. 3.3, Sec. 4.4,
Table "perf_breakdown").  Those scenes are not available, so these seeded
synthetic scenes of the same shape stand in for them.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace


@dataclass(frozen=True)
class GridCfg:
    """Multi-resolution hash grid (Sec. 3.3; Mueller et al. 2022).

    n_levels L, n_feat F features per level, table size T = 2**log2_T entries
    per level, coarsest resolution base_res, per-level growth factor.
    """
    n_levels: int
    n_feat: int
    log2_T: int
    base_res: int
    growth: float

    @property
    def T(self) -> int:
        return 1 << self.log2_T

    @property
    def n_out(self) -> int:
        return self.n_levels * self.n_feat

    @property
    def n_params(self) -> int:
        return self.n_levels * self.T * self.n_feat


@dataclass(frozen=True)
class MlpCfg:
    """Visibility MLP (Sec. 3.3): n_in -> width x n_hidden -> n_out, no biases.

    act: 'relu' or 'leaky' (slope leaky_slope) on hidden layers; the output
    layer is always a sigmoid.  dtype is the precision of weights and
    activations fed to the matrix cores ('f32', 'f16', 'bf16'); accumulation
    is always FP32.
    """
    n_in: int
    width: int
    n_hidden: int
    n_out: int
    act: str = "relu"
    leaky_slope: float = 0.01
    dtype: str = "f16"

    def layer_shapes(self):
        """[(out, in)] for every weight matrix, input layer first."""
        shapes = [(self.width, self.n_in)]
        shapes += [(self.width, self.width)] * (self.n_hidden - 1)
        shapes.append((self.n_out, self.width))
        return shapes

    @property
    def n_params(self) -> int:
        return sum(o * i for o, i in self.layer_shapes())

    @property
    def flops_per_point(self) -> int:
        return 2 * self.n_params


@dataclass(frozen=True)
class Workload:
    name: str
    grid: GridCfg
    mlp: MlpCfg
    kind: str                    # 'cube' (points in the unit cube) or 'boxes' (G-buffer of a box scene)
    n_lights: int
    n_spheres: int
    n_points: int = 0            # cube scenes
    width: int = 0               # box scenes: image size
    height: int = 0
    n_boxes: int = 0
    train_batch: int = 0
    loss: str = "bce"
    lr: float = 1e-2
    lr_end: float | None = None  # with lr_decay_steps > 0: linear decay lr -> lr_end (Sec. 3.4)
    lr_decay_steps: int = 0
    init: str = "xavier"         # MLP initialisation: 'xavier' or 'he' (Sec. 3.4)
    n_clusters: int = 0          # clustered cache (Sec. 3.6): one output per cluster of lights (0: per light)
    n_cand: int = 8              # RIS candidates of the clustered pick
    world_batch: int = 0         # world-space training points per step besides train_batch screen samples
    world_box: tuple = (0.5, 0.5, 0.5, 9.5, 9.5, 9.5)   # where they are drawn (scene units)
    beta1: float = 0.9
    beta2: float = 0.99
    adam_eps: float = 1e-8
    vis_floor: float = 1e-3      # visibility clamp (Sec. 3.1, Fig. "bias")
    frames: int = 1
    scene_seed: int = 0
    init_seed: int = 1
    rng_key: int = 2             # key of the counter-based generator (WRS picks, training pixels)
    notes: str = ""

    @property
    def n_pixels(self) -> int:
        return self.n_points if self.kind == "cube" else self.width * self.height


_GRID_1080 = GridCfg(n_levels=16, n_feat=2, log2_T=19, base_res=16, growth=1.447)
_MLP_1080 = MlpCfg(n_in=32, width=64, n_hidden=3, n_out=32, act="relu", dtype="f16")

WORKLOADS = {
    "tiny": Workload(
        name="tiny",
        grid=GridCfg(n_levels=8, n_feat=2, log2_T=14, base_res=16, growth=1.5),
        mlp=MlpCfg(n_in=16, width=32, n_hidden=2, n_out=8, act="relu", dtype="f32"),
        kind="cube", n_points=4096, n_lights=8, n_spheres=16, train_batch=1024,
        notes="4096 points in the unit cube, 8 lights, 16 spheres; FP32 on the GPU, FP64 in the oracle",
    ),
    "frame_1080p": Workload(
        name="frame_1080p", grid=_GRID_1080, mlp=_MLP_1080,
        kind="boxes", width=1920, height=1080, n_boxes=64, n_lights=32, n_spheres=256,
        train_batch=1 << 18,
        notes="1920x1080 G-buffer of 64 boxes + 4 planes in [0,10]^3, 32 point lights, 256 sphere occluders",
    ),
    "train_1080p": Workload(
        name="train_1080p", grid=_GRID_1080, mlp=_MLP_1080,
        kind="boxes", width=1920, height=1080, n_boxes=64, n_lights=32, n_spheres=256,
        train_batch=1 << 18, loss="bce",
        notes="training step on the 1080p scene: 2^18 pixels x 32 lights, BCE, Adam 0.9/0.99 lr 1e-2",
    ),
    "sweep_4k": Workload(
        name="sweep_4k",
        grid=GridCfg(n_levels=16, n_feat=2, log2_T=20, base_res=16, growth=1.447),
        mlp=MlpCfg(n_in=32, width=128, n_hidden=3, n_out=128, act="relu", dtype="f16"),
        kind="boxes", width=3840, height=2160, n_boxes=64, n_lights=128, n_spheres=256,
        train_batch=1 << 18,
        notes="3840x2160, 128 lights, width-128 MLP; FP32 / FP16 / BF16 precision sweep",
    ),
    "paper_1080p": Workload(
        name="paper_1080p",
        grid=GridCfg(n_levels=10, n_feat=4, log2_T=14, base_res=16, growth=1.19),
        mlp=MlpCfg(n_in=40, width=32, n_hidden=2, n_out=32, act="leaky", leaky_slope=0.01, dtype="f16"),
        kind="boxes", width=1920, height=1080, n_boxes=64, n_lights=32, n_spheres=256,
        train_batch=4096, world_batch=4096, loss="l2", lr=0.05, lr_end=0.001, lr_decay_steps=200, init="he",
        notes="the paper's own configuration (Sec. 3.3-3.4): ten levels x four features at base 16 (T = 2^14, "
              "growth 1.19), 40-32-32-32 MLP with leaky ReLU 0.01, L2 loss, He init, Adam with the rate lowered "
              "linearly from 0.05 to 0.001 over the first 200 steps, 4096 screen + 4096 world-space samples per "
              "frame; 1080p box scene",
    ),
    "clustered_1080p": Workload(
        name="clustered_1080p",
        grid=GridCfg(n_levels=8, n_feat=4, log2_T=14, base_res=2, growth=2.0),
        mlp=MlpCfg(n_in=32, width=32, n_hidden=2, n_out=32, act="leaky", leaky_slope=0.01, dtype="f16"),
        kind="boxes", width=1920, height=1080, n_boxes=64, n_lights=4096, n_spheres=256,
        train_batch=49152, loss="l2", lr=0.05, lr_end=0.001, lr_decay_steps=200, init="he",
        n_clusters=32, n_cand=8,
        notes="clustered cache (Sec. 3.6): 4096 point lights in 32 k-means clusters, one output per cluster, "
              "eight levels x four features at base 2 (growth 2.0, T = 2^14), 32-32-32-32 leaky MLP, L2, "
              "49,152 samples per frame, two-step pick with 8 RIS candidates; 1080p box scene",
    ),
    "loop_60f": Workload(
        name="loop_60f", grid=_GRID_1080, mlp=_MLP_1080,
        kind="boxes", width=1920, height=1080, n_boxes=64, n_lights=32, n_spheres=256,
        train_batch=1 << 18, frames=60,
        notes="60-frame loop at 1080p; light 0 moves on a radius-3 circle",
    ),
}


def get_workload(name: str, **overrides) -> Workload:
    wl = WORKLOADS[name]
    if overrides:
        mlp_over = {k[4:]: overrides.pop(k) for k in list(overrides) if k.startswith("mlp_")}
        if mlp_over:
            overrides["mlp"] = replace(wl.mlp, **mlp_over)
        wl = replace(wl, **overrides)
    return wl
