"""Scene descriptions of the standard synthetic workloads.

Every scene is a nested stack of sphere-plus-SIREN-detail SDFs
    f_j(x, t) = |x - c(t)| - r0 + a_j * N_j(input_j)
with c(t) = rho * (cos 2 pi t, sin 2 pi t, 0) (rho = 0: static) and input_j
equal to x, to x - c(t) (``follow_center``) or to (x, t) for 4-D nets.
The paper's trained scanned-model SIRENs are not available, so these scenes
stand in for them with the paper's network shapes and image sizes.

Workloads (rays; levels as (width, k) in the paper's notation):
  single_64x1_128sq   128x128; one (64,1) net, seed 0, a = 0.02
  stack3_512sq        512x512; (32,1) s1 a=.005 |> (64,1) s2 a=.015 |> (256,2) s3 a=.02,
                      delta = (0.05, 0.01)
  stack3_1080p        1920x1080; the same stack
  stack3_4096sq       4096x4096; the same stack
  anim16_1024sq       16 frames x 1024x1024, t = i/16; (64,1) s5 a=.005 on x - c(t)
                      |> 4-D (256,2) s4 a=.02, delta_1 = 0.05, rho = 0.2
  stack2_64x1_128x2_512sq
                      512x512; (64,1) s31 a=.015 |> (128,2) s32 a=.02, delta = 0.05
                      (the widths of the paper's animated example, static here)
  stack3_bigarg_512sq 512x512; the three-level stack with its (256,2) level's hidden
                      biases shifted by 300 revolutions (bias_turns = 300): the same
                      function, with hidden sine arguments near 300 revolutions
  fit_torus_256x2     fitting a (256,2) net (seed 6) to the torus; rendered at 1080p
  table3_*            the rows of the paper's Table 3 at 512x512, traced with fixed
                      iteration counts (TABLE3_ROWS gives the counts and which net is
                      used for neural normal mapping only): (64,1) s2 a=.015,
                      (256,1) s21, (256,2) s3, (256,3) s23, a=.02 for the 256-wide nets,
                      delta = (0.05, 0.01)
"""

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

from .siren_init import SirenNet, siren_init
from .camera import pinhole_rays

R0 = 0.6
STEP_SCALE = 0.9
HIT_EPS = 1e-4
FAR = 5.0
MAX_STEPS_PER_LEVEL = 64


@dataclass
class SceneLevel:
    net: SirenNet
    amplitude: float
    delta: float = 0.0           # ignored on the last traced level
    follow_center: bool = False  # net input is x - c(t)


@dataclass
class Scene:
    name: str
    levels: List[SceneLevel]
    width: int
    height: int
    frames: int = 1
    r0: float = R0
    rho: float = 0.0             # circle radius of the centre motion (period 1)
    step_scale: float = STEP_SCALE
    eps: float = HIT_EPS
    far: float = FAR
    max_steps: int = MAX_STEPS_PER_LEVEL
    base_sphere: bool = True     # include |x - c(t)| - r0 (False: f = a * N only)
    extra: dict = field(default_factory=dict)

    @property
    def n_rays(self) -> int:
        return self.width * self.height * self.frames

    def rays(self, rows=None, frames=None):
        """(o, v, t) float32; t is None for static single-frame scenes.

        ``rows`` selects image rows (same rays as the full image);
        ``frames`` selects frame indices (default: all)."""
        o1, v1 = pinhole_rays(self.width, self.height, rows=rows)
        if self.frames == 1 and self.rho == 0.0 and not any(l.net.d_in == 4 for l in self.levels):
            return o1, v1, None
        fr = np.arange(self.frames) if frames is None else np.asarray(frames)
        o = np.concatenate([o1] * len(fr), axis=0)
        v = np.concatenate([v1] * len(fr), axis=0)
        t = np.repeat((fr.astype(np.float64) / self.frames).astype(np.float32), o1.shape[0])
        return np.ascontiguousarray(o), np.ascontiguousarray(v), np.ascontiguousarray(t)

    def with_amplitudes(self, amps) -> "Scene":
        lv = [SceneLevel(l.net, float(a), l.delta, l.follow_center) for l, a in zip(self.levels, amps)]
        return Scene(self.name, lv, self.width, self.height, self.frames, self.r0, self.rho,
                     self.step_scale, self.eps, self.far, self.max_steps, self.base_sphere,
                     dict(self.extra))

    def with_size(self, width: int, height: int, frames: Optional[int] = None) -> "Scene":
        return Scene(self.name, self.levels, width, height, self.frames if frames is None else frames,
                     self.r0, self.rho, self.step_scale, self.eps, self.far, self.max_steps,
                     self.base_sphere, dict(self.extra))


def _stack3():
    return [
        SceneLevel(siren_init(1, 3, 32, 2, 0.005), 0.005, 0.05),
        SceneLevel(siren_init(2, 3, 64, 2, 0.015), 0.015, 0.01),
        SceneLevel(siren_init(3, 3, 256, 3, 0.02), 0.02, 0.0),
    ]


def _t3_net(shape):
    if shape == (64, 1):
        return SceneLevel(siren_init(2, 3, 64, 2, 0.015), 0.015, 0.05)
    seed = {1: 21, 2: 3, 3: 23}[shape[1]]
    return SceneLevel(siren_init(seed, 3, 256, shape[1] + 1, 0.02), 0.02, 0.0)


# Table 3 rows: scene name -> (nets, iterations of the traced nets, normal net)
TABLE3_ROWS = {
    "table3_256x3": ([(256, 3)], [20], 0),
    "table3_64x1": ([(64, 1)], [20], 0),
    "table3_64x1_256x1": ([(64, 1), (256, 1)], [20], 1),
    "table3_64x1_256x2": ([(64, 1), (256, 2)], [20], 1),
    "table3_64x1_256x3": ([(64, 1), (256, 3)], [20], 1),
    "table3_64x1_256x1_256x3": ([(64, 1), (256, 1), (256, 3)], [20, 5], 2),
}


def make_scene(name: str) -> Scene:
    if name in TABLE3_ROWS:
        nets = TABLE3_ROWS[name][0]
        levels = [_t3_net(sh) for sh in nets]
        if len(levels) == 3:
            levels[1] = SceneLevel(levels[1].net, levels[1].amplitude, 0.01)
        return Scene(name, levels, 512, 512)
    if name == "single_64x1_128sq":
        return Scene(name, [SceneLevel(siren_init(0, 3, 64, 2, 0.02), 0.02)], 128, 128)
    if name == "stack3_512sq":
        return Scene(name, _stack3(), 512, 512)
    if name == "stack3_1080p":
        return Scene(name, _stack3(), 1920, 1080)
    if name == "stack3_4096sq":
        return Scene(name, _stack3(), 4096, 4096)
    if name == "stack2_64x1_128x2_512sq":
        levels = [SceneLevel(siren_init(31, 3, 64, 2, 0.015), 0.015, 0.05),
                  SceneLevel(siren_init(32, 3, 128, 3, 0.02), 0.02, 0.0)]
        return Scene(name, levels, 512, 512)
    if name == "stack3_wsmid_512sq":
        # a (256,2) level in the middle of the stack: the weight-stationary
        # tracer as a non-final level (its queue sorted for the next level)
        levels = [SceneLevel(siren_init(2, 3, 64, 2, 0.015), 0.015, 0.05),
                  SceneLevel(siren_init(3, 3, 256, 3, 0.02), 0.02, 0.01),
                  SceneLevel(siren_init(23, 3, 256, 4, 0.02), 0.02, 0.0)]
        return Scene(name, levels, 512, 512)
    if name == "stack3_bigarg_512sq":
        levels = _stack3()
        levels[2] = SceneLevel(siren_init(3, 3, 256, 3, 0.02, bias_turns=300), 0.02, 0.0)
        return Scene(name, levels, 512, 512)
    if name == "anim16_1024sq":
        levels = [
            SceneLevel(siren_init(5, 3, 64, 2, 0.005), 0.005, 0.05, follow_center=True),
            SceneLevel(siren_init(4, 4, 256, 3, 0.02), 0.02, 0.0),
        ]
        return Scene(name, levels, 1024, 1024, frames=16, rho=0.2)
    if name == "fit_torus_256x2":
        net = siren_init(6, 3, 256, 3, 1.0, normalise=False)
        return Scene(name, [SceneLevel(net, 1.0)], 1920, 1080, r0=0.0, base_sphere=False,
                     extra={"n_surf": 1 << 16, "n_unif": 1 << 18, "steps": 2000, "lr": 1e-4,
                            "sample_seed": 7})
    raise KeyError(name)


WORKLOADS = ["single_64x1_128sq", "stack3_512sq", "stack3_1080p", "stack3_4096sq",
             "stack2_64x1_128x2_512sq", "stack3_bigarg_512sq", "stack3_wsmid_512sq", "anim16_1024sq", "fit_torus_256x2"] + list(TABLE3_ROWS)
