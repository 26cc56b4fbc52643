"""Seeded synthetic inputs shared by the GPU path's tests/benchmark and the oracle.

This module holds no arithmetic of the lattice Boltzmann method. It only
draws the random parameters of the randomized Taylor-Green ensemble and names
the workloads (sizes, counts, flow parameters) that tests and the benchmark
run.

Random parameters: the paper perturbs the Taylor-Green field with 24 i.i.d.
uniform variables per sample (section "Randomized Taylor-Green vortex
flow", eq. (alpha_perturbation)). Here Y ~ U[-1, 1]^24 per sample, and the
physical amplitude is applied by the method (X = amp * U0 * Y). Index
convention: p = 8*alpha + 4*i + 2*j + k for the product
a_i(2x) a_j(2y) a_k(2z) in component alpha, a_0 = sin, a_1 = cos.

Generator: SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom
number generators", OOPSLA 2014), state = seed; each draw advances the state
by the golden-gamma constant 0x9E3779B97F4A7C15 and mixes it. Draws are taken
sample by sample, parameter by parameter, and mapped to [-1, 1) as
2 * (top 53 bits * 2^-53) - 1.
"""
from dataclasses import dataclass, field
from typing import List

import numpy as np

N_PARAMS = 24
_MASK = (1 << 64) - 1


def splitmix64_stream(seed: int, count: int) -> List[int]:
    state = seed & _MASK
    out = []
    for _ in range(count):
        state = (state + 0x9E3779B97F4A7C15) & _MASK
        z = state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK
        out.append(z ^ (z >> 31))
    return out


def draw_y(seed: int, m: int) -> np.ndarray:
    """Y[m][24] in [-1, 1), float64."""
    raw = splitmix64_stream(seed, m * N_PARAMS)
    y = np.array([2.0 * ((r >> 11) * 2.0 ** -53) - 1.0 for r in raw], dtype=np.float64)
    return y.reshape(m, N_PARAMS)


def random_populations(seed: int, shape, scale: float) -> np.ndarray:
    """Uniform noise in [-scale, scale) for perturbing populations in tests."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-scale, scale, size=shape)


@dataclass
class SampleGroup:
    """`count` samples that share a resolution and flow parameters."""
    n: int            # lattice points per axis
    count: int
    u0: float         # Taylor-Green amplitude in lattice units
    re: float         # Reynolds number U0 * L / nu with L = n / (2 pi)
    amp: float        # perturbation amplitude relative to U0
    project: bool     # Leray-project the perturbation
    stride: int = 1   # advance on every stride-th tick


@dataclass
class Workload:
    name: str
    groups: List[SampleGroup]
    precision: str        # "f64" or "f32s" (FP32 shifted populations)
    ticks: int
    seed: int
    save_every: int = 0
    notes: str = ""
    lattice: int = 27     # velocities: 27 (D3Q27) or 19 (D3Q19, the paper's set)

    @property
    def m(self) -> int:
        return sum(g.count for g in self.groups)


def diffusive_u0(n: int) -> float:
    """U0 anchored at 0.05 lattice units on 32^3 and halved per doubling of n."""
    return 0.05 * 32.0 / n


WORKLOADS = {
    # single sample, FP64, pure Taylor-Green, 32^3, Re 100, 100 steps
    "tgv32_f64": Workload(
        "tgv32_f64", [SampleGroup(32, 1, 0.05, 100.0, 0.0, False)], "f64", 100, 0, 1),
    # 64 samples at 64^3, FP32 shifted, Re 1600, projected perturbation, 500 steps
    "rtgv64x64_f32": Workload(
        "rtgv64x64_f32", [SampleGroup(64, 64, diffusive_u0(64), 1600.0, 0.05, True)], "f32s", 500, 2608, 50),
    # mixed batch: 32 x 64^3 + 12 x 128^3 + 4 x 256^3, diffusive viscosity, strides 16:4:1
    "mixed48_f32": Workload(
        "mixed48_f32",
        [SampleGroup(64, 32, diffusive_u0(64), 1600.0, 0.05, True, 16),
         SampleGroup(128, 12, diffusive_u0(128), 3200.0, 0.05, True, 4),
         SampleGroup(256, 4, diffusive_u0(256), 6400.0, 0.05, True, 1)],
        "f32s", 1000, 2609, 16),
    # the 64-sample ensemble on the paper's D3Q19 lattice (same flow, seed and steps)
    "rtgv64x64_f32_d3q19": Workload(
        "rtgv64x64_f32_d3q19", [SampleGroup(64, 64, diffusive_u0(64), 1600.0, 0.05, True)], "f32s", 500, 2608, 50,
        lattice=19),
    # vanishing-viscosity sequence: 8 samples at each of 128^3, 256^3, 512^3
    # (Re = 12.5 N, diffusive U0, the same Y at every resolution), strides
    # 16:4:1; the run to t = 9 takes 234,684 ticks, the benchmark times a
    # bounded number of them and compares the resolutions at equal physical
    # time through 1-point Wasserstein distances and the relative L1 sample
    # error on the 8^3 common nodes
    "sequence512x8_f32": Workload(
        "sequence512x8_f32",
        [SampleGroup(128, 8, diffusive_u0(128), 1600.0, 0.05, True, 16),
         SampleGroup(256, 8, diffusive_u0(256), 3200.0, 0.05, True, 4),
         SampleGroup(512, 8, diffusive_u0(512), 6400.0, 0.05, True, 1)],
        "f32s", 256, 2611, 16),
    # the same sequence in acoustic scaling (the faster variant): U0 = 0.05 at
    # every N, so the time step is proportional to dx and the strides are
    # 4:2:1; Re = 12.5 N as above (the lattice viscosity is then the same at
    # every N). To t = 9: 14,688 ticks of the 512^3 lattice, saves every 1632
    # ticks (t = 1.0014 per save)
    "sequence512x8_acoustic_f32": Workload(
        "sequence512x8_acoustic_f32",
        [SampleGroup(128, 8, 0.05, 1600.0, 0.05, True, 4),
         SampleGroup(256, 8, 0.05, 3200.0, 0.05, True, 2),
         SampleGroup(512, 8, 0.05, 6400.0, 0.05, True, 1)],
        "f32s", 14688, 2611, 1632),
    # its rehearsal one resolution lower: 64^3, 128^3, 256^3, 7344 ticks to t = 9
    "sequence256x8_acoustic_f32": Workload(
        "sequence256x8_acoustic_f32",
        [SampleGroup(64, 8, 0.05, 800.0, 0.05, True, 4),
         SampleGroup(128, 8, 0.05, 1600.0, 0.05, True, 2),
         SampleGroup(256, 8, 0.05, 3200.0, 0.05, True, 1)],
        "f32s", 7344, 2611, 816),
    # adjoint workload: 8 x 128^3, FP32 forward, 1000 steps, checkpoints every 50
    "adjoint128x8_f32": Workload(
        "adjoint128x8_f32", [SampleGroup(128, 8, diffusive_u0(128), 1600.0, 0.05, True)], "f32s", 1000, 2610, 50),
}
