"""Seeded synthetic cavity workloads.

This module only describes inputs: cavity geometry, grid, layer stack and plane-wave
incidences.  It holds none of the solver's arithmetic, so both the CPU oracle and the
GPU library can take their inputs from here without sharing any code of the method.

Units follow the paper's numerical experiments (Section 7): lengths in wavelengths
(lambda = 1), wavenumber k = 2*pi, angles in radians.  Layers are listed bottom to top
as (number of z-intervals, relative permittivity); the interfaces sit on grid nodes.
Polarisation 0 is the theta-hat ("TM", "theta-theta") wave, 1 the phi-hat ("TE",
"phi-phi") wave of Section 7.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

TWO_PI = 2.0 * math.pi
TM, TE = 0, 1


@dataclasses.dataclass(frozen=True)
class Cavity:
    """One cavity problem: geometry, grid and a bottom-to-top layer stack."""

    a: float
    b: float
    c: float
    nx: int
    ny: int
    nz: int
    layer_nz: Tuple[int, ...]
    layer_eps: Tuple[complex, ...]
    k: float = TWO_PI
    tbc_oversample: int = 1
    # thickness of each layer (sum c); None: every layer has the common step c / nz
    layer_depth: Optional[Tuple[float, ...]] = None

    def __post_init__(self):
        if len(self.layer_nz) != len(self.layer_eps):
            raise ValueError("layer_nz and layer_eps differ in length")
        if self.layer_depth is not None and len(self.layer_depth) != len(self.layer_nz):
            raise ValueError("layer_depth and layer_nz differ in length")


@dataclasses.dataclass(frozen=True)
class Incidence:
    theta: float
    phi: float
    pol: int


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    cavity: Cavity
    incidences: Tuple[Incidence, ...]
    tol: float = 1e-12      # relative residual the solves stop at
    batch: int = 8          # right-hand sides iterated together
    fields: bool = True     # False: a step needs the RCS only, not the field on all nodes


def deg(x: float) -> float:
    return x * math.pi / 180.0


def _layers_by_fraction(nz: int, fractions: Sequence[float]) -> Tuple[int, ...]:
    """Split nz intervals bottom to top by fractions, interfaces at round(nz * cumsum)."""
    edges = [0]
    acc = 0.0
    for f in fractions[:-1]:
        acc += f
        edges.append(int(round(nz * acc)))
    edges.append(nz)
    return tuple(int(edges[i + 1] - edges[i]) for i in range(len(fractions)))


# -- the five benchmark workloads ------------------------------------------------------

def vacuum_1x1x05() -> Workload:
    """1 x 1 x 0.5 lambda vacuum cavity, 16 x 16 x 8 grid, normal TE incidence."""
    cav = Cavity(1.0, 1.0, 0.5, 16, 16, 8, (8,), (1.0 + 0j,))
    return Workload("vacuum_1x1x0.5_16x16x8", cav, (Incidence(0.0, 0.0, TE),))


def lossy_8x8x2() -> Workload:
    """8 x 8 x 2 lambda cavity filled with eps_r = 4+1i, 256 x 256 x 64 grid (h = lambda/32)."""
    cav = Cavity(8.0, 8.0, 2.0, 256, 256, 64, (64,), (4.0 + 1.0j,))
    inc = (Incidence(deg(30), deg(45), TM), Incidence(deg(30), deg(45), TE))
    return Workload("lossy_8x8x2_256x256x64", cav, inc)


THREE_LAYER_EPS = (4.0 + 1.0j, 2.5 + 0.5j, 1.0 + 0.0j)


def layered_16x16x4() -> Workload:
    """16 x 16 x 4 lambda cavity, three layers (25 / 50 / 25 %), 512 x 512 x 128 grid."""
    nz = 128
    cav = Cavity(16.0, 16.0, 4.0, 512, 512, nz, _layers_by_fraction(nz, (0.25, 0.5, 0.25)),
                 THREE_LAYER_EPS)
    inc = (Incidence(deg(45), 0.0, TM), Incidence(deg(45), 0.0, TE))
    return Workload("layered_16x16x4_512x512x128", cav, inc)


def batched_layered_8x8x2() -> Workload:
    """8 x 8 x 2 lambda three-layer cavity, 256 x 256 x 64 grid, 128 right-hand sides:
    theta on linspace(0, 80 deg, 8) x phi = 0:45:315 deg x {TM, TE}."""
    nz = 64
    cav = Cavity(8.0, 8.0, 2.0, 256, 256, nz, _layers_by_fraction(nz, (0.25, 0.5, 0.25)),
                 THREE_LAYER_EPS)
    inc = []
    for th in np.linspace(0.0, deg(80), 8):
        for ph in range(0, 360, 45):
            for pol in (TM, TE):
                inc.append(Incidence(float(th), deg(ph), pol))
    return Workload("batched_layered_8x8x2_256x256x64_x128", cav, tuple(inc), tol=1e-10,
                    batch=32)


# -- backscatter RCS sweeps on the geometries of the paper's numerical examples ---------
# (Section 7: phi = 0, theta stepped by 0.5 degrees, both polarisations; the mode counts
# and z-partition counts of its timing tables).

def _sweep(n_theta: int) -> Tuple[Incidence, ...]:
    return tuple(Incidence(deg(0.5 * i), 0.0, pol) for i in range(n_theta) for pol in (TM, TE))


def example1_sweep() -> Workload:
    """Example 1: 10 x 10 x 30 wavelength cavity, homogeneous (vacuum), M = N = 15
    (16 x 16 nodes), 1000 z-intervals, 100 angles x 2 polarisations."""
    cav = Cavity(10.0, 10.0, 30.0, 16, 16, 1000, (1000,), (1.0 + 0j,))
    return Workload("example1_sweep_10x10x30_16x16x1000", cav, _sweep(100), batch=32,
                    fields=False)


def example1_sweep_m21() -> Workload:
    """Example 1, the same cavity with the table's larger mode count M = N = 21 (22 x 22
    nodes; the sine/cosine transforms have length 44 = 4 x 11)."""
    cav = Cavity(10.0, 10.0, 30.0, 22, 22, 1000, (1000,), (1.0 + 0j,))
    return Workload("example1_sweep_10x10x30_22x22x1000", cav, _sweep(100), batch=32,
                    fields=False)


def example1_small_sweep() -> Workload:
    """Example 1, second cavity: 1 x 1 x 3 wavelengths, vacuum, M = N = 21, 1000
    z-intervals, 100 angles x 2 polarisations."""
    cav = Cavity(1.0, 1.0, 3.0, 22, 22, 1000, (1000,), (1.0 + 0j,))
    return Workload("example1_sweep_1x1x3_22x22x1000", cav, _sweep(100), batch=32,
                    fields=False)


def example2_sweep() -> Workload:
    """Example 2: 1 x 0.25 x 0.25 wavelength cavity, eps_r = 7 + 1.5i, M = N = 15,
    1000 z-intervals, 180 angles x 2 polarisations."""
    cav = Cavity(1.0, 0.25, 0.25, 16, 16, 1000, (1000,), (7.0 + 1.5j,))
    return Workload("example2_sweep_1x0.25x0.25_16x16x1000", cav, _sweep(180), batch=32,
                    fields=False)


def example3_sweep() -> Workload:
    """Example 3: 1 x 1 x 3 wavelength cavity, bottom layer 2 wavelengths of
    eps_r = 3 + 0.05i, top layer 1 wavelength of eps_r = 7 + 1.5i (one h: 2000 + 1000
    intervals), M = N = 21 (22 x 22 nodes), 180 angles x 2 polarisations."""
    cav = Cavity(1.0, 1.0, 3.0, 22, 22, 3000, (2000, 1000), (3.0 + 0.05j, 7.0 + 1.5j))
    return Workload("example3_sweep_1x1x3_22x22x3000", cav, _sweep(180), batch=32,
                    fields=False)


def example3_sweep_steps() -> Workload:
    """Example 3 with the other reading of its interval counts: the 2-wavelength bottom
    layer with 1000 intervals (h = 1/500) and the 1-wavelength top layer with 2000
    (h = 1/2000), each layer with its own step."""
    cav = Cavity(1.0, 1.0, 3.0, 22, 22, 3000, (1000, 2000), (3.0 + 0.05j, 7.0 + 1.5j),
                 layer_depth=(2.0, 1.0))
    return Workload("example3_sweep_steps_1x1x3_22x22x1000+2000", cav, _sweep(180), batch=32,
                    fields=False)


@dataclasses.dataclass(frozen=True)
class Request:
    arrival_s: float
    workload: Workload


def served_stream(n_requests: int = 2000, seed: int = 200801966,
                  rate_per_s: float = 40.0) -> List[Request]:
    """Poisson arrivals of single-incidence requests on random cavities.

    Draw order: first all inter-arrival gaps, then per request side, depth factor,
    number of layers, per-layer (Re eps, Im eps), theta, phi, polarisation.  Grid at
    lambda/32; layer interfaces at round(Nz * i / L)."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_per_s, size=n_requests)
    t = np.cumsum(gaps)
    out = []
    for i in range(n_requests):
        side = float(rng.choice([2.0, 4.0, 8.0, 12.0]))
        depth = float(rng.choice([0.25, 0.5])) * side
        n_layers = int(rng.integers(1, 4))
        eps = []
        for _ in range(n_layers):
            re = float(rng.uniform(1.0, 6.0))
            im = float(rng.uniform(0.0, 2.0))
            eps.append(complex(re, im))
        theta = float(rng.uniform(0.0, deg(80)))
        phi = float(rng.uniform(0.0, TWO_PI))
        pol = int(rng.integers(0, 2))
        nxy = int(round(side * 32))
        nz = int(round(depth * 32))
        cav = Cavity(side, side, depth, nxy, nxy, nz,
                     _layers_by_fraction(nz, [1.0 / n_layers] * n_layers), tuple(eps))
        out.append(Request(float(t[i]), Workload(f"req{i}", cav, (Incidence(theta, phi, pol),))))
    return out


# -- small parity cases: several tiles, ragged (non power-of-two) sizes ---------------

def small_cases() -> List[Workload]:
    cases = [
        vacuum_1x1x05(),
        Workload("ragged_rect_1.5x1x0.4_24x12x10_2layer",
                 Cavity(1.5, 1.0, 0.4, 24, 12, 10, (3, 7), (2.0 + 0.3j, 1.0 + 0j)),
                 (Incidence(deg(35), deg(20), TM), Incidence(deg(35), deg(20), TE))),
        Workload("lossy_2x1.25x0.5_40x30x13_3layer",
                 Cavity(2.0, 1.25, 0.5, 40, 30, 13, (4, 5, 4),
                        (4.0 + 1.0j, 2.5 + 0.5j, 1.0 + 0j)),
                 (Incidence(deg(60), deg(130), TM), Incidence(deg(10), deg(300), TE))),
        Workload("thin_layers_1x1x0.25_20x20x9_4layer",
                 Cavity(1.0, 1.0, 0.25, 20, 20, 9, (1, 2, 1, 5),
                        (3.0 + 0.2j, 1.5 + 0.0j, 5.0 + 2.0j, 1.0 + 0j)),
                 (Incidence(deg(45), deg(0), TE),)),
        Workload("steps_1.2x1x0.5_24x20x12_2layer",
                 Cavity(1.2, 1.0, 0.5, 24, 20, 12, (4, 8), (4.0 + 1.0j, 1.0 + 0j),
                        layer_depth=(0.3, 0.2)),
                 (Incidence(deg(40), deg(75), TM), Incidence(deg(40), deg(75), TE))),
        # node counts with the prime factors 7 and 13 (transform lengths 28 and 52)
        Workload("primes_1.4x1.3x0.45_14x26x9_2layer",
                 Cavity(1.4, 1.3, 0.45, 14, 26, 9, (3, 6), (3.0 + 0.5j, 1.0 + 0j)),
                 (Incidence(deg(25), deg(200), TM), Incidence(deg(55), deg(10), TE))),
        # the paper's M = 21 (22 nodes, length 44 = 4 x 11) and 11 nodes along y
        Workload("primes_1.1x0.9x0.3_22x11x7",
                 Cavity(1.1, 0.9, 0.3, 22, 11, 7, (7,), (2.0 + 0.2j,)),
                 (Incidence(deg(70), deg(300), TE),)),
    ]
    return cases


def by_name(name: str) -> Workload:
    table = {w.name: w for w in [vacuum_1x1x05(), lossy_8x8x2(), layered_16x16x4(),
                                 batched_layered_8x8x2(), example1_sweep(), example1_sweep_m21(),
                                 example1_small_sweep(), example2_sweep(), example3_sweep(),
                                 example3_sweep_steps()] + small_cases()}
    return table[name]
