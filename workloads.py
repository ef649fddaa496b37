"""Seeded synthetic workloads for the peridynamic beam solves.

This module holds data only: beam geometry, material constants, loading
schedules and the seeded standard-normal Karhunen-Loeve coefficients that the
random material field is built from.  It contains none of the solver's
arithmetic (no stiffness, critical stretch, damage law, field synthesis or
time stepping), so both the product library and the reference oracle can use
it without sharing any computation.

Units are SI throughout (m, kg, s, N, Pa).

The beam is the notched three-point-bending concrete specimen used for the
MC/MLMC solves (paper section 6, case study set-up; the numbers below are the
synthetic 3D stand-in for the paper's 2D specimen):

* length (x) 175 mm, thickness (y) 50 mm, depth (z) 50 mm, span 150 mm;
* a 5 mm deep notch at mid-span on the bottom face, through the thickness;
* two 5 mm support pads on the bottom face and one 5 mm load pad on top;
* E = 37 GPa, rho = 2346 kg/m^3 (section 6.2), G_F = 140 N/m,
  k = 25, alpha = 0.25 (section 6.2), horizon delta = 3.14 dx (section 6.2);
* tensile strength from the mean cylinder strength 42.3 MPa (section 6.2)
  through the usual f_t = 0.3 (f_cm - 8)^(2/3) MPa relation; the paper cites
  the fib Model Code for this map without printing it.

Levels follow the paper's uniform refinement (dx halves per level, figure of
nested meshes in section 4.2).  The time step, step count and displacement
increment scale with dx so every level sees the same load-time history at the
same fraction of its stability limit.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
from typing import List, Optional

import numpy as np

MM = 1.0e-3

# ---------------------------------------------------------------- material
E_MODULUS = 37.0e9          # Pa
DENSITY = 2346.0            # kg/m^3
FRACTURE_ENERGY = 140.0     # N/m  (0.14 N/mm)
F_CM = 42.3e6               # Pa, mean cylinder compressive strength
F_T = 0.3 * ((F_CM / 1e6) - 8.0) ** (2.0 / 3.0) * 1e6  # Pa, tensile strength
S0_MEAN = F_T / E_MODULUS   # linear elastic limit stretch
SOFT_K = 25.0
SOFT_ALPHA = 0.25
M_RATIO = 3.14              # delta / dx
DAMPING = 1.0e5             # kg m^-3 s^-1

LAW_EXPLIN = 0              # exponential + linear softening (appendix A)
LAW_TRILINEAR = 1           # piecewise-linear softening envelope


@dataclass(frozen=True)
class Material:
    """The homogeneous material values a level carries to the solver's
    parameter block (the constants above, as one record)."""
    E: float = E_MODULUS
    rho: float = DENSITY
    GF: float = FRACTURE_ENERGY
    s0: float = S0_MEAN
    k: float = SOFT_K
    alpha: float = SOFT_ALPHA
    damping: float = DAMPING


CONCRETE = Material()

# ---------------------------------------------------------------- loading
DT_L0 = 1.0e-6              # s at dx = 5 mm
STEPS_L0 = 4000
DU_LITERAL_L0 = 5.0e-11     # m per step at dx = 5 mm (5e-8 mm)
DU_FRACTURE_L0 = 2.0e-8     # m per step at dx = 5 mm (400x: peak load mid-run)

# ---------------------------------------------------------------- random field
FIELD_COV = 0.2
FIELD_CORR_LEN = 20.0 * MM
FIELD_MODES = 50


@dataclass(frozen=True)
class Beam:
    """Geometry of a notched three-point-bending beam (SI)."""
    length: float = 175.0 * MM      # x
    thickness: float = 50.0 * MM    # y
    depth: float = 50.0 * MM        # z
    span: float = 150.0 * MM
    notch_depth: float = 5.0 * MM
    pad_width: float = 5.0 * MM
    plane: bool = False             # plane body: one node through the thickness
    plane_strain: bool = False      # with plane: plane strain instead of plane stress

    @staticmethod
    def similar(depth: float) -> "Beam":
        """Size-effect family: length 3.5 D, span 3 D, thickness 50 mm,
        notch 0.2 D, pads D/10."""
        return Beam(length=3.5 * depth, thickness=50.0 * MM, depth=depth,
                    span=3.0 * depth, notch_depth=0.2 * depth,
                    pad_width=depth / 10.0)


@dataclass(frozen=True)
class Level:
    """One resolution of the beam and its time-stepping schedule."""
    beam: Beam
    dx: float
    dt: float
    n_steps: int
    du: float                 # prescribed load-pad displacement per step (m)
    law: int = LAW_TRILINEAR
    material: Material = CONCRETE

    @property
    def shape(self):
        t = self.dx if self.beam.plane else self.beam.thickness
        return tuple(int(round(L / self.dx)) for L in (self.beam.length, t, self.beam.depth))


def level(ell: int, fracture: bool = False, beam: Beam = Beam(),
          law: int = LAW_TRILINEAR, steps_scale: float = 1.0) -> Level:
    """Level ell of the hierarchy: dx = 5 mm / 2^ell with dt, steps and the
    displacement increment scaled with dx."""
    r = 2 ** ell
    du0 = DU_FRACTURE_L0 if fracture else DU_LITERAL_L0
    return Level(beam=beam, dx=5.0 * MM / r, dt=DT_L0 / r,
                 n_steps=int(round(STEPS_L0 * r * steps_scale)),
                 du=du0 / r, law=law)


@dataclass(frozen=True)
class Config:
    name: str
    levels: List[Level]
    samples: List[int]        # samples per level
    seed: int
    precision: str            # "f32" or "f64"
    random_field: bool


# ---------------------------------------------------------------- plane stress
# Specimen 3 of section 6.2 as the paper models it: a 2D plane-stress body,
# 350 x 100 mm, 50 mm thick, span 250 mm, half-notched; levels dx = 10 / 5 /
# 2.5 / 1.25 / 0.625 mm (Table discretisation: 350 ... 89,600 nodes).
SPECIMEN3 = Beam(length=350.0 * MM, thickness=50.0 * MM, depth=100.0 * MM, span=250.0 * MM,
                 notch_depth=50.0 * MM, pad_width=12.0 * MM, plane=True)
DT_2D_L0 = 2.0e-6           # s at dx = 10 mm (0.67 of the 2D stability limit)
STEPS_2D_L0 = 2000
DU_2D_L0 = 5.0e-8           # m per step at dx = 10 mm (peak load mid-run)


# The unnotched Specimen 3 of section 6.3 (case study 2, lambda = 0).
SPECIMEN3_UNNOTCHED = replace(SPECIMEN3, notch_depth=0.0)


def level2d(ell: int, law: int = LAW_TRILINEAR, steps_scale: float = 1.0, notched: bool = True) -> Level:
    """Level ell of the plane-stress Specimen 3 (half-notched, or unnotched
    with notched=False): dx = 10 mm / 2^ell with dt, steps and the
    displacement increment scaled with dx."""
    r = 2 ** ell
    return Level(beam=SPECIMEN3 if notched else SPECIMEN3_UNNOTCHED, dx=10.0 * MM / r, dt=DT_2D_L0 / r,
                 n_steps=int(round(STEPS_2D_L0 * r * steps_scale)), du=DU_2D_L0 / r, law=law)


def configs(fracture: bool = False) -> List[Config]:
    """The five workloads: plain FP64 single solve, the batched FP32 level-1
    batch, the three-level MLMC batch, the adjoint case and the size sweep."""
    sweep = [Level(beam=Beam.similar(D * MM), dx=2.5 * MM, dt=DT_L0 / 2,
                   n_steps=int(8000 * D / 50),
                   du=(DU_FRACTURE_L0 if fracture else DU_LITERAL_L0) / 2)
             for D in (50, 100, 200, 400)]
    return [
        Config("plain_fp64_L0", [level(0, fracture)], [1], 0, "f64", False),
        Config("batched_fp32_L1x64", [level(1, fracture)], [64], 1, "f32", True),
        Config("mlmc_L012", [level(0, fracture), level(1, fracture),
                             level(2, fracture)], [1024, 128, 16], 2, "f32", True),
        Config("adjoint_L1", [level(1, True)], [1], 3, "f64", True),
        Config("size_sweep", sweep, [32, 32, 32, 32], 4, "f32", True),
    ]


def kl_coefficients(seed: int, n_samples: int, n_modes: int = FIELD_MODES,
                    stream: int = 0) -> np.ndarray:
    """Standard-normal KL coefficients, one independent PCG64 stream per
    sample: sample i of stream s draws from SeedSequence(seed, spawn_key=(s,))
    child i.  Returns float64 [n_samples, n_modes].  A coupled fine/coarse
    pair uses the same row for both levels."""
    root = np.random.SeedSequence(seed, spawn_key=(stream,))
    kids = root.spawn(n_samples)
    out = np.empty((n_samples, n_modes), dtype=np.float64)
    for i, ss in enumerate(kids):
        out[i] = np.random.Generator(np.random.PCG64(ss)).standard_normal(n_modes)
    return out


def smooth_displacement(shape, dx: float, amplitude: float, seed: int) -> np.ndarray:
    """A smooth random displacement field sampled at the lattice nodes
    (cell centres), float64 [n_nodes, 3], x index fastest.  Used to probe a
    single force evaluation on a frozen configuration."""
    nx, ny, nz = shape
    rng = np.random.Generator(np.random.PCG64(seed))
    x = (np.arange(nx) + 0.5) * dx
    y = (np.arange(ny) + 0.5) * dx
    z = (np.arange(nz) + 0.5) * dx
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    Lx, Ly, Lz = nx * dx, ny * dx, nz * dx
    u = np.zeros((nz, ny, nx, 3))
    for comp in range(3):
        for _ in range(4):
            kx, ky, kz = rng.integers(1, 4, size=3)
            ph = rng.uniform(0, 2 * np.pi, size=3)
            a = rng.standard_normal()
            u[..., comp] += a * (np.sin(np.pi * kx * X / Lx + ph[0])
                                 * np.sin(np.pi * ky * Y / Ly + ph[1])
                                 * np.sin(np.pi * kz * Z / Lz + ph[2]))
    return (amplitude * u).reshape(-1, 3)
