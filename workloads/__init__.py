"""Seeded synthetic workloads shared by the tests, the benchmark and the smoke
check.  This module holds input generators and size presets only -- none of
the method's arithmetic -- so both the HIP path and the CPU oracle may consume
what it produces.

Random (h, g) draws use SplitMix64 (Steele, Lea & Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014): u_j(k) is the top 53 bits of
the SplitMix64 output for state 2k + j, scaled to [0, 1).
"""
from dataclasses import dataclass
from typing import List

MASK64 = (1 << 64) - 1


def splitmix64(state: int) -> int:
    """One SplitMix64 output for the given 64-bit state."""
    z = (state + 0x9E3779B97F4A7C15) & MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def u01(k: int, j: int) -> float:
    return (splitmix64(2 * k + j) >> 11) * (1.0 / (1 << 53))


@dataclass(frozen=True)
class Job:
    h: float
    g: float
    seed: int


# Wall-lattice-snapped periodic extents.  With wall density 1 the FCC cube is
# 4^(1/3) = 1.5874 sigma; the nominal extent is rounded to whole cubes.
BOX_SMALL = 20.636   # 13 cubes: the 2,048-atom h = 6 channel at density 0.8
BOX_SMALL_LITERAL = 12.0  # 8 cubes: the literal 12 x 12 box (774 atoms)
BOX_LARGE = 57.146   # 36 cubes: ~39k atoms at h = 15, and the batch box
BOX_LARGE_LITERAL = 40.0  # 25 cubes: the literal 40 x 40 box


def small_channel():
    """2,048 fluid atoms, h = 6, g = 0.02, 1,000 steps."""
    return dict(Lx_nom=BOX_SMALL, Lz_nom=BOX_SMALL, n_fluid=2048), Job(6.0, 0.02, 0), 1000


def paper_scale_channel():
    """h = 15 in the 57 x 57 box (39,189 atoms); g = 0.001 + 0.049 u_1(0);
    20,000 equilibration + 50,000 sampling steps."""
    return dict(Lx_nom=BOX_LARGE, Lz_nom=BOX_LARGE), Job(15.0, 0.001 + 0.049 * u01(0, 1), 0), (20000, 50000)


def batch_jobs(n: int = 64, first: int = 0) -> List[Job]:
    """Uneven batch: h_k = 4 + 16 u_0(k), g_k = 0.001 + 0.049 u_1(k), seed k."""
    return [Job(4.0 + 16.0 * u01(k, 0), 0.001 + 0.049 * u01(k, 1), k) for k in range(first, first + n)]


def batch_box():
    return dict(Lx_nom=BOX_LARGE, Lz_nom=BOX_LARGE)


def surrogate_training_jobs(n_train: int = 256, n_test: int = 64):
    """Training (seeds 0..255) and held-out (seeds 256..319) draws for the
    learned surrogate, with the batch protocol."""
    return batch_jobs(n_train, 0), batch_jobs(n_test, n_train)


@dataclass(frozen=True)
class Job3:
    h: float
    rho: float
    g: float
    seed: int


def u3(k: int, j: int) -> float:
    """Three independent draws per index k (j = 0, 1, 2) for the 3-input
    workloads: SplitMix64 state 2^40 + 3k + j, clear of the 2k + j states
    of u01 for every k below 2^38."""
    return (splitmix64((1 << 40) + 3 * k + j) >> 11) * (1.0 / (1 << 53))


def density_jobs(n: int, first: int, h_lo: float, h_hi: float, rho_lo: float, rho_hi: float,
                 g_lo: float, g_hi: float) -> List[Job3]:
    """(h, rho, g) draws for the flux database of the 3-input surrogate:
    uniform in each range, seed 100000 + k."""
    return [Job3(h_lo + (h_hi - h_lo) * u3(k, 0), rho_lo + (rho_hi - rho_lo) * u3(k, 1),
                 g_lo + (g_hi - g_lo) * u3(k, 2), 100000 + k) for k in range(first, first + n)]
