"""Problem sizes of the workloads (shapes only).

Ranges follow the paper's table of typical simulation parameters (Sec. 2):
Nkz, Nqz in [1, 21], NE in [700, 1500], Nw in [10, 100], NB in [4, 50],
Norb in [1, 30], N3D = 3.  The frequency grid is uniform with the energy grid:
phonon frequency index w shifts the energy index by s_w = w + 1.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass(frozen=True)
class Problem:
    NA: int
    NB: int
    Norb: int
    Nkz: int
    Nqz: int
    NE: int
    Nw: int
    N3D: int = 3
    shift: tuple = field(default=None)

    def shifts(self) -> np.ndarray:
        if self.shift is not None:
            return np.asarray(self.shift, dtype=np.int32)
        return np.arange(1, self.Nw + 1, dtype=np.int32)

    @property
    def NN(self) -> int:
        return self.Norb * self.Norb

    def g_elems(self) -> int:
        return self.Nkz * self.NE * self.NA * self.NN

    def d_elems(self) -> int:
        return self.Nqz * self.Nw * self.NA * self.NB * self.N3D * self.N3D

    def flops_corr(self) -> int:
        """Tap work: 9 complex scalar filters over Norb^2 channels, per
        (k, e, q, w, a, b): 8 * N3D^2 * Norb^2 real flops."""
        return 8 * self.N3D ** 2 * self.NN * self.Nkz * self.Nqz * self.NE * self.Nw * \
            self.NA * self.NB

    def flops_sandwich(self) -> int:
        """dH sandwich per (k, e, a, b): 4 N3D^2 Norb^3 (left products, real x
        complex) + 4 N3D Norb^3 (right products)."""
        return (4 * self.N3D ** 2 + 4 * self.N3D) * self.Norb ** 3 * self.Nkz * self.NE * \
            self.NA * self.NB

    def flops(self, antiherm: bool = False) -> int:
        """Algorithmic flops of one component in the reassociated form; with an
        anti-Hermitian D~ (D~_ji = -conj(D~_ij)) the tap work halves: three
        complex filters split into real and imaginary parts (4 real x complex
        products) plus three imaginary diagonals, 4.5 complex filters in all."""
        corr = self.flops_corr() // 2 if antiherm else self.flops_corr()
        return corr + self.flops_sandwich()

    def flops_plain(self) -> int:
        """Flops of the plain definition as the oracle evaluates it: per (k, e, q,
        w, a, b) and each of the 9 (i, j) pairs, two Norb^3 real x complex
        products (4 Norb^3 flops each) and one complex scale-add of Norb^2
        elements (8 Norb^2)."""
        return 9 * (8 * self.Norb ** 3 + 8 * self.NN) * self.Nkz * self.Nqz * self.NE * \
            self.Nw * self.NA * self.NB

    def flops_paper_form(self) -> int:
        """Flops of the paper's own final form (Sec. 4.2; its published flop
        formula divided by the four of {Sigma, Pi} x {<, >}): 8 N3D Norb^3 per
        (k, e, q, w, a, b) for the Norb x Norb Nw x Norb GEMMs plus 8 N3D Norb^3 per
        (k, e, a, b) for the dH G products."""
        pts = self.Nkz * self.NE * self.NA * self.NB
        return 8 * self.N3D * self.Norb ** 3 * pts * (self.Nqz * self.Nw + 1)

    def bytes_compulsory(self, elem_bytes: int = 16) -> int:
        """Read G, D~, dH and neigh once; write Sigma once (one component)."""
        return (2 * self.g_elems() + self.d_elems()) * elem_bytes + \
            self.NA * self.NB * self.N3D * self.NN * 8 + self.NA * self.NB * 4


# CPU-scale plain configuration (full oracle in well under a second).
SMALL = Problem(NA=16, NB=4, Norb=4, Nkz=3, Nqz=3, NE=64, Nw=4)
# Device-scale plain configuration: Sigma of shape [7, 1000, 1024, 10, 10].
DEVICE = Problem(NA=1024, NB=4, Norb=10, Nkz=7, Nqz=7, NE=1000, Nw=30)
SEED = 1912


def batch_instances(seed: int = SEED, n: int = 48):
    """Uneven instances: NA ~ U{64..2048}, NE ~ U{200..1500}, Nw ~ U{10..40},
    Norb = 10, NB = 4, Nkz = Nqz = 5 (seeded)."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        out.append(Problem(NA=int(rng.integers(64, 2049)), NB=4, Norb=10, Nkz=5, Nqz=5,
                           NE=int(rng.integers(200, 1501)), Nw=int(rng.integers(10, 41))))
    return out


def small_instances(seed: int = SEED, n: int = 24):
    """Small serving jobs that do not fill the GPU: NA ~ U{64..160}, NE ~ U{200..320},
    Nw ~ U{10..20}, Norb = 10, NB = 4, Nkz = Nqz = 5 (seeded)."""
    rng = np.random.default_rng(seed)
    return [Problem(NA=int(rng.integers(64, 161)), NB=4, Norb=10, Nkz=5, Nqz=5,
                    NE=int(rng.integers(200, 321)), Nw=int(rng.integers(10, 21)))
            for _ in range(n)]


def tiny_instances(seed: int = SEED, n: int = 48):
    """Jobs with fewer output tiles than the GPU has compute units (one job alone
    leaves most of the GPU idle): NA ~ U{8..16}, NE ~ U{30..60}, Nw ~ U{4..10},
    Norb = 10, NB = 4, Nkz = Nqz = 3 (seeded)."""
    rng = np.random.default_rng(seed)
    return [Problem(NA=int(rng.integers(8, 17)), NB=4, Norb=10, Nkz=3, Nqz=3,
                    NE=int(rng.integers(30, 61)), Nw=int(rng.integers(4, 11)))
            for _ in range(n)]
