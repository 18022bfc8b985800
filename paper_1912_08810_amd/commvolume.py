"""Communication volume of the SSE phase across processes (Sec. 4.1), on the CPU.

Two data distributions between the GF and SSE phases, with the per-process
byte counts of Sec. 4.1 (64 bytes = a lesser/greater pair of complex128
values):

* the momentum/energy ("natural") distribution: each of P processes receives
  64 (Nkz NE / P) Nqz Nw NA Norb^2 bytes of electron Green's functions and
  exchanges 64 Nqz Nw NA NB N3D^2 bytes of phonon Green's functions and
  self-energies;
* the atom x energy tiling of the transformed program, P = T_E T_A tiles: each
  process contributes 64 Nkz (NE / T_E + 2 Nw)(NA / T_A + NB) Norb^2 bytes for
  G and Sigma (its energy range plus the frequency halo on both sides, its
  atoms plus the neighbour halo) and 64 Nqz Nw (NA / T_A + NB) NB N3D^2 bytes
  for D and Pi.

``best_tiling`` searches every factorisation P = T_E T_A exhaustively (the
paper searches its feasible tile sizes exhaustively, Sec. 4.1).  The tables of
Sec. 5 (weak and strong scaling of the communication volume, in TiB) follow
from these formulas with T_E = Nkz, T_A = P / T_E (weak) and T_E = 7,
T_A = P / 7 (strong); the text's own statement of those tilings is garbled
(it gives T_A = 7 and T_A = 32 P / 112, neither of which multiplies with T_E
to P).
"""
from __future__ import annotations

from dataclasses import dataclass

TIB = 2.0 ** 40


@dataclass(frozen=True)
class Sizes:
    NA: int
    NB: int
    Norb: int
    Nkz: int
    Nqz: int
    NE: int
    Nw: int
    N3D: int = 3


def omen_bytes(s: Sizes, P: int) -> float:
    """Total bytes moved by the momentum/energy distribution over P processes."""
    g = 64.0 * (s.Nkz * s.NE / P) * s.Nqz * s.Nw * s.NA * s.Norb ** 2
    d = 64.0 * s.Nqz * s.Nw * s.NA * s.NB * s.N3D ** 2
    return P * (g + d)


def tiled_bytes(s: Sizes, TE: int, TA: int) -> float:
    """Total bytes of the atom x energy tiling with T_E energy and T_A atom tiles."""
    halo_a = s.NA / TA + s.NB
    g = 64.0 * s.Nkz * (s.NE / TE + 2 * s.Nw) * halo_a * s.Norb ** 2
    d = 64.0 * s.Nqz * s.Nw * halo_a * s.NB * s.N3D ** 2
    return TE * TA * (g + d)


def tilings(s: Sizes, P: int):
    """Every feasible (T_E, T_A) with T_E T_A = P, T_E <= NE, T_A <= NA."""
    return [(te, P // te) for te in range(1, P + 1)
            if P % te == 0 and te <= s.NE and P // te <= s.NA]


def best_tiling(s: Sizes, P: int):
    """(bytes, T_E, T_A) of the cheapest feasible tiling; ties go to the smaller T_E."""
    cands = tilings(s, P)
    if not cands:
        raise ValueError(f"no feasible tiling of {P} processes")
    return min((tiled_bytes(s, te, ta), te, ta) for te, ta in cands)


# The silicon structure of the paper's communication tables (Sec. 5).
SI = dict(NA=4864, NB=34, Norb=12, NE=706, Nw=70)


def weak_table():
    """Rows of the weak-scaling table: Nkz = Nqz in 3..11, P = 256 Nkz."""
    rows = []
    for nkz in (3, 5, 7, 9, 11):
        s = Sizes(Nkz=nkz, Nqz=nkz, **SI)
        P = 256 * nkz
        rows.append({"Nkz": nkz, "P": P, "omen_tib": omen_bytes(s, P) / TIB,
                     "tiled_tib": tiled_bytes(s, nkz, P // nkz) / TIB,
                     "best": best_tiling(s, P)})
    return rows


def strong_table():
    """Rows of the strong-scaling table: Nkz = Nqz = 7, P in 224..2688, T_E = 7."""
    rows = []
    s = Sizes(Nkz=7, Nqz=7, **SI)
    for P in (224, 448, 896, 1792, 2688):
        rows.append({"P": P, "omen_tib": omen_bytes(s, P) / TIB,
                     "tiled_tib": tiled_bytes(s, 7, P // 7) / TIB,
                     "best": best_tiling(s, P)})
    return rows


if __name__ == "__main__":
    for r in weak_table():
        b, te, ta = r["best"]
        print(f"weak   Nkz={r['Nkz']:2d} P={r['P']:4d}: momentum/energy {r['omen_tib']:7.2f} TiB, "
              f"tiled {r['tiled_tib']:5.2f} TiB; best T_E={te} T_A={ta} {b / TIB:5.2f} TiB")
    for r in strong_table():
        b, te, ta = r["best"]
        print(f"strong P={r['P']:4d}: momentum/energy {r['omen_tib']:7.2f} TiB, "
              f"tiled {r['tiled_tib']:5.2f} TiB; best T_E={te} T_A={ta} {b / TIB:5.2f} TiB")
