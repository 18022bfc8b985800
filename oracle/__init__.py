"""ORACLE -- test infrastructure only.

Plain binary64 CPU evaluations of the scattering self-energies of Ziogas et
al. (SC'19, Sec. 2), written out as their definitions: the electron
self-energy of Eq. (3) (``sse_oracle.c``), the phonon self-energy of Eqs. (4)
and (5) (``pi_oracle.c``), the combination of the phonon Green's function
blocks that Eq. (3) consumes, and the retarded components.  Only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import this package; the product library never does, and the two share no
code.  Parity of every function here is pinned by ``tests/test_oracle_pins.py``
against closed forms, symmetry invariants, textbook reductions and brute
force on tiny inputs.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(_HERE, "libsse_oracle.so")
SRC = os.path.join(_HERE, "sse_oracle.c")


PI_LIB = os.path.join(_HERE, "libpi_oracle.so")
PI_SRC = os.path.join(_HERE, "pi_oracle.c")


def build(src: str = None, out: str = None) -> str:
    """Compile an oracle source with gcc: -O2, OpenMP over output blocks, no FMA
    contraction.  Without arguments both oracles are built."""
    if src is None:
        build(PI_SRC, PI_LIB)
        src, out = SRC, LIB
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-o", out + ".tmp", src]
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


_libs: dict = {}


def _lib(path: str = LIB):
    if path not in _libs:
        if path in (LIB, PI_LIB) and not os.path.exists(path):
            build(SRC if path == LIB else PI_SRC, path)
        L = ctypes.CDLL(path)
        c = ctypes
        if hasattr(L, "sse_oracle"):
            L.sse_oracle.argtypes = [c.c_int] * 8 + [c.c_void_p] * 6 + [c.c_double, c.c_double,
                                                                       c.c_int64, c.c_void_p,
                                                                       c.c_void_p, c.c_int]
            L.sse_oracle.restype = c.c_int
        if hasattr(L, "pi_oracle"):
            L.pi_oracle.argtypes = [c.c_int] * 8 + [c.c_void_p] * 6 + [c.c_double, c.c_double,
                                                                     c.c_int64, c.c_void_p,
                                                                     c.c_void_p, c.c_int]
            L.pi_oracle.restype = c.c_int
        _libs[path] = L
    return _libs[path]


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def sigma(neigh, dH, G, D, shift, Nkz: int, NE: int, alpha=1j, blocks=None, gslot=None,
          nthreads: int = 0, lib: str = LIB) -> np.ndarray:
    """Sigma[k, e, a] of Eq. (3).

    neigh int32 [NA, NB]; dH float64 [NA, NB, N3D, Norb, Norb];
    D complex [Nqz, Nw, NA, NB, N3D, N3D]; shift int32 [Nw] (energy index shift
    of frequency w); G complex, either the full [Nkz, NE, NA, Norb, Norb] tensor
    (gslot None) or a stack of blocks [n, Norb, Norb] with gslot int64
    [Nkz * NE * NA] giving each block's position (-1 = not supplied).
    blocks: None (every output block; result [Nkz, NE, NA, Norb, Norb]) or an
    int array [n, 3] of (k, e, a) (result [n, Norb, Norb]).
    """
    neigh = np.ascontiguousarray(neigh, dtype=np.int32)
    dH = np.ascontiguousarray(dH, dtype=np.float64)
    G = np.ascontiguousarray(G, dtype=np.complex128)
    D = np.ascontiguousarray(D, dtype=np.complex128)
    shift = np.ascontiguousarray(shift, dtype=np.int32)
    NA, NB, N3D, Norb, _ = dH.shape
    Nqz, Nw = D.shape[0], D.shape[1]
    assert neigh.shape == (NA, NB) and D.shape == (Nqz, Nw, NA, NB, N3D, N3D)
    assert shift.shape == (Nw,)
    if gslot is None:
        assert G.shape == (Nkz, NE, NA, Norb, Norb)
    else:
        gslot = np.ascontiguousarray(gslot, dtype=np.int64)
        assert gslot.shape == (Nkz * NE * NA,)
    if blocks is None:
        out = np.empty((Nkz, NE, NA, Norb, Norb), dtype=np.complex128)
        blk, nblk = None, Nkz * NE * NA
    else:
        blk = np.ascontiguousarray(np.asarray(blocks, dtype=np.int32).reshape(-1, 3))
        nblk = blk.shape[0]
        out = np.empty((nblk, Norb, Norb), dtype=np.complex128)
    alpha = complex(alpha)
    rc = _lib(lib).sse_oracle(NA, NB, Norb, N3D, Nkz, Nqz, NE, Nw, _p(shift), _p(neigh), _p(dH),
                              _p(G), _p(gslot), _p(D), alpha.real, alpha.imag, nblk, _p(blk),
                              _p(out), nthreads)
    if rc == 1:
        raise ValueError("oracle: index out of range (neighbour table or block list)")
    if rc == 2:
        raise ValueError("oracle: a needed G block was not supplied")
    return out


def needed_g_blocks(neigh, shift, Nkz: int, Nqz: int, NE: int, NA: int, blocks) -> np.ndarray:
    """Flat indices (k * NE + e) * NA + f of every G block that the listed output
    blocks read (bookkeeping for sampled evaluation; no arithmetic of Eq. (3))."""
    blocks = np.asarray(blocks, dtype=np.int64).reshape(-1, 3)
    shift = np.asarray(shift, dtype=np.int64)
    need = set()
    for k, e, a in blocks:
        for f in neigh[a]:
            for q in range(Nqz):
                kk = (k - q) % Nkz
                for s in shift:
                    ee = e - s
                    if 0 <= ee < NE:
                        need.add((kk * NE + ee) * NA + int(f))
    return np.array(sorted(need), dtype=np.int64)


def pi(neigh, dH, X, Y, shift, Nkz: int, Nqz: int, NE: int, beta=1j, blocks=None, gslot=None,
       nthreads: int = 0, lib: str = PI_LIB) -> np.ndarray:
    """Pi[q, w, a] of Eqs. (4) and (5): NB neighbour blocks and, in slot NB, the
    diagonal block, each N3D x N3D.

    X, Y: the two opposite components of the electron Green's function -- Pi<
    takes X = G<, Y = G>; Pi> takes X = G>, Y = G< -- each either a full
    [Nkz, NE, NA, Norb, Norb] tensor (gslot None) or a stack of blocks with
    gslot int64 [Nkz * NE * NA] giving each block's slot in both stacks.
    neigh int32 [NA, NB]; dH float64 [NA, NB, N3D, Norb, Norb]; shift int32 [Nw].
    blocks: None (result [Nqz, Nw, NA, NB + 1, N3D, N3D]) or an int array [n, 3]
    of (q, w, a) (result [n, NB + 1, N3D, N3D]).
    """
    neigh = np.ascontiguousarray(neigh, dtype=np.int32)
    dH = np.ascontiguousarray(dH, dtype=np.float64)
    X = np.ascontiguousarray(X, dtype=np.complex128)
    Y = np.ascontiguousarray(Y, dtype=np.complex128)
    shift = np.ascontiguousarray(shift, dtype=np.int32)
    NA, NB, N3D, Norb, _ = dH.shape
    Nw = shift.size
    assert neigh.shape == (NA, NB) and X.shape == Y.shape
    if gslot is None:
        assert X.shape == (Nkz, NE, NA, Norb, Norb)
    else:
        gslot = np.ascontiguousarray(gslot, dtype=np.int64)
        assert gslot.shape == (Nkz * NE * NA,)
    if blocks is None:
        out = np.empty((Nqz, Nw, NA, NB + 1, N3D, N3D), dtype=np.complex128)
        blk, nblk = None, Nqz * Nw * NA
    else:
        blk = np.ascontiguousarray(np.asarray(blocks, dtype=np.int32).reshape(-1, 3))
        nblk = blk.shape[0]
        out = np.empty((nblk, NB + 1, N3D, N3D), dtype=np.complex128)
    beta = complex(beta)
    rc = _lib(lib).pi_oracle(NA, NB, Norb, N3D, Nkz, Nqz, NE, Nw, _p(shift), _p(neigh), _p(dH),
                             _p(X), _p(Y), _p(gslot), beta.real, beta.imag, nblk, _p(blk),
                             _p(out), nthreads)
    if rc == 1:
        raise ValueError("oracle: index out of range (neighbour table or block list)")
    if rc == 2:
        raise ValueError("oracle: a needed G block was not supplied")
    return out


def needed_g_blocks_pi(neigh, shift, Nkz: int, NE: int, NA: int, blocks) -> np.ndarray:
    """Flat indices (k * NE + e) * NA + atom of every G block that the listed
    (q, w, a) blocks of Pi read, in either component (bookkeeping for sampled
    evaluation; no arithmetic of Eqs. (4)-(5))."""
    blocks = np.asarray(blocks, dtype=np.int64).reshape(-1, 3)
    shift = np.asarray(shift, dtype=np.int64)
    need = set()
    for q, w, a in blocks:
        s = int(shift[w])
        for k in range(Nkz):
            kk = (k + q) % Nkz
            for e in range(NE):
                ee = e + s
                if 0 <= ee < NE:
                    need.add((kk * NE + ee) * NA + int(a))
                    for f in neigh[a]:
                        need.add((k * NE + e) * NA + int(f))
    return np.array(sorted(need), dtype=np.int64)


def dtilde(D, neigh) -> np.ndarray:
    """The combination of phonon Green's function blocks that Eq. (3) sums over
    (Sec. 2, below Eq. (3); Sec. 4.2 names it as the kernel's input):

        Dt[q, w, a, b, i, j] = D_ba - D_bb - D_aa + D_ab   (each at (i, j))

    with D [Nqz, Nw, NA, NB + 1, N3D, N3D] holding, per atom a, the blocks
    D_a,neigh[a, b] in slots b < NB and the diagonal block D_aa in slot NB.
    For f = neigh[a, b]: D_ab = D[.., a, b], D_bb = D[.., f, NB], D_aa =
    D[.., a, NB], and D_ba = D[.., f, r] where r is the slot of a in f's row of
    the neighbour table (the table must be symmetric: ValueError otherwise).
    The sum is formed left to right as written."""
    D = np.asarray(D, dtype=np.complex128)
    neigh = np.asarray(neigh)
    Nqz, Nw, NA, NB1 = D.shape[:4]
    NB = NB1 - 1
    assert neigh.shape == (NA, NB)
    out = np.empty((Nqz, Nw, NA, NB) + D.shape[4:], dtype=np.complex128)
    for a in range(NA):
        for b in range(NB):
            f = int(neigh[a, b])
            slots = [r for r in range(NB) if int(neigh[f, r]) == a]
            if not slots:
                raise ValueError(f"atom {a} is not a neighbour of its neighbour {f}")
            r = slots[0]
            out[:, :, a, b] = D[:, :, f, r] - D[:, :, f, NB] - D[:, :, a, NB] + D[:, :, a, b]
    return out


def retarded(lesser, greater) -> np.ndarray:
    """The retarded component from the lesser and greater ones (Sec. 2, after
    Eq. (5); the same relation for Sigma and Pi): (X> - X<) / 2, elementwise."""
    return (np.asarray(greater, dtype=np.complex128) - np.asarray(lesser, dtype=np.complex128)) / 2
