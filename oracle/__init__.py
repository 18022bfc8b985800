"""ORACLE -- test infrastructure only.

Plain binary64 CPU evaluation of the electron scattering self-energy, Eq. (3)
of Ziogas et al. (SC'19, Sec. 2), written out as the definition (see
``sse_oracle.c``).  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package; the product
library never does, and the two share no code.  Parity of every function here
is pinned by ``tests/test_oracle_pins.py`` against closed forms, symmetry
invariants, textbook reductions and brute force on tiny inputs.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(_HERE, "libsse_oracle.so")
SRC = os.path.join(_HERE, "sse_oracle.c")


def build(src: str = SRC, out: str = LIB) -> str:
    """Compile the oracle with gcc: -O2, OpenMP over output blocks, no FMA contraction."""
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-o", out + ".tmp", src]
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


_libs: dict = {}


def _lib(path: str = LIB):
    if path not in _libs:
        if path == LIB and not os.path.exists(LIB):
            build()
        L = ctypes.CDLL(path)
        c = ctypes
        L.sse_oracle.argtypes = [c.c_int] * 8 + [c.c_void_p] * 6 + [c.c_double, c.c_double,
                                                                   c.c_int64, c.c_void_p,
                                                                   c.c_void_p, c.c_int]
        L.sse_oracle.restype = c.c_int
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
