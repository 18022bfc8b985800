"""Seeded synthetic inputs for the SSE self-energy kernel.

Counter-based (Philox4x32-10) generator, implemented once in ``ssegen_core.h``
and compiled for the host (``libssegen_host.so``, gcc) and for the device
(``libssegen_device.so``, hipcc).  Both produce identical bits: every step is
integer arithmetic or exactly rounded binary64 +, -, *, /.

The inputs follow the paper's tensor statement (Sec. 2, the five- and six-
dimensional G and D tensors; Sec. 3, the typed signature of the Sigma
program): neighbour table int32 [NA, NB]; dH float64 [NA, NB, N3D, Norb, Norb];
G complex [Nkz, NE, NA, Norb, Norb]; D~ complex [Nqz, Nw, NA, NB, N3D, N3D].
Distributions: neighbours are NB distinct atoms other than a, drawn uniformly;
dH real approximately N(0,1); G and D~ blocks are (X - X^H)/2 of complex
approximately-normal X (anti-Hermitian, as lesser/greater Green's functions
are); optionally each G block is scaled by (1 + u) 2^n, n uniform in
{-20..6}, to spread magnitudes over about eight decades.

This module contains no self-energy arithmetic; it is the only code shared by
the oracle side and the GPU side.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
HOST_LIB = os.path.join(_HERE, "libssegen_host.so")
DEVICE_LIB = os.path.join(_HERE, "libssegen_device.so")

S_NEIGH, S_DH, S_G, S_GSCALE, S_D, S_PERT_G, S_PERT_D = 1, 2, 16, 24, 32, 64, 72


def build_host() -> None:
    """Compile the host generator (gcc, OpenMP, no FMA contraction)."""
    src = os.path.join(_HERE, "ssegen_host.c")
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-o", HOST_LIB + ".tmp", src, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(HOST_LIB + ".tmp", HOST_LIB)


def build_device(hipcc: str = "/opt/rocm/bin/hipcc") -> None:
    """Compile the device generator for gfx950."""
    src = os.path.join(_HERE, "ssegen_device.hip")
    cmd = [hipcc, "--offload-arch=gfx950", "-O3", "-fPIC", "-shared", "-std=c++17",
           "-ffp-contract=off", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-o", DEVICE_LIB + ".tmp", src]
    subprocess.run(cmd, check=True)
    os.replace(DEVICE_LIB + ".tmp", DEVICE_LIB)


_host = None
_dev = None


def _hostlib():
    global _host
    if _host is None:
        if not os.path.exists(HOST_LIB):
            build_host()
        L = ctypes.CDLL(HOST_LIB)
        c = ctypes
        L.ssegen_host_neigh.argtypes = [c.c_uint64, c.c_int, c.c_int, c.c_void_p]
        L.ssegen_host_neigh.restype = c.c_int
        L.ssegen_host_dH.argtypes = [c.c_uint64, c.c_int64, c.c_void_p]
        L.ssegen_host_G_blocks.argtypes = [c.c_uint64, c.c_int, c.c_int, c.c_int, c.c_int64,
                                           c.c_void_p, c.c_void_p]
        L.ssegen_host_D.argtypes = [c.c_uint64, c.c_int, c.c_int, c.c_int64, c.c_void_p]
        L.ssegen_host_perturb.argtypes = [c.c_uint64, c.c_int, c.c_uint32, c.c_int, c.c_int64,
                                          c.c_void_p, c.c_void_p]
        L.ssegen_host_philox.argtypes = [c.c_void_p, c.c_void_p, c.c_void_p]
        L.ssegen_host_normal.argtypes = [c.c_uint64, c.c_uint64, c.c_uint32]
        L.ssegen_host_normal.restype = c.c_double
        _host = L
    return _host


def _devlib():
    global _dev
    if _dev is None:
        if not os.path.exists(DEVICE_LIB):
            raise RuntimeError("libssegen_device.so is not built (run __graft_entry__.build())")
        # bind to the HIP runtime PyTorch carries (it supplies memory and streams)
        import torch  # noqa: F401
        L = ctypes.CDLL(DEVICE_LIB)
        with open("/proc/self/maps") as fh:
            rts = sorted({ln.split()[-1] for ln in fh if "libamdhip64" in ln})
        if len(rts) > 1:
            raise RuntimeError("two HIP runtimes are loaded in this process: " + ", ".join(rts))
        c = ctypes
        L.ssegen_dev_fill_dH.argtypes = [c.c_uint64, c.c_int64, c.c_void_p, c.c_void_p]
        L.ssegen_dev_fill_G.argtypes = [c.c_uint64, c.c_int, c.c_int, c.c_int64, c.c_int, c.c_int,
                                        c.c_void_p, c.c_void_p]
        L.ssegen_dev_fill_D.argtypes = [c.c_uint64, c.c_int, c.c_int, c.c_int64, c.c_int,
                                        c.c_void_p, c.c_void_p]
        L.ssegen_dev_perturb.argtypes = [c.c_uint64, c.c_int, c.c_uint32, c.c_int, c.c_int64,
                                         c.c_int, c.c_void_p, c.c_void_p]
        for f in (L.ssegen_dev_fill_dH, L.ssegen_dev_fill_G, L.ssegen_dev_fill_D,
                  L.ssegen_dev_perturb):
            f.restype = c.c_int
        _dev = L
    return _dev


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


# ---------------------------------------------------------------- host side

def philox4x32_10(ctr, key):
    """Raw Philox4x32-10 output for a 4-word counter and 2-word key."""
    c = np.asarray(ctr, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    o = np.zeros(4, dtype=np.uint32)
    _hostlib().ssegen_host_philox(_ptr(c), _ptr(k), _ptr(o))
    return o


def normal(seed: int, idx: int, stream: int) -> float:
    return _hostlib().ssegen_host_normal(seed, idx, stream)


def neigh(seed: int, NA: int, NB: int) -> np.ndarray:
    out = np.empty((NA, NB), dtype=np.int32)
    if _hostlib().ssegen_host_neigh(seed, NA, NB, _ptr(out)) != 0:
        raise ValueError("need 1 <= NB <= NA - 1 for a table without self-neighbours")
    return out


def neigh_symmetric(seed: int, NA: int, NB: int) -> np.ndarray:
    """A symmetric neighbour table: the atoms on a ring in a seeded random
    order, each joined to the NB/2 nearest atoms on either side (NB even,
    NA > NB), so atom a is in the row of each of its neighbours.  Column order
    per row: +1, -1, +2, -2, ... along the ring."""
    if NB % 2 or NA <= NB:
        raise ValueError("need an even NB and NA > NB")
    order = np.random.default_rng(seed).permutation(NA)
    pos = np.argsort(order)
    offs = [o for d in range(1, NB // 2 + 1) for o in (d, -d)]
    return np.array([[order[(pos[a] + o) % NA] for o in offs] for a in range(NA)],
                    dtype=np.int32)


def dH(seed: int, NA: int, NB: int, Norb: int, N3D: int = 3) -> np.ndarray:
    out = np.empty((NA, NB, N3D, Norb, Norb), dtype=np.float64)
    _hostlib().ssegen_host_dH(seed, out.size, _ptr(out))
    return out


def D(seed: int, comp: int, Nqz: int, Nw: int, NA: int, NB: int, N3D: int = 3) -> np.ndarray:
    out = np.empty((Nqz, Nw, NA, NB, N3D, N3D), dtype=np.complex128)
    _hostlib().ssegen_host_D(seed, comp, N3D, Nqz * Nw * NA * NB, _ptr(out))
    return out


def G_blocks(seed: int, comp: int, NE: int, NA: int, Norb: int, blocks, scaled: bool = False):
    """G blocks for an array of (k, e, a) triples (shape [n, 3]); returns [n, Norb, Norb]."""
    b = np.asarray(blocks, dtype=np.int64).reshape(-1, 3)
    flat = np.ascontiguousarray((b[:, 0] * NE + b[:, 1]) * NA + b[:, 2])
    out = np.empty((flat.size, Norb, Norb), dtype=np.complex128)
    _hostlib().ssegen_host_G_blocks(seed, comp, Norb, int(scaled), flat.size, _ptr(flat),
                                    _ptr(out))
    return out


def G_flat_blocks(seed: int, comp: int, Norb: int, flat, scaled: bool = False):
    flat = np.ascontiguousarray(np.asarray(flat, dtype=np.int64).ravel())
    out = np.empty((flat.size, Norb, Norb), dtype=np.complex128)
    _hostlib().ssegen_host_G_blocks(seed, comp, Norb, int(scaled), flat.size, _ptr(flat),
                                    _ptr(out))
    return out


def G(seed: int, comp: int, Nkz: int, NE: int, NA: int, Norb: int, scaled: bool = False):
    flat = np.arange(Nkz * NE * NA, dtype=np.int64)
    return G_flat_blocks(seed, comp, Norb, flat, scaled).reshape(Nkz, NE, NA, Norb, Norb)


def perturb(seed: int, iteration: int, stream: int, blocks: np.ndarray, flat_index) -> None:
    """In-place host perturbation of complex128 blocks [n, s, s] keyed by flat_index."""
    assert blocks.dtype == np.complex128 and blocks.flags.c_contiguous
    n_side = blocks.shape[-1]
    flat = np.ascontiguousarray(np.asarray(flat_index, dtype=np.int64).ravel())
    assert flat.size * n_side * n_side == blocks.size
    _hostlib().ssegen_host_perturb(seed, iteration, stream, n_side, flat.size, _ptr(flat),
                                   _ptr(blocks))


# -------------------------------------------------------------- device side

def _chk(rc: int, what: str):
    if rc != 0:
        raise RuntimeError(f"{what} failed with hipError {rc}")


def dev_fill_dH(seed: int, n: int, ptr: int, stream: int = 0):
    _chk(_devlib().ssegen_dev_fill_dH(seed, n, ptr, stream), "ssegen_dev_fill_dH")


def dev_fill_G(seed: int, comp: int, Norb: int, nblk: int, ptr: int, fp32: bool = False,
               scaled: bool = False, stream: int = 0):
    _chk(_devlib().ssegen_dev_fill_G(seed, comp, Norb, nblk, int(scaled), int(fp32), ptr, stream),
         "ssegen_dev_fill_G")


def dev_fill_D(seed: int, comp: int, nblk: int, ptr: int, fp32: bool = False, N3D: int = 3,
               stream: int = 0):
    _chk(_devlib().ssegen_dev_fill_D(seed, comp, N3D, nblk, int(fp32), ptr, stream),
         "ssegen_dev_fill_D")


def dev_perturb(seed: int, iteration: int, stream_word: int, n_side: int, nblk: int, ptr: int,
                fp32: bool = False, stream: int = 0):
    _chk(_devlib().ssegen_dev_perturb(seed, iteration, stream_word, n_side, nblk, int(fp32), ptr,
                                      stream), "ssegen_dev_perturb")
