"""Thin ctypes binding of libsse.so (include/sse.h): argument marshalling only.

Every step of the computation runs in the library's HIP kernels.  Tensors are
passed as device pointers (torch tensors' ``data_ptr()`` or plain ints) and
streams as ``hipStream_t`` handles (``torch.cuda.current_stream().cuda_stream``
under ROCm).  Importing this module fails loudly when the library is missing.
"""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libsse.so")

OK, PENDING, ERR_ARG, ERR_SHAPE, ERR_NEIGH, ERR_NOMEM, ERR_BUSY, ERR_TOLERANCE, ERR_DEVICE, \
    ERR_UNSUPPORTED = range(10)
FP64, FP32, BF16X3, FP64C64 = 0, 1, 2, 3
STATUS_NAMES = ["SSE_OK", "SSE_PENDING", "SSE_ERR_ARG", "SSE_ERR_SHAPE", "SSE_ERR_NEIGH",
                "SSE_ERR_NOMEM", "SSE_ERR_BUSY", "SSE_ERR_TOLERANCE", "SSE_ERR_DEVICE",
                "SSE_ERR_UNSUPPORTED"]


class sse_desc(ctypes.Structure):
    _fields_ = [("NA", ctypes.c_int32), ("NB", ctypes.c_int32), ("Norb", ctypes.c_int32),
                ("N3D", ctypes.c_int32), ("Nkz", ctypes.c_int32), ("Nqz", ctypes.c_int32),
                ("NE", ctypes.c_int32), ("Nw", ctypes.c_int32), ("ncomp", ctypes.c_int32),
                ("prec", ctypes.c_int32), ("tile_e", ctypes.c_int32),
                ("chunk_taps", ctypes.c_int32), ("dt_antiherm", ctypes.c_int32),
                ("alpha_re", ctypes.c_double),
                ("alpha_im", ctypes.c_double)]


class sse_args(ctypes.Structure):
    _fields_ = [("neigh", ctypes.c_void_p), ("dH", ctypes.c_void_p), ("G", ctypes.c_void_p),
                ("Dt", ctypes.c_void_p), ("Sigma", ctypes.c_void_p)]


class SSEError(RuntimeError):
    def __init__(self, status: int, where: str, text: str):
        self.status = status
        super().__init__(f"{where}: {STATUS_NAMES[status] if 0 <= status < 10 else status}: {text}")


def hip_runtimes_mapped():
    """Distinct HIP runtime libraries mapped into this process."""
    try:
        with open("/proc/self/maps") as fh:
            return sorted({ln.split()[-1] for ln in fh if "libamdhip64" in ln})
    except OSError:
        return []


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
    # Device memory and streams come from PyTorch, whose wheel carries its own HIP
    # runtime.  Load it first so libsse binds to that same runtime: with two HIP
    # runtimes in one process, a torch stream handle is a foreign object to ours.
    import torch  # noqa: F401
    L = ctypes.CDLL(LIB_PATH)
    rts = hip_runtimes_mapped()
    if len(rts) > 1:
        raise ImportError("two HIP runtimes are loaded in this process (" + ", ".join(rts) +
                          "); import torch before any other HIP library")
    c = ctypes
    vp = c.c_void_p
    L.sse_plan.argtypes = [c.POINTER(sse_desc), vp, c.POINTER(vp), c.POINTER(c.c_size_t)]
    L.sse_plan_batch.argtypes = [c.POINTER(sse_desc), c.POINTER(vp), c.c_int32, c.POINTER(vp),
                                 c.POINTER(c.c_size_t)]
    L.sse_compute.argtypes = [vp, vp, vp, vp, vp, vp, vp, c.c_size_t, vp]
    L.sse_compute_noalloc.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    L.sse_pi_submit.argtypes = [vp, vp, vp, vp, vp, vp, c.c_size_t, vp, c.POINTER(c.c_uint64)]
    L.sse_pi_compute.argtypes = [vp, vp, vp, vp, vp, vp, c.c_size_t, vp]
    L.sse_dtilde_submit.argtypes = [vp, vp, vp, vp, vp, c.c_size_t, vp, c.POINTER(c.c_uint64)]
    L.sse_retarded.argtypes = [vp, c.c_int32, vp, vp, vp]
    L.sse_ablation_compute.argtypes = [vp, vp, vp, vp, vp, vp, vp, c.c_size_t, vp]
    L.sse_submit.argtypes = [vp, c.POINTER(sse_args), vp, c.c_size_t, vp,
                             c.POINTER(c.c_uint64)]
    L.sse_check_submit.argtypes = [vp, c.POINTER(sse_args), vp, c.c_int32, c.c_double, vp, vp,
                                   c.c_size_t, vp, c.POINTER(c.c_uint64)]
    L.sse_poll.argtypes = [c.c_uint64]
    L.sse_wait.argtypes = [c.c_uint64]
    L.sse_plan_destroy.argtypes = [vp]
    L.sse_plan_destroy.restype = None
    L.sse_last_error.restype = c.c_char_p
    for f in (L.sse_plan, L.sse_plan_batch, L.sse_compute, L.sse_compute_noalloc, L.sse_submit,
              L.sse_poll, L.sse_wait, L.sse_check_submit, L.sse_pi_submit, L.sse_pi_compute,
              L.sse_dtilde_submit, L.sse_retarded, L.sse_ablation_compute):
        f.restype = c.c_int
    return L


lib = _load()

# Every symbol include/sse.h declares (checked by the CPU test of the library).
EXPORTS = ["sse_ablation_compute", "sse_check_submit", "sse_compute", "sse_compute_noalloc",
           "sse_dtilde_submit",
           "sse_last_error", "sse_pi_compute", "sse_pi_submit", "sse_plan", "sse_plan_batch",
           "sse_plan_destroy", "sse_poll", "sse_retarded", "sse_submit", "sse_wait"]
NOALLOC_SCRATCH_BYTES = 32 << 20  # SSE_NOALLOC_SCRATCH_BYTES


def last_error() -> str:
    return lib.sse_last_error().decode()


def _check(st: int, where: str):
    if st != OK:
        raise SSEError(st, where, last_error())
    return st


def _ptr(x):
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


def _stream(s):
    if s is None:
        return None
    if isinstance(s, int):
        return s
    return s.cuda_stream


def make_desc(NA, NB, Norb, Nkz, Nqz, NE, Nw, ncomp=1, prec=FP64, alpha=1j, N3D=3, tile_e=0,
              chunk_taps=0, dt_antiherm=0):
    alpha = complex(alpha)
    return sse_desc(NA, NB, Norb, N3D, Nkz, Nqz, NE, Nw, ncomp, prec, tile_e, chunk_taps,
                    int(dt_antiherm), alpha.real, alpha.imag)


class Plan:
    """Owns an sse_plan_t; ``workspace_bytes`` is the device workspace each call needs."""

    def __init__(self, desc, w_shift=None, descs=None, w_shifts=None):
        self.handle = ctypes.c_void_p()
        ws = ctypes.c_size_t()
        if descs is None:
            import numpy as np
            self._shift = np.ascontiguousarray(w_shift, dtype=np.int32)
            st = lib.sse_plan(ctypes.byref(desc), self._shift.ctypes.data_as(ctypes.c_void_p),
                              ctypes.byref(self.handle), ctypes.byref(ws))
            _check(st, "sse_plan")
            self.n = 1
            self.descs = [desc]
        else:
            import numpy as np
            n = len(descs)
            arr = (sse_desc * n)(*descs)
            self._shifts = [np.ascontiguousarray(s, dtype=np.int32) for s in w_shifts]
            ptrs = (ctypes.c_void_p * n)(*[s.ctypes.data for s in self._shifts])
            st = lib.sse_plan_batch(arr, ptrs, n, ctypes.byref(self.handle), ctypes.byref(ws))
            _check(st, "sse_plan_batch")
            self.n = n
            self.descs = list(descs)
        self.workspace_bytes = ws.value

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value and lib is not None:
            lib.sse_plan_destroy(h)
            self.handle = None


def sse_plan(desc, w_shift) -> Plan:
    return Plan(desc, w_shift)


def sse_plan_batch(descs, w_shifts) -> Plan:
    return Plan(None, descs=descs, w_shifts=w_shifts)


def sse_compute(plan: Plan, neigh, dH, G, Dt, Sigma, workspace, stream=None, check=True) -> int:
    st = lib.sse_compute(plan.handle, _ptr(neigh), _ptr(dH), _ptr(G), _ptr(Dt), _ptr(Sigma),
                         _ptr(workspace), plan.workspace_bytes, _stream(stream))
    return _check(st, "sse_compute") if check else st


def sse_compute_noalloc(plan: Plan, neigh, dH, G, Dt, Sigma, stream=None, check=True) -> int:
    """sse_compute with the library's static device scratch instead of a workspace."""
    st = lib.sse_compute_noalloc(plan.handle, _ptr(neigh), _ptr(dH), _ptr(G), _ptr(Dt),
                                 _ptr(Sigma), _stream(stream))
    return _check(st, "sse_compute_noalloc") if check else st


def pi_elems(desc) -> int:
    """Complex elements of one component of Pi: [Nqz, Nw, NA, NB + 1, 3, 3]."""
    return desc.Nqz * desc.Nw * desc.NA * (desc.NB + 1) * 9


def sse_pi_compute(plan: Plan, neigh, dH, G, Pi, workspace, stream=None, check=True) -> int:
    """Phonon self-energy (Eqs. (4)-(5)); G holds both components, Pi ncomp."""
    nbytes = workspace.numel() * workspace.element_size() if hasattr(workspace, "numel") \
        else plan.workspace_bytes
    st = lib.sse_pi_compute(plan.handle, _ptr(neigh), _ptr(dH), _ptr(G), _ptr(Pi),
                            _ptr(workspace), nbytes, _stream(stream))
    return _check(st, "sse_pi_compute") if check else st


def sse_pi_submit(plan: Plan, neigh, dH, G, Pi, workspace, stream=None) -> int:
    t = ctypes.c_uint64()
    nbytes = workspace.numel() * workspace.element_size() if hasattr(workspace, "numel") \
        else plan.workspace_bytes
    _check(lib.sse_pi_submit(plan.handle, _ptr(neigh), _ptr(dH), _ptr(G), _ptr(Pi),
                             _ptr(workspace), nbytes, _stream(stream), ctypes.byref(t)),
           "sse_pi_submit")
    return t.value


def dtilde_workspace_bytes(desc) -> int:
    return 256 + 4 * desc.NA * desc.NB


def sse_dtilde_submit(plan: Plan, neigh, D, Dt, workspace, stream=None) -> int:
    """D [ncomp][Nqz, Nw, NA, NB + 1, 3, 3] -> Dt [ncomp][Nqz, Nw, NA, NB, 3, 3]; a ticket."""
    t = ctypes.c_uint64()
    nbytes = workspace.numel() * workspace.element_size()
    _check(lib.sse_dtilde_submit(plan.handle, _ptr(neigh), _ptr(D), _ptr(Dt), _ptr(workspace),
                                 nbytes, _stream(stream), ctypes.byref(t)), "sse_dtilde_submit")
    return t.value


def sse_retarded(plan: Plan, which: int, X, XR, stream=None, check=True) -> int:
    """XR = (X[1] - X[0]) / 2; which 0 = Sigma, 1 = Pi."""
    st = lib.sse_retarded(plan.handle, which, _ptr(X), _ptr(XR), _stream(stream))
    return _check(st, "sse_retarded") if check else st


def ablation_workspace_bytes(desc, atoms: int) -> int:
    """Workspace of sse_ablation_compute holding the transients of `atoms` atoms."""
    per = desc.NB * 3 * (desc.Nkz * desc.NE + desc.Nqz * desc.Nw) * desc.Norb ** 2 * 16
    return 256 + per * atoms


def sse_ablation_compute(plan: Plan, neigh, dH, G, Dt, Sigma, workspace, stream=None,
                         check=True) -> int:
    nbytes = workspace.numel() * workspace.element_size()
    st = lib.sse_ablation_compute(plan.handle, _ptr(neigh), _ptr(dH), _ptr(G), _ptr(Dt),
                                  _ptr(Sigma), _ptr(workspace), nbytes, _stream(stream))
    return _check(st, "sse_ablation_compute") if check else st


def _args(items):
    arr = (sse_args * len(items))()
    for t, (neigh, dH, G, Dt, Sigma) in enumerate(items):
        arr[t] = sse_args(_ptr(neigh), _ptr(dH), _ptr(G), _ptr(Dt), _ptr(Sigma))
    return arr


def sse_submit(plan: Plan, items, workspace, stream=None) -> int:
    """items: one (neigh, dH, G, Dt, Sigma) tuple per instance; returns a ticket."""
    t = ctypes.c_uint64()
    arr = _args(items)
    _check(lib.sse_submit(plan.handle, arr, _ptr(workspace), plan.workspace_bytes,
                          _stream(stream), ctypes.byref(t)), "sse_submit")
    return t.value


def sse_poll(ticket: int) -> int:
    st = lib.sse_poll(ticket)
    if st not in (OK, PENDING):
        raise SSEError(st, "sse_poll", last_error())
    return st


def sse_wait(ticket: int, check=True) -> int:
    st = lib.sse_wait(ticket)
    return _check(st, "sse_wait") if check else st


def check_workspace_bytes(nblocks: int, ncomp: int) -> int:
    return 256 + 16 * nblocks * ncomp


class CheckTicket:
    """A pending sse_check_submit: ``rel_err`` is filled when it finishes."""

    def __init__(self, ticket: int, rel_err):
        self.ticket = ticket
        self.rel_err = rel_err


def sse_check_submit(plan: Plan, item, blocks, tol, workspace, stream=None) -> CheckTicket:
    """item: (neigh, dH, G, Dt, Sigma); blocks: device int32 tensor [n, 3]."""
    ncomp = plan.descs[0].ncomp
    rel = (ctypes.c_double * ncomp)()
    t = ctypes.c_uint64()
    arr = _args([item])
    n = int(blocks.shape[0]) if hasattr(blocks, "shape") else len(blocks) // 3
    _check(lib.sse_check_submit(plan.handle, arr, _ptr(blocks), n, float(tol),
                                ctypes.cast(rel, ctypes.c_void_p), _ptr(workspace),
                                workspace.numel() * workspace.element_size()
                                if hasattr(workspace, "numel") else check_workspace_bytes(n, ncomp),
                                _stream(stream), ctypes.byref(t)), "sse_check_submit")
    return CheckTicket(t.value, rel)
