"""Helpers of the GPU parity tests: device inputs from the seeded generator,
library calls through the C ABI, oracle evaluation on the host and the
comparison measure (relative Frobenius error)."""
from __future__ import annotations

import numpy as np

import oracle
import ssegen
from paper_1912_08810_amd import configs
from ssegen import device_problem as _dp


def torch_mod():
    import torch
    return torch


def rel_fro(x, y) -> float:
    x = np.asarray(x)
    y = np.asarray(y)
    return float(np.linalg.norm((x - y).ravel()) / max(np.linalg.norm(y.ravel()), 1e-300))


def max_elem_rel(x, y) -> float:
    """Largest element-wise deviation, relative to the largest |y| element."""
    return float(np.abs(x - y).max() / max(np.abs(y).max(), 1e-300))


DeviceProblem = _dp.DeviceProblem


def oracle_full(dp, comp: int, alpha=1j) -> np.ndarray:
    """Oracle Sigma of every block of one component of a DeviceProblem."""
    p = dp.prob
    dH, D = dp.host_inputs(comp)
    G = dp._round(ssegen.G(dp.seed, comp, p.Nkz, p.NE, p.NA, p.Norb, scaled=dp.scaled))
    return oracle.sigma(dp.neigh_h, dH, G, D, p.shifts(), p.Nkz, p.NE, alpha=alpha)


def oracle_blocks(dp, comp: int, blocks, alpha=1j) -> np.ndarray:
    """Oracle Sigma of the listed (k, e, a) blocks; only the G blocks they read
    are generated on the host."""
    p = dp.prob
    dH, D = dp.host_inputs(comp)
    need = oracle.needed_g_blocks(dp.neigh_h, p.shifts(), p.Nkz, p.Nqz, p.NE, p.NA, blocks)
    Gb = dp._round(ssegen.G_flat_blocks(dp.seed, comp, p.Norb, need, scaled=dp.scaled))
    gslot = np.full(p.Nkz * p.NE * p.NA, -1, dtype=np.int64)
    gslot[need] = np.arange(need.size)
    return oracle.sigma(dp.neigh_h, dH, Gb, D, p.shifts(), p.Nkz, p.NE, alpha=alpha,
                        blocks=blocks, gslot=gslot)


def sample_blocks(prob: configs.Problem, seed: int, n_e: int = 16, n_a: int = 8):
    """All k, n_e energies (always including 0, s_max - 1, s_max, NE - 1 and the
    two ends of an interior tile boundary) and n_a atoms (including 0 and NA - 1)."""
    rng = np.random.default_rng(seed)
    s = prob.shifts()
    smax = int(s.max())
    es = {0, max(smax - 1, 0), min(smax, prob.NE - 1), prob.NE - 1, prob.NE // 2,
          prob.NE // 2 - 1}
    while len(es) < min(n_e, prob.NE):
        es.add(int(rng.integers(0, prob.NE)))
    as_ = {0, prob.NA - 1}
    while len(as_) < min(n_a, prob.NA):
        as_.add(int(rng.integers(0, prob.NA)))
    return np.array([(k, e, a) for k in range(prob.Nkz) for e in sorted(es) for a in sorted(as_)],
                    dtype=np.int32)


def run_sse(dp, alpha=1j, prec=0, tile_e=0):
    """sse_plan + sse_compute through the C ABI on the current stream; returns the status."""
    import torch
    from paper_1912_08810_amd import sse
    p = dp.prob
    desc = sse.make_desc(p.NA, p.NB, p.Norb, p.Nkz, p.Nqz, p.NE, p.Nw, ncomp=dp.ncomp, prec=prec,
                         alpha=alpha, tile_e=tile_e)
    plan = sse.sse_plan(desc, p.shifts())
    ws = torch.empty(max(plan.workspace_bytes, 1), dtype=torch.uint8, device="cuda")
    print(f"[case] NA={p.NA} NB={p.NB} Norb={p.Norb} Nkz={p.Nkz} Nqz={p.Nqz} NE={p.NE} "
          f"Nw={p.Nw} ncomp={dp.ncomp} prec={prec}", flush=True)
    st = sse.sse_compute(plan, dp.neigh, dp.dH, dp.G, dp.D, dp.Sigma, ws,
                         torch.cuda.current_stream(), check=False)
    torch.cuda.synchronize()
    return st


# ---------------------------------------------------------------- phonon self-energy

def pi_host(Pi, comp: int, prob) -> np.ndarray:
    """One component of a device Pi tensor as complex128 [Nqz, Nw, NA, NB + 1, 3, 3]."""
    s = Pi[comp].cpu().numpy().astype(np.float64)
    return (s[0::2] + 1j * s[1::2]).reshape(prob.Nqz, prob.Nw, prob.NA, prob.NB + 1, 3, 3)


def _xy(comp: int, G0, G1):
    """Pi< pairs the shifted G< with G>; Pi> the shifted G> with G<."""
    return (G0, G1) if comp == 0 else (G1, G0)


def oracle_pi_full(dp, comp: int, beta=1j) -> np.ndarray:
    p = dp.prob
    dH, _ = dp.host_inputs(0)
    G0 = ssegen.G(dp.seed, 0, p.Nkz, p.NE, p.NA, p.Norb)
    G1 = ssegen.G(dp.seed, 1, p.Nkz, p.NE, p.NA, p.Norb)
    X, Y = _xy(comp, G0, G1)
    return oracle.pi(dp.neigh_h, dH, X, Y, p.shifts(), p.Nkz, p.Nqz, p.NE, beta=beta)


def oracle_pi_blocks(dp, comp: int, blocks, beta=1j) -> np.ndarray:
    """Oracle Pi of the listed (q, w, a) blocks; only the G blocks they read are generated."""
    p = dp.prob
    dH, _ = dp.host_inputs(0)
    need = oracle.needed_g_blocks_pi(dp.neigh_h, p.shifts(), p.Nkz, p.NE, p.NA, blocks)
    G0 = ssegen.G_flat_blocks(dp.seed, 0, p.Norb, need)
    G1 = ssegen.G_flat_blocks(dp.seed, 1, p.Norb, need)
    gslot = np.full(p.Nkz * p.NE * p.NA, -1, dtype=np.int64)
    gslot[need] = np.arange(need.size)
    X, Y = _xy(comp, G0, G1)
    return oracle.pi(dp.neigh_h, dH, X, Y, p.shifts(), p.Nkz, p.Nqz, p.NE, beta=beta,
                     blocks=blocks, gslot=gslot)


def run_pi(dp, ncomp: int = 2, beta=1j):
    """sse_plan + sse_pi_compute through the C ABI; returns (status, Pi tensor)."""
    import torch
    from paper_1912_08810_amd import sse
    p = dp.prob
    assert dp.ncomp == 2, "the phonon self-energy reads both components of G"
    desc = sse.make_desc(p.NA, p.NB, p.Norb, p.Nkz, p.Nqz, p.NE, p.Nw, ncomp=ncomp,
                         prec=sse.FP64, alpha=beta)
    plan = sse.sse_plan(desc, p.shifts())
    ws = torch.empty(max(plan.workspace_bytes, 256), dtype=torch.uint8, device="cuda")
    Pi = torch.full((ncomp, sse.pi_elems(desc) * 2), float("nan"), dtype=torch.float64,
                    device="cuda")
    print(f"[case] pi NA={p.NA} NB={p.NB} Norb={p.Norb} Nkz={p.Nkz} Nqz={p.Nqz} NE={p.NE} "
          f"Nw={p.Nw} ncomp={ncomp}", flush=True)
    st = sse.sse_pi_compute(plan, dp.neigh, dp.dH, dp.G, Pi, ws, torch.cuda.current_stream(),
                            check=False)
    torch.cuda.synchronize()
    return st, Pi


def sample_pi_blocks(prob, seed: int, n_a: int = 2, n_w: int = 3):
    """All q, n_w frequencies (the smallest and largest shift among them) and
    n_a atoms (0 and NA - 1 among them)."""
    rng = np.random.default_rng(seed)
    s = prob.shifts()
    ws = {int(np.argmin(s)), int(np.argmax(s))}
    while len(ws) < min(n_w, prob.Nw):
        ws.add(int(rng.integers(0, prob.Nw)))
    as_ = {0, prob.NA - 1}
    while len(as_) < min(n_a, prob.NA):
        as_.add(int(rng.integers(0, prob.NA)))
    return np.array([(q, w, a) for q in range(prob.Nqz) for w in sorted(ws) for a in sorted(as_)],
                    dtype=np.int32)
