"""Seeded device tensors of one problem, filled on the GPU by the device
generator, plus the matching host-side inputs (same generator, host side).
Allocation uses torch (device memory only); no self-energy arithmetic here."""
from __future__ import annotations

import numpy as np

import ssegen


def torch_mod():
    import torch
    return torch


class DeviceProblem:
    """Seeded device tensors of one problem (all components)."""

    def __init__(self, prob: configs.Problem, seed: int, ncomp: int = 1, fp32: bool = False,
                 scaled: bool = False, neigh=None, sync: bool = True):
        torch = torch_mod()
        self.prob, self.seed, self.ncomp, self.fp32, self.scaled = prob, seed, ncomp, fp32, scaled
        p = prob
        stream = torch.cuda.current_stream().cuda_stream
        self.neigh_h = ssegen.neigh(seed, p.NA, p.NB) if neigh is None else np.asarray(
            neigh, dtype=np.int32)
        self.neigh = torch.from_numpy(self.neigh_h).cuda()
        self.dH = torch.empty(p.NA * p.NB * p.N3D * p.NN, dtype=torch.float64, device="cuda")
        ssegen.dev_fill_dH(seed, self.dH.numel(), self.dH.data_ptr(), stream)
        rdt = torch.float32 if fp32 else torch.float64
        esz = 4 if fp32 else 8
        self.G = torch.empty(ncomp, p.g_elems() * 2, dtype=rdt, device="cuda")
        self.D = torch.empty(ncomp, p.d_elems() * 2, dtype=rdt, device="cuda")
        for c in range(ncomp):
            ssegen.dev_fill_G(seed, c, p.Norb, p.Nkz * p.NE * p.NA,
                              self.G.data_ptr() + c * p.g_elems() * 2 * esz, fp32=fp32,
                              scaled=scaled, stream=stream)
            ssegen.dev_fill_D(seed, c, p.Nqz * p.Nw * p.NA * p.NB,
                              self.D.data_ptr() + c * p.d_elems() * 2 * esz, fp32=fp32,
                              stream=stream)
        self.Sigma = torch.full_like(self.G, float("nan"))
        if sync:
            torch.cuda.synchronize()

    def sigma_host(self, comp: int) -> np.ndarray:
        p = self.prob
        s = self.Sigma[comp].cpu().numpy().astype(np.float64)
        return (s[0::2] + 1j * s[1::2]).reshape(p.Nkz, p.NE, p.NA, p.Norb, p.Norb)

    # ---- host inputs for the oracle (same generator, host side)
    def _round(self, x):
        return x.astype(np.complex64).astype(np.complex128) if self.fp32 else x

    def host_inputs(self, comp: int):
        p = self.prob
        dH = ssegen.dH(self.seed, p.NA, p.NB, p.Norb)
        D = self._round(ssegen.D(self.seed, comp, p.Nqz, p.Nw, p.NA, p.NB))
        return dH, D

    def device_blocks(self, comp: int, blocks) -> np.ndarray:
        """The listed output blocks of the device result (gathered on the device)."""
        torch = torch_mod()
        p = self.prob
        b = np.asarray(blocks, dtype=np.int64).reshape(-1, 3)
        flat = torch.from_numpy((b[:, 0] * p.NE + b[:, 1]) * p.NA + b[:, 2]).cuda()
        S = self.Sigma[comp].view(-1, p.NN * 2)
        s = S.index_select(0, flat).cpu().numpy().astype(np.float64)
        return (s[:, 0::2] + 1j * s[:, 1::2]).reshape(-1, p.Norb, p.Norb)
