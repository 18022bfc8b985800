"""The paper's own final form of Eq. (3) (dH G and dH D precomputed, then the
Norb x Norb Nw x Norb GEMMs on the matrix cores) against the oracle at the
binary64 bar, including atom chunks forced by a small workspace, odd shapes,
and the device-scale configuration on sampled blocks."""
import numpy as np
import pytest

from paper_1912_08810_amd import configs
from tests import gpu_util as gu

pytestmark = pytest.mark.gpu
TOL = 1e-12


def run_ablation(dp, atoms=None, alpha=1j):
    import torch
    from paper_1912_08810_amd import sse
    p = dp.prob
    desc = sse.make_desc(p.NA, p.NB, p.Norb, p.Nkz, p.Nqz, p.NE, p.Nw, ncomp=dp.ncomp,
                         alpha=alpha)
    plan = sse.sse_plan(desc, p.shifts())
    ws = torch.empty(sse.ablation_workspace_bytes(desc, atoms or p.NA), dtype=torch.uint8,
                     device="cuda")
    print(f"[case] ablation NA={p.NA} Norb={p.Norb} NE={p.NE} Nw={p.Nw} atoms/chunk={atoms}",
          flush=True)
    st = sse.sse_ablation_compute(plan, dp.neigh, dp.dH, dp.G, dp.D, dp.Sigma, ws,
                                  torch.cuda.current_stream(), check=False)
    torch.cuda.synchronize()
    return st


@pytest.mark.parametrize("prob,atoms", [
    (configs.SMALL, None),
    (configs.SMALL, 3),
    (configs.Problem(NA=9, NB=3, Norb=10, Nkz=4, Nqz=3, NE=29, Nw=7, shift=(3, 1, -2, 7, 5, 2, 4)), 4),
    (configs.Problem(NA=5, NB=2, Norb=1, Nkz=2, Nqz=2, NE=11, Nw=3), None),
    (configs.Problem(NA=4, NB=2, Norb=16, Nkz=2, Nqz=1, NE=9, Nw=2), None),
    (configs.Problem(NA=51, NB=50, Norb=4, Nkz=2, Nqz=2, NE=6, Nw=3), 17),
], ids=["small", "small_chunks", "norb10_ragged", "norb1", "norb16", "nb50"])
def test_ablation_matches_oracle(prob, atoms):
    dp = gu.DeviceProblem(prob, 91, ncomp=2)
    assert run_ablation(dp, atoms) == 0
    for c in range(2):
        e1 = gu.rel_fro(dp.sigma_host(c), gu.oracle_full(dp, c))
        e2 = gu.max_elem_rel(dp.sigma_host(c), gu.oracle_full(dp, c))
        print(f"  comp {c}: rel_fro={e1:.3e} max_elem={e2:.3e}", flush=True)
        assert e1 <= TOL and e2 <= TOL, (c, e1, e2)


def test_ablation_device_scale_sampled():
    prob = configs.DEVICE
    dp = gu.DeviceProblem(prob, configs.SEED, ncomp=1)
    assert run_ablation(dp, atoms=160) == 0
    blocks = gu.sample_blocks(prob, 5, n_e=8, n_a=4)
    got = dp.device_blocks(0, blocks)
    want = gu.oracle_blocks(dp, 0, blocks)
    e = gu.rel_fro(got, want)
    print(f"  {len(blocks)} blocks rel_fro={e:.3e}", flush=True)
    assert e <= TOL, e


def test_ablation_limits():
    import torch
    from paper_1912_08810_amd import sse
    p = configs.SMALL
    desc = sse.make_desc(p.NA, p.NB, p.Norb, p.Nkz, p.Nqz, p.NE, p.Nw)
    plan = sse.sse_plan(desc, p.shifts())
    ws = torch.empty(512, dtype=torch.uint8, device="cuda")
    assert sse.sse_ablation_compute(plan, 1, 1, 1, 1, 1, ws, None, check=False) == sse.ERR_ARG
    big = sse.sse_plan(sse.make_desc(4, 2, 17, 2, 2, 8, 2), np.array([1, 2]))
    assert sse.sse_ablation_compute(big, 1, 1, 1, 1, 1, ws, None, check=False) == \
        sse.ERR_UNSUPPORTED
