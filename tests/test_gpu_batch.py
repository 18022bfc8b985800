"""Persistent batched launch (sse_plan_batch + sse_submit): uneven instances in
one launch per component, checked per instance against the oracle and bitwise
against the same instance computed alone with the same tile shape."""
import numpy as np
import pytest

from paper_1912_08810_amd import configs
from tests import gpu_util as gu

pytestmark = pytest.mark.gpu
TOL = {0: 1e-12, 1: 1e-5, 2: 1e-3}


def uneven_instances(n, seed, Norb):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        NE = int(rng.integers(12, 60))
        Nw = int(rng.integers(2, 14))
        out.append(configs.Problem(NA=int(rng.integers(5, 40)), NB=3, Norb=Norb, Nkz=3, Nqz=3,
                                   NE=NE, Nw=Nw))
    return out


def run_batch(dps, prec, tile_e=None):
    import torch
    from paper_1912_08810_amd import sse
    descs = [sse.make_desc(dp.prob.NA, dp.prob.NB, dp.prob.Norb, dp.prob.Nkz, dp.prob.Nqz,
                           dp.prob.NE, dp.prob.Nw, ncomp=dp.ncomp, prec=prec,
                           tile_e=0 if tile_e is None else tile_e[i])
             for i, dp in enumerate(dps)]
    plan = sse.sse_plan_batch(descs, [dp.prob.shifts() for dp in dps])
    ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device="cuda")
    print(f"[case] batch of {len(dps)} prec={prec}", flush=True)
    t = sse.sse_submit(plan, [(dp.neigh, dp.dH, dp.G, dp.D, dp.Sigma) for dp in dps], ws,
                       torch.cuda.current_stream())
    st = sse.sse_wait(t, check=False)
    torch.cuda.synchronize()
    return st


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_uneven_batch_matches_oracle_and_single(prec):
    import torch
    fp32 = prec != 0
    probs = uneven_instances(7, 10 + prec, Norb=4 if prec == 0 else 10)
    dps = [gu.DeviceProblem(p, 300 + i, ncomp=2, fp32=fp32, scaled=fp32)
           for i, p in enumerate(probs)]
    tiles = [int(t) for t in np.random.default_rng(prec).integers(1, 6, len(dps))]
    assert run_batch(dps, prec, tile_e=tiles) == 0
    for i, dp in enumerate(dps):
        for c in range(2):
            got = dp.sigma_host(c)
            want = gu.oracle_full(dp, c)
            e = gu.rel_fro(got, want)
            print(f"  inst {i} {dp.prob} comp {c}: rel_fro={e:.3e}", flush=True)
            assert e <= TOL[prec]
    # the same instance alone (one-shot kernel, same tile shape) gives the same bits
    for i in (0, 3, 6):
        dp = dps[i]
        batched = dp.Sigma.clone()
        dp.Sigma.fill_(float("nan"))
        assert gu.run_sse(dp, prec=prec, tile_e=tiles[i]) == 0
        assert bool((batched == dp.Sigma).all()), i


def test_batch_of_one_and_bad_neighbour_in_batch():
    from paper_1912_08810_amd import sse
    probs = uneven_instances(3, 77, Norb=3)
    dps = [gu.DeviceProblem(p, 400 + i) for i, p in enumerate(probs)]
    assert run_batch(dps[:1], 0) == 0
    assert gu.rel_fro(dps[0].sigma_host(0), gu.oracle_full(dps[0], 0)) <= 1e-12
    bad = dps[1].neigh_h.copy()
    bad[0, 0] = dps[1].prob.NA + 5
    dps[1].neigh.copy_(__import__("torch").from_numpy(bad))
    assert run_batch(dps, 0) == sse.ERR_NEIGH


@pytest.mark.parametrize("prec", [0, 2])
def test_batch_with_empty_work_queues(prec):
    """Five atoms in all: three of the eight work queues are empty, so the
    workgroups that start on them move on to the others at once."""
    fp32 = prec != 0
    probs = [configs.Problem(NA=3, NB=2, Norb=5, Nkz=3, Nqz=2, NE=23, Nw=6),
             configs.Problem(NA=2, NB=1, Norb=5, Nkz=4, Nqz=3, NE=17, Nw=4)]
    dps = [gu.DeviceProblem(p, 500 + i, ncomp=1, fp32=fp32, scaled=fp32)
           for i, p in enumerate(probs)]
    assert run_batch(dps, prec, tile_e=[2, 3]) == 0
    for i, dp in enumerate(dps):
        e = gu.rel_fro(dp.sigma_host(0), gu.oracle_full(dp, 0))
        print(f"  inst {i} {dp.prob}: rel_fro={e:.3e}", flush=True)
        assert e <= TOL[prec]
        batched = dp.Sigma.clone()
        dp.Sigma.fill_(float("nan"))
        assert gu.run_sse(dp, prec=prec, tile_e=[2, 3][i]) == 0
        assert bool((batched == dp.Sigma).all()), i


@pytest.mark.parametrize("prec", [0, 2])
def test_batch_of_different_neighbour_counts(prec):
    """Instances with 1, 50 (the ABI's largest count) and 7 neighbours per
    atom in one launch; each against the oracle and bitwise against itself
    alone."""
    fp32 = prec != 0
    probs = [configs.Problem(NA=9, NB=1, Norb=4, Nkz=3, Nqz=2, NE=14, Nw=3),
             configs.Problem(NA=51, NB=50, Norb=4, Nkz=2, Nqz=2, NE=6, Nw=3),
             configs.Problem(NA=12, NB=7, Norb=4, Nkz=3, Nqz=3, NE=9, Nw=5)]
    dps = [gu.DeviceProblem(p, 600 + i, ncomp=2, fp32=fp32, scaled=fp32)
           for i, p in enumerate(probs)]
    tiles = [3, 2, 4]
    assert run_batch(dps, prec, tile_e=tiles) == 0
    for i, dp in enumerate(dps):
        for c in range(2):
            e = gu.rel_fro(dp.sigma_host(c), gu.oracle_full(dp, c))
            print(f"  inst {i} {dp.prob} comp {c}: rel_fro={e:.3e}", flush=True)
            assert e <= TOL[prec]
        batched = dp.Sigma.clone()
        dp.Sigma.fill_(float("nan"))
        assert gu.run_sse(dp, prec=prec, tile_e=tiles[i]) == 0
        assert bool((batched == dp.Sigma).all()), i
