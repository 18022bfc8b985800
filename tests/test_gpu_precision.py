"""Parity of the complex64-storage MFMA paths (SSE_FP32, SSE_BF16X3) with the
binary64 oracle, through the C ABI.

The oracle is evaluated on the same stored (complex64) inputs, so the figure
is the error of the kernel's arithmetic; it is printed per result.  Bars
(relative Frobenius error per component): fp32 products <= 1e-5, bf16 hi/lo
split products <= 1e-3.  The G magnitudes of the stress cases spread over
about eight decades (per-block scale (1 + u) 2^n, n in -20..6).
"""
import numpy as np
import pytest

from paper_1912_08810_amd import configs
from tests import gpu_util as gu

pytestmark = pytest.mark.gpu
FP32, BF16X3 = 1, 2
TOL = {FP32: 1e-5, BF16X3: 1e-3}


def check_full(dp, prec, alpha=1j):
    worst = 0.0
    for c in range(dp.ncomp):
        got = dp.sigma_host(c)
        want = gu.oracle_full(dp, c, alpha=alpha)
        e1 = gu.rel_fro(got, want)
        print(f"  prec={prec} comp {c}: rel_fro={e1:.3e} max_elem={gu.max_elem_rel(got, want):.3e}",
              flush=True)
        assert e1 <= TOL[prec], (c, e1)
        worst = max(worst, e1)
    return worst


@pytest.mark.parametrize("prec", [FP32, BF16X3])
@pytest.mark.parametrize("scaled", [False, True])
def test_small_config_full(prec, scaled):
    dp = gu.DeviceProblem(configs.SMALL, configs.SEED, ncomp=2, fp32=True, scaled=scaled)
    assert gu.run_sse(dp, prec=prec) == 0
    check_full(dp, prec)


@pytest.mark.parametrize("prec", [FP32, BF16X3])
def test_ragged_tiles_unsorted_negative_shifts(prec):
    prob = configs.Problem(NA=37, NB=5, Norb=10, Nkz=4, Nqz=3, NE=47, Nw=11,
                           shift=(3, 1, -2, 7, 5, 2, 4, 9, 11, 6, 8))
    dp = gu.DeviceProblem(prob, 7, fp32=True, scaled=True)
    assert gu.run_sse(dp, prec=prec) == 0
    check_full(dp, prec)


@pytest.mark.parametrize("prec", [FP32, BF16X3])
@pytest.mark.parametrize("Norb", [1, 3, 7, 16, 22])
def test_orbital_counts(prec, Norb):
    prob = configs.Problem(NA=9, NB=3, Norb=Norb, Nkz=3, Nqz=2, NE=23, Nw=13)
    dp = gu.DeviceProblem(prob, 100 + Norb, fp32=True)
    assert gu.run_sse(dp, prec=prec) == 0
    check_full(dp, prec)


@pytest.mark.parametrize("prec", [FP32, BF16X3])
@pytest.mark.parametrize("Norb,NE", [(1, 600), (2, 300), (4, 150), (17, 20), (21, 9)])
def test_sandwich_tile_limits(prec, Norb, NE):
    # small Norb with long energy grids: the energy tile is cut to what the
    # sandwich's LDS region and output tiles hold; Norb > 16: two row tiles;
    # every case ends in a ragged energy tile
    prob = configs.Problem(NA=5, NB=3, Norb=Norb, Nkz=2, Nqz=2, NE=NE, Nw=7)
    dp = gu.DeviceProblem(prob, 200 + Norb, fp32=True, scaled=True)
    assert gu.run_sse(dp, prec=prec) == 0
    check_full(dp, prec)


@pytest.mark.parametrize("prec", [FP32, BF16X3])
def test_general_alpha(prec):
    prob = configs.Problem(NA=11, NB=4, Norb=5, Nkz=3, Nqz=3, NE=19, Nw=5)
    dp = gu.DeviceProblem(prob, 21, fp32=True)
    assert gu.run_sse(dp, prec=prec, alpha=0.25 - 2.0j) == 0
    check_full(dp, prec, alpha=0.25 - 2.0j)


@pytest.mark.parametrize("prec", [FP32, BF16X3])
def test_device_scale_sampled_scaled_magnitudes(prec):
    """Device-scale shapes with G magnitudes spread over eight decades."""
    prob = configs.DEVICE
    dp = gu.DeviceProblem(prob, configs.SEED, ncomp=1, fp32=True, scaled=True)
    assert gu.run_sse(dp, prec=prec) == 0
    blocks = gu.sample_blocks(prob, 4, n_e=12, n_a=5)
    got = dp.device_blocks(0, blocks)
    want = gu.oracle_blocks(dp, 0, blocks)
    e1 = gu.rel_fro(got, want)
    print(f"  prec={prec}: {len(blocks)} blocks rel_fro={e1:.3e}", flush=True)
    assert e1 <= TOL[prec]
    import torch
    assert not bool(torch.isnan(dp.Sigma).any())


@pytest.mark.parametrize("prec", [FP32, BF16X3])
def test_bitwise_deterministic(prec):
    prob = configs.Problem(NA=20, NB=4, Norb=10, Nkz=3, Nqz=3, NE=33, Nw=8)
    dp = gu.DeviceProblem(prob, 5, fp32=True)
    assert gu.run_sse(dp, prec=prec) == 0
    first = dp.Sigma.clone()
    assert gu.run_sse(dp, prec=prec) == 0
    assert bool((first == dp.Sigma).all())


def test_large_orbital_count_is_unsupported_not_wrong():
    from paper_1912_08810_amd import sse
    d = sse.make_desc(4, 2, 23, 2, 2, 8, 3, prec=FP32)
    with pytest.raises(sse.SSEError) as ei:
        sse.sse_plan(d, np.arange(1, 4))
    assert ei.value.status == sse.ERR_UNSUPPORTED
