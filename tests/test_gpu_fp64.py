"""Parity of the binary64 HIP path with the oracle, through the C ABI.

Tolerance: relative Frobenius error <= 1e-12 per component and element-wise
deviation <= 1e-12 of the largest |Sigma| element (the FP64 bar of the
precision targets).  Sizes span several energy tiles with a ragged last tile,
negative and unsorted shift tables, every supported orbital count class, the
device-scale configuration on sampled blocks, and the error paths.
"""
import numpy as np
import pytest

from paper_1912_08810_amd import configs
from tests import gpu_util as gu

pytestmark = pytest.mark.gpu
TOL = 1e-12


def _sse():
    from paper_1912_08810_amd import sse
    return sse


def run(dp: gu.DeviceProblem, alpha=1j, prec=0):
    return gu.run_sse(dp, alpha=alpha, prec=prec)


def check_full(dp, alpha=1j):
    for c in range(dp.ncomp):
        got = dp.sigma_host(c)
        want = gu.oracle_full(dp, c, alpha=alpha)
        e1, e2 = gu.rel_fro(got, want), gu.max_elem_rel(got, want)
        print(f"  comp {c}: rel_fro={e1:.3e} max_elem={e2:.3e}", flush=True)
        assert e1 <= TOL and e2 <= TOL, (c, e1, e2)


def test_small_config_full_both_components():
    dp = gu.DeviceProblem(configs.SMALL, configs.SEED, ncomp=2)
    assert run(dp) == 0
    check_full(dp)
    # the lesser self-energy keeps the anti-Hermitian symmetry of its inputs
    s = dp.sigma_host(0)
    assert np.linalg.norm(s + np.conj(np.swapaxes(s, -1, -2))) <= 1e-13 * np.linalg.norm(s)


def test_ragged_tiles_unsorted_negative_shifts():
    prob = configs.Problem(NA=37, NB=5, Norb=10, Nkz=4, Nqz=3, NE=47, Nw=7,
                           shift=(3, 1, -2, 7, 5, 2, 4))
    dp = gu.DeviceProblem(prob, 7)
    assert run(dp) == 0
    check_full(dp)


def test_wide_shift_spread_many_chunks():
    # shift spread 78 at Norb=10: the taps are cut into several windows per
    # (b, q); shifts of +-39 with NE=40 read almost only zero-padded rows
    prob = configs.Problem(NA=6, NB=3, Norb=10, Nkz=2, Nqz=2, NE=40, Nw=9,
                           shift=(0, 8, 16, 24, 32, 39, -8, -16, -39))
    dp = gu.DeviceProblem(prob, 13)
    assert run(dp) == 0
    check_full(dp)


@pytest.mark.parametrize("Norb", [1, 3, 7, 12, 16, 23, 24, 30])
def test_orbital_counts(Norb):
    prob = configs.Problem(NA=9, NB=3, Norb=Norb, Nkz=3, Nqz=2, NE=23, Nw=6)
    dp = gu.DeviceProblem(prob, 100 + Norb)
    assert run(dp) == 0
    check_full(dp)


def test_hermitian_prefactor_and_general_alpha():
    prob = configs.Problem(NA=11, NB=4, Norb=5, Nkz=3, Nqz=3, NE=19, Nw=5)
    for alpha in (1.0, 0.25 - 2.0j):
        dp = gu.DeviceProblem(prob, 21)
        assert run(dp, alpha=alpha) == 0
        check_full(dp, alpha=alpha)


def test_bitwise_deterministic():
    prob = configs.Problem(NA=20, NB=4, Norb=10, Nkz=3, Nqz=3, NE=33, Nw=8)
    dp = gu.DeviceProblem(prob, 5)
    assert run(dp) == 0
    first = dp.Sigma.clone()
    assert run(dp) == 0
    assert bool((first == dp.Sigma).all())


def test_device_scale_sampled():
    """The device-scale configuration, Sigma [7, 1000, 1024, 10, 10], both
    components, checked on sampled blocks that include the energy edges."""
    prob = configs.DEVICE
    dp = gu.DeviceProblem(prob, configs.SEED, ncomp=2)
    assert run(dp) == 0
    blocks = gu.sample_blocks(prob, 3, n_e=16, n_a=6)
    for c in range(2):
        got = dp.device_blocks(c, blocks)
        want = gu.oracle_blocks(dp, c, blocks)
        e1, e2 = gu.rel_fro(got, want), gu.max_elem_rel(got, want)
        print(f"  comp {c}: {len(blocks)} blocks rel_fro={e1:.3e} max_elem={e2:.3e}", flush=True)
        assert e1 <= TOL and e2 <= TOL
    # no output left unwritten
    import torch
    assert not bool(torch.isnan(dp.Sigma).any())


def test_bad_neighbour_is_reported_not_faulted():
    sse = _sse()
    prob = configs.Problem(NA=8, NB=2, Norb=3, Nkz=2, Nqz=2, NE=10, Nw=3)
    neigh = np.array([[1, 2], [0, 3], [4, 5], [6, 7], [0, 1], [2, 8], [3, 4], [5, 6]])  # 8 >= NA
    dp = gu.DeviceProblem(prob, 3, neigh=neigh)
    assert run(dp) == sse.ERR_NEIGH
    assert "neighbour" in sse.last_error()
