"""Binary64 arithmetic on complex64 storage (SSE_FP64C64, the serving
fallback) and the sampled binary64 check (sse_check_submit)."""
import numpy as np
import pytest

from paper_1912_08810_amd import configs
from tests import gpu_util as gu

pytestmark = pytest.mark.gpu


def _sse():
    from paper_1912_08810_amd import sse
    return sse


def test_fp64_arithmetic_on_complex64_storage():
    prob = configs.Problem(NA=21, NB=4, Norb=10, Nkz=3, Nqz=3, NE=37, Nw=9)
    dp = gu.DeviceProblem(prob, 41, ncomp=2, fp32=True, scaled=True)
    assert gu.run_sse(dp, prec=3) == 0
    for c in range(2):
        got = dp.sigma_host(c)
        want = gu.oracle_full(dp, c)
        # binary64 arithmetic; the only rounding left is the final store to complex64
        e = gu.rel_fro(got, want)
        print(f"  fp64c64 comp {c}: rel_fro={e:.3e}", flush=True)
        assert e <= 1e-7


@pytest.mark.parametrize("Norb,shift", [(5, (0, 9, 18, 27, 36, 43, -9, 3)),
                                         (10, (0, 12, 24, 36, 43, -12, 5, -43))])
def test_fp64_arithmetic_on_complex64_storage_wide_spread(Norb, shift):
    # odd Norb^2 rows of complex64 are copied in 4-byte units; the spreads cut
    # the taps into several windows
    prob = configs.Problem(NA=7, NB=3, Norb=Norb, Nkz=2, Nqz=2, NE=44, Nw=len(shift),
                           shift=shift)
    dp = gu.DeviceProblem(prob, 43 + Norb, ncomp=1, fp32=True, scaled=True)
    assert gu.run_sse(dp, prec=3) == 0
    got = dp.sigma_host(0)
    want = gu.oracle_full(dp, 0)
    e = gu.rel_fro(got, want)
    print(f"  fp64c64 Norb={Norb}: rel_fro={e:.3e}", flush=True)
    assert e <= 1e-7


def setup_check(prec):
    import torch
    sse = _sse()
    prob = configs.Problem(NA=30, NB=4, Norb=10, Nkz=3, Nqz=3, NE=41, Nw=8)
    dp = gu.DeviceProblem(prob, 52, ncomp=2, fp32=True, scaled=True)
    assert gu.run_sse(dp, prec=prec) == 0
    desc = sse.make_desc(prob.NA, prob.NB, prob.Norb, prob.Nkz, prob.Nqz, prob.NE, prob.Nw,
                         ncomp=2, prec=prec)
    plan = sse.sse_plan(desc, prob.shifts())
    blocks_h = gu.sample_blocks(prob, 9, n_e=6, n_a=4)
    blocks = torch.from_numpy(blocks_h).cuda()
    ws = torch.empty(sse.check_workspace_bytes(len(blocks_h), 2), dtype=torch.uint8,
                     device="cuda")
    return sse, dp, plan, blocks_h, blocks, ws


@pytest.mark.parametrize("prec", [1, 2])
def test_sampled_check_agrees_with_host_error(prec):
    import torch
    sse, dp, plan, blocks_h, blocks, ws = setup_check(prec)
    item = (dp.neigh, dp.dH, dp.G, dp.D, dp.Sigma)
    ct = sse.sse_check_submit(plan, item, blocks, 1e-2, ws, torch.cuda.current_stream())
    assert sse.sse_wait(ct.ticket) == 0
    for c in range(2):
        host = gu.rel_fro(dp.device_blocks(c, blocks_h), gu.oracle_blocks(dp, c, blocks_h))
        print(f"  prec {prec} comp {c}: device check {ct.rel_err[c]:.4e} host {host:.4e}",
              flush=True)
        assert abs(ct.rel_err[c] - host) <= 1e-3 * host + 1e-12
    # same inputs, same bits of the error
    ct2 = sse.sse_check_submit(plan, item, blocks, 1e-2, ws, torch.cuda.current_stream())
    assert sse.sse_wait(ct2.ticket) == 0
    assert list(ct2.rel_err) == list(ct.rel_err)
    # a zero tolerance is missed
    ct3 = sse.sse_check_submit(plan, item, blocks, 0.0, ws, torch.cuda.current_stream())
    assert sse.sse_wait(ct3.ticket, check=False) == sse.ERR_TOLERANCE


def test_sampled_check_catches_a_corrupted_result_and_bad_blocks():
    import torch
    sse, dp, plan, blocks_h, blocks, ws = setup_check(1)
    dp.Sigma.mul_(1.001)
    item = (dp.neigh, dp.dH, dp.G, dp.D, dp.Sigma)
    ct = sse.sse_check_submit(plan, item, blocks, 1e-5, ws, torch.cuda.current_stream())
    assert sse.sse_wait(ct.ticket, check=False) == sse.ERR_TOLERANCE
    assert 0.9e-3 < ct.rel_err[0] < 1.1e-3
    bad = blocks.clone()
    bad[1, 1] = dp.prob.NE  # energy out of range
    ct = sse.sse_check_submit(plan, item, bad, 1.0, ws, torch.cuda.current_stream())
    assert sse.sse_wait(ct.ticket, check=False) == sse.ERR_ARG


def test_pending_poll_then_more_launches():
    """Regression: a poll that finds the submission still running must not make
    the next launch (the library's, the generator's or torch's) report an error."""
    import torch
    import ssegen
    sse = _sse()
    prob = configs.Problem(NA=256, NB=4, Norb=10, Nkz=5, Nqz=5, NE=300, Nw=20)
    dp = gu.DeviceProblem(prob, 61)
    desc = sse.make_desc(prob.NA, prob.NB, prob.Norb, prob.Nkz, prob.Nqz, prob.NE, prob.Nw)
    plan = sse.sse_plan(desc, prob.shifts())
    ws = torch.empty(max(plan.workspace_bytes, 256), dtype=torch.uint8, device="cuda")
    item = [(dp.neigh, dp.dH, dp.G, dp.D, dp.Sigma)]
    st = torch.cuda.current_stream()
    t1 = sse.sse_submit(plan, item, ws, st)
    saw_pending = sse.sse_poll(t1) == sse.PENDING
    x = torch.ones(1024, device="cuda")
    x.add_(1.0)                                     # torch launch
    ssegen.dev_fill_dH(3, dp.dH.numel(), dp.dH.data_ptr(), st.cuda_stream)  # generator launch
    sse.sse_wait(t1)
    t2 = sse.sse_submit(plan, item, ws, st)         # library launch
    while sse.sse_poll(t2) == sse.PENDING:
        pass
    torch.cuda.synchronize()
    assert float(x[0]) == 2.0
    print(f"  first poll pending: {saw_pending}", flush=True)
