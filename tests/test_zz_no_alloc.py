"""sse_compute_noalloc (the entry point for callers that cannot allocate) against
sse_compute: the same kernels with the scratch in the library's static device
array instead of a caller workspace, so the results must be identical, bit for
bit.  Two calls in a row per precision, the second on a smaller problem, so
what the first call left in the shared scratch must not leak into the second."""
import pytest

from paper_1912_08810_amd import configs

pytestmark = pytest.mark.gpu

# (larger, smaller) problem pairs; the complex64 (MFMA) ones need scratch for
# their A fragments and, in bf16x3, for the split copy of G.
PAIRS = {
    0: (configs.Problem(NA=40, NB=4, Norb=5, Nkz=3, Nqz=2, NE=90, Nw=6),
        configs.Problem(NA=16, NB=4, Norb=4, Nkz=3, Nqz=3, NE=64, Nw=4)),
    3: (configs.Problem(NA=40, NB=4, Norb=5, Nkz=3, Nqz=2, NE=90, Nw=6),
        configs.Problem(NA=16, NB=4, Norb=4, Nkz=3, Nqz=3, NE=64, Nw=4)),
    2: (configs.Problem(NA=48, NB=4, Norb=10, Nkz=3, Nqz=3, NE=120, Nw=12),
        configs.Problem(NA=20, NB=3, Norb=6, Nkz=2, Nqz=2, NE=50, Nw=5)),
    1: (configs.Problem(NA=48, NB=4, Norb=10, Nkz=3, Nqz=3, NE=120, Nw=12),
        configs.Problem(NA=20, NB=3, Norb=6, Nkz=2, Nqz=2, NE=50, Nw=5)),
}


def _both(prob, prec, seed):
    import torch
    from paper_1912_08810_amd import sse
    from tests import gpu_util as gu
    fp32 = prec != sse.FP64
    dp = gu.DeviceProblem(prob, seed, ncomp=2, fp32=fp32)
    desc = sse.make_desc(prob.NA, prob.NB, prob.Norb, prob.Nkz, prob.Nqz, prob.NE, prob.Nw,
                         ncomp=2, prec=prec)
    plan = sse.sse_plan(desc, prob.shifts())
    assert plan.workspace_bytes <= sse.NOALLOC_SCRATCH_BYTES
    print(f"[case] noalloc prec={prec} NA={prob.NA} NB={prob.NB} Norb={prob.Norb} "
          f"NE={prob.NE} Nw={prob.Nw} ws={plan.workspace_bytes}", flush=True)
    ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()
    sse.sse_compute(plan, dp.neigh, dp.dH, dp.G, dp.D, dp.Sigma, ws, stream)
    torch.cuda.synchronize()
    ref = dp.Sigma.clone()
    dp.Sigma.fill_(float("nan"))
    torch.cuda.synchronize()
    sse.sse_compute_noalloc(plan, dp.neigh, dp.dH, dp.G, dp.D, dp.Sigma, stream)
    out = dp.Sigma.clone()
    torch.cuda.synchronize()
    return dp, ref, out


@pytest.mark.parametrize("prec", [0, 3, 2, 1])
def test_noalloc_matches_workspace_path_twice(prec):
    from tests import gpu_util as gu
    for n, prob in enumerate(PAIRS[prec]):
        dp, ref, out = _both(prob, prec, configs.SEED + 31 * n + prec)
        import torch
        ity = torch.int64 if ref.dtype == torch.float64 else torch.int32
        assert torch.equal(out.view(ity), ref.view(ity)), \
            f"call {n}: noalloc result differs from sse_compute"
        # and the workspace path itself is right (the oracle on one component)
        if n == 1:
            # binary64 arithmetic; SSE_FP64C64 stores complex64 (rounding ~6e-8)
            tol = {0: 1e-12, 3: 1e-7, 1: 1e-5, 2: 1e-3}[prec]
            err = gu.rel_fro(dp.sigma_host(1), gu.oracle_full(dp, 1))
            assert err <= tol, err


def test_noalloc_rejects_plans_beyond_the_scratch():
    from paper_1912_08810_amd import sse
    p = configs.DEVICE
    desc = sse.make_desc(p.NA, p.NB, p.Norb, p.Nkz, p.Nqz, p.NE, p.Nw, ncomp=1, prec=sse.BF16X3)
    plan = sse.sse_plan(desc, p.shifts())
    assert plan.workspace_bytes > sse.NOALLOC_SCRATCH_BYTES
    st = sse.sse_compute_noalloc(plan, 1, 1, 1, 1, 1, None, check=False)
    assert st == sse.ERR_UNSUPPORTED
    assert "scratch" in sse.last_error()
    big = configs.Problem(NA=64, NB=4, Norb=4, Nkz=3, Nqz=3, NE=64, Nw=4)
    bplan = sse.sse_plan_batch([sse.make_desc(big.NA, big.NB, big.Norb, big.Nkz, big.Nqz,
                                              big.NE, big.Nw)], [big.shifts()])
    assert sse.sse_compute_noalloc(bplan, 1, 1, 1, 1, 1, None, check=False) == sse.ERR_ARG
