"""The opt-in anti-Hermitian D~ mode of the binary64 kernels (dt_antiherm = 1):
half the tap arithmetic, the same result on anti-Hermitian D~ (the generator's
blocks are), checked against the oracle at the binary64 bar; on a general D~
only the entries i < j and the imaginary diagonal are read, which the oracle
reproduces on the anti-Hermitian completion of that triangle."""
import numpy as np
import pytest

import oracle
import ssegen
from paper_1912_08810_amd import configs
from tests import gpu_util as gu

pytestmark = pytest.mark.gpu
TOL = 1e-12


def run_ah(dp, prec=0, alpha=1j):
    import torch
    from paper_1912_08810_amd import sse
    p = dp.prob
    desc = sse.make_desc(p.NA, p.NB, p.Norb, p.Nkz, p.Nqz, p.NE, p.Nw, ncomp=dp.ncomp, prec=prec,
                         alpha=alpha, dt_antiherm=1)
    plan = sse.sse_plan(desc, p.shifts())
    ws = torch.empty(max(plan.workspace_bytes, 256), dtype=torch.uint8, device="cuda")
    print(f"[case] antiherm NA={p.NA} Norb={p.Norb} NE={p.NE} Nw={p.Nw} prec={prec}", flush=True)
    st = sse.sse_compute(plan, dp.neigh, dp.dH, dp.G, dp.D, dp.Sigma, ws,
                         torch.cuda.current_stream(), check=False)
    torch.cuda.synchronize()
    return st


@pytest.mark.parametrize("prob", [
    configs.SMALL,
    configs.Problem(NA=37, NB=5, Norb=10, Nkz=4, Nqz=3, NE=47, Nw=7, shift=(3, 1, -2, 7, 5, 2, 4)),
    configs.Problem(NA=6, NB=3, Norb=10, Nkz=2, Nqz=2, NE=40, Nw=9,
                    shift=(0, 8, 16, 24, 32, 39, -8, -16, -39)),
], ids=["small", "ragged", "many_chunks"])
def test_antihermitian_mode_matches_oracle(prob):
    dp = gu.DeviceProblem(prob, 61, ncomp=2)
    assert run_ah(dp) == 0
    for c in range(2):
        e = gu.rel_fro(dp.sigma_host(c), gu.oracle_full(dp, c))
        print(f"  comp {c}: rel_fro={e:.3e}", flush=True)
        assert e <= TOL, e


def test_antihermitian_mode_complex64_storage():
    prob = configs.Problem(NA=20, NB=4, Norb=6, Nkz=3, Nqz=3, NE=33, Nw=6)
    dp = gu.DeviceProblem(prob, 67, ncomp=1, fp32=True)
    assert run_ah(dp, prec=3) == 0
    e = gu.rel_fro(dp.sigma_host(0), gu.oracle_full(dp, 0))
    assert e <= 1e-7, e   # binary64 arithmetic, complex64 result


def test_general_Dt_reads_only_the_upper_triangle():
    import torch
    prob = configs.Problem(NA=8, NB=3, Norb=4, Nkz=2, Nqz=2, NE=12, Nw=3)
    dp = gu.DeviceProblem(prob, 71, ncomp=1)
    rng = np.random.default_rng(3)
    D = (rng.standard_normal((prob.Nqz, prob.Nw, prob.NA, prob.NB, 3, 3))
         + 1j * rng.standard_normal((prob.Nqz, prob.Nw, prob.NA, prob.NB, 3, 3)))
    dp.D.copy_(torch.from_numpy(np.ascontiguousarray(D).view(np.float64).reshape(1, -1)).cuda())
    assert run_ah(dp) == 0
    # the anti-Hermitian completion of the strict upper triangle and imaginary diagonal
    U = np.triu(D, 1)
    Dc = U - np.conj(np.swapaxes(U, -1, -2)) + 1j * np.imag(D) * np.eye(3)
    dH = ssegen.dH(71, prob.NA, prob.NB, prob.Norb)
    G = ssegen.G(71, 0, prob.Nkz, prob.NE, prob.NA, prob.Norb)
    want = oracle.sigma(dp.neigh_h, dH, G, Dc, prob.shifts(), prob.Nkz, prob.NE)
    e = gu.rel_fro(dp.sigma_host(0), want)
    assert e <= TOL, e


def test_antihermitian_batch_matches_one_shot_bitwise():
    import torch
    from paper_1912_08810_amd import sse
    probs = [configs.Problem(NA=30, NB=4, Norb=10, Nkz=3, Nqz=3, NE=41, Nw=9),
             configs.Problem(NA=11, NB=4, Norb=10, Nkz=3, Nqz=2, NE=25, Nw=14)]
    dps = [gu.DeviceProblem(p, 80 + i, ncomp=1) for i, p in enumerate(probs)]
    descs = [sse.make_desc(p.NA, p.NB, p.Norb, p.Nkz, p.Nqz, p.NE, p.Nw, dt_antiherm=1)
             for p in probs]
    plan = sse.sse_plan_batch(descs, [p.shifts() for p in probs])
    ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device="cuda")
    t = sse.sse_submit(plan, [(d.neigh, d.dH, d.G, d.D, d.Sigma) for d in dps], ws,
                       torch.cuda.current_stream())
    sse.sse_wait(t)
    batched = [d.Sigma.clone() for d in dps]
    for d, b in zip(dps, batched):
        assert run_ah(d) == 0
        assert torch.equal(d.Sigma.view(torch.int64), b.view(torch.int64))
        e = gu.rel_fro(d.sigma_host(0), gu.oracle_full(d, 0))
        assert e <= TOL, e


def test_antihermitian_mode_refused_on_the_matrix_cores():
    from paper_1912_08810_amd import sse
    for prec in (sse.FP32, sse.BF16X3):
        with pytest.raises(sse.SSEError) as ei:
            sse.sse_plan(sse.make_desc(16, 4, 4, 3, 3, 64, 4, prec=prec, dt_antiherm=1),
                         np.arange(1, 5))
        assert ei.value.status == sse.ERR_UNSUPPORTED
