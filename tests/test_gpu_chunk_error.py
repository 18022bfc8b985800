"""The two-level accumulation of the complex64 matrix-core forms as a function
of the tap-chunk length (chunk_taps: at most this many frequencies summed in
fp32 before the partial sum is added into binary64): device-scale shapes with
G magnitudes over eight decades, one component, sampled blocks against the
oracle.  Every chunk length meets the form's bar; the printed table (error and
launch time per chunk length) is the record of how the error depends on it."""
import numpy as np
import pytest

from paper_1912_08810_amd import configs
from tests import gpu_util as gu

pytestmark = pytest.mark.gpu
TOL = {1: 1e-5, 2: 1e-3}
CHUNKS = [1, 2, 4, 8, 15, 0]   # 0 = as many as the LDS window holds (30 at this size)


@pytest.mark.parametrize("prec", [1, 2])
def test_error_against_chunk_length(prec):
    import torch
    from paper_1912_08810_amd import sse
    prob = configs.DEVICE
    dp = gu.DeviceProblem(prob, configs.SEED, ncomp=1, fp32=True, scaled=True)
    blocks = gu.sample_blocks(prob, 23, n_e=8, n_a=4)
    want = gu.oracle_blocks(dp, 0, blocks)
    stream = torch.cuda.current_stream()
    rows = []
    for ct in CHUNKS:
        desc = sse.make_desc(prob.NA, prob.NB, prob.Norb, prob.Nkz, prob.Nqz, prob.NE, prob.Nw,
                             prec=prec, chunk_taps=ct)
        plan = sse.sse_plan(desc, prob.shifts())
        ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device="cuda")
        print(f"[case] prec={prec} chunk_taps={ct}", flush=True)
        sse.sse_compute(plan, dp.neigh, dp.dH, dp.G, dp.D, dp.Sigma, ws, stream)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        sse.sse_compute(plan, dp.neigh, dp.dH, dp.G, dp.D, dp.Sigma, ws, stream)
        e1.record(stream)
        e1.synchronize()
        got = dp.device_blocks(0, blocks)
        err = gu.rel_fro(got, want)
        rows.append((ct, err, e0.elapsed_time(e1)))
        del ws
    print(f"prec {prec}: chunk_taps | rel. Frobenius error over {len(blocks)} blocks | ms/launch")
    for ct, err, ms in rows:
        print(f"  {ct if ct else 'all (30)':>8} | {err:.3e} | {ms:.1f}", flush=True)
    for ct, err, ms in rows:
        assert err <= TOL[prec], (ct, err)
