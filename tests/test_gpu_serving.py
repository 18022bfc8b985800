"""Serving loop: results are the same alone and in a mix (bitwise), match the
oracle after perturbed SCBA iterations, the sampled check triggers the binary64
fallback, and admission respects the HBM budget."""
import numpy as np
import pytest

import oracle
import ssegen
from paper_1912_08810_amd import configs
from tests import gpu_util as gu

pytestmark = pytest.mark.gpu


def small_jobs(n, seed, iterations=3):
    from paper_1912_08810_amd import serving
    rng = np.random.default_rng(seed)
    probs = [configs.Problem(NA=int(rng.integers(20, 60)), NB=4, Norb=10, Nkz=3, Nqz=3,
                             NE=int(rng.integers(40, 90)), Nw=int(rng.integers(4, 12)))
             for _ in range(n)]
    jobs = serving.make_jobs(probs, rate=1e6, seed=seed, iterations=iterations)
    for j in jobs:
        j.arrival = 0.0
    return jobs


def test_same_result_alone_and_in_the_mix():
    from paper_1912_08810_amd import serving
    jobs = small_jobs(4, 5)
    mix = serving.Server(slots=4, keep_results=True)
    res = mix.run(jobs)
    assert all(r.status == 0 for r in res)
    for j in jobs:
        alone = serving.Server(slots=1, keep_results=True)
        r = alone.run([j])
        assert r[0].status == 0
        assert bool((alone.sigma[j.jid] == mix.sigma[j.jid]).all()), j.jid
    print(serving.summarize(res), flush=True)


def host_inputs_after(job, comp, iterations, blocks_needed_flat):
    """Inputs of the job's last iteration on the host: complex64-rounded
    generation, then the same counter-based perturbation per iteration (each
    step rounded back to complex64, as stored on the device)."""
    p = job.prob
    r64 = lambda x: x.astype(np.complex64).astype(np.complex128)
    G = r64(ssegen.G_flat_blocks(job.seed, comp, p.Norb, blocks_needed_flat))
    D = r64(ssegen.D(job.seed, comp, p.Nqz, p.Nw, p.NA, p.NB)).reshape(-1, 3, 3).copy()
    dflat = np.arange(D.shape[0])
    for it in range(1, iterations):
        G = np.ascontiguousarray(G)
        ssegen.perturb(job.seed, it - 1, ssegen.S_PERT_G + comp, G, blocks_needed_flat)
        G = r64(G)
        ssegen.perturb(job.seed, it - 1, ssegen.S_PERT_D + comp, D, dflat)
        D = r64(D)
    return G, D.reshape(p.Nqz, p.Nw, p.NA, p.NB, 3, 3)


def test_served_job_matches_oracle_after_perturbed_iterations():
    from paper_1912_08810_amd import serving
    job = small_jobs(1, 9, iterations=3)[0]
    srv = serving.Server(slots=1, keep_results=True)
    res = srv.run([job])
    assert res[0].status == 0
    p = job.prob
    sig = srv.sigma[job.jid].numpy().astype(np.float64)
    blocks = gu.sample_blocks(p, 2, n_e=8, n_a=6)
    neigh = ssegen.neigh(job.seed, p.NA, p.NB)
    dH = ssegen.dH(job.seed, p.NA, p.NB, p.Norb)
    need = oracle.needed_g_blocks(neigh, p.shifts(), p.Nkz, p.Nqz, p.NE, p.NA, blocks)
    for c in range(2):
        G, D = host_inputs_after(job, c, job.iterations, need)
        gslot = np.full(p.Nkz * p.NE * p.NA, -1, dtype=np.int64)
        gslot[need] = np.arange(need.size)
        want = oracle.sigma(neigh, dH, G, D, p.shifts(), p.Nkz, p.NE, blocks=blocks, gslot=gslot)
        s = sig[c, 0::2] + 1j * sig[c, 1::2]
        s = s.reshape(p.Nkz, p.NE, p.NA, p.Norb, p.Norb)
        got = np.stack([s[k, e, a] for k, e, a in blocks])
        err = gu.rel_fro(got, want)
        print(f"  served job comp {c}: rel_fro={err:.3e} check={res[0].max_check_err:.3e}",
              flush=True)
        assert err <= 1e-5


def test_tolerance_miss_falls_back_to_binary64():
    from paper_1912_08810_amd import serving
    job = small_jobs(1, 11, iterations=2)[0]
    srv = serving.Server(slots=1, tol=1e-7, keep_results=True)  # bf16x3 misses 1e-7
    res = srv.run([job])
    assert res[0].status == 0 and res[0].fallbacks == 2
    srv64 = serving.Server(slots=1, prec=3, keep_results=True)  # binary64 throughout
    r64 = srv64.run([job])
    assert r64[0].fallbacks == 0
    assert bool((srv.sigma[job.jid] == srv64.sigma[job.jid]).all())


def test_admission_respects_budget():
    from paper_1912_08810_amd import serving
    jobs = small_jobs(3, 13, iterations=1)
    size = {j.jid: serving.job_bytes(j.prob) for j in jobs}
    # the resident set never exceeds the budget at any admission instant
    budget = max(size.values()) * 1.5
    res = serving.Server(budget_bytes=budget, slots=3).run(jobs)
    for r in res:
        resident = sum(size[x.jid] for x in res if x.admitted <= r.admitted < x.done)
        assert resident <= budget, (r.jid, resident, budget)
    # three jobs of one size and room for one and a half: they run one at a time
    same = serving.make_jobs([jobs[0].prob] * 3, rate=1e6, seed=21, iterations=1)
    one = serving.job_bytes(jobs[0].prob)
    res = sorted(serving.Server(budget_bytes=one * 1.5, slots=3).run(same),
                 key=lambda r: r.admitted)
    for a, b in zip(res, res[1:]):
        assert b.admitted >= a.done
    with pytest.raises(ValueError):
        serving.Server(budget_bytes=min(size.values()) * 0.5).run(jobs[:1])
