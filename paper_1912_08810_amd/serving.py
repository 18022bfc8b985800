"""Continuous-batching serving loop for self-energy jobs on one GPU.

A job is one device (one problem size) iterated self-consistently: in every
iteration the Green's functions are refreshed and Sigma lesser/greater are
recomputed (the GF <-> SSE alternation of Sec. 2; here the GF phase is stood in
for by a 1% on-device perturbation of the resident G and D~).  The loop

* admits arrived jobs first-come-first-served while the job fits the HBM
  budget and a slot (stream) is free; admission allocates the job's tensors and
  generates its inputs on the device, where they stay for all iterations;
* keeps several jobs in flight, each on its own HIP stream, so their kernels
  overlap on the device (a new job starts as soon as memory and a slot free up);
* runs each iteration as: perturb (iterations >= 1) -> complex64 compute
  (sse_submit) -> sampled binary64 check (sse_check_submit) -> on a tolerance
  miss, a binary64-arithmetic recompute (SSE_FP64C64) and a re-check;
* records per-job latency (arrival to completion) and reports p50/p99 beside
  throughput.

Every step on the GPU goes through libsse (compute, check) or the seeded
generator (input generation and perturbation); this module only schedules.
Kernels are deterministic and the check reduces in a fixed order, so a job's
result is the same alone and in a mix.
"""
from __future__ import annotations

import dataclasses
import math
import time

import numpy as np

import ssegen
from . import configs, sse


@dataclasses.dataclass
class JobSpec:
    jid: int
    prob: configs.Problem
    seed: int
    arrival: float            # seconds after the start of the run
    iterations: int = 10


@dataclasses.dataclass
class JobResult:
    jid: int
    arrival: float
    admitted: float
    done: float
    flops: float
    fallbacks: int
    max_check_err: float
    status: int

    @property
    def latency(self) -> float:
        return self.done - self.arrival


def job_bytes(prob: configs.Problem, ncomp: int = 2, nsample: int = 64) -> int:
    """Device bytes a job holds while admitted (complex64 storage)."""
    g = prob.g_elems() * 8 * ncomp
    d = prob.d_elems() * 8 * ncomp
    dh = prob.NA * prob.NB * prob.N3D * prob.NN * 8
    groups = sum(math.ceil(n / 8) for n in [prob.Nw])  # one chunk at these sizes
    afrag = prob.NA * prob.NB * prob.Nqz * groups * 64 * 32
    split = prob.g_elems() * 8  # bf16 (hi, lo) copy of one component's G
    return 2 * g + d + dh + afrag + split + 512 + sse.check_workspace_bytes(nsample, ncomp) + \
        prob.NA * prob.NB * 4


def poisson_arrivals(n: int, rate: float, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=n)) - 0.0


def make_jobs(probs, rate: float, seed: int, iterations: int = 10):
    arr = poisson_arrivals(len(probs), rate, seed)
    return [JobSpec(i, p, seed * 1000 + i, float(arr[i]), iterations)
            for i, p in enumerate(probs)]


class _Active:
    """An admitted job: resident tensors, plans, its stream and iteration state."""

    def __init__(self, spec: JobSpec, prec: int, stream, nsample: int, now: float):
        import torch
        from ssegen.device_problem import DeviceProblem
        self.spec = spec
        self.admitted = now
        p = spec.prob
        self.stream = stream
        mk = lambda pr: sse.make_desc(p.NA, p.NB, p.Norb, p.Nkz, p.Nqz, p.NE, p.Nw, ncomp=2,
                                      prec=pr)
        self.plan = sse.sse_plan(mk(prec), p.shifts())
        self.plan_fb = sse.sse_plan(mk(sse.FP64C64), p.shifts())
        nbytes = max(self.plan.workspace_bytes, self.plan_fb.workspace_bytes, 256)
        rng = np.random.default_rng(spec.seed + 17)
        blocks = np.stack([rng.integers(0, p.Nkz, nsample), rng.integers(0, p.NE, nsample),
                           rng.integers(0, p.NA, nsample)], axis=1).astype(np.int32)
        # every allocation and the input generation are ordered on the job's stream
        with torch.cuda.stream(stream):
            self.dp = DeviceProblem(p, spec.seed, ncomp=2, fp32=True, sync=False)
            self.ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
            self.blocks = torch.from_numpy(blocks).cuda()
            self.cws = torch.empty(sse.check_workspace_bytes(nsample, 2), dtype=torch.uint8,
                                   device="cuda")
        self.item = (self.dp.neigh, self.dp.dH, self.dp.G, self.dp.D, self.dp.Sigma)
        self.it = 0
        self.phase = None
        self.ticket = None
        self.check = None
        self.fallbacks = 0
        self.max_err = 0.0
        self.status = sse.OK

    def perturb(self):
        p = self.spec.prob
        st = self.stream.cuda_stream
        esz = 8
        for c in range(2):
            ssegen.dev_perturb(self.spec.seed, self.it - 1, ssegen.S_PERT_G + c, p.Norb,
                               p.Nkz * p.NE * p.NA,
                               self.dp.G.data_ptr() + c * p.g_elems() * esz, fp32=True,
                               stream=st)
            ssegen.dev_perturb(self.spec.seed, self.it - 1, ssegen.S_PERT_D + c, p.N3D,
                               p.Nqz * p.Nw * p.NA * p.NB,
                               self.dp.D.data_ptr() + c * p.d_elems() * esz, fp32=True,
                               stream=st)

    def start_iteration(self):
        if self.it > 0:
            self.perturb()
        self.ticket = sse.sse_submit(self.plan, [self.item], self.ws, self.stream)
        self.phase = "compute"

    def submit_check(self, tol):
        self.check = sse.sse_check_submit(self.plan, self.item, self.blocks, tol, self.cws,
                                          self.stream)
        self.ticket = self.check.ticket

    def drain(self):
        """Wait for the job's submission in flight (used when the loop is aborted)."""
        if self.ticket is not None:
            sse.lib.sse_wait(self.ticket)
            self.ticket = None

    def step(self, tol) -> bool:
        """Advance if the current submission finished; True when the job is done."""
        st = sse.lib.sse_poll(self.ticket)
        if st == sse.PENDING:
            return False
        if self.phase in ("compute", "fallback"):
            if st != sse.OK:
                self.status = st
                return True
            self.submit_check(tol)
            self.phase = "check" if self.phase == "compute" else "recheck"
            return False
        # a check finished
        err = max(self.check.rel_err[0], self.check.rel_err[1])
        self.max_err = max(self.max_err, err if err == err else float("inf"))
        if st == sse.ERR_TOLERANCE and self.phase == "check":
            self.fallbacks += 1
            self.ticket = sse.sse_submit(self.plan_fb, [self.item], self.ws, self.stream)
            self.phase = "fallback"
            return False
        if st != sse.OK:
            self.status = st
            return True
        self.it += 1
        if self.it >= self.spec.iterations:
            return True
        self.start_iteration()
        return False


class Server:
    """Continuous-batching loop over a list of jobs with arrival times."""

    def __init__(self, budget_bytes: float = 200e9, slots: int = 4, prec: int = sse.BF16X3,
                 tol: float = 1e-5, nsample: int = 64, keep_results: bool = False):
        self.budget = budget_bytes
        self.slots = slots
        self.prec = prec
        self.tol = tol
        self.nsample = nsample
        self.keep = keep_results
        self.sigma = {}

    def run(self, jobs, log=None):
        import torch
        streams = [torch.cuda.Stream() for _ in range(self.slots)]
        free_streams = list(range(self.slots))
        pending = sorted(jobs, key=lambda j: (j.arrival, j.jid))
        for j in pending:
            if job_bytes(j.prob, nsample=self.nsample) > self.budget:
                raise ValueError(f"job {j.jid} needs more than the HBM budget")
        active, results = {}, []
        try:
            return self._loop(pending, active, results, streams, free_streams, log)
        except BaseException:
            # never free a job's tensors while its work is still on the device
            for a in active.values():
                a.drain()
            torch.cuda.synchronize()
            raise

    def _loop(self, pending, active, results, streams, free_streams, log):
        import torch
        used = 0
        t0 = time.perf_counter()
        while pending or active:
            now = time.perf_counter() - t0
            # admission: first come first served, by budget and free slot
            while pending and free_streams and pending[0].arrival <= now:
                need = job_bytes(pending[0].prob, nsample=self.nsample)
                if used + need > self.budget:
                    break
                spec = pending.pop(0)
                si = free_streams.pop(0)
                a = _Active(spec, self.prec, streams[si], self.nsample, now)
                a.si, a.need = si, need
                used += need
                a.start_iteration()
                active[spec.jid] = a
                if log:
                    log(f"t={now:7.3f}s admit job {spec.jid} ({spec.prob.NA} atoms, "
                        f"{spec.prob.NE} energies, {spec.prob.Nw} frequencies)")
            progressed = False
            for jid in list(active):
                a = active[jid]
                if a.step(self.tol):
                    progressed = True
                    torch.cuda.current_stream().wait_stream(a.stream)
                    t_done = time.perf_counter() - t0
                    p = a.spec.prob
                    flops = 2.0 * p.flops() * a.spec.iterations
                    results.append(JobResult(jid, a.spec.arrival, a.admitted, t_done, flops,
                                             a.fallbacks, a.max_err, a.status))
                    if self.keep:
                        self.sigma[jid] = a.dp.Sigma.cpu()
                    if log:
                        log(f"t={t_done:7.3f}s done job {jid} latency "
                            f"{t_done - a.spec.arrival:.3f}s fallbacks {a.fallbacks} "
                            f"check {a.max_err:.2e}")
                    free_streams.append(a.si)
                    used -= a.need
                    del active[jid]
            if not progressed:
                wait = 2e-4
                if pending and not active:
                    wait = max(0.0, min(0.05, pending[0].arrival - now))
                time.sleep(wait)
        torch.cuda.synchronize()
        return results


def summarize(results, t_first: float = None):
    lat = np.array([r.latency for r in results])
    done = max(r.done for r in results)
    start = min(r.arrival for r in results) if t_first is None else t_first
    span = done - start
    flops = sum(r.flops for r in results)
    return {
        "jobs": len(results),
        "makespan_s": round(span, 3),
        "jobs_per_s": round(len(results) / span, 4),
        "tflops": round(flops / span / 1e12, 3),
        "latency_p50_s": round(float(np.percentile(lat, 50)), 3),
        "latency_p99_s": round(float(np.percentile(lat, 99)), 3),
        "fallbacks": int(sum(r.fallbacks for r in results)),
        "max_check_err": float(max(r.max_check_err for r in results)),
        "failed": int(sum(r.status != 0 for r in results)),
    }
