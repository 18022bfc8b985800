// sse_runtime.hip -- host runtime of libsse: plan validation and tile
// geometry, submission onto the caller's stream, tickets, error state.
// Implements the C ABI declared in include/sse.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <mutex>
#include <new>
#include <string>
#include <unordered_map>
#include <vector>

#include "sse_internal.h"

using namespace sse;

namespace {

thread_local std::string g_err;

sse_status fail(sse_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

sse_status hip_fail(hipError_t e, const char *what)
{
    return fail(SSE_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

// One problem instance of a plan.
struct Instance {
    sse_desc d;
    TapTable taps;  // sorted and chunked for this instance's tile geometry
    TileGeom geom;
};

constexpr size_t kStatusBytes = 256;  // status word region at the start of the workspace

}  // namespace

struct sse_plan_s {
    std::vector<Instance> inst;
    size_t ws_bytes = kStatusBytes;
};

namespace {

struct Ticket {
    hipEvent_t ev = nullptr;
    uint32_t *host_status = nullptr;  // pinned
};

std::mutex g_mu;
std::unordered_map<uint64_t, Ticket> g_tickets;
std::vector<uint32_t *> g_pinned_free;
std::vector<hipEvent_t> g_event_free;
uint64_t g_next_ticket = 1;
constexpr size_t kMaxInFlight = 4096;

bool fits62(std::initializer_list<int64_t> dims)
{
    long double p = 1;
    for (int64_t v : dims)
        p *= (long double)v;
    return p < (long double)(1LL << 62);
}

sse_status check_desc(const sse_desc *d, const int32_t *w_shift)
{
    if (!d || !w_shift)
        return fail(SSE_ERR_ARG, "sse_plan: desc and w_shift must be non-NULL");
    if (d->prec < SSE_FP64 || d->prec > SSE_BF16X3)
        return fail(SSE_ERR_ARG, "sse_plan: unknown precision %d", d->prec);
    if (d->NA < 1 || d->Nkz < 1 || d->NE < 1)
        return fail(SSE_ERR_SHAPE, "sse_plan: NA, Nkz, NE must be >= 1 (got %d, %d, %d)", d->NA,
                    d->Nkz, d->NE);
    if (d->NB < 1 || d->NB > kMaxNB)
        return fail(SSE_ERR_SHAPE, "sse_plan: NB=%d outside 1..%d", d->NB, kMaxNB);
    if (d->Norb < 1 || d->Norb > kMaxNorb)
        return fail(SSE_ERR_SHAPE, "sse_plan: Norb=%d outside 1..%d", d->Norb, kMaxNorb);
    if (d->N3D != kN3D)
        return fail(SSE_ERR_SHAPE, "sse_plan: N3D=%d, must be 3", d->N3D);
    if (d->Nqz < 1 || d->Nqz > d->Nkz)
        return fail(SSE_ERR_SHAPE, "sse_plan: Nqz=%d outside 1..Nkz=%d", d->Nqz, d->Nkz);
    if (d->Nw < 1 || d->Nw > kMaxTaps)
        return fail(SSE_ERR_SHAPE, "sse_plan: Nw=%d outside 1..%d", d->Nw, kMaxTaps);
    if (d->ncomp != 1 && d->ncomp != 2)
        return fail(SSE_ERR_SHAPE, "sse_plan: ncomp=%d, must be 1 or 2", d->ncomp);
    for (int w = 0; w < d->Nw; ++w)
        if (w_shift[w] <= -d->NE || w_shift[w] >= d->NE)
            return fail(SSE_ERR_SHAPE, "sse_plan: |w_shift[%d]|=%d not below NE=%d", w, w_shift[w],
                        d->NE);
    const int64_t NN = (int64_t)d->Norb * d->Norb;
    if (!fits62({d->ncomp, d->Nkz, d->NE, d->NA, NN}) ||
        !fits62({d->ncomp, d->Nqz, d->Nw, d->NA, d->NB, kNF}))
        return fail(SSE_ERR_SHAPE, "sse_plan: tensor too large");
    return SSE_OK;
}

TapTable sorted_taps(const sse_desc &d, const int32_t *w_shift)
{
    TapTable t{};
    t.n = d.Nw;
    std::vector<int> order(d.Nw);
    for (int w = 0; w < d.Nw; ++w)
        order[w] = w;
    std::stable_sort(order.begin(), order.end(),
                     [&](int x, int y) { return w_shift[x] > w_shift[y]; });
    for (int u = 0; u < d.Nw; ++u) {
        t.w[u] = order[u];
        t.s[u] = w_shift[order[u]];
    }
    return t;
}

sse_status build_instance(const sse_desc *d, const int32_t *w_shift, int te_request, Instance *out)
{
    sse_status st = check_desc(d, w_shift);
    if (st != SSE_OK)
        return st;
    out->d = *d;
    TapTable t = sorted_taps(*d, w_shift);
    if (d->prec == SSE_FP64) {
        out->geom = fp64_geometry(d->Norb, d->NE, t, te_request, &out->taps);
    } else {
        return fail(SSE_ERR_UNSUPPORTED, "sse_plan: precision %d not available in this build",
                    d->prec);
    }
    const int64_t nwg = (int64_t)out->geom.n_etiles * d->Nkz * d->NA;
    if (nwg > 0x7fffffffLL)
        return fail(SSE_ERR_SHAPE, "sse_plan: %lld tiles exceed one launch", (long long)nwg);
    return SSE_OK;
}

size_t elem_bytes(int prec) { return prec == SSE_FP64 ? 16 : 8; }

sse_status enqueue_instance(const Instance &I, const sse_args &a, uint32_t *dstatus, hipStream_t s)
{
    const sse_desc &d = I.d;
    hipError_t e = launch_validate_neigh(a.neigh, (int64_t)d.NA * d.NB, d.NA, dstatus, s);
    if (e != hipSuccess)
        return hip_fail(e, "validate_neigh launch");
    const size_t NN = (size_t)d.Norb * d.Norb;
    const size_t g_elems = (size_t)d.Nkz * d.NE * d.NA * NN;
    const size_t d_elems = (size_t)d.Nqz * d.Nw * d.NA * d.NB * kNF;
    const size_t eb = elem_bytes(d.prec);
    for (int c = 0; c < d.ncomp; ++c) {
        const char *G = (const char *)a.G + c * g_elems * eb;
        const char *D = (const char *)a.Dt + c * d_elems * eb;
        char *S = (char *)a.Sigma + c * g_elems * eb;
        if (d.prec == SSE_FP64) {
            Fp64Params p{};
            p.neigh = a.neigh;
            p.dH = a.dH;
            p.G = (const double2 *)G;
            p.D = (const double2 *)D;
            p.Sigma = (double2 *)S;
            p.NA = d.NA;
            p.NB = d.NB;
            p.Norb = d.Norb;
            p.NN = (int)NN;
            p.Nkz = d.Nkz;
            p.Nqz = d.Nqz;
            p.NE = d.NE;
            p.Nw = d.Nw;
            p.TE = I.geom.TE;
            p.n_etiles = I.geom.n_etiles;
            p.n_wg = (int64_t)I.geom.n_etiles * d.Nkz * d.NA;
            p.lds_win = I.geom.lds_win;
            p.alpha_re = d.alpha_re;
            p.alpha_im = d.alpha_im;
            p.taps = I.taps;
            e = fp64_launch(p, I.geom.lds_bytes, s);
            if (e != hipSuccess)
                return hip_fail(e, "fp64 kernel launch");
        } else {
            return fail(SSE_ERR_UNSUPPORTED, "precision %d not available", d.prec);
        }
    }
    return SSE_OK;
}

}  // namespace

extern "C" {

const char *sse_last_error(void) { return g_err.c_str(); }

sse_status sse_plan(const sse_desc *desc, const int32_t *w_shift, sse_plan_t *plan,
                    size_t *workspace_bytes)
{
    if (!plan)
        return fail(SSE_ERR_ARG, "sse_plan: plan must be non-NULL");
    *plan = nullptr;
    sse_plan_s *p = new (std::nothrow) sse_plan_s;
    if (!p)
        return fail(SSE_ERR_NOMEM, "sse_plan: out of host memory");
    p->inst.resize(1);
    sse_status st = build_instance(desc, w_shift, 0, &p->inst[0]);
    if (st != SSE_OK) {
        delete p;
        return st;
    }
    *plan = p;
    if (workspace_bytes)
        *workspace_bytes = p->ws_bytes;
    return SSE_OK;
}

sse_status sse_plan_batch(const sse_desc *descs, const int32_t *const *w_shift, int32_t n,
                          sse_plan_t *plan, size_t *workspace_bytes)
{
    if (!plan || !descs || !w_shift || n < 1)
        return fail(SSE_ERR_ARG, "sse_plan_batch: NULL argument or n < 1");
    *plan = nullptr;
    sse_plan_s *p = new (std::nothrow) sse_plan_s;
    if (!p)
        return fail(SSE_ERR_NOMEM, "sse_plan_batch: out of host memory");
    p->inst.resize(n);
    for (int t = 0; t < n; ++t) {
        const sse_desc &d0 = descs[0], &dt = descs[t];
        if (dt.Norb != d0.Norb || dt.ncomp != d0.ncomp || dt.prec != d0.prec ||
            dt.alpha_re != d0.alpha_re || dt.alpha_im != d0.alpha_im) {
            delete p;
            return fail(SSE_ERR_ARG, "sse_plan_batch: instance %d differs in Norb/ncomp/prec/alpha",
                        t);
        }
        sse_status st = build_instance(&descs[t], w_shift[t], 0, &p->inst[t]);
        if (st != SSE_OK) {
            delete p;
            return st;
        }
    }
    *plan = p;
    if (workspace_bytes)
        *workspace_bytes = p->ws_bytes;
    return SSE_OK;
}

void sse_plan_destroy(sse_plan_t plan) { delete plan; }

sse_status sse_submit(sse_plan_t plan, const sse_args *args, void *workspace,
                      size_t workspace_bytes, void *stream, uint64_t *ticket)
{
    if (!plan || !args || !ticket)
        return fail(SSE_ERR_ARG, "sse_submit: NULL plan, args or ticket");
    if (!workspace || workspace_bytes < plan->ws_bytes)
        return fail(SSE_ERR_ARG, "sse_submit: workspace of %zu bytes needed", plan->ws_bytes);
    for (size_t t = 0; t < plan->inst.size(); ++t) {
        const sse_args &a = args[t];
        if (!a.neigh || !a.dH || !a.G || !a.Dt || !a.Sigma)
            return fail(SSE_ERR_ARG, "sse_submit: NULL tensor pointer for instance %zu", t);
    }
    hipStream_t s = (hipStream_t)stream;
    Ticket tk;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        if (g_tickets.size() >= kMaxInFlight)
            return fail(SSE_ERR_BUSY, "sse_submit: %zu submissions in flight", g_tickets.size());
        if (!g_pinned_free.empty()) {
            tk.host_status = g_pinned_free.back();
            g_pinned_free.pop_back();
        }
        if (!g_event_free.empty()) {
            tk.ev = g_event_free.back();
            g_event_free.pop_back();
        }
    }
    hipError_t e;
    if (!tk.host_status) {
        e = hipHostMalloc((void **)&tk.host_status, sizeof(uint32_t), hipHostMallocDefault);
        if (e != hipSuccess)
            return hip_fail(e, "hipHostMalloc");
    }
    if (!tk.ev) {
        e = hipEventCreateWithFlags(&tk.ev, hipEventDisableTiming);
        if (e != hipSuccess)
            return hip_fail(e, "hipEventCreate");
    }
    auto give_back = [&]() {
        std::lock_guard<std::mutex> lk(g_mu);
        g_pinned_free.push_back(tk.host_status);
        g_event_free.push_back(tk.ev);
    };
    *tk.host_status = 0xffffffffu;
    uint32_t *dstatus = (uint32_t *)workspace;
    e = launch_clear_status(dstatus, s);
    if (e != hipSuccess) {
        give_back();
        return hip_fail(e, "clear_status launch");
    }
    for (size_t t = 0; t < plan->inst.size(); ++t) {
        sse_status st = enqueue_instance(plan->inst[t], args[t], dstatus, s);
        if (st != SSE_OK) {
            give_back();
            return st;
        }
    }
    e = hipMemcpyAsync(tk.host_status, dstatus, sizeof(uint32_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipEventRecord(tk.ev, s);
    if (e != hipSuccess) {
        give_back();
        return hip_fail(e, "status copy / event record");
    }
    std::lock_guard<std::mutex> lk(g_mu);
    *ticket = g_next_ticket++;
    g_tickets[*ticket] = tk;
    return SSE_OK;
}

static sse_status finish_ticket(uint64_t ticket, bool block)
{
    Ticket tk;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        auto it = g_tickets.find(ticket);
        if (it == g_tickets.end())
            return fail(SSE_ERR_ARG, "unknown ticket %llu", (unsigned long long)ticket);
        tk = it->second;
    }
    hipError_t e = block ? hipEventSynchronize(tk.ev) : hipEventQuery(tk.ev);
    if (e == hipErrorNotReady)
        return SSE_PENDING;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        auto it = g_tickets.find(ticket);
        if (it == g_tickets.end())
            return fail(SSE_ERR_ARG, "ticket %llu already finished", (unsigned long long)ticket);
        g_tickets.erase(it);
    }
    const uint32_t hs = *tk.host_status;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        g_pinned_free.push_back(tk.host_status);
        g_event_free.push_back(tk.ev);
    }
    if (e != hipSuccess)
        return hip_fail(e, "waiting for a submission");
    if (hs & kStatusBadNeigh)
        return fail(SSE_ERR_NEIGH, "a neighbour index is outside [0, NA)");
    if (hs != 0)
        return fail(SSE_ERR_DEVICE, "device status word 0x%x", hs);
    return SSE_OK;
}

sse_status sse_poll(uint64_t ticket) { return finish_ticket(ticket, false); }

sse_status sse_wait(uint64_t ticket) { return finish_ticket(ticket, true); }

sse_status sse_compute(sse_plan_t plan, const int32_t *neigh, const double *dH, const void *G,
                       const void *Dt, void *Sigma, void *workspace, size_t workspace_bytes,
                       void *stream)
{
    if (!plan)
        return fail(SSE_ERR_ARG, "sse_compute: NULL plan");
    if (plan->inst.size() != 1)
        return fail(SSE_ERR_ARG, "sse_compute: batch plan; use sse_submit with one sse_args per instance");
    sse_args a{neigh, dH, G, Dt, Sigma};
    uint64_t t = 0;
    sse_status st = sse_submit(plan, &a, workspace, workspace_bytes, stream, &t);
    if (st != SSE_OK)
        return st;
    return sse_wait(t);
}

}  // extern "C"
