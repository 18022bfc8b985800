// sse_runtime.hip -- host runtime of libsse: plan validation and tile
// geometry, submission onto the caller's stream, tickets, error state.
// Implements the C ABI declared in include/sse.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <cstdarg>
#include <cstdio>
#include <mutex>
#include <new>
#include <string>
#include <unordered_map>
#include <vector>

#include "sse_internal.h"
#include "sse_mfma.h"

using namespace sse;

// Device scratch of sse_compute_noalloc: the status word and, for the complex64
// precisions, the MFMA auxiliary data that sse_compute takes from the caller's
// workspace.  One copy per GPU, held for the life of the process.  In host code
// the name stands for a host-side shadow, never a device address: kernels get
// the address that hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) unsigned char scratch[SSE_NOALLOC_SCRATCH_BYTES];

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
    TapTable taps;      // sorted and chunked for this instance's tile geometry
    GroupTable groups;  // MFMA path: tap groups per chunk
    TileGeom geom;
    size_t afrag_bytes = 0;  // MFMA path: workspace for the A fragments (+ split G, bf16x3)
    int32_t shift[kMaxTaps] = {};  // the caller's shift table, in frequency order
};

constexpr size_t kStatusBytes = 256;  // status word region at the start of the workspace

}  // namespace

struct sse_plan_s {
    std::vector<Instance> inst;
    size_t ws_bytes = kStatusBytes;
    bool batch = false;
    // ---- batch plans: device tables, built at the first submission
    std::once_flag tables_once;
    hipError_t tables_err = hipSuccess;
    void *d_params = nullptr;
    int32_t *d_chunk_inst = nullptr, *d_chunk_atom = nullptr;
    int64_t *d_chunk_start = nullptr;
    int32_t qbeg[kQueues + 1] = {};
    int64_t qcount[kQueues] = {};
    std::vector<size_t> afrag_off;  // per instance, offset of its A fragments in the workspace
    size_t lds_bytes = 0;
    int grid = 0;
    ~sse_plan_s()
    {
        // nothing useful can be done with a failure while destroying a plan
        (void)hipFree(d_params);
        (void)hipFree(d_chunk_inst);
        (void)hipFree(d_chunk_atom);
        (void)hipFree(d_chunk_start);
    }
};

namespace {

struct Ticket {
    hipEvent_t ev = nullptr;
    uint32_t *host_status = nullptr;  // pinned 64-byte block: status word, then check sums
    int ncheck = 0;                   // sse_check_submit: components checked
    double tol = 0.0;
    double *rel_out = nullptr;        // caller's host array for the errors
};
constexpr size_t kHostBlock = 64;

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
    if (d->prec < SSE_FP64 || d->prec > SSE_FP64C64)
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
    if (d->tile_e < 0 || d->chunk_taps < 0)
        return fail(SSE_ERR_ARG, "sse_plan: tile_e and chunk_taps must be >= 0");
    if (d->dt_antiherm != 0 && d->dt_antiherm != 1)
        return fail(SSE_ERR_ARG, "sse_plan: dt_antiherm must be 0 or 1");
    if (d->dt_antiherm && d->prec != SSE_FP64 && d->prec != SSE_FP64C64)
        return fail(SSE_ERR_UNSUPPORTED,
                    "sse_plan: dt_antiherm is a binary64-kernel mode (the matrix-core forms' tap "
                    "products are dense real GEMMs whose row count it would not change)");
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

sse_status build_instance(const sse_desc *d, const int32_t *w_shift, Instance *out)
{
    const int te_request = d ? d->tile_e : 0;
    sse_status st = check_desc(d, w_shift);
    if (st != SSE_OK)
        return st;
    out->d = *d;
    for (int w = 0; w < d->Nw; ++w)
        out->shift[w] = w_shift[w];
    TapTable t = sorted_taps(*d, w_shift);
    if (d->prec == SSE_FP64 || d->prec == SSE_FP64C64) {
        out->geom = fp64_geometry(d->Norb, d->NE, t, te_request, d->chunk_taps, &out->taps);
    } else {
        if (d->Norb > 22)
            return fail(SSE_ERR_UNSUPPORTED,
                        "sse_plan: the complex64 (MFMA) precisions support Norb <= 22 (got %d)",
                        d->Norb);
        out->geom = mfma_geometry(d->Norb, d->NE, t, te_request, d->chunk_taps, &out->taps,
                                  &out->groups);
        out->afrag_bytes = mfma_aux_bytes(d->prec, d->NA, d->NB, d->Nqz, d->Nkz, d->NE, d->Norb,
                                          out->groups);
    }
    const int64_t nwg = (int64_t)out->geom.n_etiles * d->Nkz * d->NA;
    if (nwg > 0x7fffffffLL)
        return fail(SSE_ERR_SHAPE, "sse_plan: %lld tiles exceed one launch", (long long)nwg);
    return SSE_OK;
}

size_t elem_bytes(int prec) { return prec == SSE_FP64 ? 16 : 8; }
bool fp64_arith(int prec) { return prec == SSE_FP64 || prec == SSE_FP64C64; }

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

sse_status enqueue_instance(const Instance &I, const sse_args &a, uint32_t *dstatus, void *wsfree,
                            hipStream_t s)
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
        if (d.prec == SSE_FP64 || d.prec == SSE_FP64C64) {
            Fp64Params p{};
            p.neigh = a.neigh;
            p.dH = a.dH;
            p.G = G;
            p.D = D;
            p.Sigma = S;
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
            fill_tap_pairs(p);
            e = fp64_launch(p, d.prec == SSE_FP64C64, d.dt_antiherm != 0, I.geom.lds_bytes, s);
            if (e != hipSuccess)
                return hip_fail(e, "fp64 kernel launch");
        } else {
            MfmaPrepParams pp{};
            pp.D = (const float2 *)D;
            pp.zero = wsfree;
            pp.afrag = (char *)wsfree + mfmak::kZeroPage;
            pp.NA = d.NA;
            pp.NB = d.NB;
            pp.Nqz = d.Nqz;
            pp.Nw = d.Nw;
            pp.taps = I.taps;
            pp.groups = I.groups;
            e = mfma_prep_launch(d.prec, pp, s);
            if (e != hipSuccess)
                return hip_fail(e, "MFMA prep launch");
            const void *Gm = G;
            if (d.prec == SSE_BF16X3) {
                char *split = (char *)wsfree + mfma_split_offset(d.prec, d.NA, d.NB, d.Nqz,
                                                                 I.groups);
                e = mfma_split_launch((const float2 *)G, split, (int64_t)g_elems, s);
                if (e != hipSuccess)
                    return hip_fail(e, "G split launch");
                Gm = split;
            }
            MfmaParams p{};
            p.neigh = a.neigh;
            p.dH = a.dH;
            p.G = Gm;
            p.afrag = wsfree;
            p.Sigma = (float2 *)S;
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
            p.groups = I.groups;
            e = mfma_launch(d.prec, p, I.geom.lds_bytes, s);
            if (e != hipSuccess)
                return hip_fail(e, "MFMA kernel launch");
        }
    }
    return SSE_OK;
}

// Per-instance static launch parameters (sizes, taps, geometry; no pointers).
Fp64Params fp64_params(const Instance &I)
{
    const sse_desc &d = I.d;
    Fp64Params p{};
    p.NA = d.NA;
    p.NB = d.NB;
    p.Norb = d.Norb;
    p.NN = d.Norb * d.Norb;
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
    fill_tap_pairs(p);
    return p;
}

MfmaParams mfma_params(const Instance &I)
{
    const sse_desc &d = I.d;
    MfmaParams p{};
    p.NA = d.NA;
    p.NB = d.NB;
    p.Norb = d.Norb;
    p.NN = d.Norb * d.Norb;
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
    p.groups = I.groups;
    return p;
}

// Work queues of a batch plan: atoms of all instances, instances in order of
// decreasing tile cost, dealt round-robin to the eight queues.
hipError_t build_batch_tables(sse_plan_s *P)
{
    const int n = (int)P->inst.size();
    std::vector<int> order(n);
    for (int t = 0; t < n; ++t)
        order[t] = t;
    auto cost = [&](int t) {
        const sse_desc &d = P->inst[t].d;
        return (double)d.NB * d.Nqz * d.Nw * P->inst[t].geom.TE;
    };
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return cost(x) > cost(y); });
    std::vector<std::vector<int32_t>> qi(kQueues), qa(kQueues);
    std::vector<std::vector<int64_t>> qs(kQueues);
    std::vector<int64_t> qtot(kQueues, 0);
    int64_t c = 0;
    for (int t : order) {
        const Instance &I = P->inst[t];
        const int64_t tiles = (int64_t)I.d.Nkz * I.geom.n_etiles;
        for (int a = 0; a < I.d.NA; ++a, ++c) {
            const int x = (int)(c % kQueues);
            qi[x].push_back(t);
            qa[x].push_back(a);
            qs[x].push_back(qtot[x]);
            qtot[x] += tiles;
        }
    }
    std::vector<int32_t> ci, ca;
    std::vector<int64_t> cs;
    for (int x = 0; x < kQueues; ++x) {
        P->qbeg[x] = (int32_t)ci.size();
        P->qcount[x] = qtot[x];
        ci.insert(ci.end(), qi[x].begin(), qi[x].end());
        ca.insert(ca.end(), qa[x].begin(), qa[x].end());
        cs.insert(cs.end(), qs[x].begin(), qs[x].end());
    }
    P->qbeg[kQueues] = (int32_t)ci.size();
    const bool fp64 = fp64_arith(P->inst[0].d.prec);
    const size_t psz = fp64 ? sizeof(Fp64Params) : sizeof(MfmaParams);
    std::vector<unsigned char> params(psz * n);
    for (int t = 0; t < n; ++t) {
        if (fp64) {
            Fp64Params fp = fp64_params(P->inst[t]);
            memcpy(params.data() + psz * t, &fp, psz);
        } else {
            MfmaParams mp = mfma_params(P->inst[t]);
            memcpy(params.data() + psz * t, &mp, psz);
        }
    }
    hipError_t e;
    if ((e = hipMalloc(&P->d_params, params.size())) != hipSuccess ||
        (e = hipMalloc((void **)&P->d_chunk_inst, ci.size() * 4)) != hipSuccess ||
        (e = hipMalloc((void **)&P->d_chunk_atom, ca.size() * 4)) != hipSuccess ||
        (e = hipMalloc((void **)&P->d_chunk_start, cs.size() * 8)) != hipSuccess)
        return e;
    if ((e = hipMemcpy(P->d_params, params.data(), params.size(), hipMemcpyHostToDevice)) !=
            hipSuccess ||
        (e = hipMemcpy(P->d_chunk_inst, ci.data(), ci.size() * 4, hipMemcpyHostToDevice)) !=
            hipSuccess ||
        (e = hipMemcpy(P->d_chunk_atom, ca.data(), ca.size() * 4, hipMemcpyHostToDevice)) !=
            hipSuccess ||
        (e = hipMemcpy(P->d_chunk_start, cs.data(), cs.size() * 8, hipMemcpyHostToDevice)) !=
            hipSuccess)
        return e;
    int dev = 0, cus = 0;
    if ((e = hipGetDevice(&dev)) != hipSuccess ||
        (e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess)
        return e;
    // two binary64 workgroups per CU (256 threads each), one MFMA workgroup (512)
    P->grid = std::max(8, (fp64_arith(P->inst[0].d.prec) ? 2 : 1) * cus);
    return hipSuccess;
}

sse_status enqueue_batch(sse_plan_s *P, const sse_args *args, char *ws, uint32_t *dstatus,
                         hipStream_t s)
{
    std::call_once(P->tables_once, [&] { P->tables_err = build_batch_tables(P); });
    if (P->tables_err != hipSuccess)
        return hip_fail(P->tables_err, "building the batch tables");
    const int n = (int)P->inst.size();
    const sse_desc &d0 = P->inst[0].d;
    hipError_t e;
    {
        // every instance's neighbour table in one launch
        const int32_t *tabs[kMaxBatch];
        int64_t cnt[kMaxBatch];
        int32_t na[kMaxBatch];
        for (int t = 0; t < n; ++t) {
            tabs[t] = args[t].neigh;
            cnt[t] = (int64_t)P->inst[t].d.NA * P->inst[t].d.NB;
            na[t] = P->inst[t].d.NA;
        }
        e = launch_validate_neigh_batch(tabs, cnt, na, n, dstatus, s);
        if (e != hipSuccess)
            return hip_fail(e, "validate_neigh launch");
    }
    unsigned long long *counters = (unsigned long long *)(ws + kStatusBytes);
    const size_t eb = elem_bytes(d0.prec);
    for (int c = 0; c < d0.ncomp; ++c) {
        BatchLaunch bl{};
        bl.params = P->d_params;
        bl.chunk_inst = P->d_chunk_inst;
        bl.chunk_atom = P->d_chunk_atom;
        bl.chunk_start = P->d_chunk_start;
        bl.counters = counters;
        for (int x = 0; x <= kQueues; ++x)
            bl.qbeg[x] = P->qbeg[x];
        for (int x = 0; x < kQueues; ++x)
            bl.qcount[x] = P->qcount[x];
        // bf16x3: every instance's G split in one launch after the loop
        const float2 *split_in[kMaxBatch];
        void *split_out[kMaxBatch];
        int64_t split_n[kMaxBatch];
        int nsplit = 0;
        for (int t = 0; t < n; ++t) {
            const sse_desc &d = P->inst[t].d;
            const size_t NN = (size_t)d.Norb * d.Norb;
            const size_t g_elems = (size_t)d.Nkz * d.NE * d.NA * NN;
            const size_t d_elems = (size_t)d.Nqz * d.Nw * d.NA * d.NB * kNF;
            bl.nkz[t] = d.Nkz;
            bl.ptr[t].neigh = args[t].neigh;
            bl.ptr[t].dH = args[t].dH;
            bl.ptr[t].G = (const char *)args[t].G + c * g_elems * eb;
            bl.ptr[t].D = (const char *)args[t].Dt + c * d_elems * eb;
            bl.ptr[t].Sigma = (char *)args[t].Sigma + c * g_elems * eb;
            bl.ptr[t].aux = ws + P->afrag_off[t];
            if (d.prec == SSE_BF16X3) {
                char *split = ws + P->afrag_off[t] +
                              mfma_split_offset(d.prec, d.NA, d.NB, d.Nqz, P->inst[t].groups);
                split_in[nsplit] = (const float2 *)bl.ptr[t].G;
                split_out[nsplit] = split;
                split_n[nsplit] = (int64_t)g_elems;
                ++nsplit;
                bl.ptr[t].G = split;
            }
        }
        if (nsplit > 0) {
            e = mfma_split_batch_launch(split_in, split_out, split_n, nsplit, s);
            if (e != hipSuccess)
                return hip_fail(e, "G split launch");
        }
        if (!fp64_arith(d0.prec)) {
            // every instance's A fragments in one launch
            e = mfma_prep_batch_launch(d0.prec, bl, n, s);
            if (e != hipSuccess)
                return hip_fail(e, "MFMA prep launch");
        }
        e = launch_clear_u64(counters, kQueues, s);
        if (e != hipSuccess)
            return hip_fail(e, "counter clear launch");
        if (fp64_arith(d0.prec))
            e = fp64_persistent_launch(bl, d0.prec == SSE_FP64C64, d0.dt_antiherm != 0, P->grid,
                                       P->lds_bytes, s);
        else
            e = mfma_persistent_launch(d0.prec, bl, P->grid, P->lds_bytes, s);
        if (e != hipSuccess)
            return hip_fail(e, "persistent kernel launch");
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
    sse_status st = build_instance(desc, w_shift, &p->inst[0]);
    if (st != SSE_OK) {
        delete p;
        return st;
    }
    p->ws_bytes = kStatusBytes + align256(p->inst[0].afrag_bytes);
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
    if (n > kMaxBatch)
        return fail(SSE_ERR_ARG, "sse_plan_batch: n=%d above %d instances", n, kMaxBatch);
    *plan = nullptr;
    sse_plan_s *p = new (std::nothrow) sse_plan_s;
    if (!p)
        return fail(SSE_ERR_NOMEM, "sse_plan_batch: out of host memory");
    p->batch = true;
    p->inst.resize(n);
    p->afrag_off.resize(n);
    size_t ws = 2 * kStatusBytes;  // status word, then the queue counters
    for (int t = 0; t < n; ++t) {
        const sse_desc &d0 = descs[0], &dt = descs[t];
        if (dt.Norb != d0.Norb || dt.ncomp != d0.ncomp || dt.prec != d0.prec ||
            dt.alpha_re != d0.alpha_re || dt.alpha_im != d0.alpha_im || dt.N3D != d0.N3D ||
            dt.dt_antiherm != d0.dt_antiherm) {
            delete p;
            return fail(SSE_ERR_ARG, "sse_plan_batch: instance %d differs in Norb/ncomp/prec/alpha/dt_antiherm",
                        t);
        }
        sse_status st = build_instance(&descs[t], w_shift[t], &p->inst[t]);
        if (st != SSE_OK) {
            delete p;
            return st;
        }
        p->afrag_off[t] = ws;
        ws += align256(p->inst[t].afrag_bytes);
        p->lds_bytes = std::max(p->lds_bytes, p->inst[t].geom.lds_bytes);
    }
    p->ws_bytes = ws;
    *plan = p;
    if (workspace_bytes)
        *workspace_bytes = p->ws_bytes;
    return SSE_OK;
}

void sse_plan_destroy(sse_plan_t plan) { delete plan; }

static sse_status ticket_acquire(Ticket *tk)
{
    {
        std::lock_guard<std::mutex> lk(g_mu);
        if (g_tickets.size() >= kMaxInFlight)
            return fail(SSE_ERR_BUSY, "sse_submit: %zu submissions in flight", g_tickets.size());
        if (!g_pinned_free.empty()) {
            tk->host_status = g_pinned_free.back();
            g_pinned_free.pop_back();
        }
        if (!g_event_free.empty()) {
            tk->ev = g_event_free.back();
            g_event_free.pop_back();
        }
    }
    hipError_t e;
    if (!tk->host_status) {
        e = hipHostMalloc((void **)&tk->host_status, kHostBlock, hipHostMallocDefault);
        if (e != hipSuccess)
            return hip_fail(e, "hipHostMalloc");
    }
    if (!tk->ev) {
        e = hipEventCreateWithFlags(&tk->ev, hipEventDisableTiming);
        if (e != hipSuccess)
            return hip_fail(e, "hipEventCreate");
    }
    *tk->host_status = 0xffffffffu;
    return SSE_OK;
}

static void ticket_release(const Ticket &tk)
{
    std::lock_guard<std::mutex> lk(g_mu);
    if (tk.host_status)
        g_pinned_free.push_back(tk.host_status);
    if (tk.ev)
        g_event_free.push_back(tk.ev);
}

// Copies the device status (and check sums) to the ticket's pinned block,
// records its event and registers it.
static sse_status ticket_finish_enqueue(Ticket &tk, const void *dstatus, size_t bytes,
                                        hipStream_t s, uint64_t *ticket)
{
    hipError_t e = hipMemcpyAsync(tk.host_status, dstatus, bytes, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipEventRecord(tk.ev, s);
    if (e != hipSuccess) {
        ticket_release(tk);
        return hip_fail(e, "status copy / event record");
    }
    std::lock_guard<std::mutex> lk(g_mu);
    *ticket = g_next_ticket++;
    g_tickets[*ticket] = tk;
    return SSE_OK;
}

sse_status sse_check_submit(sse_plan_t plan, const sse_args *args, const int32_t *blocks,
                            int32_t nblocks, double tol, double *rel_err, void *workspace,
                            size_t workspace_bytes, void *stream, uint64_t *ticket)
{
    if (!plan || !args || !blocks || !rel_err || !ticket || nblocks < 1)
        return fail(SSE_ERR_ARG, "sse_check_submit: NULL argument or nblocks < 1");
    if (plan->batch || plan->inst.size() != 1)
        return fail(SSE_ERR_ARG, "sse_check_submit: needs a single-instance plan");
    const Instance &I = plan->inst[0];
    const sse_desc &d = I.d;
    if (d.prec == SSE_FP64)
        return fail(SSE_ERR_ARG, "sse_check_submit: checks complex64 results only");
    if (d.Norb > 22)
        return fail(SSE_ERR_UNSUPPORTED, "sse_check_submit: Norb <= 22");
    const size_t need = kStatusBytes + (size_t)16 * nblocks * d.ncomp;
    if (!workspace || workspace_bytes < need)
        return fail(SSE_ERR_ARG, "sse_check_submit: workspace of %zu bytes needed", need);
    const sse_args &a = args[0];
    if (!a.neigh || !a.dH || !a.G || !a.Dt || !a.Sigma)
        return fail(SSE_ERR_ARG, "sse_check_submit: NULL tensor pointer");
    hipStream_t s = (hipStream_t)stream;
    Ticket tk;
    sse_status st = ticket_acquire(&tk);
    if (st != SSE_OK)
        return st;
    tk.ncheck = d.ncomp;
    tk.tol = tol;
    tk.rel_out = rel_err;
    char *ws = (char *)workspace;
    uint32_t *dstatus = (uint32_t *)ws;
    double *sums = (double *)(ws + 16);
    hipError_t e = launch_clear_status(dstatus, s);
    if (e == hipSuccess)
        e = launch_validate_neigh(a.neigh, (int64_t)d.NA * d.NB, d.NA, dstatus, s);
    const size_t NN = (size_t)d.Norb * d.Norb;
    const size_t g_elems = (size_t)d.Nkz * d.NE * d.NA * NN;
    const size_t d_elems = (size_t)d.Nqz * d.Nw * d.NA * d.NB * kNF;
    for (int c = 0; c < d.ncomp && e == hipSuccess; ++c) {
        CheckParams cp{};
        cp.neigh = a.neigh;
        cp.dH = a.dH;
        cp.G = (const float2 *)a.G + c * g_elems;
        cp.D = (const float2 *)a.Dt + c * d_elems;
        cp.Sigma = (const float2 *)a.Sigma + c * g_elems;
        cp.blocks = blocks;
        cp.nblocks = nblocks;
        cp.partial = (double *)(ws + kStatusBytes) + (size_t)2 * nblocks * c;
        cp.status = dstatus;
        cp.NA = d.NA;
        cp.NB = d.NB;
        cp.Norb = d.Norb;
        cp.NN = (int)NN;
        cp.Nkz = d.Nkz;
        cp.Nqz = d.Nqz;
        cp.NE = d.NE;
        cp.Nw = d.Nw;
        cp.alpha_re = d.alpha_re;
        cp.alpha_im = d.alpha_im;
        for (int t = 0; t < I.taps.n; ++t)
            cp.shift[I.taps.w[t]] = I.taps.s[t];
        e = check_launch(cp, sums + 2 * c, s);
    }
    if (e != hipSuccess) {
        ticket_release(tk);
        return hip_fail(e, "check launch");
    }
    return ticket_finish_enqueue(tk, ws, 16 + 16 * d.ncomp, s, ticket);
}

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
    sse_status st = ticket_acquire(&tk);
    if (st != SSE_OK)
        return st;
    uint32_t *dstatus = (uint32_t *)workspace;
    hipError_t e = launch_clear_status(dstatus, s);
    if (e != hipSuccess) {
        ticket_release(tk);
        return hip_fail(e, "clear_status launch");
    }
    if (plan->batch)
        st = enqueue_batch(plan, args, (char *)workspace, dstatus, s);
    else
        st = enqueue_instance(plan->inst[0], args[0], dstatus, (char *)workspace + kStatusBytes, s);
    if (st != SSE_OK) {
        ticket_release(tk);
        return st;
    }
    return ticket_finish_enqueue(tk, dstatus, sizeof(uint32_t), s, ticket);
}

// Status of a finished submission from its device status word.
static sse_status status_from_word(uint32_t hs)
{
    if (hs & kStatusBadNeigh)
        return fail(SSE_ERR_NEIGH, "a neighbour index is outside [0, NA)");
    if (hs & kStatusBadBlock)
        return fail(SSE_ERR_ARG, "sse_check_submit: a listed block is outside the output");
    if (hs & kStatusAsymNeigh)
        return fail(SSE_ERR_NEIGH, "the neighbour table is not symmetric: an atom is missing "
                                   "from the row of one of its neighbours");
    if (hs != 0)
        return fail(SSE_ERR_DEVICE, "device status word 0x%x", hs);
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
    if (e == hipErrorNotReady) {
        // HIP records the query's "not ready" as the thread's last error; clear it so
        // the next launch check (ours or the caller's) does not read it as a failure.
        (void)hipGetLastError();
        return SSE_PENDING;
    }
    {
        std::lock_guard<std::mutex> lk(g_mu);
        auto it = g_tickets.find(ticket);
        if (it == g_tickets.end())
            return fail(SSE_ERR_ARG, "ticket %llu already finished", (unsigned long long)ticket);
        g_tickets.erase(it);
    }
    const uint32_t hs = *tk.host_status;
    double sums[4] = {0, 0, 0, 0};
    for (int c = 0; c < 2 * tk.ncheck; ++c)
        sums[c] = ((const double *)((const char *)tk.host_status + 16))[c];
    ticket_release(tk);
    if (e != hipSuccess)
        return hip_fail(e, "waiting for a submission");
    const sse_status hst = status_from_word(hs);
    if (hst != SSE_OK)
        return hst;
    if (tk.ncheck > 0) {
        bool miss = false;
        for (int c = 0; c < tk.ncheck; ++c) {
            const double d2 = sums[2 * c], r2 = sums[2 * c + 1];
            const double rel = r2 > 0.0 ? sqrt(d2 / r2) : sqrt(d2);
            tk.rel_out[c] = rel;
            miss |= !(rel <= tk.tol);
        }
        if (miss)
            return fail(SSE_ERR_TOLERANCE, "sampled error above tolerance %g", tk.tol);
    }
    return SSE_OK;
}

sse_status sse_poll(uint64_t ticket) { return finish_ticket(ticket, false); }

sse_status sse_wait(uint64_t ticket) { return finish_ticket(ticket, true); }

}  // extern "C"

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// The device address of `scratch` on the current device, looked up once per
// device (with that device current) and kept.
sse_status scratch_for_current_device(void **out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices)
        return fail(SSE_ERR_UNSUPPORTED, "sse_compute_noalloc: device %d above %d", dev,
                    kMaxDevices - 1);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess)
            return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p)
            return fail(SSE_ERR_DEVICE, "hipGetSymbolAddress(scratch) gave NULL");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return SSE_OK;
}

}  // namespace

extern "C" {

sse_status sse_compute_noalloc(sse_plan_t plan, const int32_t *neigh, const double *dH,
                               const void *G, const void *Dt, void *Sigma, void *stream)
{
    if (!plan)
        return fail(SSE_ERR_ARG, "sse_compute_noalloc: NULL plan");
    if (plan->batch || plan->inst.size() != 1)
        return fail(SSE_ERR_ARG, "sse_compute_noalloc: needs a single-instance plan");
    if (!neigh || !dH || !G || !Dt || !Sigma)
        return fail(SSE_ERR_ARG, "sse_compute_noalloc: NULL tensor pointer");
    if (plan->ws_bytes > (size_t)SSE_NOALLOC_SCRATCH_BYTES)
        return fail(SSE_ERR_UNSUPPORTED,
                    "sse_compute_noalloc: the plan needs %zu bytes of scratch, the static scratch "
                    "holds %zu (use sse_compute with a workspace)",
                    plan->ws_bytes, (size_t)SSE_NOALLOC_SCRATCH_BYTES);
    void *ws = nullptr;
    sse_status st = scratch_for_current_device(&ws);
    if (st != SSE_OK)
        return st;
    hipStream_t s = (hipStream_t)stream;
    uint32_t *dstatus = (uint32_t *)ws;
    hipError_t e = launch_clear_status(dstatus, s);
    if (e != hipSuccess)
        return hip_fail(e, "clear_status launch");
    sse_args a{neigh, dH, G, Dt, Sigma};
    st = enqueue_instance(plan->inst[0], a, dstatus, (char *)ws + kStatusBytes, s);
    if (st != SSE_OK)
        return st;
    uint32_t hs = 0xffffffffu;
    e = hipMemcpyAsync(&hs, dstatus, sizeof hs, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);
    if (e != hipSuccess)
        return hip_fail(e, "sse_compute_noalloc: waiting for the computation");
    return status_from_word(hs);
}

sse_status sse_pi_submit(sse_plan_t plan, const int32_t *neigh, const double *dH, const void *G,
                         void *Pi, void *workspace, size_t workspace_bytes, void *stream,
                         uint64_t *ticket)
{
    if (!plan || !ticket || !neigh || !dH || !G || !Pi)
        return fail(SSE_ERR_ARG, "sse_pi_submit: NULL argument");
    if (plan->batch || plan->inst.size() != 1)
        return fail(SSE_ERR_ARG, "sse_pi_submit: needs a single-instance plan");
    const Instance &I = plan->inst[0];
    const sse_desc &d = I.d;
    if (d.prec != SSE_FP64)
        return fail(SSE_ERR_UNSUPPORTED, "sse_pi_submit: the phonon self-energy is SSE_FP64 only");
    if (d.Norb > pik::kMaxNorb)
        return fail(SSE_ERR_UNSUPPORTED, "sse_pi_submit: Norb <= %d (got %d)", pik::kMaxNorb,
                    d.Norb);
    if (!workspace || workspace_bytes < kStatusBytes)
        return fail(SSE_ERR_ARG, "sse_pi_submit: workspace of %zu bytes needed", kStatusBytes);
    const PiGeom gm = pi_geometry(d.Norb, d.NB, I.shift, d.Nw);
    if (!gm.ok)
        return fail(SSE_ERR_UNSUPPORTED, "sse_pi_submit: Norb=%d leaves no room for the ring",
                    d.Norb);
    const int nbgroups = (d.NB + gm.nbw - 1) / gm.nbw;
    const int64_t n_wg = (int64_t)d.NA * d.Nqz * nbgroups * gm.nchunk;
    if (n_wg > 0x7fffffffLL)
        return fail(SSE_ERR_SHAPE, "sse_pi_submit: %lld workgroups exceed one launch",
                    (long long)n_wg);
    hipStream_t s = (hipStream_t)stream;
    Ticket tk;
    sse_status st = ticket_acquire(&tk);
    if (st != SSE_OK)
        return st;
    uint32_t *dstatus = (uint32_t *)workspace;
    hipError_t e = launch_clear_status(dstatus, s);
    if (e == hipSuccess)
        e = launch_validate_neigh(neigh, (int64_t)d.NA * d.NB, d.NA, dstatus, s);
    const size_t NN = (size_t)d.Norb * d.Norb;
    const size_t g_elems = (size_t)d.Nkz * d.NE * d.NA * NN;
    const size_t pi_elems = (size_t)d.Nqz * d.Nw * d.NA * (d.NB + 1) * kNF;
    for (int c = 0; c < d.ncomp && e == hipSuccess; ++c) {
        PiParams pp{};
        pp.X = (const double2 *)G + (size_t)c * g_elems;
        pp.Y = (const double2 *)G + (size_t)(1 - c) * g_elems;
        pp.dH = dH;
        pp.neigh = neigh;
        pp.Pi = (double2 *)Pi + (size_t)c * pi_elems;
        pp.NA = d.NA;
        pp.NB = d.NB;
        pp.Norb = d.Norb;
        pp.NN = (int)NN;
        pp.Nkz = d.Nkz;
        pp.Nqz = d.Nqz;
        pp.NE = d.NE;
        pp.Nw = d.Nw;
        pp.nchunk = gm.nchunk;
        pp.R = gm.R;
        pp.nbw = gm.nbw;
        pp.nbgroups = nbgroups;
        pp.mtiles = gm.mtiles;
        memcpy(pp.cb, gm.cb, sizeof pp.cb);
        memcpy(pp.tw, gm.tw, sizeof pp.tw);
        memcpy(pp.ts, gm.ts, sizeof pp.ts);
        pp.n_wg = n_wg;
        pp.beta_re = d.alpha_re;
        pp.beta_im = d.alpha_im;
        e = pi_launch(pp, gm.lds_bytes, s);
    }
    if (e != hipSuccess) {
        ticket_release(tk);
        return hip_fail(e, "phonon kernel launch");
    }
    return ticket_finish_enqueue(tk, dstatus, sizeof(uint32_t), s, ticket);
}

sse_status sse_pi_compute(sse_plan_t plan, const int32_t *neigh, const double *dH, const void *G,
                          void *Pi, void *workspace, size_t workspace_bytes, void *stream)
{
    uint64_t t = 0;
    sse_status st = sse_pi_submit(plan, neigh, dH, G, Pi, workspace, workspace_bytes, stream, &t);
    if (st != SSE_OK)
        return st;
    return sse_wait(t);
}

sse_status sse_dtilde_submit(sse_plan_t plan, const int32_t *neigh, const void *D, void *Dt,
                             void *workspace, size_t workspace_bytes, void *stream,
                             uint64_t *ticket)
{
    if (!plan || !ticket || !neigh || !D || !Dt)
        return fail(SSE_ERR_ARG, "sse_dtilde_submit: NULL argument");
    if (plan->batch || plan->inst.size() != 1)
        return fail(SSE_ERR_ARG, "sse_dtilde_submit: needs a single-instance plan");
    const sse_desc &d = plan->inst[0].d;
    const size_t need = kStatusBytes + (size_t)4 * d.NA * d.NB;
    if (!workspace || workspace_bytes < need)
        return fail(SSE_ERR_ARG, "sse_dtilde_submit: workspace of %zu bytes needed", need);
    hipStream_t s = (hipStream_t)stream;
    Ticket tk;
    sse_status st = ticket_acquire(&tk);
    if (st != SSE_OK)
        return st;
    uint32_t *dstatus = (uint32_t *)workspace;
    int32_t *rmap = (int32_t *)((char *)workspace + kStatusBytes);
    const bool c64 = d.prec != SSE_FP64;
    const size_t eb = c64 ? 8 : 16;
    const int64_t nqw = (int64_t)d.Nqz * d.Nw;
    const size_t d_in = (size_t)nqw * d.NA * (d.NB + 1) * kNF;
    const size_t d_out = (size_t)nqw * d.NA * d.NB * kNF;
    hipError_t e = launch_clear_status(dstatus, s);
    for (int c = 0; c < d.ncomp && e == hipSuccess; ++c)
        e = dtilde_launch((const char *)D + c * d_in * eb, (char *)Dt + c * d_out * eb, neigh,
                          rmap, dstatus, nqw, d.NA, d.NB, c64, s);
    if (e != hipSuccess) {
        ticket_release(tk);
        return hip_fail(e, "D~ kernel launch");
    }
    return ticket_finish_enqueue(tk, dstatus, sizeof(uint32_t), s, ticket);
}

sse_status sse_retarded(sse_plan_t plan, int32_t which, const void *X, void *XR, void *stream)
{
    if (!plan || !X || !XR)
        return fail(SSE_ERR_ARG, "sse_retarded: NULL argument");
    if (plan->batch || plan->inst.size() != 1)
        return fail(SSE_ERR_ARG, "sse_retarded: needs a single-instance plan");
    if (which != 0 && which != 1)
        return fail(SSE_ERR_ARG, "sse_retarded: which must be 0 (Sigma) or 1 (Pi)");
    const sse_desc &d = plan->inst[0].d;
    if (which == 1 && d.prec != SSE_FP64)
        return fail(SSE_ERR_UNSUPPORTED, "sse_retarded: Pi is complex128 (SSE_FP64) only");
    const int64_t n = which == 0 ? (int64_t)d.Nkz * d.NE * d.NA * d.Norb * d.Norb
                                 : (int64_t)d.Nqz * d.Nw * d.NA * (d.NB + 1) * kNF;
    hipError_t e = retarded_launch(X, XR, n, d.prec != SSE_FP64, (hipStream_t)stream);
    if (e != hipSuccess)
        return hip_fail(e, "retarded kernel launch");
    return SSE_OK;
}

sse_status sse_ablation_compute(sse_plan_t plan, const int32_t *neigh, const double *dH,
                                const void *G, const void *Dt, void *Sigma, void *workspace,
                                size_t workspace_bytes, void *stream)
{
    if (!plan || !neigh || !dH || !G || !Dt || !Sigma || !workspace)
        return fail(SSE_ERR_ARG, "sse_ablation_compute: NULL argument");
    if (plan->batch || plan->inst.size() != 1)
        return fail(SSE_ERR_ARG, "sse_ablation_compute: needs a single-instance plan");
    const Instance &I = plan->inst[0];
    const sse_desc &d = I.d;
    if (d.prec != SSE_FP64 || d.dt_antiherm)
        return fail(SSE_ERR_UNSUPPORTED, "sse_ablation_compute: SSE_FP64 with a general Dt only");
    if (2 * d.Norb > 16 * pik::kAblNT)
        return fail(SSE_ERR_UNSUPPORTED, "sse_ablation_compute: Norb <= %d", 8 * pik::kAblNT);
    const size_t NN = (size_t)d.Norb * d.Norb;
    AblParams p{};
    p.NA = d.NA;
    p.NB = d.NB;
    p.Norb = d.Norb;
    p.NN = (int)NN;
    p.Nkz = d.Nkz;
    p.Nqz = d.Nqz;
    p.NE = d.NE;
    p.Nw = d.Nw;
    p.TE = std::max(1, pik::kAblRows / d.Norb);
    p.n_etiles = (d.NE + p.TE - 1) / p.TE;
    int smin = I.shift[0], smax = I.shift[0];
    for (int w = 0; w < d.Nw; ++w) {
        smin = std::min(smin, I.shift[w]);
        smax = std::max(smax, I.shift[w]);
        p.shift[w] = I.shift[w];
    }
    p.smax = smax;
    p.win_rows = p.TE + smax - smin;
    p.alpha_re = d.alpha_re;
    p.alpha_im = d.alpha_im;
    const size_t kp = (size_t)d.Nw * d.Norb + ((size_t)d.Nw * d.Norb & 1);
    const size_t lds = std::max((size_t)(p.win_rows + 1) * NN * 16 +
                                    (kp + 2) * 16 * pik::kAblNT * 8 + 4 * (kp + 4),
                                (size_t)pik::kAblRows * 16 * pik::kAblNT * 8);
    if (lds > pik::kLdsBudgetOne)
        return fail(SSE_ERR_UNSUPPORTED,
                    "sse_ablation_compute: window and N_i blocks need %zu bytes of LDS", lds);
    const size_t per_atom = (size_t)d.NB * kN3D * ((size_t)d.Nkz * d.NE + (size_t)d.Nqz * d.Nw) *
                            NN * 16;
    if (workspace_bytes < kStatusBytes + per_atom)
        return fail(SSE_ERR_ARG, "sse_ablation_compute: workspace of at least %zu bytes needed",
                    kStatusBytes + per_atom);
    const int chunk = (int)std::min<size_t>(d.NA, (workspace_bytes - kStatusBytes) / per_atom);
    p.M = (double2 *)((char *)workspace + kStatusBytes);
    p.N = p.M + (size_t)chunk * d.NB * kN3D * d.Nkz * d.NE * NN;
    p.neigh = neigh;
    p.dH = dH;
    hipStream_t s = (hipStream_t)stream;
    uint32_t *dstatus = (uint32_t *)workspace;
    hipError_t e = launch_clear_status(dstatus, s);
    if (e == hipSuccess)
        e = launch_validate_neigh(neigh, (int64_t)d.NA * d.NB, d.NA, dstatus, s);
    const size_t g_elems = (size_t)d.Nkz * d.NE * d.NA * NN;
    const size_t d_elems = (size_t)d.Nqz * d.Nw * d.NA * d.NB * kNF;
    for (int c = 0; c < d.ncomp && e == hipSuccess; ++c) {
        p.G = (const double2 *)G + c * g_elems;
        p.D = (const double2 *)Dt + c * d_elems;
        p.Sigma = (double2 *)Sigma + c * g_elems;
        e = ablation_launch(p, lds, chunk, s);
    }
    if (e != hipSuccess)
        return hip_fail(e, "ablation kernel launch");
    uint32_t hs = 0xffffffffu;
    e = hipMemcpyAsync(&hs, dstatus, sizeof hs, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);
    if (e != hipSuccess)
        return hip_fail(e, "sse_ablation_compute: waiting for the computation");
    return status_from_word(hs);
}

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
