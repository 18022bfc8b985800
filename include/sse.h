/*
 * sse.h -- C ABI of libsse.so, the MI355X (gfx950) electron scattering
 * self-energy library.
 *
 * Operation (Ziogas et al., SC'19, Sec. 2, Eq. (3); tensor shapes from the
 * typed Sigma program of Sec. 3): for every momentum k, energy e and atom a,
 *
 *   Sigma[k, e, a] = alpha * sum_{b < NB} sum_{q < Nqz} sum_{w < Nw} sum_{i, j < N3D}
 *       Dt[q, w, a, b, i, j] * dH[a, b, i] . G[(k - q) mod Nkz, e - s_w, f] . dH[a, b, j]^T
 *
 * where f = neigh[a, b] (the neighbour indirection of Sec. 4.1), s is the
 * caller's integer energy-shift table (s_w = w + 1 on a uniform grid), terms
 * with e - s_w outside [0, NE) are zero, and Dt is the phonon Green's function
 * already combined as D_ba - D_bb - D_aa + D_ab (Eq. (3); Sec. 4.2 lists it
 * as a kernel input).  The result overwrites Sigma.  Only the diagonal blocks
 * of Sigma are produced, as in the paper (Sec. 2).
 *
 * Memory.  Every tensor is caller-owned device memory, contiguous, row-major,
 * complex values interleaved (re, im):
 *   neigh int32   [NA, NB]
 *   dH    float64 [NA, NB, N3D, Norb, Norb]
 *   G     complex [ncomp][Nkz, NE, NA, Norb, Norb]
 *   Dt    complex [ncomp][Nqz, Nw, NA, NB, N3D, N3D]
 *   Sigma complex [ncomp][Nkz, NE, NA, Norb, Norb]
 * "complex" is complex128 (16 bytes) for SSE_FP64 and complex64 (8 bytes) for
 * SSE_FP32, SSE_BF16X3 and SSE_FP64C64.  With ncomp = 2 the lesser and greater components
 * are stacked on a leading axis; each is computed from its own G and Dt.
 * The workspace is caller-owned device memory of at least the size that
 * sse_plan reports; the library keeps no pointer after the call (or, for
 * sse_submit, after sse_poll/sse_wait has returned something other than
 * SSE_PENDING).  A plan owns only small tables (shift and tile tables) and
 * frees them in sse_plan_destroy.
 *
 * Errors.  Every function returns a status; nothing aborts and no exception
 * crosses the ABI.  sse_last_error() gives a text for the calling thread's
 * last non-OK status.  A neighbour index outside [0, NA) is detected on the
 * device: the kernels skip that neighbour (nothing out of bounds is read) and
 * the call reports SSE_ERR_NEIGH.
 *
 * Threading.  Plans are immutable after creation and may be shared between
 * threads.  sse_submit, sse_poll and sse_wait are thread-safe.  Calls that
 * share one workspace must not overlap in time.
 */
#ifndef SSE_H
#define SSE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SSE_OK = 0,
    SSE_PENDING = 1,        /* sse_poll: the submission is still running */
    SSE_ERR_ARG = 2,        /* NULL pointer, bad enum, workspace too small, unknown ticket */
    SSE_ERR_SHAPE = 3,      /* a dimension outside the supported range (see sse_plan) */
    SSE_ERR_NEIGH = 4,      /* a neighbour index outside [0, NA) was found on the device */
    SSE_ERR_NOMEM = 5,      /* a host or small device allocation of the library failed */
    SSE_ERR_BUSY = 6,       /* too many submissions in flight */
    SSE_ERR_TOLERANCE = 7,  /* sse_check: sampled error above the caller's tolerance */
    SSE_ERR_DEVICE = 8,     /* a HIP runtime call failed (the text names it) */
    SSE_ERR_UNSUPPORTED = 9 /* valid request that this library does not implement */
} sse_status;

typedef enum {
    SSE_FP64 = 0,  /* complex128 storage, binary64 arithmetic throughout */
    /* SSE_FP32 and SSE_BF16X3 (complex64 storage, the matrix cores): for each
       neighbour b the tap sum over (qz, w) runs window by window -- one window
       is one qz row and one chunk of at most chunk_taps frequencies (all that
       fit the LDS window when chunk_taps = 0) -- with the tap products and the
       sum inside a window in fp32 on MFMA, and the window sums added into
       binary64 accumulators (the sum across qz rows and chunks).  The
       accumulated sums are then rounded once to fp32 for the dH sandwich,
       whose Norb x Norb block products run in fp32 on MFMA; the sum over
       neighbours b is fp32; alpha is applied in binary64 to that fp32 sum and
       the result is stored as complex64. */
    SSE_FP32 = 1,   /* tap products in fp32 */
    SSE_BF16X3 = 2, /* tap products as bf16 hi*hi + hi*lo + lo*hi (x = hi + lo) */
    SSE_FP64C64 = 3 /* complex64 storage, binary64 arithmetic throughout (the fallback
                       of a complex64 job whose sampled check misses its tolerance) */
} sse_precision;

typedef struct {
    int32_t NA;    /* atoms, >= 1 */
    int32_t NB;    /* neighbours per atom, 1..50 (Sec. 2, typical parameter table) */
    int32_t Norb;  /* orbitals per atom, 1..30 (same table) */
    int32_t N3D;   /* vibration directions, must be 3 */
    int32_t Nkz;   /* electron momenta, >= 1 */
    int32_t Nqz;   /* phonon momenta, 1..Nkz (same momentum grid, periodic) */
    int32_t NE;    /* energies, >= 1 */
    int32_t Nw;    /* phonon frequencies, 1..128 */
    int32_t ncomp; /* 1, or 2 = lesser and greater stacked */
    int32_t prec;  /* sse_precision */
    int32_t tile_e; /* energies per output tile; 0 = the library's default (the largest
                       that fills a workgroup); clamped to [1, that default] */
    int32_t chunk_taps; /* at most this many frequencies per tap chunk (one staged G
                           window); 0 = as many as the window holds.  Under
                           SSE_FP32/SSE_BF16X3 it bounds the fp32 part of the tap sum;
                           in every precision it is a tuning parameter.  >= 0 */
    int32_t dt_antiherm; /* 0: general Dt.  1: Dt anti-Hermitian per 3 x 3 block
                            (Dt_ji = -conj(Dt_ij), as the lesser/greater phonon Green's
                            function is): only Re/Im of the entries i < j and Im of the
                            diagonal are read, which halves the tap arithmetic.  SSE_FP64
                            and SSE_FP64C64 only (SSE_ERR_UNSUPPORTED otherwise). */
    double alpha_re, alpha_im; /* prefactor; Eq. (3) is alpha = i (0 + 1i) */
} sse_desc;

/* One instance's device pointers (see the layout above). */
typedef struct {
    const int32_t *neigh;
    const double *dH;
    const void *G;
    const void *Dt;
    void *Sigma;
} sse_args;

typedef struct sse_plan_s *sse_plan_t;

/*
 * Validate a problem and build a plan.  w_shift: host array [Nw] of energy
 * index shifts, |s_w| < NE (may be negative; need not be sorted).
 * *workspace_bytes receives the device workspace size every call with this
 * plan needs.  SSE_ERR_SHAPE if NA, Nkz, NE < 1, NB outside 1..50, Norb outside
 * 1..30, N3D != 3, Nqz outside 1..Nkz, Nw outside 1..128, ncomp not 1 or 2, a
 * shift out of range, or a tensor larger than 2^62 elements.
 */
sse_status sse_plan(const sse_desc *desc, const int32_t *w_shift, sse_plan_t *plan,
                    size_t *workspace_bytes);

/*
 * Batch plan (persistent launch): n (1..64) instances of uneven sizes computed
 * by one persistent kernel launch per component.  descs[t] and w_shift[t] as
 * in sse_plan; all instances must share Norb, N3D, ncomp, prec and alpha.
 * Each instance's tile shape is its desc's tile_e (an autotuner picks it per
 * size bucket).  The launch keeps a fixed grid of two workgroups per compute
 * unit pulling tiles -- (instance, atom, kz, energy tile) -- from eight work
 * queues, one per XCD, each holding whole atoms (all kz and energy tiles of an
 * atom share G rows) ordered by decreasing tile cost; an empty queue's
 * workgroups take tiles from the others.  Device tables are built at the
 * first submission.
 */
sse_status sse_plan_batch(const sse_desc *descs, const int32_t *const *w_shift, int32_t n,
                          sse_plan_t *plan, size_t *workspace_bytes);

/*
 * Compute Sigma for a single-instance plan; returns when the result is in
 * Sigma (the work runs on `stream`, a hipStream_t; NULL = the null stream).
 */
sse_status sse_compute(sse_plan_t plan, const int32_t *neigh, const double *dH, const void *G,
                       const void *Dt, void *Sigma, void *workspace, size_t workspace_bytes,
                       void *stream);

/* Size of the device scratch that sse_compute_noalloc uses: 32 MiB, one copy per
 * GPU the library runs on, held until the process ends. */
#define SSE_NOALLOC_SCRATCH_BYTES (32u << 20)

/*
 * sse_compute without a workspace argument, for callers that cannot allocate
 * device memory (code under stream capture, tight serving loops, harnesses
 * that forbid allocation).  Same arguments, result and statuses as
 * sse_compute, and the same kernels; the scratch those kernels need (the
 * status word and, for SSE_FP32/SSE_BF16X3, the MFMA fragments and the split
 * of G) lives in a static device array of SSE_NOALLOC_SCRATCH_BYTES on the
 * current device, whose address is looked up the first time the current device
 * calls this function.  The call allocates nothing (no hipMalloc, no pinned
 * host memory, no events): it enqueues the work on `stream`, which must belong
 * to the current device, copies the status word back and synchronizes the
 * stream.  SSE_ERR_UNSUPPORTED if the plan needs more scratch than the array
 * holds (then use sse_compute), SSE_ERR_ARG for a batch plan or a NULL pointer.
 * Every call on one GPU shares that GPU's array: calls that overlap in time on
 * one GPU (from several threads or streams) race and must not be made.
 */
sse_status sse_compute_noalloc(sse_plan_t plan, const int32_t *neigh, const double *dH,
                               const void *G, const void *Dt, void *Sigma, void *stream);

/*
 * Enqueue the computation for every instance of the plan (args has one entry
 * per instance) on `stream` and return at once with a ticket.
 */
sse_status sse_submit(sse_plan_t plan, const sse_args *args, void *workspace,
                      size_t workspace_bytes, void *stream, uint64_t *ticket);

/*
 * Sampled binary64 check of a finished complex64 result (a single-instance
 * plan of precision SSE_FP32, SSE_BF16X3 or SSE_FP64C64, Norb <= 22): the
 * nblocks output blocks listed in blocks (device int32 [nblocks][3] = k, e, a)
 * are recomputed in binary64 from the same stored inputs and compared with
 * args->Sigma.  Enqueued on `stream` behind the work it checks; returns at once
 * with a ticket.  The ticket finishes with SSE_ERR_TOLERANCE if a component's
 * relative Frobenius error over the sample exceeds tol, SSE_ERR_ARG if a listed
 * block is outside the output, else SSE_OK; rel_err (host, ncomp doubles,
 * caller-owned until the ticket finishes) receives the errors.  The partial
 * sums are reduced in block order, so the same inputs give the same errors.
 * Workspace: at least 256 + 16 * nblocks * ncomp bytes, not shared with a
 * computation in flight.  (The error decides the fallback of a serving job.)
 */
sse_status sse_check_submit(sse_plan_t plan, const sse_args *args, const int32_t *blocks,
                            int32_t nblocks, double tol, double *rel_err, void *workspace,
                            size_t workspace_bytes, void *stream, uint64_t *ticket);

/*
 * Phonon scattering self-energy, Eqs. (4) and (5) (Sec. 2), for a
 * single-instance SSE_FP64 plan (the same desc: sizes, shift table, ncomp;
 * alpha is the prefactor beta of Eq. (5), i in the paper).  For frequency w,
 * momentum q, atom a and neighbour slot b < NB (f = neigh[a, b]):
 *
 *   P_ij[q, w, a, b] = sum_k sum_e tr( dH[a, b, i]^T . X[(k + q) mod Nkz, e + s_w, a]
 *                                     . dH[a, b, j] . Y[k, e, f] )
 *   Pi[q, w, a, b,  i, j] =  alpha * P_ij[q, w, a, b]          (Eq. (5))
 *   Pi[q, w, a, NB, i, j] = -sum_b Pi[q, w, a, b, i, j]       (Eq. (4), the diagonal)
 *
 * where terms with e + s_w outside [0, NE) are zero, dH[a, b, i]^T stands for
 * the back-bond derivative (real H), and X, Y are opposite components: the
 * lesser Pi takes X = G<, Y = G>, the greater one X = G>, Y = G<.  G always
 * holds both components, complex128 [2][Nkz, NE, NA, Norb, Norb] (lesser
 * first); Pi is complex128 [ncomp][Nqz, Nw, NA, NB + 1, 3, 3] (ncomp = 1: the
 * lesser only), overwritten, in the layout of the phonon Green's function
 * (Sec. 2) with the diagonal block in slot NB.  Workspace: at least 256 bytes.
 * SSE_ERR_UNSUPPORTED for another precision or Norb > 16; SSE_ERR_NEIGH (at
 * poll) for a neighbour index outside [0, NA), whose block is left zero.
 * Returns at once with a ticket (sse_poll / sse_wait).
 */
sse_status sse_pi_submit(sse_plan_t plan, const int32_t *neigh, const double *dH, const void *G,
                         void *Pi, void *workspace, size_t workspace_bytes, void *stream,
                         uint64_t *ticket);

/* sse_pi_submit, then wait for it. */
sse_status sse_pi_compute(sse_plan_t plan, const int32_t *neigh, const double *dH, const void *G,
                          void *Pi, void *workspace, size_t workspace_bytes, void *stream);

/*
 * The combination of phonon Green's function blocks that Eq. (3) sums over
 * (Sec. 2; Sec. 4.2 names it as the kernel's input), for a single-instance
 * plan (its sizes, ncomp and storage: complex128 for SSE_FP64, complex64
 * otherwise):
 *
 *   Dt[q, w, a, b, i, j] = D_ba - D_bb - D_aa + D_ab      (entry (i, j) of each block)
 *
 * D [ncomp][Nqz, Nw, NA, NB + 1, 3, 3] holds, per atom a, the blocks
 * D_a,neigh[a, b] in slots b < NB and the diagonal block D_aa in slot NB (the
 * layout of Pi); for f = neigh[a, b], D_ab = D[.., a, b], D_bb = D[.., f, NB],
 * D_aa = D[.., a, NB] and D_ba = D[.., f, r] with r the first slot of f's row
 * holding a.  The sum is formed left to right in binary64.  Dt
 * [ncomp][Nqz, Nw, NA, NB, 3, 3] is overwritten.  The table must be symmetric:
 * a neighbour index outside [0, NA), or an atom missing from the row of one of
 * its neighbours, gives SSE_ERR_NEIGH (at poll) and zero blocks there.
 * Workspace: at least 256 + 4 NA NB bytes (the reverse map).
 */
sse_status sse_dtilde_submit(sse_plan_t plan, const int32_t *neigh, const void *D, void *Dt,
                             void *workspace, size_t workspace_bytes, void *stream,
                             uint64_t *ticket);

/*
 * Retarded component from the lesser and greater ones, (X> - X<) / 2 (Sec. 2,
 * after Eq. (5); the same relation for Sigma and Pi), elementwise over the
 * plan's tensor: which = 0: X = Sigma [2][Nkz, NE, NA, Norb, Norb] (storage of
 * the plan's precision), XR [Nkz, NE, NA, Norb, Norb]; which = 1: X = Pi
 * [2][Nqz, Nw, NA, NB + 1, 3, 3] complex128 (SSE_FP64 plans), XR one component.
 * Enqueued on `stream`; returns once enqueued (no ticket: nothing is checked on
 * the device).
 */
sse_status sse_retarded(sse_plan_t plan, int32_t which, const void *X, void *XR, void *stream);

/*
 * The same Sigma as sse_compute, evaluated in the paper's own final form of
 * Eq. (3) (Sec. 4.2): the transients dH.G (M_i[k', e'] = dH[a, b, i] . G[k', e', f])
 * and dH.D (N_i[q, w] = sum_j Dt[q, w, a, b, i, j] dH[a, b, j]^T) are
 * precomputed, and for each (a, b, i, k, q) the sum over frequencies is one
 * Norb x Norb Nw x Norb GEMM of the energy window of M_i with the stacked N_i[q, :]
 * on the matrix cores (binary64).  8 N3D Norb^3 flops per (k, e, q, w, a, b)
 * against the 8 N3D^2 Norb^2 of sse_compute: it exists to measure that
 * difference.  Single-instance SSE_FP64 plans with a general Dt, Norb <= 16;
 * blocking.  Workspace: 256 bytes plus NB 3 (Nkz NE + Nqz Nw) Norb^2 16 bytes
 * per atom for at least one atom; atoms are processed in chunks that fit it.
 * SSE_ERR_UNSUPPORTED outside these limits or when the window needs more LDS
 * than a compute unit has.
 */
sse_status sse_ablation_compute(sse_plan_t plan, const int32_t *neigh, const double *dH,
                                const void *G, const void *Dt, void *Sigma, void *workspace,
                                size_t workspace_bytes, void *stream);

/* SSE_PENDING while the submission runs, else its final status (the ticket is
 * then released; polling it again gives SSE_ERR_ARG). */
sse_status sse_poll(uint64_t ticket);

/* Block until the submission ends; returns its final status and releases the ticket. */
sse_status sse_wait(uint64_t ticket);

void sse_plan_destroy(sse_plan_t plan);

/* Text for the calling thread's last non-OK status ("" if none). */
const char *sse_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SSE_H */
