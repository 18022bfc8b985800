// Host-side runtime test: plans, submissions, sampled-check tickets and batch
// plans through the C ABI with stand-in launchers.  Exits non-zero on failure.
#include "sse.h"
#include <cstdio>
#include <cstdlib>
#include <vector>
int main() {
  sse_desc d{}; d.NA = 30; d.NB = 4; d.Norb = 10; d.N3D = 3; d.Nkz = 3; d.Nqz = 3; d.NE = 41; d.Nw = 8;
  d.ncomp = 2; d.prec = SSE_BF16X3; d.alpha_re = 0; d.alpha_im = 1;
  int32_t sh[8] = {1,2,3,4,5,6,7,8};
  sse_plan_t p, pf; size_t ws, wsf;
  if (sse_plan(&d, sh, &p, &ws)) { printf("plan: %s\n", sse_last_error()); return 1; }
  d.prec = SSE_FP64C64; sse_plan(&d, sh, &pf, &wsf);
  std::vector<char> W(ws + 4096), C(256 + 16 * 64 * 2 + 64);
  std::vector<int32_t> neigh(120), blocks(64 * 3);
  std::vector<double> dH(1), G(1), D(1), S(1);
  sse_args a{neigh.data(), dH.data(), G.data(), D.data(), S.data()};
  for (int it = 0; it < 200; ++it) {
    uint64_t t1, t2, t3;
    if (sse_submit(p, &a, W.data(), ws, nullptr, &t1)) { printf("submit: %s\n", sse_last_error()); return 1; }
    double rel[2] = {-1, -1};
    if (sse_check_submit(p, &a, blocks.data(), 64, 1e-5, rel, C.data(), C.size(), nullptr, &t2)) { printf("check: %s\n", sse_last_error()); return 1; }
    if (sse_submit(pf, &a, W.data(), ws, nullptr, &t3)) return 1;
    int s1, s3, s2 = sse_wait(t2);
    while ((s1 = sse_poll(t1)) == SSE_PENDING) {}
    while ((s3 = sse_poll(t3)) == SSE_PENDING) {}
    if (s1 || s2 || s3 || rel[0] != 1e-6) { printf("it %d: %d %d %d rel %g\n", it, s1, s2, s3, rel[0]); return 1; }
  }
  sse_plan_t p2; size_t ws2; d.prec = SSE_BF16X3; sse_plan(&d, sh, &p2, &ws2);
  sse_plan_destroy(p); sse_plan_destroy(pf);
  // batch plan path
  sse_desc ds[3] = {d, d, d}; for (auto &x : ds) { x.prec = SSE_BF16X3; x.ncomp = 1; }
  ds[1].NA = 17; ds[2].NE = 77; ds[2].Nw = 5;
  const int32_t *shs[3] = {sh, sh, sh};
  sse_plan_t pb; size_t wsb;
  if (sse_plan_batch(ds, shs, 3, &pb, &wsb)) { printf("batch: %s\n", sse_last_error()); return 1; }
  std::vector<char> WB(wsb);
  sse_args aa[3] = {a, a, a};
  uint64_t tb; if (sse_submit(pb, aa, WB.data(), wsb, nullptr, &tb)) { printf("bsubmit %s\n", sse_last_error()); return 1; }
  printf("batch poll %d\n", sse_wait(tb));
  sse_plan_destroy(pb);
  {
    // binary64 batch of 3 + 2 atoms: three of the eight work queues stay empty
    sse_desc e[2] = {d, d};
    for (auto &x : e) { x.prec = SSE_FP64; x.ncomp = 1; x.NA = 3; }
    e[1].NA = 2; e[1].NE = 9;
    const int32_t *she[2] = {sh, sh};
    sse_plan_t pe; size_t wse;
    if (sse_plan_batch(e, she, 2, &pe, &wse)) { printf("batch64: %s\n", sse_last_error()); return 1; }
    std::vector<char> WE(wse);
    sse_args ae[2] = {a, a};
    uint64_t te;
    if (sse_submit(pe, ae, WE.data(), wse, nullptr, &te)) { printf("bsubmit64 %s\n", sse_last_error()); return 1; }
    if (sse_wait(te)) return 5;
    sse_plan_destroy(pe);
  }
  {
    uint64_t ta, tb2;
    if (sse_submit(p2, &a, W.data(), ws, nullptr, &ta)) return 2;
    if (sse_poll(ta) != SSE_PENDING) return 3;
    if (sse_submit(p2, &a, W.data(), ws, nullptr, &tb2)) { printf("submit after a pending poll: %s\n", sse_last_error()); return 4; }
    sse_wait(ta); sse_wait(tb2);
  }
  {
    // allocation-free variant: the plan's scratch comes from the static array
    sse_desc n1 = d; n1.prec = SSE_FP64; n1.ncomp = 2;
    sse_plan_t pn; size_t wsn;
    if (sse_plan(&n1, sh, &pn, &wsn)) return 6;
    for (int it = 0; it < 3; ++it)
      if (sse_compute_noalloc(pn, neigh.data(), dH.data(), G.data(), D.data(), S.data(), nullptr)) {
        printf("noalloc: %s\n", sse_last_error()); return 7; }
    if (sse_compute_noalloc(pn, nullptr, dH.data(), G.data(), D.data(), S.data(), nullptr) != SSE_ERR_ARG) return 8;
    sse_plan_destroy(pn);
    sse_desc big = d; big.prec = SSE_BF16X3; big.NA = 1024; big.NE = 1000; big.Nkz = 7; big.Nqz = 7;
    sse_plan_t pbig; size_t wsbig;
    if (sse_plan(&big, sh, &pbig, &wsbig)) return 9;
    if (wsbig <= SSE_NOALLOC_SCRATCH_BYTES) return 10;
    if (sse_compute_noalloc(pbig, neigh.data(), dH.data(), G.data(), D.data(), S.data(), nullptr) != SSE_ERR_UNSUPPORTED) return 11;
    sse_plan_destroy(pbig);
  }
  {
    // phonon self-energy, D~ and the retarded relation through the C ABI
    sse_desc pd = d; pd.prec = SSE_FP64; pd.ncomp = 2; pd.Norb = 4; pd.Nw = 8;
    int32_t psh[8] = {3, -2, 1, 5, 0, 7, 2, 2};
    sse_plan_t pp; size_t wsp;
    if (sse_plan(&pd, psh, &pp, &wsp)) return 12;
    std::vector<char> PW(256 + 4 * pd.NA * pd.NB);
    uint64_t t1, t2;
    if (sse_pi_submit(pp, neigh.data(), dH.data(), G.data(), S.data(), PW.data(), PW.size(), nullptr, &t1)) { printf("pi: %s\n", sse_last_error()); return 13; }
    if (sse_wait(t1)) return 14;
    if (sse_dtilde_submit(pp, neigh.data(), D.data(), S.data(), PW.data(), PW.size(), nullptr, &t2)) { printf("dtilde: %s\n", sse_last_error()); return 15; }
    if (sse_wait(t2)) return 16;
    if (sse_dtilde_submit(pp, neigh.data(), D.data(), S.data(), PW.data(), 256, nullptr, &t2) != SSE_ERR_ARG) return 17;
    if (sse_retarded(pp, 1, G.data(), S.data(), nullptr)) return 18;
    if (sse_retarded(pp, 2, G.data(), S.data(), nullptr) != SSE_ERR_ARG) return 19;
    sse_plan_destroy(pp);
    pd.Norb = 17;
    if (sse_plan(&pd, psh, &pp, &wsp)) return 20;
    if (sse_pi_submit(pp, neigh.data(), dH.data(), G.data(), S.data(), PW.data(), PW.size(), nullptr, &t1) != SSE_ERR_UNSUPPORTED) return 21;
    sse_plan_destroy(pp);
  }
  printf("OK\n");
  return 0;
}
