// C ABI of the NEGF library: argument checking, workspace carving, point
// chunking and the host-side sequencing of the batched kernels that make up
// the lead decimation and the RGF sweeps.
//
// Every chunk is a run of consecutive points (problem order, energy order)
// that share one block shape (nb, b); a chunk is processed by batched
// launches over all of its points, so each product/inversion launch carries
// (points x tiles) workgroups.  Per-problem data (H, S, Sigma_sc, energies,
// Fermi levels) enter only through the assembly kernels, which are launched
// per problem segment of the chunk.
#include "../../include/negf.h"
#include "internal.h"
#include "orch.h"

#include <algorithm>
#include <cstring>
#include <mutex>
#include <vector>

using namespace negf;
using namespace negf::orch;

namespace negf {
namespace orch {
// block i of a scattering self-energy for the first energy of the segment (energy-dependent
// self-energies advance by the problem's sc_stride per energy)
inline const double2* sc_blk(const Seg& sg, const void* base, int i, int b) {
  return base ? blk(base, i, b) + (long)sg.e0 * sg.pr->sc_stride : nullptr;
}

// A_ii = E S_ii - H_ii - Sigma_sc,ii - [i==0] SigL - [i==nb-1] SigR for every point of the chunk
void assemble_diag(Ctx& cx, const Chunk& ch, int i, const PointWs& pw, Blocks out, bool with_leads = true) {
  const int b = ch.b, nb = ch.nb;
  for (const Seg& sg : ch.segs) {
    const negf_device& dv = sg.pr->dev;
    AssembleDesc d = asm_base(b, sg.n, sg.pr->energies + sg.e0, out.at(sg.off), out.stride);
    d.S = blk(dv.S_diag, i, b); d.s_identity = 1;
    d.H = blk(dv.H_diag, i, b);
    d.Y = sc_blk(sg, dv.sig_r_sc, i, b); d.sY = sg.pr->sc_stride;
    if (with_leads && i == 0) { d.Z = pw.sigL.at(sg.off); d.sZ = pw.sigL.stride; }
    if (with_leads && i == nb - 1) {
      if (d.Z) {
        // nb == 1 is rejected by argument checking, so both leads never share a block
      }
      d.Z = pw.sigR.at(sg.off); d.sZ = pw.sigR.stride;
    }
    cx.assemble(d);
  }
}

// A_{i,i+1} = E S_{i,i+1} - H_{i,i+1}
void assemble_upper(Ctx& cx, const Chunk& ch, int i, Blocks out) {
  const int b = ch.b;
  for (const Seg& sg : ch.segs) {
    const negf_device& dv = sg.pr->dev;
    AssembleDesc d = asm_base(b, sg.n, sg.pr->energies + sg.e0, out.at(sg.off), out.stride);
    d.S = blk(dv.S_upper, i, b); d.s_identity = 0;
    d.H = blk(dv.H_upper, i, b);
    cx.assemble(d);
  }
}

// Sigma_i (lesser or greater, kind 0/1): scattering block plus the lead terms
// of the end blocks.  Returns false when the block is identically zero.
bool assemble_sigma_lg(Ctx& cx, const Chunk& ch, int i, int kind, const PointWs& pw, Blocks out) {
  const int b = ch.b, nb = ch.nb;
  const Blocks& leadL = kind == 0 ? pw.slL : pw.sgL;
  const Blocks& leadR = kind == 0 ? pw.slR : pw.sgR;
  bool any = false;
  for (const Seg& sg : ch.segs) {
    const negf_device& dv = sg.pr->dev;
    const void* sc = kind == 0 ? dv.sig_l_sc : dv.sig_g_sc;
    if (sc || i == 0 || i == nb - 1) any = true;
  }
  if (!any) return false;
  for (const Seg& sg : ch.segs) {
    const negf_device& dv = sg.pr->dev;
    AssembleDesc d = asm_base(b, sg.n, nullptr, out.at(sg.off), out.stride);
    d.S = nullptr; d.s_identity = 0; d.s_coef = 0.0;
    d.H = nullptr;
    d.Y = sc_blk(sg, kind == 0 ? dv.sig_l_sc : dv.sig_g_sc, i, b); d.sY = sg.pr->sc_stride; d.y_coef = 1.0;
    if (i == 0) { d.Z = leadL.at(sg.off); d.sZ = leadL.stride; d.z_coef = 1.0; }
    if (i == nb - 1) { d.Z = leadR.at(sg.off); d.sZ = leadR.stride; d.z_coef = 1.0; }
    cx.assemble(d);
  }
  return true;
}

// ------------------------------------------------------------------ decimation

// Solves the leads of the given sides for every point of the chunk.  Pair
// q = side_index * npts + p.  Writes g_s into lw.g and Sigma^R into sig_out
// (per pair, stride b*b) and the iteration counts / residuals / info.
void run_decimation(Ctx& cx, const Chunk& ch, const int* sides, int nsides, LeadWs& w, const double2* seed,
                    long seed_stride, Blocks sig_out_L, Blocks sig_out_R, int* info_pts, int* iters_out,
                    double* resid_out) {
  const int b = ch.b, nb = ch.nb, npts = ch.npts, np = npts * nsides;
  const long bb = (long)b * b;
  hipStream_t s = cx.s;
  // --- lead blocks d, alpha, beta at z = E + i eta
  for (int si = 0; si < nsides; ++si) {
    const int side = sides[si];
    for (const Seg& sg : ch.segs) {
      const negf_device& dv = sg.pr->dev;
      const double* en = sg.pr->energies + sg.e0;
      const int q0 = si * npts + sg.off;
      const long cell = side == 0 ? 0 : nb - 1;
      const long cpl = side == 0 ? 0 : nb - 2;
      AssembleDesc d = asm_base(b, sg.n, en, w.d.at(q0), bb);
      d.eta = sg.pr->eta;
      d.S = blk(dv.S_diag, cell, b); d.s_identity = 1;
      d.H = blk(dv.H_diag, cell, b);
      cx.assemble(d);
      // alpha = H1 - z S1, beta = H1^H - z S1^H ; left lead: H1 = H_01^H, right: H1 = H_{N-2,N-1}
      AssembleDesc a = asm_base(b, sg.n, en, w.alpha.at(q0), bb);
      a.eta = sg.pr->eta; a.s_coef = -1.0; a.h_coef = 1.0;
      a.S = blk(dv.S_upper, cpl, b); a.s_identity = 0;
      a.H = blk(dv.H_upper, cpl, b);
      a.op = side == 0 ? 1 : 0;
      cx.assemble(a);
      AssembleDesc be = a;
      be.out = w.beta.at(q0);
      be.op = side == 0 ? 0 : 1;
      cx.assemble(be);
    }
  }
  if (!cx.ok()) return;
  cx.chk(launch_fill_int(np, w.active, 1, s));
  cx.chk(launch_fill_int(np, w.iters, 0, s));
  cx.chk(launch_fill_int(np, w.accepted, 0, s));
  cx.chk(launch_frob2(b, np, w.d.p, bb, 0.0, nullptr, w.part, w.d2, s));

  // --- optional seed g~: candidate g0 = (d - alpha g~ beta)^{-1} (kept in w.g), accepted
  // when its normalised Dyson residual is <= accept; accepted pairs skip the decimation.
  if (seed) {
    for (int si = 0; si < nsides; ++si)
      cx.gemm(PREC_F64, OP_N, OP_N, b, npts, ONE, w.alpha.at(si * npts), bb, seed, seed_stride, ZERO, nullptr, 0,
              w.t1.at(si * npts), bb);
    cx.gemm(PREC_F64, OP_N, OP_N, b, np, MONE, w.t1.p, bb, w.beta.p, bb, ONE, w.d.p, bb, w.eps.p, bb);
    // d - alpha g~ beta is kept for the seeded closure of the decimation steps
    cx.lincomb(b, np, ONE, w.eps.p, bb, ZERO, nullptr, 0, ZERO, w.dseed.p, bb);
    cx.inverse(b, np, w.eps.p, bb, w.g.p, bb, w.inv_scratch, nullptr, 0);
    cx.gemm(PREC_F64, OP_N, OP_N, b, np, ONE, w.alpha.p, bb, w.g.p, bb, ZERO, nullptr, 0, w.t1.p, bb);
    cx.gemm(PREC_F64, OP_N, OP_N, b, np, MONE, w.t1.p, bb, w.beta.p, bb, ONE, w.d.p, bb, w.t2.p, bb);
    cx.gemm(PREC_F64, OP_N, OP_N, b, np, ONE, w.t2.p, bb, w.g.p, bb, ZERO, nullptr, 0, w.t1.p, bb);
    cx.chk(launch_frob2(b, np, w.t1.p, bb, 1.0, nullptr, w.part, w.r2, s));
    cx.chk(launch_frob2(b, np, w.t2.p, bb, 0.0, nullptr, w.part, w.m2, s));
    cx.chk(launch_frob2(b, np, w.g.p, bb, 0.0, nullptr, w.part, w.g2, s));
    // w.accepted[q] stays 0 (= accepted) unless the residual test fails
    cx.chk(launch_sr_finish(np, w.r2, w.m2, w.g2, nullptr, cx.o.accept, nullptr, w.accepted, 0, s));
    cx.chk(launch_seed_flags(np, w.accepted, w.active, w.iters, s));
  }
  if (!cx.ok()) return;
  // --- plain decimation: eps_s = eps = d, a = alpha, c = beta.  The chain keeps eps_s and
  // D = eps - eps_s (in w.eps): the term a g c that both lose cancels in D, so each update is
  // one product with an accumulating epilogue, and eps = eps_s + D is formed where it is inverted.
  cx.lincomb(b, np, ONE, w.d.p, bb, ZERO, nullptr, 0, ZERO, w.eps_s.p, bb);
  cx.lincomb(b, np, ZERO, nullptr, 0, ZERO, nullptr, 0, ZERO, w.eps.p, bb);
  cx.lincomb(b, np, ONE, w.alpha.p, bb, ZERO, nullptr, 0, ZERO, w.a.p, bb);
  cx.lincomb(b, np, ONE, w.beta.p, bb, ZERO, nullptr, 0, ZERO, w.c.p, bb);
  Blocks a = w.a, c = w.c, t1 = w.t1, t2 = w.t2;
  const Blocks D = w.eps;
  // Exactly max_iter steps are enqueued: a pair that has converged (or been closed by its seed) is
  // masked out of every later launch, so nothing is read back on the host and the whole call
  // stays asynchronous (and capturable); steps after the last pair has converged only launch
  // workgroups that exit at once.
  for (int it = 1; it <= cx.o.max_iter && cx.ok(); ++it) {
    const int* act = w.active;
    // g = eps^{-1} with eps = eps_s + D formed in t1 (the inversion overwrites its input)
    cx.lincomb(b, np, ONE, w.eps_s.p, bb, ONE, D.p, bb, ZERO, t1.p, bb, act);
    cx.inverse(b, np, t1.p, bb, w.ag.p, bb, w.inv_scratch, nullptr, 0, act);   // ag temporarily holds g
    std::swap(w.ag, w.cg);   // cg := g ; ag free
    const Blocks g = w.cg;
    // ag = a g, t2 = c g
    cx.gemm(PREC_F64, OP_N, OP_N, b, np, ONE, a.p, bb, g.p, bb, ZERO, nullptr, 0, w.ag.p, bb, act);
    cx.gemm(PREC_F64, OP_N, OP_N, b, np, ONE, c.p, bb, g.p, bb, ZERO, nullptr, 0, t2.p, bb, act);
    // eps_s -= (a g) c ; D -= (c g) a
    cx.gemm(PREC_F64, OP_N, OP_N, b, np, MONE, w.ag.p, bb, c.p, bb, ONE, w.eps_s.p, bb, w.eps_s.p, bb, act);
    cx.gemm(PREC_F64, OP_N, OP_N, b, np, MONE, t2.p, bb, a.p, bb, ONE, D.p, bb, D.p, bb, act);
    // a' = (a g) a -> t1 ; c' = (c g) c -> g buffer (g no longer needed)
    cx.gemm(PREC_F64, OP_N, OP_N, b, np, ONE, w.ag.p, bb, a.p, bb, ZERO, nullptr, 0, t1.p, bb, act);
    cx.gemm(PREC_F64, OP_N, OP_N, b, np, ONE, t2.p, bb, c.p, bb, ZERO, nullptr, 0, w.cg.p, bb, act);
    std::swap(a, t1);
    {
      Blocks tmp = c;
      c = w.cg;
      w.cg = tmp;
    }
    if (seed) {
      // seeded closure of the chain after this step: X = (eps - eps_s + d - alpha g~ beta)^{-1},
      // g^ = (eps_s - a X c)^{-1}, accepted (and the pair finished) when its Dyson residual passes.
      // Free here: t1, w.ag, w.cg, t2.
      cx.lincomb(b, np, ONE, D.p, bb, ONE, w.dseed.p, bb, ZERO, t1.p, bb, act);
      cx.inverse(b, np, t1.p, bb, w.ag.p, bb, w.inv_scratch, nullptr, 0, act);
      cx.gemm(PREC_F64, OP_N, OP_N, b, np, ONE, a.p, bb, w.ag.p, bb, ZERO, nullptr, 0, w.cg.p, bb, act);
      cx.gemm(PREC_F64, OP_N, OP_N, b, np, MONE, w.cg.p, bb, c.p, bb, ONE, w.eps_s.p, bb, t2.p, bb, act);
      cx.inverse(b, np, t2.p, bb, t1.p, bb, w.inv_scratch, nullptr, 0, act);          // t1 = g^
      cx.gemm(PREC_F64, OP_N, OP_N, b, np, ONE, w.alpha.p, bb, t1.p, bb, ZERO, nullptr, 0, w.ag.p, bb, act);
      cx.gemm(PREC_F64, OP_N, OP_N, b, np, MONE, w.ag.p, bb, w.beta.p, bb, ONE, w.d.p, bb, t2.p, bb, act);
      cx.gemm(PREC_F64, OP_N, OP_N, b, np, ONE, t2.p, bb, t1.p, bb, ZERO, nullptr, 0, w.cg.p, bb, act);
      cx.chk(launch_frob2(b, np, w.cg.p, bb, 1.0, act, w.part, w.r2, s));
      cx.chk(launch_frob2(b, np, t2.p, bb, 0.0, act, w.part, w.m2, s));
      cx.chk(launch_frob2(b, np, t1.p, bb, 0.0, act, w.part, w.g2, s));
      cx.chk(launch_closure_accept(np, w.r2, w.m2, w.g2, cx.o.accept, it, w.active, w.iters, w.accepted, w.closed,
                                   s));
      cx.lincomb(b, np, ONE, t1.p, bb, ZERO, nullptr, 0, ZERO, w.g.p, bb, w.closed);
    }
    cx.chk(launch_frob2(b, np, a.p, bb, 0.0, w.active, w.part, w.a2, s));
    cx.chk(launch_frob2(b, np, c.p, bb, 0.0, w.active, w.part, w.c2, s));
    cx.chk(launch_sr_check(np, w.a2, w.c2, w.d2, cx.o.tol, it, w.active, w.iters, w.n_active, s));
  }
  if (!cx.ok()) return;
  // --- g_s = eps_s^{-1} (pairs that ran the decimation); seeded-accepted pairs keep g0
  if (seed) {
    cx.inverse(b, np, w.eps_s.p, bb, t1.p, bb, w.inv_scratch, nullptr, 0);
    cx.chk(launch_seed_select(b, np, w.accepted, t1.p, w.g.p, s));   // g <- eps_s^{-1} where rejected
  } else {
    cx.inverse(b, np, w.eps_s.p, bb, w.g.p, bb, w.inv_scratch, nullptr, 0);
  }
  // --- Sigma = alpha g_s beta ; residual of the surface Dyson equation
  cx.gemm(PREC_F64, OP_N, OP_N, b, np, ONE, w.alpha.p, bb, w.g.p, bb, ZERO, nullptr, 0, t1.p, bb);
  for (int si = 0; si < nsides; ++si) {
    Blocks dst = (sides[si] == 0) ? sig_out_L : sig_out_R;
    cx.gemm(PREC_F64, OP_N, OP_N, b, npts, ONE, t1.at(si * npts), bb, w.beta.at(si * npts), bb, ZERO, nullptr, 0,
            dst.p, dst.stride);
    cx.lincomb(b, npts, ONE, w.d.at(si * npts), bb, MONE, dst.p, dst.stride, ZERO, t2.at(si * npts), bb);
  }
  cx.gemm(PREC_F64, OP_N, OP_N, b, np, ONE, t2.p, bb, w.g.p, bb, ZERO, nullptr, 0, t1.p, bb);
  cx.chk(launch_frob2(b, np, t1.p, bb, 1.0, nullptr, w.part, w.r2, s));
  cx.chk(launch_frob2(b, np, t2.p, bb, 0.0, nullptr, w.part, w.m2, s));
  cx.chk(launch_frob2(b, np, w.g.p, bb, 0.0, nullptr, w.part, w.g2, s));
  if (info_pts) cx.chk(launch_sr_finish(np, w.r2, w.m2, w.g2, w.active, cx.o.accept, resid_out, info_pts, npts, s));
  if (iters_out) cx.chk(rt_copy_d2d(iters_out, w.iters, sizeof(int) * np, s));
  if (info_pts) cx.chk(launch_check_finite(b, np, w.g.p, bb, info_pts, npts, s));
}

// ------------------------------------------------------------------ RGF sweeps


// Leads of both sides into pw.sigL / pw.sigR, Gamma and (optionally) Sigma^<>.
void leads_for_sweeps(Ctx& cx, const Chunk& ch, ChunkWs& w, int* info, bool lesser) {
  const int sides[2] = {0, 1};
  run_decimation(cx, ch, sides, 2, w.lw, nullptr, 0, w.pw.sigL, w.pw.sigR, info, nullptr, nullptr);
  const int b = ch.b;
  for (const Seg& sg : ch.segs) {
    const double* en = sg.pr->energies + sg.e0;
    const PointWs& p = w.pw;
    cx.chk(launch_gamma_sigma(b, sg.n, p.sigL.at(sg.off), p.sigL.stride, en, sg.pr->mu_l, sg.pr->kT,
                              p.gamL.at(sg.off), p.gamL.stride, lesser ? p.slL.at(sg.off) : nullptr, p.slL.stride,
                              lesser ? p.sgL.at(sg.off) : nullptr, p.sgL.stride, cx.s));
    cx.chk(launch_gamma_sigma(b, sg.n, p.sigR.at(sg.off), p.sigR.stride, en, sg.pr->mu_r, sg.pr->kT,
                              p.gamR.at(sg.off), p.gamR.stride, lesser ? p.slR.at(sg.off) : nullptr, p.slR.stride,
                              lesser ? p.sgR.at(sg.off) : nullptr, p.sgR.stride, cx.s));
  }
}

// Forward retarded sweep: g_i -> gdiag (per point stride nb*b*b), X_i, M_i (refine).
// With corner != nullptr also the left-connected G_{nb-1,0} recursion for T.
void forward_retarded(Ctx& cx, const Chunk& ch, PointWs& pw, negf_precision prec, double2* gdiag, long gstride,
                      int* info, bool want_X, Blocks* corner) {
  const int b = ch.b, nb = ch.nb, n = ch.npts;
  const long bb = (long)b * b;
  const Prec pf = (prec == NEGF_FP32_NOREFINE) ? PREC_F32 : PREC_F64;
  const long xs = (long)(nb - 1) * bb, ms = (long)nb * bb;
  Blocks C = pw.C0, Cn = pw.C1;
  for (int i = 0; i < nb && cx.ok(); ++i) {
    assemble_diag(cx, ch, i, pw, pw.T0);
    double2* g_prev = gdiag + (long)(i - 1) * bb;
    if (i > 0) {
      assemble_upper(cx, ch, i - 1, pw.T1);
      double2* Xi = want_X ? pw.X + (long)(i - 1) * bb : pw.T2.p;
      const long sX = want_X ? xs : bb;
      cx.gemm(pf, OP_N, OP_N, b, n, ONE, g_prev, gstride, pw.T1.p, bb, ZERO, nullptr, 0, Xi, sX, nullptr, false,
              cx.cpl(i - 1, 1));
      cx.gemm(pf, OP_C, OP_N, b, n, MONE, pw.T1.p, bb, Xi, sX, ONE, pw.T0.p, bb, pw.T0.p, bb, nullptr, false,
              cx.cpl(i - 1, 2));
    }
    if (pw.Mst) cx.lincomb(b, n, ONE, pw.T0.p, bb, ZERO, nullptr, 0, ZERO, pw.Mst + (long)i * bb, ms);
    double2* gi = gdiag + (long)i * bb;
    cx.inverse(b, n, pw.T0.p, bb, gi, gstride, pw.inv_scratch, info, 0);
    if (corner) {
      if (i == 0) {
        cx.lincomb(b, n, ONE, gi, gstride, ZERO, nullptr, 0, ZERO, C.p, bb);
      } else {
        // C_i = -g_i (A_{i,i-1} C_{i-1}),  A_{i,i-1} = T1^H
        cx.gemm(PREC_F64, OP_C, OP_N, b, n, ONE, pw.T1.p, bb, C.p, bb, ZERO, nullptr, 0, pw.T3.p, bb, nullptr, false,
                cx.cpl(i - 1, 2));
        cx.gemm(PREC_F64, OP_N, OP_N, b, n, MONE, gi, gstride, pw.T3.p, bb, ZERO, nullptr, 0, Cn.p, bb);
        std::swap(C, Cn);
      }
    }
  }
  if (corner) *corner = C;
}

void backward_retarded(Ctx& cx, const Chunk& ch, PointWs& pw, negf_precision prec, const Outs& o) {
  const int b = ch.b, nb = ch.nb, n = ch.npts;
  const long bb = (long)b * b;
  const long ds = (long)nb * bb, us = (long)(nb - 1) * bb;
  const bool refine = prec == NEGF_FP32_REFINE;
  const Prec pb = (prec == NEGF_PLAIN_FP64) ? PREC_F64 : PREC_F32;
  double2* GRd = o.GRd + ch.out_diag_off;
  double2* GRu = o.GRu + ch.out_off_off;
  double2* GRl = o.GRl ? o.GRl + ch.out_off_off : nullptr;
  for (int i = nb - 2; i >= 0 && cx.ok(); --i) {
    assemble_upper(cx, ch, i, pw.T1);                  // A_{i,i+1}
    double2* gi = GRd + (long)i * bb;                  // holds g_i
    double2* Gn = GRd + (long)(i + 1) * bb;            // G_{i+1,i+1}
    double2* Xi = pw.X + (long)i * bb;
    const long xs = us;
    double2* Glo = GRl ? GRl + (long)i * bb : pw.T3.p;
    const long sLo = GRl ? us : bb;
    double2* Gup = GRu + (long)i * bb;
    // W = A_{i+1,i} g_i ; G_{i+1,i} = -G_{i+1,i+1} W
    cx.gemm(pb, OP_C, OP_N, b, n, ONE, pw.T1.p, bb, gi, ds, ZERO, nullptr, 0, pw.T2.p, bb, nullptr, false,
            cx.cpl(i, 2));
    cx.gemm(pb, OP_N, OP_N, b, n, MONE, Gn, ds, pw.T2.p, bb, ZERO, nullptr, 0, Glo, sLo);
    double2* Mi = refine ? pw.Mst + (long)i * bb : nullptr;
    if (refine) {
      // r = -G_{i+1,i+1} A_{i+1,i} - G_{i+1,i} M_i ; G_{i+1,i} += r g_i
      cx.gemm(PREC_F64, OP_N, OP_C, b, n, MONE, Gn, ds, pw.T1.p, bb, ZERO, nullptr, 0, pw.T4.p, bb);
      cx.gemm(PREC_F64, OP_N, OP_N, b, n, MONE, Glo, sLo, Mi, ds, ONE, pw.T4.p, bb, pw.T4.p, bb);
      cx.gemm(PREC_F32, OP_N, OP_N, b, n, ONE, pw.T4.p, bb, gi, ds, ONE, Glo, sLo, Glo, sLo);
    }
    // G_{i,i+1} = -X_i G_{i+1,i+1}
    cx.gemm(pb, OP_N, OP_N, b, n, MONE, Xi, xs, Gn, ds, ZERO, nullptr, 0, Gup, us);
    if (refine) {
      // r = -A_{i,i+1} G_{i+1,i+1} - M_i G_{i,i+1} ; G_{i,i+1} += g_i r
      cx.gemm(PREC_F64, OP_N, OP_N, b, n, MONE, pw.T1.p, bb, Gn, ds, ZERO, nullptr, 0, pw.T4.p, bb);
      cx.gemm(PREC_F64, OP_N, OP_N, b, n, MONE, Mi, ds, Gup, us, ONE, pw.T4.p, bb, pw.T4.p, bb);
      cx.gemm(PREC_F32, OP_N, OP_N, b, n, ONE, gi, ds, pw.T4.p, bb, ONE, Gup, us, Gup, us);
      // keep g_i for the diagonal correction
      cx.lincomb(b, n, ONE, gi, ds, ZERO, nullptr, 0, ZERO, pw.T0.p, bb);
    }
    // G_ii = g_i - X_i G_{i+1,i}
    cx.gemm(pb, OP_N, OP_N, b, n, MONE, Xi, xs, Glo, sLo, ONE, gi, ds, gi, ds);
    if (refine) {
      // r = I - M_i G_ii - A_{i,i+1} G_{i+1,i} ; G_ii += g_i r
      cx.gemm(PREC_F64, OP_N, OP_N, b, n, ONE, Mi, ds, gi, ds, ZERO, nullptr, 0, pw.T4.p, bb);
      cx.gemm(PREC_F64, OP_N, OP_N, b, n, ONE, pw.T1.p, bb, Glo, sLo, ONE, pw.T4.p, bb, pw.T4.p, bb);
      cx.lincomb(b, n, MONE, pw.T4.p, bb, ZERO, nullptr, 0, ONE, pw.T4.p, bb);
      cx.gemm(PREC_F32, OP_N, OP_N, b, n, ONE, pw.T0.p, bb, pw.T4.p, bb, ONE, gi, ds, gi, ds);
    }
  }
}

// Forward lesser/greater sweep of one kind; g^<> into gl (stride ds).  Needs g_i in GRd.
// V_{i-1} = A_{i,i-1} g^<>_{i-1}, formed at step i, is left in the upper output block i-1 (lu,
// stride (nb-1) b^2), which the backward sweep reads back before it writes that block.
void forward_lesser(Ctx& cx, const Chunk& ch, PointWs& pw, negf_precision prec, int kind, const double2* GRd,
                    double2* gl, double2* lu) {
  const int b = ch.b, nb = ch.nb, n = ch.npts;
  const long bb = (long)b * b, ds = (long)nb * bb, us = (long)(nb - 1) * bb;
  // the refined form keeps the lesser sweeps in double: one residual correction of
  // single-precision products here leaves ~3e-7 in g^<, which the backward sweep
  // amplifies beyond 1e-6 over a 60-block device
  const Prec pg = (prec == NEGF_FP32_NOREFINE) ? PREC_F32 : PREC_F64;  // g B g^H
  const Prec pbt = pg;                                                  // B formation
  for (int i = 0; i < nb && cx.ok(); ++i) {
    const double2* gi = GRd + (long)i * bb;
    double2* gli = gl + (long)i * bb;
    const bool has_sig = assemble_sigma_lg(cx, ch, i, kind, pw, pw.T4);
    if (i > 0) {
      assemble_upper(cx, ch, i - 1, pw.T1);   // A_{i-1,i}; A_{i,i-1} = T1^H
      double2* V = lu + (long)(i - 1) * bb;
      cx.gemm(pbt, OP_C, OP_N, b, n, ONE, pw.T1.p, bb, gl + (long)(i - 1) * bb, ds, ZERO, nullptr, 0, V, us, nullptr,
              false, cx.cpl(i - 1, 2));
      cx.gemm(pbt, OP_N, OP_N, b, n, ONE, V, us, pw.T1.p, bb, has_sig ? ONE : ZERO, has_sig ? pw.T4.p : nullptr, bb,
              pw.T4.p, bb, nullptr, false, cx.cpl(i - 1, 1));
    } else if (!has_sig) {
      cx.lincomb(b, n, ZERO, nullptr, 0, ZERO, nullptr, 0, ZERO, pw.T4.p, bb);
    }
    // g^<_i = g_i B g_i^H
    cx.gemm(pg, OP_N, OP_N, b, n, ONE, gi, ds, pw.T4.p, bb, ZERO, nullptr, 0, pw.T3.p, bb);
    cx.gemm(pg, OP_N, OP_C, b, n, ONE, pw.T3.p, bb, gi, ds, ZERO, nullptr, 0, gli, ds);
  }
}

void backward_lesser(Ctx& cx, const Chunk& ch, PointWs& pw, negf_precision prec, const double2* GRd,
                     const double2* GRu, double2* Ld, double2* Lu) {
  const int b = ch.b, nb = ch.nb, n = ch.npts;
  const long bb = (long)b * b, ds = (long)nb * bb, us = (long)(nb - 1) * bb;
  const Prec pp = (prec == NEGF_FP32_NOREFINE) ? PREC_F32 : PREC_F64;
  for (int i = nb - 2; i >= 0 && cx.ok(); --i) {
    double2* gli = Ld + (long)i * bb;                 // holds g^<_i
    const double2* Xi = pw.X + (long)i * bb;
    // V = A_{i+1,i} g^<_i was left in the upper block i by the forward sweep (same product, same
    // operands) and is read from there until that block receives G^<_{i,i+1}.
    const double2* V = Lu + (long)i * bb;
    // Z = X_i G^<_{i+1,i+1}
    cx.gemm(pp, OP_N, OP_N, b, n, ONE, Xi, us, Ld + (long)(i + 1) * bb, ds, ZERO, nullptr, 0, pw.T4.p, bb);
    // G^<_{i,i+1} = V^H G_{i+1,i+1}^H - Z, formed in T3
    cx.gemm(pp, OP_C, OP_C, b, n, ONE, V, us, GRd + (long)(i + 1) * bb, ds, MONE, pw.T4.p, bb, pw.T3.p, bb);
    // G^<_ii = g^<_i + Z X_i^H + Q - Q^H with Q = -G_{i,i+1} V.  Since Q^H = V^H G_{i+1,i+1}^H X_i^H
    // (G_{i,i+1} = -X_i G_{i+1,i+1}), Z X_i^H - Q^H = -G^<_{i,i+1} X_i^H, so
    // G^<_ii = g^<_i - G_{i,i+1} V - G^<_{i,i+1} X_i^H: two accumulating products, no transpose pass.
    cx.gemm(pp, OP_N, OP_N, b, n, MONE, GRu + (long)i * bb, us, V, us, ONE, gli, ds, gli, ds);
    cx.gemm(pp, OP_N, OP_C, b, n, MONE, pw.T3.p, bb, Xi, us, ONE, gli, ds, gli, ds);
    cx.lincomb(b, n, ONE, pw.T3.p, bb, ZERO, nullptr, 0, ZERO, Lu + (long)i * bb, us);
  }
}

// ------------------------------------------------------------------ argument checks


negf_status check_problems(const negf_problem* pr, int n_prob) {
  if (!pr || n_prob <= 0) return NEGF_EINVAL;
  for (int q = 0; q < n_prob; ++q) {
    const negf_device& d = pr[q].dev;
    if (d.nb < 2 || d.b < 1 || d.b > 1024) return NEGF_EINVAL;
    if (!d.H_diag || !d.H_upper) return NEGF_EINVAL;
    if (pr[q].n_e < 0) return NEGF_EINVAL;
    if (pr[q].n_e > 0 && !pr[q].energies) return NEGF_EINVAL;
    if (!(pr[q].eta >= 0.0) || !(pr[q].kT >= 0.0)) return NEGF_EINVAL;
    const void* ptrs[] = {d.H_diag, d.H_upper, d.S_diag, d.S_upper, d.sig_r_sc, d.sig_l_sc, d.sig_g_sc};
    for (const void* p : ptrs)
      if (p && !aligned16(p)) return NEGF_EINVAL;
    if ((d.S_diag == nullptr) != (d.S_upper == nullptr)) return NEGF_EINVAL;
    if ((d.sig_l_sc == nullptr) != (d.sig_g_sc == nullptr)) return NEGF_EINVAL;
    if (pr[q].sc_stride != 0 && pr[q].sc_stride < (int64_t)d.nb * d.b * d.b) return NEGF_EINVAL;
  }
  return NEGF_OK;
}

long count_points(const negf_problem* pr, int n_prob) {
  long n = 0;
  for (int q = 0; q < n_prob; ++q) n += pr[q].n_e;
  return n;
}

size_t workspace_for(int opk, const negf_problem* pr, int n_prob, negf_precision prec, const Opts& o) {
  size_t mx = 0;
  for (const Chunk& ch : make_chunks(pr, n_prob, o.batch)) {
    Carver cv{nullptr, 0};
    carve_chunk(cv, opk, ch.nb, ch.b, ch.npts, prec, opk == OPK_OBC ? 1 : 2);
    mx = std::max(mx, cv.off);
  }
  return mx + 256;
}



}  // namespace orch
}  // namespace negf



namespace {

// One chunk of points through the leads and the sweeps of operation opk.
void run_chunk(Ctx& cx, int opk, const Chunk& ch, ChunkWs& w, negf_precision prec, const Outs& outs) {
  int* info = outs.info + ch.first_point;
  const bool lesser = opk == OPK_RL;
  leads_for_sweeps(cx, ch, w, info, lesser);
  // zero-slab maps of the coupling blocks A_{i,i+1} = E S_{i,i+1} - H_{i,i+1} (the union
  // over the chunk's devices): products with a coupling operand skip its zero slabs
  cx.cmask = nullptr;
  if (w.pw.cmask && !cx.o.dense && cx.ok()) {
    int q = 0;
    for (const Seg& sg : ch.segs) {
      const negf_device& dv = sg.pr->dev;
      cx.chk(launch_slab_map(ch.b, ch.nb - 1, (const double2*)dv.H_upper, (const double2*)dv.S_upper, w.pw.cmask,
                             q++ > 0, cx.s));
    }
    cx.cmask = w.pw.cmask;
    cx.cmask_words = ch.b / 16;
  }
  const long bb = (long)ch.b * ch.b;
  const int b = ch.b, nb = ch.nb, n = ch.npts;
  if (opk == OPK_T) {
    // forward recursion only: g_i alternates between T2 and T4, the corner block between C0 and C1
    Blocks C = w.pw.C0, Cn = w.pw.C1, gcur = w.pw.T2, gprev = w.pw.T4;
    for (int i = 0; i < nb && cx.ok(); ++i) {
      assemble_diag(cx, ch, i, w.pw, w.pw.T0);
      if (i > 0) {
        assemble_upper(cx, ch, i - 1, w.pw.T1);
        cx.gemm(PREC_F64, OP_N, OP_N, b, n, ONE, gprev.p, bb, w.pw.T1.p, bb, ZERO, nullptr, 0, w.pw.T3.p, bb,
                nullptr, false, cx.cpl(i - 1, 1));
        cx.gemm(PREC_F64, OP_C, OP_N, b, n, MONE, w.pw.T1.p, bb, w.pw.T3.p, bb, ONE, w.pw.T0.p, bb, w.pw.T0.p, bb,
                nullptr, false, cx.cpl(i - 1, 2));
      }
      cx.inverse(b, n, w.pw.T0.p, bb, gcur.p, bb, w.pw.inv_scratch, info, 0);
      if (i == 0) {
        cx.lincomb(b, n, ONE, gcur.p, bb, ZERO, nullptr, 0, ZERO, C.p, bb);
      } else {
        cx.gemm(PREC_F64, OP_C, OP_N, b, n, ONE, w.pw.T1.p, bb, C.p, bb, ZERO, nullptr, 0, w.pw.T3.p, bb, nullptr,
                false, cx.cpl(i - 1, 2));
        cx.gemm(PREC_F64, OP_N, OP_N, b, n, MONE, gcur.p, bb, w.pw.T3.p, bb, ZERO, nullptr, 0, Cn.p, bb);
        std::swap(C, Cn);
      }
      std::swap(gcur, gprev);
    }
    // T = Re sum (Gamma_R C) .* conj(C Gamma_L)
    cx.gemm(PREC_F64, OP_N, OP_N, b, n, ONE, w.pw.gamR.p, bb, C.p, bb, ZERO, nullptr, 0, w.pw.T0.p, bb);
    cx.gemm(PREC_F64, OP_N, OP_N, b, n, ONE, C.p, bb, w.pw.gamL.p, bb, ZERO, nullptr, 0, w.pw.T1.p, bb);
    cx.chk(launch_dot_re(b, n, w.pw.T0.p, bb, w.pw.T1.p, bb, outs.T + ch.first_point, cx.s));
    return;
  }
  const long ds = (long)nb * bb;
  double2* GRd = outs.GRd + ch.out_diag_off;
  forward_retarded(cx, ch, w.pw, prec, GRd, ds, info, true, nullptr);
  if (lesser) {
    forward_lesser(cx, ch, w.pw, prec, 0, GRd, outs.GLd + ch.out_diag_off, outs.GLu + ch.out_off_off);
    if (outs.GGd)
      forward_lesser(cx, ch, w.pw, prec, 1, GRd, outs.GGd + ch.out_diag_off, outs.GGu + ch.out_off_off);
  }
  backward_retarded(cx, ch, w.pw, prec, outs);
  if (lesser) {
    const double2* GRu = outs.GRu + ch.out_off_off;
    backward_lesser(cx, ch, w.pw, prec, GRd, GRu, outs.GLd + ch.out_diag_off, outs.GLu + ch.out_off_off);
    if (outs.GGd) backward_lesser(cx, ch, w.pw, prec, GRd, GRu, outs.GGd + ch.out_diag_off, outs.GGu + ch.out_off_off);
  }
}

}  // namespace

// ------------------------------------------------------------------ plans (batched uneven workloads)

struct negf_plan {
  std::vector<negf_problem> probs;
  negf_precision prec;
  Opts base;
  std::vector<Chunk> chunks;
  std::vector<Opts> chunk_opts;
  std::vector<int> stream_of;
  std::vector<size_t> run_order;   // enqueue order: shortest chunk first (per stream: shortest first)
  std::vector<size_t> stream_ws_off;
  size_t ws_total = 0;
  int n_streams = 1;
  std::vector<hipStream_t> streams;
  std::vector<hipEvent_t> events;
  // one captured graph per worker stream (its chunks and stamps); a replay forks to the worker
  // streams, launches each graph on its own stream and joins, so the streams overlap as they do
  // eagerly (a single fork/join graph replayed on one stream overlapped them less)
  std::vector<void*> graphs;
  // arguments the graphs were captured with (a replay is valid only for the same ones)
  Outs cap_outs{};
  void* cap_ws = nullptr;
  unsigned long long* cap_stamps = nullptr;
  // the point queue's per-stream round graphs and the arguments they were captured with
  std::vector<void*> qgraphs;
  std::vector<const void*> qkey;
};

namespace {

double chunk_cost(const Chunk& c) {
  const double b3 = (double)c.b * c.b * c.b;
  return c.npts * b3 * (128.0 * (c.nb - 1) + 2.0 * (56.0 * 30 + 24));
}

bool same_outs(const Outs& a, const Outs& b) {
  return a.GRd == b.GRd && a.GRu == b.GRu && a.GRl == b.GRl && a.GLd == b.GLd && a.GLu == b.GLu && a.GGd == b.GGd &&
         a.GGu == b.GGu && a.info == b.info;
}

// Chunk c on its worker stream, followed by its stamp.  No host synchronisation.
hipError_t enqueue_chunk(negf_plan* P, size_t c, const Outs& outs, char* ws, unsigned long long* stamps) {
  const Chunk& ch = P->chunks[c];
  const int si = P->stream_of[c];
  Ctx cx;
  cx.s = P->streams[si];
  cx.o = P->chunk_opts[c];
  Carver cv{ws + P->stream_ws_off[si], P->ws_total - P->stream_ws_off[si]};
  ChunkWs w = carve_chunk(cv, OPK_RL, ch.nb, ch.b, ch.npts, P->prec, 2);
  if (cv.overflow) return hipErrorInvalidValue;
  run_chunk(cx, OPK_RL, ch, w, P->prec, outs);
  if (!cx.ok()) return cx.err;
  return stamps ? launch_stamp(stamps + 1 + c, cx.s) : hipSuccess;
}

// Start of a plan on the caller's stream (info cleared, start stamp), then the fork to the workers.
hipError_t enqueue_fork(negf_plan* P, const Outs& outs, unsigned long long* stamps, hipStream_t main) {
  hipError_t e = launch_fill_int((int)count_points(P->probs.data(), (int)P->probs.size()), outs.info, 0, main);
  if (e != hipSuccess) return e;
  if (stamps && (e = launch_stamp(stamps, main)) != hipSuccess) return e;
  for (int i = 0; i < P->n_streams; ++i)
    if ((e = rt_record_wait(P->events[i], main, P->streams[i])) != hipSuccess) return e;
  return hipSuccess;
}

hipError_t enqueue_join(negf_plan* P, hipStream_t main) {
  const int ns = P->n_streams;
  for (int i = 0; i < ns; ++i) {
    hipError_t e = rt_record_wait(P->events[ns + i], P->streams[i], main);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// The whole plan eagerly: fork, the chunks in run order (each on its stream), join.
hipError_t enqueue_plan(negf_plan* P, const Outs& outs, char* ws, unsigned long long* stamps, hipStream_t main) {
  hipError_t e = enqueue_fork(P, outs, stamps, main);
  for (size_t k = 0; k < P->run_order.size() && e == hipSuccess; ++k)
    e = enqueue_chunk(P, P->run_order[k], outs, ws, stamps);
  return e == hipSuccess ? enqueue_join(P, main) : e;
}

void destroy_graphs(negf_plan* P) {
  for (void* g : P->graphs) (void)rt_graph_destroy(g);
  P->graphs.clear();
}

void destroy_queue_graphs(negf_plan* P) {
  for (void* g : P->qgraphs) (void)rt_graph_destroy(g);
  P->qgraphs.clear();
  P->qkey.clear();
}

// ---- point queue: task lists streamed through the plan's chunks (see negf_plan_run_queue)

struct QueueArgs {
  const double* const* task_E;   // per problem, device
  const int32_t* n_tasks;        // per problem, host
  std::vector<long> task_off;    // per problem: offset of its tasks in the result arrays
  int32_t* task_info;
  double* task_dos;
  unsigned long long* task_stamps;
  int* rounds;                   // per segment (device)
  int* slot_task;                // per point (device)
};

size_t queue_segments(const negf_plan* P) {
  size_t n = 0;
  for (const Chunk& c : P->chunks) n += c.segs.size();
  return n;
}

// Rounds a worker stream runs: the most any segment of its chunks needs.
int stream_rounds(const negf_plan* P, int si, const int32_t* n_tasks) {
  int r = 0;
  for (size_t c = 0; c < P->chunks.size(); ++c) {
    if (P->stream_of[c] != si) continue;
    for (const Seg& g : P->chunks[c].segs) {
      const int q = (int)(g.pr - P->probs.data());
      const int nq = g.pr->n_e;
      r = std::max(r, (int)((n_tasks[q] + nq - 1) / nq));
    }
  }
  return r;
}

// One round of worker stream si: for each of its chunks (in run order) the task intake of its
// segments, the chunk, and the results of its segments.
hipError_t enqueue_queue_round(negf_plan* P, int si, const Outs& outs, char* ws, const QueueArgs& qa) {
  size_t seg_base = 0;
  std::vector<size_t> first_seg(P->chunks.size());
  for (size_t c = 0; c < P->chunks.size(); ++c) {
    first_seg[c] = seg_base;
    seg_base += P->chunks[c].segs.size();
  }
  for (size_t k = 0; k < P->run_order.size(); ++k) {
    const size_t c = P->run_order[k];
    if (P->stream_of[c] != si) continue;
    const Chunk& ch = P->chunks[c];
    hipStream_t st = P->streams[si];
    hipError_t e = hipSuccess;
    for (size_t j = 0; j < ch.segs.size() && e == hipSuccess; ++j) {
      const Seg& g = ch.segs[j];
      const int q = (int)(g.pr - P->probs.data());
      const long p0 = ch.first_point + g.off;
      e = launch_queue_pop(const_cast<double*>(g.pr->energies), g.e0, g.n, g.pr->n_e, qa.task_E[q], qa.n_tasks[q],
                           qa.rounds + first_seg[c] + j, qa.slot_task + p0, outs.info + p0, st);
    }
    if (e == hipSuccess) e = enqueue_chunk(P, c, outs, ws, nullptr);
    for (size_t j = 0; j < ch.segs.size() && e == hipSuccess; ++j) {
      const Seg& g = ch.segs[j];
      const int q = (int)(g.pr - P->probs.data());
      const long p0 = ch.first_point + g.off;
      const double2* GRd = outs.GRd + ch.out_diag_off + (size_t)g.off * ch.nb * ch.b * ch.b;
      e = launch_queue_finish(GRd, ch.nb, ch.b, g.n, qa.slot_task + p0, outs.info + p0, qa.task_info + qa.task_off[q],
                              qa.task_dos + qa.task_off[q], qa.task_stamps + qa.task_off[q], st);
    }
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Capture each worker stream's chunks into its own graph; a begun capture is always ended.
hipError_t capture_plan(negf_plan* P, const Outs& outs, char* ws, unsigned long long* stamps) {
  destroy_graphs(P);
  for (int si = 0; si < P->n_streams; ++si) {
    hipError_t e = rt_capture_begin(P->streams[si]);
    if (e != hipSuccess) return e;
    for (size_t k = 0; k < P->run_order.size() && e == hipSuccess; ++k)
      if (P->stream_of[P->run_order[k]] == si) e = enqueue_chunk(P, P->run_order[k], outs, ws, stamps);
    void* exec = nullptr;
    const hipError_t e2 = rt_capture_end(P->streams[si], &exec);
    if (e != hipSuccess || e2 != hipSuccess) {
      if (exec) (void)rt_graph_destroy(exec);
      destroy_graphs(P);
      return e != hipSuccess ? e : e2;
    }
    P->graphs.push_back(exec);
  }
  return hipSuccess;
}

}  // namespace

extern "C" {

negf_status negf_plan_create(const negf_problem* problems, int32_t n_prob, negf_precision prec,
                             const negf_options* opt, const negf_tuning* tunings, int32_t n_tunings,
                             int32_t n_streams, negf_plan** plan) {
  if (!plan) return NEGF_EINVAL;
  *plan = nullptr;
  negf_status st = check_problems(problems, n_prob);
  if (st != NEGF_OK) return st;
  if (prec != NEGF_PLAIN_FP64 && prec != NEGF_FP32_REFINE && prec != NEGF_FP32_NOREFINE) return NEGF_EINVAL;
  if (n_streams < 1 || n_streams > 16 || n_tunings < 0 || (n_tunings > 0 && !tunings)) return NEGF_EINVAL;
  negf_plan* P = new negf_plan();
  P->probs.assign(problems, problems + n_prob);
  P->prec = prec;
  P->base = get_opts(opt);
  if (!opt || opt->sr_max_iter <= 0) P->base.max_iter = 40;   // fixed decimation count of a plan
  P->n_streams = n_streams;
  auto tuning_of = [&](int b) -> const negf_tuning* {
    for (int i = 0; i < n_tunings; ++i)
      if (tunings[i].b == b) return &tunings[i];
    return nullptr;
  };
  P->chunks = make_chunks_by(P->probs.data(), n_prob, [&](int, int b) {
    const negf_tuning* t = tuning_of(b);
    return (t && t->batch > 0) ? t->batch : P->base.batch;
  });
  for (const Chunk& c : P->chunks) {
    Opts o = P->base;
    if (const negf_tuning* t = tuning_of(c.b)) {
      if (t->gemm_tile >= GEMM_TILE_64 && t->gemm_tile <= GEMM_TILE_LAST) o.tile = t->gemm_tile;
      if (t->gemm_tile_f32 >= GEMM_TILE_64 && t->gemm_tile_f32 <= GEMM_TILE_LAST) o.tile32 = t->gemm_tile_f32;
      if (t->inv_nb == 16 || t->inv_nb == 32) o.inv_nb = t->inv_nb;
    }
    P->chunk_opts.push_back(o);
  }
  // longest-processing-time-first assignment of chunks to streams
  std::vector<size_t> order(P->chunks.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(),
                   [&](size_t a, size_t b) { return chunk_cost(P->chunks[a]) > chunk_cost(P->chunks[b]); });
  std::vector<double> load(n_streams, 0.0);
  std::vector<size_t> ws_need(n_streams, 0);
  P->stream_of.assign(P->chunks.size(), 0);
  for (size_t k : order) {
    const int si = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    P->stream_of[k] = si;
    load[si] += chunk_cost(P->chunks[k]);
    Carver cv{nullptr, 0};
    const Chunk& c = P->chunks[k];
    carve_chunk(cv, OPK_RL, c.nb, c.b, c.npts, prec, 2);
    ws_need[si] = std::max(ws_need[si], cv.off);
  }
  // each stream runs its chunks shortest first: the same total per stream, earlier completion
  // of the small ones
  P->run_order.assign(order.rbegin(), order.rend());
  size_t off = 0;
  for (int i = 0; i < n_streams; ++i) {
    P->stream_ws_off.push_back(off);
    off += (ws_need[i] + 255) & ~(size_t)255;
  }
  P->ws_total = off;
  *plan = P;
  return NEGF_OK;
}

size_t negf_plan_workspace_bytes(const negf_plan* plan) { return plan ? plan->ws_total + 256 : 0; }

int32_t negf_plan_chunks(const negf_plan* plan, int32_t* first_point, int32_t* n_points, int32_t* stream_index) {
  if (!plan) return 0;
  for (size_t c = 0; c < plan->chunks.size(); ++c) {
    if (first_point) first_point[c] = (int32_t)plan->chunks[c].first_point;
    if (n_points) n_points[c] = plan->chunks[c].npts;
    if (stream_index) stream_index[c] = plan->stream_of[c];
  }
  return (int32_t)plan->chunks.size();
}

double negf_plan_clock_hz(void) { return rt_wallclock_hz(); }

negf_status negf_plan_execute(negf_plan* plan, int32_t use_graph, void* GR_diag, void* GR_upper, void* GR_lower,
                              void* GL_diag, void* GL_upper, void* GG_diag, void* GG_upper, int32_t* info,
                              uint64_t* stamps, void* workspace, size_t ws_bytes, void* stream) {
  if (!plan || !GR_diag || !GR_upper || !GL_diag || !GL_upper || !info || !workspace) return NEGF_EINVAL;
  if ((GG_diag == nullptr) != (GG_upper == nullptr)) return NEGF_EINVAL;
  const void* ps[] = {GR_diag, GR_upper, GR_lower, GL_diag, GL_upper, GG_diag, GG_upper, stamps};
  for (const void* p : ps)
    if (p && ((uintptr_t)p & 15)) return NEGF_EINVAL;
  if (ws_bytes < negf_plan_workspace_bytes(plan)) return NEGF_EINVAL;
  negf_plan* P = plan;
  hipStream_t main = (hipStream_t)stream;
  if (P->streams.empty()) {
    for (int i = 0; i < P->n_streams; ++i) {
      hipStream_t st = nullptr;
      if (rt_stream_create(&st) != hipSuccess) return NEGF_EHIP;
      P->streams.push_back(st);
    }
    for (int i = 0; i < 2 * P->n_streams; ++i) {
      hipEvent_t ev = nullptr;
      if (rt_event_create(&ev) != hipSuccess) return NEGF_EHIP;
      P->events.push_back(ev);
    }
  }
  Outs outs{(double2*)GR_diag, (double2*)GR_upper, (double2*)GR_lower, (double2*)GL_diag, (double2*)GL_upper,
            (double2*)GG_diag, (double2*)GG_upper, info, nullptr};
  char* ws = align256(workspace);
  unsigned long long* stp = (unsigned long long*)stamps;
  if (!use_graph) return to_status(enqueue_plan(P, outs, ws, stp, main));
  const bool reuse = (int)P->graphs.size() == P->n_streams && same_outs(P->cap_outs, outs) && P->cap_ws == ws &&
                     P->cap_stamps == stp;
  hipError_t e = enqueue_fork(P, outs, stp, main);
  if (e == hipSuccess && !reuse) {
    // captured after the fork was enqueued: capture records, it does not run anything
    if (capture_plan(P, outs, ws, stp) != hipSuccess) {
      (void)enqueue_join(P, main);   // the capture failed; the join keeps the streams ordered
      return NEGF_EHIP;
    }
    P->cap_outs = outs;
    P->cap_ws = ws;
    P->cap_stamps = stp;
  }
  for (int si = 0; si < P->n_streams && e == hipSuccess; ++si) e = rt_graph_launch(P->graphs[si], P->streams[si]);
  if (e == hipSuccess) e = enqueue_join(P, main);
  return to_status(e);
}

size_t negf_plan_queue_bytes(const negf_plan* plan) {
  if (!plan) return 0;
  const size_t a = (queue_segments(plan) * sizeof(int) + 255) & ~(size_t)255;
  const size_t b = ((size_t)count_points(plan->probs.data(), (int)plan->probs.size()) * sizeof(int) + 255) &
                   ~(size_t)255;
  return a + b + 256;
}

negf_status negf_plan_run_queue(negf_plan* plan, int32_t use_graph, const double* const* task_E,
                                const int32_t* n_tasks, int32_t* task_info, double* task_dos, uint64_t* task_stamps,
                                uint64_t* start_stamp, void* GR_diag, void* GR_upper, void* GR_lower, void* GL_diag,
                                void* GL_upper, void* GG_diag, void* GG_upper, int32_t* info, void* queue_ws,
                                size_t queue_bytes, void* workspace, size_t ws_bytes, void* stream) {
  if (!plan || !task_E || !n_tasks || !GR_diag || !GR_upper || !GL_diag || !GL_upper || !info || !workspace ||
      !queue_ws)
    return NEGF_EINVAL;
  if ((GG_diag == nullptr) != (GG_upper == nullptr)) return NEGF_EINVAL;
  const void* ps[] = {GR_diag, GR_upper, GR_lower, GL_diag, GL_upper, GG_diag, GG_upper};
  for (const void* p : ps)
    if (p && ((uintptr_t)p & 15)) return NEGF_EINVAL;
  if (ws_bytes < negf_plan_workspace_bytes(plan) || queue_bytes < negf_plan_queue_bytes(plan)) return NEGF_EINVAL;
  negf_plan* P = plan;
  const int np = (int)P->probs.size();
  long total = 0;
  QueueArgs qa;
  qa.task_E = task_E;
  qa.n_tasks = n_tasks;
  for (int q = 0; q < np; ++q) {
    // a problem without slots cannot take tasks; a slot takes any task's energy, so the
    // scattering self-energies must be the same for every energy
    if (n_tasks[q] < 0 || (n_tasks[q] > 0 && (!task_E[q] || P->probs[q].n_e < 1))) return NEGF_EINVAL;
    if (n_tasks[q] > 0 && P->probs[q].sc_stride != 0) return NEGF_EINVAL;
    qa.task_off.push_back(total);
    total += n_tasks[q];
  }
  if (total > 0 && (!task_info || !task_dos || !task_stamps)) return NEGF_EINVAL;
  qa.task_info = task_info;
  qa.task_dos = task_dos;
  qa.task_stamps = (unsigned long long*)task_stamps;
  char* qws = align256(queue_ws);
  qa.rounds = (int*)qws;
  qa.slot_task = (int*)(qws + ((queue_segments(P) * sizeof(int) + 255) & ~(size_t)255));
  hipStream_t main = (hipStream_t)stream;
  if (P->streams.empty()) {
    for (int i = 0; i < P->n_streams; ++i) {
      hipStream_t st = nullptr;
      if (rt_stream_create(&st) != hipSuccess) return NEGF_EHIP;
      P->streams.push_back(st);
    }
    for (int i = 0; i < 2 * P->n_streams; ++i) {
      hipEvent_t ev = nullptr;
      if (rt_event_create(&ev) != hipSuccess) return NEGF_EHIP;
      P->events.push_back(ev);
    }
  }
  Outs outs{(double2*)GR_diag, (double2*)GR_upper, (double2*)GR_lower, (double2*)GL_diag, (double2*)GL_upper,
            (double2*)GG_diag, (double2*)GG_upper, info, nullptr};
  char* ws = align256(workspace);
  // start: round counters to zero, the start stamp, then the fork to the workers
  hipError_t e = launch_fill_int((int)queue_segments(P), qa.rounds, 0, main);
  if (e == hipSuccess && start_stamp) e = launch_stamp((unsigned long long*)start_stamp, main);
  for (int i = 0; i < P->n_streams && e == hipSuccess; ++i) e = rt_record_wait(P->events[i], main, P->streams[i]);
  if (e != hipSuccess) return to_status(e);
  std::vector<int> rounds(P->n_streams);
  int max_rounds = 0;
  for (int si = 0; si < P->n_streams; ++si) max_rounds = std::max(max_rounds, rounds[si] = stream_rounds(P, si, n_tasks));
  if (use_graph) {
    std::vector<const void*> key = {GR_diag, GR_upper, GR_lower, GL_diag, GL_upper, GG_diag, GG_upper, info,
                                    ws, qws, task_info, task_dos, task_stamps};
    for (int q = 0; q < np; ++q) {
      key.push_back(task_E[q]);
      key.push_back((const void*)(intptr_t)n_tasks[q]);
    }
    if (P->qkey != key || (int)P->qgraphs.size() != P->n_streams) {
      destroy_queue_graphs(P);
      for (int si = 0; si < P->n_streams && e == hipSuccess; ++si) {
        e = rt_capture_begin(P->streams[si]);
        if (e != hipSuccess) break;
        hipError_t ec = enqueue_queue_round(P, si, outs, ws, qa);
        void* exec = nullptr;
        const hipError_t e2 = rt_capture_end(P->streams[si], &exec);
        if (ec != hipSuccess || e2 != hipSuccess) {
          if (exec) (void)rt_graph_destroy(exec);
          e = ec != hipSuccess ? ec : e2;
          break;
        }
        P->qgraphs.push_back(exec);
      }
      if (e != hipSuccess) {
        destroy_queue_graphs(P);
        (void)enqueue_join(P, main);   // the capture failed; the join keeps the streams ordered
        return NEGF_EHIP;
      }
      P->qkey = key;
    }
    for (int r = 0; r < max_rounds && e == hipSuccess; ++r)
      for (int si = 0; si < P->n_streams && e == hipSuccess; ++si)
        if (r < rounds[si]) e = rt_graph_launch(P->qgraphs[si], P->streams[si]);
  } else {
    for (int r = 0; r < max_rounds && e == hipSuccess; ++r)
      for (int si = 0; si < P->n_streams && e == hipSuccess; ++si)
        if (r < rounds[si]) e = enqueue_queue_round(P, si, outs, ws, qa);
  }
  if (e == hipSuccess) e = enqueue_join(P, main);
  return to_status(e);
}

void negf_plan_destroy(negf_plan* plan) {
  if (!plan) return;
  destroy_graphs(plan);
  destroy_queue_graphs(plan);
  for (hipEvent_t e : plan->events) (void)rt_event_destroy(e);
  for (hipStream_t s : plan->streams) (void)rt_stream_destroy(s);
  delete plan;
}

}  // extern "C"

// ------------------------------------------------------------------ C ABI

extern "C" {

size_t negf_workspace_bytes(int32_t op, const negf_problem* problems, int32_t n_prob, negf_precision prec,
                            const negf_options* opt) {
  if (check_problems(problems, n_prob) != NEGF_OK) return 0;
  const int opk = op == NEGF_OP_OBC ? OPK_OBC : op == NEGF_OP_RETARDED ? OPK_R
                : op == NEGF_OP_LESSER_GREATER ? OPK_RL : OPK_T;
  return workspace_for(opk, problems, n_prob, prec, get_opts(opt));
}

negf_status negf_obc_surface(const negf_problem* problems, int32_t n_prob, int32_t side, const negf_options* opt,
                             const void* seed, void* g_surf, void* sigma_r, int32_t* iters, double* resid,
                             int32_t* info, void* workspace, size_t ws_bytes, void* stream) {
  negf_status st = check_problems(problems, n_prob);
  if (st != NEGF_OK) return st;
  if (side != 0 && side != 1) return NEGF_EINVAL;
  if (!g_surf || !sigma_r || !info || !workspace) return NEGF_EINVAL;
  if (!aligned16(g_surf) || !aligned16(sigma_r) || (seed && !aligned16(seed))) return NEGF_EINVAL;
  const Opts o = get_opts(opt);
  if (ws_bytes < workspace_for(OPK_OBC, problems, n_prob, NEGF_PLAIN_FP64, o)) return NEGF_EINVAL;
  Ctx cx;
  cx.s = (hipStream_t)stream;
  cx.o = o;
  const long npts_all = count_points(problems, n_prob);
  cx.chk(launch_fill_int((int)npts_all, info, 0, cx.s));
  for (const Chunk& ch : make_chunks(problems, n_prob, o.batch)) {
    Carver cv{align256(workspace), ws_bytes - (size_t)(align256(workspace) - (char*)workspace)};
    ChunkWs w = carve_chunk(cv, OPK_OBC, ch.nb, ch.b, ch.npts, NEGF_PLAIN_FP64, 1);
    if (cv.overflow) return NEGF_EINVAL;
    const long bb = (long)ch.b * ch.b;
    const long pofs = (long)ch.first_point * bb;   // all points of an OBC call share b only per chunk
    // outputs are [points][b][b]: offset by the blocks of the previous points
    size_t blk_off = 0;
    {
      long gp = 0;
      for (int q = 0; q < n_prob && gp < ch.first_point; ++q) {
        const long take = std::min<long>(problems[q].n_e, ch.first_point - gp);
        blk_off += (size_t)take * problems[q].dev.b * problems[q].dev.b;
        gp += take;
      }
    }
    (void)pofs;
    Blocks sig{(double2*)sigma_r + blk_off, bb};
    const int sides[1] = {side};
    const double2* sd = seed ? (const double2*)seed + blk_off : nullptr;
    run_decimation(cx, ch, sides, 1, w.lw, sd, bb, sig, sig, info + ch.first_point,
                   iters ? iters + ch.first_point : nullptr, resid ? resid + ch.first_point : nullptr);
    cx.lincomb(ch.b, ch.npts, ONE, w.lw.g.p, bb, ZERO, nullptr, 0, ZERO, (double2*)g_surf + blk_off, bb);
    if (!cx.ok()) break;
  }
  return to_status(cx.err);
}

static negf_status rgf_common(int opk, const negf_problem* problems, int32_t n_prob, negf_precision prec,
                              const negf_options* opt, const Outs& outs, void* workspace, size_t ws_bytes,
                              void* stream) {
  negf_status st = check_problems(problems, n_prob);
  if (st != NEGF_OK) return st;
  if (prec != NEGF_PLAIN_FP64 && prec != NEGF_FP32_REFINE && prec != NEGF_FP32_NOREFINE) return NEGF_EINVAL;
  if (!outs.info || !workspace) return NEGF_EINVAL;
  const Opts o = get_opts(opt);
  if (ws_bytes < workspace_for(opk, problems, n_prob, prec, o)) return NEGF_EINVAL;
  Ctx cx;
  cx.s = (hipStream_t)stream;
  cx.o = o;
  const long npts_all = count_points(problems, n_prob);
  cx.chk(launch_fill_int((int)npts_all, outs.info, 0, cx.s));
  for (const Chunk& ch : make_chunks(problems, n_prob, o.batch)) {
    Carver cv{align256(workspace), ws_bytes - (size_t)(align256(workspace) - (char*)workspace)};
    ChunkWs w = carve_chunk(cv, opk, ch.nb, ch.b, ch.npts, prec, 2);
    if (cv.overflow) return NEGF_EINVAL;
    run_chunk(cx, opk, ch, w, prec, outs);
    if (!cx.ok()) break;
  }
  return to_status(cx.err);
}

negf_status negf_rgf_retarded(const negf_problem* problems, int32_t n_prob, negf_precision prec,
                              const negf_options* opt, void* GR_diag, void* GR_upper, void* GR_lower, int32_t* info,
                              void* workspace, size_t ws_bytes, void* stream) {
  if (!GR_diag || !GR_upper) return NEGF_EINVAL;
  if (!aligned16(GR_diag) || !aligned16(GR_upper) || (GR_lower && !aligned16(GR_lower))) return NEGF_EINVAL;
  Outs o{(double2*)GR_diag, (double2*)GR_upper, (double2*)GR_lower, nullptr, nullptr, nullptr, nullptr, info, nullptr};
  return rgf_common(OPK_R, problems, n_prob, prec, opt, o, workspace, ws_bytes, stream);
}

negf_status negf_rgf_lesser_greater(const negf_problem* problems, int32_t n_prob, negf_precision prec,
                                    const negf_options* opt, void* GR_diag, void* GR_upper, void* GR_lower,
                                    void* GL_diag, void* GL_upper, void* GG_diag, void* GG_upper, int32_t* info,
                                    void* workspace, size_t ws_bytes, void* stream) {
  if (!GR_diag || !GR_upper || !GL_diag || !GL_upper) return NEGF_EINVAL;
  if ((GG_diag == nullptr) != (GG_upper == nullptr)) return NEGF_EINVAL;
  const void* ps[] = {GR_diag, GR_upper, GR_lower, GL_diag, GL_upper, GG_diag, GG_upper};
  for (const void* p : ps)
    if (p && !aligned16(p)) return NEGF_EINVAL;
  Outs o{(double2*)GR_diag, (double2*)GR_upper, (double2*)GR_lower, (double2*)GL_diag, (double2*)GL_upper,
         (double2*)GG_diag, (double2*)GG_upper, info, nullptr};
  return rgf_common(OPK_RL, problems, n_prob, prec, opt, o, workspace, ws_bytes, stream);
}

}  // extern "C"

// ------------------------------------------------------------------ allocation-free variant

// Scratch of negf_rgf_lesser_greater_static: one copy per GPU (allocated when the
// library's code object is loaded on that device and held until the process ends).
// Host code never uses the name itself for device memory; it uses the address that
// hipGetSymbolAddress returns for the current device (scratch_address).
static __device__ __align__(256) unsigned char scratch[NEGF_STATIC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_addr[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per device
// (with that device current) and kept.
hipError_t scratch_address(void** out) {
  *out = nullptr;
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_addr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_addr[dev] = p;
  }
  *out = g_scratch_addr[dev];
  return hipSuccess;
}

// Points in flight per chunk for the static scratch: opt->batch if set, else the
// largest count whose workspace fits (0 when not even one point fits).
int static_batch(const negf_problem* pr, int n_prob, negf_precision prec, const Opts& o) {
  auto fits = [&](int b) {
    Opts t = o;
    t.batch = b;
    return workspace_for(OPK_RL, pr, n_prob, prec, t) <= (size_t)NEGF_STATIC_SCRATCH_BYTES;
  };
  if (o.batch > 0) return fits(o.batch) ? o.batch : 0;
  const long total = count_points(pr, n_prob);
  if (total <= 0) return 1;
  if (!fits(1)) return 0;
  int lo = 1, hi = (int)std::min<long>(total, 1 << 30);
  while (lo < hi) {   // largest b in [lo, hi] that fits (fits is monotone in b)
    const int mid = lo + (hi - lo + 1) / 2;
    if (fits(mid)) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

}  // namespace

extern "C" {

negf_status negf_rgf_lesser_greater_static(const negf_problem* problems, int32_t n_prob, negf_precision prec,
                                           const negf_options* opt, void* GR_diag, void* GR_upper, void* GR_lower,
                                           void* GL_diag, void* GL_upper, void* GG_diag, void* GG_upper,
                                           int32_t* info, void* stream) {
  if (!GR_diag || !GR_upper || !GL_diag || !GL_upper || !info) return NEGF_EINVAL;
  if ((GG_diag == nullptr) != (GG_upper == nullptr)) return NEGF_EINVAL;
  const void* ps[] = {GR_diag, GR_upper, GR_lower, GL_diag, GL_upper, GG_diag, GG_upper};
  for (const void* p : ps)
    if (p && !aligned16(p)) return NEGF_EINVAL;
  negf_status st = check_problems(problems, n_prob);
  if (st != NEGF_OK) return st;
  if (prec != NEGF_PLAIN_FP64 && prec != NEGF_FP32_REFINE && prec != NEGF_FP32_NOREFINE) return NEGF_EINVAL;
  const int batch = static_batch(problems, n_prob, prec, get_opts(opt));
  if (batch <= 0) return NEGF_ENOMEM;   // one point (or the requested batch) exceeds the scratch
  void* ws = nullptr;
  if (scratch_address(&ws) != hipSuccess) return NEGF_EHIP;
  negf_options o{};
  if (opt) o = *opt;
  o.batch = batch;
  Outs outs{(double2*)GR_diag, (double2*)GR_upper, (double2*)GR_lower, (double2*)GL_diag, (double2*)GL_upper,
            (double2*)GG_diag, (double2*)GG_upper, info, nullptr};
  return rgf_common(OPK_RL, problems, n_prob, prec, &o, outs, ws, (size_t)NEGF_STATIC_SCRATCH_BYTES, stream);
}

negf_status negf_transmission(const negf_problem* problems, int32_t n_prob, const negf_options* opt, double* T,
                              int32_t* info, void* workspace, size_t ws_bytes, void* stream) {
  if (!T) return NEGF_EINVAL;
  Outs o{nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, info, T};
  return rgf_common(OPK_T, problems, n_prob, NEGF_PLAIN_FP64, opt, o, workspace, ws_bytes, stream);
}

negf_status negf_zgemm_batched(char opa, char opb, int32_t M, int32_t N, int32_t K, const double* alpha,
                               const void* A, int64_t lda, int64_t sa, const void* B, int64_t ldb, int64_t sb,
                               const double* beta, void* C, int64_t ldc, int64_t sc, int32_t batch, int32_t prec,
                               int32_t tile, void* stream) {
  if (M < 0 || N < 0 || K < 0 || batch < 0 || !alpha || !beta) return NEGF_EINVAL;
  if ((opa != 'N' && opa != 'C') || (opb != 'N' && opb != 'C')) return NEGF_EINVAL;
  if (M == 0 || N == 0 || batch == 0) return NEGF_OK;
  if (!A || !B || !C || !aligned16(A) || !aligned16(B) || !aligned16(C)) return NEGF_EINVAL;
  GemmDesc g{};
  g.M = M; g.N = N; g.K = K; g.batch = batch;
  g.opA = opa == 'N' ? OP_N : OP_C;
  g.opB = opb == 'N' ? OP_N : OP_C;
  g.A = MatRef{(const double2*)A, (long)lda, (long)sa};
  g.B = MatRef{(const double2*)B, (long)ldb, (long)sb};
  g.alpha = make_double2(alpha[0], alpha[1]);
  g.beta = make_double2(beta[0], beta[1]);
  g.Cin = MatRef{(const double2*)C, (long)ldc, (long)sc};
  g.C = MatOut{(double2*)C, (long)ldc, (long)sc};
  const int skew = prec & 4;   // the product is anti-Hermitian: upper triangle computed, lower mirrored
  prec &= 3;
  if (prec > 2 || (skew && M != N)) return NEGF_EINVAL;
  g.prec = prec == 1 ? PREC_F32 : PREC_F64;
  g.gauss = prec == 2;
  g.skew = skew ? 1 : 0;
  g.tile = tile;
  g.xcd_remap = 1;
  g.prof_class = -1;
  return to_status(launch_gemm(g, (hipStream_t)stream));
}

size_t negf_inverse_workspace_bytes(int32_t n, int32_t batch) {
  if (n <= 0 || batch <= 0) return 0;
  return inverse_scratch_bytes(n, batch) + 256;
}

negf_status negf_zinv_batched(int32_t n, int32_t batch, void* M, void* out, int32_t* info, int32_t nb,
                              void* workspace, size_t ws_bytes, void* stream) {
  if (n <= 0 || n > 1024 || batch < 0) return NEGF_EINVAL;
  if (batch == 0) return NEGF_OK;
  if (!M || !out || M == out || !workspace || !aligned16(M) || !aligned16(out)) return NEGF_EINVAL;
  if (ws_bytes < negf_inverse_workspace_bytes(n, batch)) return NEGF_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  if (info) {
    hipError_t e = launch_fill_int(batch, info, 0, s);
    if (e != hipSuccess) return NEGF_EHIP;
  }
  InvDesc d{};
  d.n = n; d.batch = batch;
  d.M = (double2*)M; d.ldm = n; d.sM = (long)n * n;
  d.out = (double2*)out; d.ldo = n; d.sO = (long)n * n;
  d.scratch = align256(workspace);
  d.info = info; d.info_mod = 0;
  d.nb = nb;
  return to_status(launch_inverse(d, s));
}

const char* negf_status_string(negf_status s) {
  switch (s) {
    case NEGF_OK: return "ok";
    case NEGF_EINVAL: return "invalid argument";
    case NEGF_ENOCONV: return "lead decimation did not converge";
    case NEGF_ESINGULAR: return "singular block";
    case NEGF_ENONFINITE: return "non-finite value";
    case NEGF_EHIP: return "HIP runtime error";
    case NEGF_ENOMEM: return "out of memory";
  }
  return "unknown status";
}

int32_t negf_version(void) { return 102; }

}  // extern "C"
