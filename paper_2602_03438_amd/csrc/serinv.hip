// Partitioned selected inversion on one GPU (the parallel solver the paper
// builds on Schur complements of block-tridiagonal matrices, Fig. 3 and the
// paragraph after it in Section II): the device is split into P partitions,
// each partition eliminates its interior independently, the boundary blocks
// form a small reduced block-tridiagonal system that is solved sequentially,
// and each partition then recovers its selected blocks of G^R and G^<> with
// the exact boundary self-energies the reduced system provides.  On one GPU
// the partitions are a batch axis next to the energy points, so that a few
// energies (down to one) still give every launch P times more work.
//
// Layout (period T = ceil((nb + 1) / P), blocks numbered from 0):
//   partition p has interior blocks [p T, p T + m_p) with m_p = T - 2 for
//   p < P - 1 and m_{P-1} = nb - (P - 1) T; its top boundary is p T - 1
//   (p >= 1) and its bottom boundary p T + T - 2 (p <= P - 2).  The boundary
//   blocks e_0, s_1, e_1, ..., s_{P-1} form the reduced system.
// Items are (partition, energy point) pairs, partition-major: item
// q = p * npts + k.  Every step of the lock-stepped loops is active on one
// contiguous range of items (whole partitions), so no masks are needed.
//
// 1. Interior elimination (all items): the left-connected recursion over the
//    interior, carrying the corner blocks of the interior inverse L and of
//    Gamma = L Sigma^<> L^H (first row, last column): L_11, L_1m, L_m1, L_mm,
//    Gamma_11, Gamma_1m, Gamma_mm.  Step i (A = A_{i-1,i}):
//      g_i = (A_ii - A^H g_{i-1} A)^{-1};  RA = R A;  R <- -RA g_i
//      V = A^H C;  C <- -g_i V;  D <- D - R V                 (D = L_11)
//      gam_i = g_i (Sigma_i + A^H gam_{i-1} A) g_i^H
//      T1 = G1 A;  G1 <- -T1 g_i^H - RA gam_i                  (G1 = Gamma_1i)
//      G11 <- G11 - T1 R^H + (T1 R^H)^H + (RA gam_i) RA^H
// 2. Reduced system on the boundary blocks (Schur complements, with the
//    Keldysh form of the lesser part, whose reduced Sigma^<> couples s_p and
//    e_p inside a partition):
//      S_ss = A_ss - A_{s,s+1} L_11 A_{s+1,s},  S_se = -A_{s,s+1} L_1m A_{e-1,e}
//      S_es = -A_{e,e-1} L_m1 A_{s+1,s},        S_ee = A_ee - A_{e,e-1} L_mm A_{e-1,e}
//      Sigma_ss = Sigma_s + A_{s,s+1} Gamma_11 A_{s,s+1}^H,
//      Sigma_se = A_{s,s+1} Gamma_1m A_{e-1,e},  Sigma_ee = Sigma_e + A_{e,e-1} Gamma_mm A_{e,e-1}^H
//    then left-connected (forward) and right-connected (backward) sweeps over
//    it; for a block-tridiagonal Sigma^<> the left-connected lesser step is
//      gam_r = g_r (Sigma_rr + L gam_{r-1} L^H - Y + Y^H) g_r^H,  Y = L g_{r-1} Sigma_{r-1,r}
//    with L the coupling from block r - 1 to r (and its mirror from the right).
// 3. Each partition runs the plain RGF sweeps over its own blocks with the
//    boundary self-energies from step 2 (retarded A g A^H and lesser A gam A^H
//    of the left- and right-connected neighbours) where the device leads
//    would be: this gives every selected block inside the partition.
// 4. The blocks that couple two partitions, G_{e,e+1}, G_{e+1,e} and
//    G^<>_{e,e+1}, from the left-connected g_e, gam_e of step 2 and the
//    first block of the next partition (the backward-step formulas).
// Results are then copied into the point-major outputs.
#include "orch.h"

using namespace negf;
using namespace negf::orch;

namespace {

struct Layout {
  int P, T, mlast, nb, b, npts, Q;
  long bb;
};

bool make_layout(int nb, int b, int npts, int P, Layout& L) {
  if (P < 2) return false;
  const int T = (nb + 1 + P - 1) / P;
  const int mlast = nb - (P - 1) * T;
  if (T < 3 || mlast < 1) return false;
  L = Layout{P, T, mlast, nb, b, npts, P * npts, (long)b * b};
  return true;
}

struct SerinvWs {
  PointWs pw;            // lead self-energies of every point (sigL, sigR, Gamma, Sigma^<>)
  LeadWs lw;             // decimation scratch (shared region)
  // step 1, per item
  Blocks g, D, R, C, A0, Ac, X, RA, V, T1, B, W, As, Ae;
  Blocks gam[2], G11[2], G1m[2];
  // reduced system, per (partition, point)
  Blocks DS, DE, USE, LES, UE, SS[2], SE[2], SSE[2];
  Blocks glS, glE, grS, grE, ylS[2], ylE[2], yrS[2], yrE[2];
  // step 3, per item: sub-device blocks (stride T or T - 1 blocks) and temporaries
  double2 *Gd, *Gu, *Gl, *X3, *Ld[2], *Lu[2];
  Blocks U0, U1, U2, U3, U4, SigTop, SigBot, STop[2], SBot[2];
  // step 4, per boundary pair
  Blocks GuX, GlX, LuX[2];
  void* inv_scratch;
};

SerinvWs carve_serinv(Carver& cv, const Layout& L, int nk) {
  SerinvWs w{};
  const int b = L.b, Q = L.Q, npts = L.npts;
  PointWs& p = w.pw;
  Blocks* pers[] = {&p.sigL, &p.sigR, &p.gamL, &p.gamR, &p.slL, &p.slR, &p.sgL, &p.sgR};
  for (Blocks* x : pers) *x = take_blocks(cv, b, npts);
  p.dot = cv.take<double>(npts);
  // the decimation runs before anything below is used: its scratch shares their region
  Carver sub{cv.base ? cv.base + cv.off : nullptr, cv.base ? cv.cap - std::min(cv.cap, cv.off) : 0};
  w.lw = carve_leads(sub, b, 2 * npts, false);
  Carver s2{cv.base ? cv.base + cv.off : nullptr, cv.base ? cv.cap - std::min(cv.cap, cv.off) : 0};
  Blocks* s1[] = {&w.g, &w.D, &w.R, &w.C, &w.A0, &w.Ac, &w.X, &w.RA, &w.V, &w.T1, &w.B, &w.W, &w.As, &w.Ae};
  for (Blocks* x : s1) *x = take_blocks(s2, b, Q);
  for (int k = 0; k < nk; ++k) {
    w.gam[k] = take_blocks(s2, b, Q);
    w.G11[k] = take_blocks(s2, b, Q);
    w.G1m[k] = take_blocks(s2, b, Q);
  }
  Blocks* red[] = {&w.DS, &w.DE, &w.USE, &w.LES, &w.UE, &w.glS, &w.glE, &w.grS, &w.grE};
  for (Blocks* x : red) *x = take_blocks(s2, b, Q);
  for (int k = 0; k < nk; ++k) {
    Blocks* rk[] = {&w.SS[k], &w.SE[k], &w.SSE[k], &w.ylS[k], &w.ylE[k], &w.yrS[k], &w.yrE[k]};
    for (Blocks* x : rk) *x = take_blocks(s2, b, Q);
  }
  const long bb = L.bb, T = L.T;
  w.Gd = s2.take<double2>((size_t)Q * T * bb);
  w.Gu = s2.take<double2>((size_t)Q * (T - 1) * bb);
  w.Gl = s2.take<double2>((size_t)Q * (T - 1) * bb);
  w.X3 = s2.take<double2>((size_t)Q * (T - 1) * bb);
  for (int k = 0; k < nk; ++k) {
    w.Ld[k] = s2.take<double2>((size_t)Q * T * bb);
    w.Lu[k] = s2.take<double2>((size_t)Q * (T - 1) * bb);
  }
  Blocks* s3[] = {&w.U0, &w.U1, &w.U2, &w.U3, &w.U4, &w.SigTop, &w.SigBot, &w.GuX, &w.GlX};
  for (Blocks* x : s3) *x = take_blocks(s2, b, Q);
  for (int k = 0; k < nk; ++k) {
    w.STop[k] = take_blocks(s2, b, Q);
    w.SBot[k] = take_blocks(s2, b, Q);
    w.LuX[k] = take_blocks(s2, b, Q);
  }
  w.inv_scratch = s2.take<char>(inverse_scratch_bytes(b, Q));
  cv.take<char>(std::max(sub.off, s2.off));
  if (sub.overflow || s2.overflow) cv.overflow = true;
  return w;
}

// Blocks of item range [q0, q0 + n) of a per-item array.
inline double2* at(const Blocks& x, int q0) { return x.p + (long)q0 * x.stride; }

struct Serinv {
  Ctx& cx;
  const negf_problem& pr;
  const Layout& L;
  SerinvWs& w;
  int nk;
  int* info;

  const negf_device& dev() const { return pr.dev; }

  // A-blocks of block index blk0 + g T for the items [q0, q0 + n) (g = item group relative to q0):
  // kind 0 diagonal E S - H - Sigma^R_sc, 1 coupling E S_{i,i+1} - H_{i,i+1}, 2 / 3 the lesser /
  // greater scattering self-energy (zero when the device has none)
  void assemble(int kind, int blk0, int q0, int n, double2* out) {
    if (n <= 0 || !cx.ok()) return;
    const int b = L.b;
    const negf_device& d = dev();
    AssembleDesc a = asm_base(b, n, pr.energies, out, L.bb);
    a.inner = L.npts;
    a.sHo = (long)L.T * L.bb;
    if (kind == 0) {
      a.S = blk(d.S_diag, blk0, b); a.s_identity = 1;
      a.H = blk(d.H_diag, blk0, b);
      a.Y = blk(d.sig_r_sc, blk0, b); a.sY = pr.sc_stride;
    } else if (kind == 1) {
      a.S = blk(d.S_upper, blk0, b); a.s_identity = 0;
      a.H = blk(d.H_upper, blk0, b);
    } else {
      a.energies = nullptr;
      a.S = nullptr; a.s_identity = 0; a.s_coef = 0.0;
      a.H = nullptr;
      a.Y = blk(kind == 2 ? d.sig_l_sc : d.sig_g_sc, blk0, b); a.sY = pr.sc_stride; a.y_coef = 1.0;
    }
    cx.assemble(a);
  }

  // C = alpha op(A) op(B) + beta Cin over n items with strides sA, sB, sCin, sC (elements)
  void mm(Op oa, Op ob, int n, double2 alpha, const double2* A, long sA, const double2* B, long sB, double2 beta,
          const double2* Cin, long sCi, double2* C, long sC) {
    if (n <= 0) return;
    cx.gemm(PREC_F64, oa, ob, L.b, n, alpha, A, sA, B, sB, beta, Cin, sCi, C, sC);
  }
  void mm(Op oa, Op ob, int n, double2 alpha, const double2* A, const double2* B, double2 beta, const double2* Cin,
          double2* C) {
    mm(oa, ob, n, alpha, A, L.bb, B, L.bb, beta, Cin, L.bb, C, L.bb);
  }
  void inv(int n, double2* M, double2* out, long sO) {
    if (n <= 0) return;
    cx.inverse(L.b, n, M, L.bb, out, sO, w.inv_scratch, info, L.npts);
  }
  void axpy(int n, double2 c, const double2* X, long sX, double2* out, long sOut) {   // out += c X
    if (n <= 0) return;
    cx.lincomb(L.b, n, c, X, sX, ONE, out, sOut, ZERO, out, sOut);
  }
  void copy(int n, const double2* X, long sX, double2* out, long sOut) {
    if (n <= 0) return;
    cx.lincomb(L.b, n, ONE, X, sX, ZERO, nullptr, 0, ZERO, out, sOut);
  }
  void adj_add(int n, double2 c, const double2* Wm, double2* out) {   // out += c Wm^H
    if (n <= 0 || !cx.ok()) return;
    cx.chk(launch_add_adjoint(L.b, n, c, Wm, L.bb, out, L.bb, cx.s));
  }
  const Blocks& lead_lesser(int k, int side) const {
    return side == 0 ? (k == 0 ? w.pw.slL : w.pw.sgL) : (k == 0 ? w.pw.slR : w.pw.sgR);
  }

  // ---------------------------------------------------------------- 1. interior elimination
  void eliminate_interiors() {
    const int np = L.npts, P = L.P, T = L.T, Q = L.Q;
    const int mmax = std::max(T - 2, L.mlast);
    const long bb = L.bb;
    for (int j = 0; j < mmax && cx.ok(); ++j) {
      const int lo = j < T - 2 ? 0 : (P - 1) * np;
      const int hi = j < L.mlast ? Q : (P - 1) * np;
      if (lo >= hi) continue;
      const int n = hi - lo;
      const int glo = lo / np;
      double2* A0 = at(w.A0, lo);
      assemble(0, glo * T + j, lo, n, A0);
      if (j == 0 && lo == 0) axpy(np, MONE, w.pw.sigL.p, bb, A0, bb);                    // left lead, block 0
      if (j == L.mlast - 1 && hi == Q) axpy(np, MONE, w.pw.sigR.p, bb, at(w.A0, (P - 1) * np), bb);
      double2 *g = at(w.g, lo), *D = at(w.D, lo), *R = at(w.R, lo), *C = at(w.C, lo);
      if (j == 0) {
        inv(n, A0, g, bb);
        copy(n, g, bb, D, bb);
        copy(n, g, bb, R, bb);
        copy(n, g, bb, C, bb);
      } else {
        double2 *Ac = at(w.Ac, lo), *X = at(w.X, lo), *RA = at(w.RA, lo), *V = at(w.V, lo);
        assemble(1, glo * T + j - 1, lo, n, Ac);                                              // A_{i-1,i}
        mm(OP_N, OP_N, n, ONE, g, Ac, ZERO, nullptr, X);
        mm(OP_C, OP_N, n, MONE, Ac, X, ONE, A0, A0);
        inv(n, A0, g, bb);                                                                    // g_i
        mm(OP_N, OP_N, n, ONE, R, Ac, ZERO, nullptr, RA);
        mm(OP_N, OP_N, n, MONE, RA, g, ZERO, nullptr, R);
        mm(OP_C, OP_N, n, ONE, Ac, C, ZERO, nullptr, V);
        mm(OP_N, OP_N, n, MONE, g, V, ZERO, nullptr, C);
        mm(OP_N, OP_N, n, MONE, R, V, ONE, D, D);
      }
      for (int k = 0; k < nk; ++k) {
        double2 *gam = at(w.gam[k], lo), *G11 = at(w.G11[k], lo), *G1m = at(w.G1m[k], lo);
        double2 *Bm = at(w.B, lo), *T1 = at(w.T1, lo), *Wm = at(w.W, lo), *Ac = at(w.Ac, lo), *X = at(w.X, lo);
        assemble(2 + k, glo * T + j, lo, n, Bm);                                              // Sigma_sc,i
        if (j == 0 && lo == 0) axpy(np, ONE, lead_lesser(k, 0).p, bb, Bm, bb);
        if (j == L.mlast - 1 && hi == Q) axpy(np, ONE, lead_lesser(k, 1).p, bb, at(w.B, (P - 1) * np), bb);
        if (j > 0) {
          mm(OP_C, OP_N, n, ONE, Ac, gam, ZERO, nullptr, X);                                  // A^H gam_{i-1}
          mm(OP_N, OP_N, n, ONE, X, Ac, ONE, Bm, Bm);
        }
        mm(OP_N, OP_N, n, ONE, g, Bm, ZERO, nullptr, Wm);
        mm(OP_N, OP_C, n, ONE, Wm, g, ZERO, nullptr, gam);                                    // gam_i
        if (j == 0) {
          copy(n, gam, bb, G11, bb);
          copy(n, gam, bb, G1m, bb);
        } else {
          double2* RA = at(w.RA, lo);
          mm(OP_N, OP_N, n, ONE, G1m, Ac, ZERO, nullptr, T1);                                 // T1 = G1 A
          mm(OP_N, OP_C, n, MONE, T1, g, ZERO, nullptr, G1m);
          mm(OP_N, OP_N, n, MONE, RA, gam, ONE, G1m, G1m);                                    // G1 = -T1 g^H - RA gam
          mm(OP_N, OP_C, n, ONE, T1, R, ZERO, nullptr, Wm);                                   // W = T1 R^H
          axpy(n, MONE, Wm, bb, G11, bb);
          adj_add(n, ONE, Wm, G11);
          mm(OP_N, OP_N, n, ONE, RA, gam, ZERO, nullptr, Wm);
          mm(OP_N, OP_C, n, ONE, Wm, RA, ONE, G11, G11);
        }
      }
    }
  }

  // ---------------------------------------------------------------- 2. reduced system
  void reduce() {
    const int np = L.npts, P = L.P, T = L.T, Q = L.Q;
    // top boundaries s_p = p T - 1 (p >= 1): items [np, Q)
    {
      const int q0 = np, n = Q - np;
      double2 *As = at(w.As, q0), *tmp = at(w.X, q0), *A0 = at(w.A0, q0);
      assemble(0, T - 1, q0, n, A0);                                                          // A_ss
      assemble(1, T - 1, q0, n, As);                                                          // A_{s,s+1}
      mm(OP_N, OP_N, n, ONE, As, at(w.D, q0), ZERO, nullptr, tmp);
      mm(OP_N, OP_C, n, MONE, tmp, As, ONE, A0, at(w.DS, q0));
      for (int k = 0; k < nk; ++k) {
        assemble(2 + k, T - 1, q0, n, at(w.SS[k], q0));                                       // Sigma_s
        mm(OP_N, OP_N, n, ONE, As, at(w.G11[k], q0), ZERO, nullptr, tmp);
        mm(OP_N, OP_C, n, ONE, tmp, As, ONE, at(w.SS[k], q0), at(w.SS[k], q0));
      }
    }
    // bottom boundaries e_p = p T + T - 2 (p <= P - 2): items [0, (P - 1) np)
    {
      const int n = (P - 1) * np;
      double2 *Ae = at(w.Ae, 0), *tmp = at(w.X, 0), *A0 = at(w.A0, 0);
      assemble(0, T - 2, 0, n, A0);                                                           // A_ee
      assemble(1, T - 3, 0, n, Ae);                                                           // A_{e-1,e}
      assemble(1, T - 2, 0, n, at(w.UE, 0));                                                  // A_{e,e+1}
      mm(OP_C, OP_N, n, ONE, Ae, at(w.g, 0), ZERO, nullptr, tmp);
      mm(OP_N, OP_N, n, MONE, tmp, Ae, ONE, A0, at(w.DE, 0));
      for (int k = 0; k < nk; ++k) {
        assemble(2 + k, T - 2, 0, n, at(w.SE[k], 0));                                         // Sigma_e
        mm(OP_C, OP_N, n, ONE, Ae, at(w.gam[k], 0), ZERO, nullptr, tmp);
        mm(OP_N, OP_N, n, ONE, tmp, Ae, ONE, at(w.SE[k], 0), at(w.SE[k], 0));
      }
    }
    // fill-in between the two boundaries of the middle partitions: items [np, (P - 1) np)
    if (P >= 3) {
      const int q0 = np, n = (P - 2) * np;
      double2 *As = at(w.As, q0), *Ae = at(w.Ae, q0), *tmp = at(w.X, q0);
      mm(OP_N, OP_N, n, MONE, As, at(w.R, q0), ZERO, nullptr, tmp);
      mm(OP_N, OP_N, n, ONE, tmp, Ae, ZERO, nullptr, at(w.USE, q0));                          // S_se
      mm(OP_C, OP_N, n, MONE, Ae, at(w.C, q0), ZERO, nullptr, tmp);
      mm(OP_N, OP_C, n, ONE, tmp, As, ZERO, nullptr, at(w.LES, q0));                          // S_es
      for (int k = 0; k < nk; ++k) {
        mm(OP_N, OP_N, n, ONE, As, at(w.G1m[k], q0), ZERO, nullptr, tmp);
        mm(OP_N, OP_N, n, ONE, tmp, Ae, ZERO, nullptr, at(w.SSE[k], q0));                     // Sigma_se
      }
    }
  }

  // gam = g Bm g^H
  void sandwich(double2* g, double2* Bm, double2* tmp, double2* out) {
    mm(OP_N, OP_N, L.npts, ONE, g, Bm, ZERO, nullptr, tmp);
    mm(OP_N, OP_C, L.npts, ONE, tmp, g, ZERO, nullptr, out);
  }

  void reduced_sweeps() {
    const int np = L.npts, P = L.P;
    const long bb = L.bb;
    auto slot = [&](const Blocks& x, int p) { return at(x, p * np); };
    double2 *M = at(w.U0, 0), *t = at(w.U1, 0), *Bm = at(w.U2, 0), *t2 = at(w.U3, 0);
    // left-connected, forward over e_0, s_1, e_1, ..., s_{P-1}
    copy(np, slot(w.DE, 0), bb, M, bb);
    inv(np, M, slot(w.glE, 0), bb);
    for (int k = 0; k < nk; ++k) sandwich(slot(w.glE, 0), slot(w.SE[k], 0), t, slot(w.ylE[k], 0));
    for (int p = 1; p < P && cx.ok(); ++p) {
      double2* UE = slot(w.UE, p - 1);
      mm(OP_C, OP_N, np, ONE, UE, slot(w.glE, p - 1), ZERO, nullptr, t);
      mm(OP_N, OP_N, np, MONE, t, UE, ONE, slot(w.DS, p), M);
      inv(np, M, slot(w.glS, p), bb);
      for (int k = 0; k < nk; ++k) {
        mm(OP_C, OP_N, np, ONE, UE, slot(w.ylE[k], p - 1), ZERO, nullptr, t);
        mm(OP_N, OP_N, np, ONE, t, UE, ONE, slot(w.SS[k], p), Bm);
        sandwich(slot(w.glS, p), Bm, t, slot(w.ylS[k], p));
      }
      if (p <= P - 2) {
        double2 *LE = slot(w.LES, p), *US = slot(w.USE, p);
        mm(OP_N, OP_N, np, ONE, LE, slot(w.glS, p), ZERO, nullptr, t);                        // t = L g_s
        mm(OP_N, OP_N, np, MONE, t, US, ONE, slot(w.DE, p), M);
        inv(np, M, slot(w.glE, p), bb);
        for (int k = 0; k < nk; ++k) {
          mm(OP_N, OP_N, np, ONE, LE, slot(w.ylS[k], p), ZERO, nullptr, t2);
          mm(OP_N, OP_C, np, ONE, t2, LE, ONE, slot(w.SE[k], p), Bm);                         // Sigma + L gam L^H
          mm(OP_N, OP_N, np, ONE, t, slot(w.SSE[k], p), ZERO, nullptr, t2);                   // Y = L g Sigma_se
          axpy(np, MONE, t2, bb, Bm, bb);
          adj_add(np, ONE, t2, Bm);
          sandwich(slot(w.glE, p), Bm, t2, slot(w.ylE[k], p));
        }
      }
    }
    // right-connected, backward over s_{P-1}, e_{P-2}, s_{P-2}, ..., e_0
    copy(np, slot(w.DS, P - 1), bb, M, bb);
    inv(np, M, slot(w.grS, P - 1), bb);
    for (int k = 0; k < nk; ++k) sandwich(slot(w.grS, P - 1), slot(w.SS[k], P - 1), t, slot(w.yrS[k], P - 1));
    for (int p = P - 2; p >= 0 && cx.ok(); --p) {
      double2* UE = slot(w.UE, p);
      mm(OP_N, OP_N, np, ONE, UE, slot(w.grS, p + 1), ZERO, nullptr, t);
      mm(OP_N, OP_C, np, MONE, t, UE, ONE, slot(w.DE, p), M);
      inv(np, M, slot(w.grE, p), bb);
      for (int k = 0; k < nk; ++k) {
        mm(OP_N, OP_N, np, ONE, UE, slot(w.yrS[k], p + 1), ZERO, nullptr, t);
        mm(OP_N, OP_C, np, ONE, t, UE, ONE, slot(w.SE[k], p), Bm);
        sandwich(slot(w.grE, p), Bm, t, slot(w.yrE[k], p));
      }
      if (p >= 1) {
        double2 *LE = slot(w.LES, p), *US = slot(w.USE, p);
        mm(OP_N, OP_N, np, ONE, US, slot(w.grE, p), ZERO, nullptr, t);                        // t = U g_e
        mm(OP_N, OP_N, np, MONE, t, LE, ONE, slot(w.DS, p), M);
        inv(np, M, slot(w.grS, p), bb);
        for (int k = 0; k < nk; ++k) {
          mm(OP_N, OP_N, np, ONE, US, slot(w.yrE[k], p), ZERO, nullptr, t2);
          mm(OP_N, OP_C, np, ONE, t2, US, ONE, slot(w.SS[k], p), Bm);                         // Sigma + U gam U^H
          mm(OP_N, OP_C, np, MONE, t, slot(w.SSE[k], p), ZERO, nullptr, t2);                  // Y' = -U g Sigma_se^H
          axpy(np, MONE, t2, bb, Bm, bb);
          adj_add(np, ONE, t2, Bm);
          sandwich(slot(w.grS, p), Bm, t2, slot(w.yrS[k], p));
        }
      }
    }
  }

  // ---------------------------------------------------------------- 3. partitions with boundary terms
  void boundary_terms() {
    const int np = L.npts, P = L.P;
    const int n = (P - 1) * np;
    double2* t = at(w.U0, 0);
    // top of partitions 1..P-1: A_{e,s}^H g_e A_{e,s} from the left neighbour's e (items z -> partition z/np + 1)
    mm(OP_C, OP_N, n, ONE, at(w.UE, 0), at(w.glE, 0), ZERO, nullptr, t);
    mm(OP_N, OP_N, n, ONE, t, at(w.UE, 0), ZERO, nullptr, at(w.SigTop, 0));
    for (int k = 0; k < nk; ++k) {
      mm(OP_C, OP_N, n, ONE, at(w.UE, 0), at(w.ylE[k], 0), ZERO, nullptr, t);
      mm(OP_N, OP_N, n, ONE, t, at(w.UE, 0), ZERO, nullptr, at(w.STop[k], 0));
    }
    // bottom of partitions 0..P-2: A_{e,s} g_s A_{e,s}^H from the right neighbour's s
    mm(OP_N, OP_N, n, ONE, at(w.UE, 0), at(w.grS, np), ZERO, nullptr, t);
    mm(OP_N, OP_C, n, ONE, t, at(w.UE, 0), ZERO, nullptr, at(w.SigBot, 0));
    for (int k = 0; k < nk; ++k) {
      mm(OP_N, OP_N, n, ONE, at(w.UE, 0), at(w.yrS[k], np), ZERO, nullptr, t);
      mm(OP_N, OP_C, n, ONE, t, at(w.UE, 0), ZERO, nullptr, at(w.SBot[k], 0));
    }
  }

  void partition_sweeps() {
    const int np = L.npts, P = L.P, T = L.T, Q = L.Q;
    const long bb = L.bb, sD = (long)T * bb, sU = (long)(T - 1) * bb;
    // forward: sub-device step j is block p T - 1 + j (partition 0 starts at j = 1, the last one ends at mlast)
    for (int j = 0; j < T && cx.ok(); ++j) {
      const int lo = j == 0 ? np : 0;
      const int hi = j <= L.mlast ? Q : (P - 1) * np;
      const int n = hi - lo, glo = lo / np;
      double2* A0 = at(w.U0, lo);
      assemble(0, glo * T - 1 + j, lo, n, A0);
      if (j == 1) axpy(np, MONE, w.pw.sigL.p, bb, A0, bb);                                    // left lead at block 0
      if (j == L.mlast) axpy(np, MONE, w.pw.sigR.p, bb, at(w.U0, (P - 1) * np), bb);          // right lead
      if (j == 0) axpy(Q - np, MONE, at(w.SigTop, 0), bb, at(w.U0, np), bb);
      if (j == T - 1) axpy((P - 1) * np, MONE, at(w.SigBot, 0), bb, at(w.U0, 0), bb);
      // coupled to the previous step: every item of the range except partition 0 at its first step
      const int clo = (j == 1) ? std::max(lo, np) : lo;
      const int cn = j > 0 ? hi - clo : 0, cglo = clo / np;
      double2* Ac = at(w.U1, clo);
      double2* gj = w.Gd + (long)lo * sD + (long)j * bb;
      if (cn > 0) {
        assemble(1, cglo * T - 2 + j, clo, cn, Ac);                                           // A_{i-1,i}
        double2* Xp = w.X3 + (long)clo * sU + (long)(j - 1) * bb;
        mm(OP_N, OP_N, cn, ONE, w.Gd + (long)clo * sD + (long)(j - 1) * bb, sD, Ac, bb, ZERO, nullptr, 0, Xp, sU);
        mm(OP_C, OP_N, cn, MONE, Ac, bb, Xp, sU, ONE, at(w.U0, clo), bb, at(w.U0, clo), bb);
      }
      cx.inverse(L.b, n, A0, bb, gj, sD, w.inv_scratch, info, np);
      for (int k = 0; k < nk; ++k) {
        double2* Bm = at(w.U4, lo);
        assemble(2 + k, glo * T - 1 + j, lo, n, Bm);
        if (j == 1) axpy(np, ONE, lead_lesser(k, 0).p, bb, Bm, bb);
        if (j == L.mlast) axpy(np, ONE, lead_lesser(k, 1).p, bb, at(w.U4, (P - 1) * np), bb);
        if (j == 0) axpy(Q - np, ONE, at(w.STop[k], 0), bb, at(w.U4, np), bb);
        if (j == T - 1) axpy((P - 1) * np, ONE, at(w.SBot[k], 0), bb, at(w.U4, 0), bb);
        if (cn > 0) {
          // V = A_{i,i-1} g^<_{i-1}, kept in the upper lesser block j - 1 for the backward sweep
          double2* Vp = w.Lu[k] + (long)clo * sU + (long)(j - 1) * bb;
          mm(OP_C, OP_N, cn, ONE, Ac, bb, w.Ld[k] + (long)clo * sD + (long)(j - 1) * bb, sD, ZERO, nullptr, 0, Vp,
             sU);
          mm(OP_N, OP_N, cn, ONE, Vp, sU, Ac, bb, ONE, at(w.U4, clo), bb, at(w.U4, clo), bb);
        }
        double2* t3 = at(w.U3, lo);
        mm(OP_N, OP_N, n, ONE, gj, sD, Bm, bb, ZERO, nullptr, 0, t3, bb);
        mm(OP_N, OP_C, n, ONE, t3, bb, gj, sD, ZERO, nullptr, 0, w.Ld[k] + (long)lo * sD + (long)j * bb, sD);
      }
    }
    // backward
    for (int j = T - 2; j >= 0 && cx.ok(); --j) {
      const int lo = j == 0 ? np : 0;
      const int hi = j < L.mlast ? Q : (P - 1) * np;
      const int n = hi - lo, glo = lo / np;
      double2* Ac = at(w.U1, lo);
      assemble(1, glo * T - 1 + j, lo, n, Ac);                                                 // A_{i,i+1}
      const long od = (long)lo * sD, ou = (long)lo * sU;
      double2 *gi = w.Gd + od + (long)j * bb, *Gn = w.Gd + od + (long)(j + 1) * bb;
      double2 *Xi = w.X3 + ou + (long)j * bb, *Glo = w.Gl + ou + (long)j * bb, *Gup = w.Gu + ou + (long)j * bb;
      double2* Wt = at(w.U2, lo);
      mm(OP_C, OP_N, n, ONE, Ac, bb, gi, sD, ZERO, nullptr, 0, Wt, bb);                        // W = A_{i+1,i} g_i
      mm(OP_N, OP_N, n, MONE, Gn, sD, Wt, bb, ZERO, nullptr, 0, Glo, sU);                      // G_{i+1,i}
      mm(OP_N, OP_N, n, MONE, Xi, sU, Gn, sD, ZERO, nullptr, 0, Gup, sU);                      // G_{i,i+1}
      mm(OP_N, OP_N, n, MONE, Xi, sU, Glo, sU, ONE, gi, sD, gi, sD);                           // G_ii
      for (int k = 0; k < nk; ++k) {
        double2 *gli = w.Ld[k] + od + (long)j * bb, *Lnext = w.Ld[k] + od + (long)(j + 1) * bb;
        double2* Vp = w.Lu[k] + ou + (long)j * bb;
        double2 *Z = at(w.U3, lo), *T3 = at(w.U4, lo);
        mm(OP_N, OP_N, n, ONE, Xi, sU, Lnext, sD, ZERO, nullptr, 0, Z, bb);
        mm(OP_C, OP_C, n, ONE, Vp, sU, Gn, sD, MONE, Z, bb, T3, bb);                           // G^<_{i,i+1}
        mm(OP_N, OP_N, n, MONE, Gup, sU, Vp, sU, ONE, gli, sD, gli, sD);
        mm(OP_N, OP_C, n, MONE, T3, bb, Xi, sU, ONE, gli, sD, gli, sD);                        // G^<_ii
        copy(n, T3, bb, Vp, sU);
      }
    }
  }

  // ---------------------------------------------------------------- 4. blocks between partitions
  void cross_blocks() {
    const int np = L.npts, P = L.P, T = L.T;
    const long bb = L.bb, sD = (long)T * bb;
    const int n = (P - 1) * np;
    double2 *t = at(w.U0, 0), *t2 = at(w.U1, 0);
    const double2* Gs = w.Gd + (long)np * sD;   // first block of the next partition
    mm(OP_N, OP_N, n, ONE, at(w.glE, 0), bb, at(w.UE, 0), bb, ZERO, nullptr, 0, t, bb);        // g_e A_{e,s}
    mm(OP_N, OP_N, n, MONE, t, bb, Gs, sD, ZERO, nullptr, 0, at(w.GuX, 0), bb);
    mm(OP_N, OP_C, n, ONE, Gs, sD, at(w.UE, 0), bb, ZERO, nullptr, 0, t2, bb);
    mm(OP_N, OP_N, n, MONE, t2, bb, at(w.glE, 0), bb, ZERO, nullptr, 0, at(w.GlX, 0), bb);
    for (int k = 0; k < nk; ++k) {
      const double2* Ls = w.Ld[k] + (long)np * sD;
      mm(OP_C, OP_N, n, ONE, at(w.UE, 0), bb, at(w.ylE[k], 0), bb, ZERO, nullptr, 0, t2, bb);  // V = A_{s,e} gam_e
      mm(OP_C, OP_C, n, ONE, t2, bb, Gs, sD, ZERO, nullptr, 0, at(w.LuX[k], 0), bb);
      mm(OP_N, OP_N, n, MONE, t, bb, Ls, sD, ONE, at(w.LuX[k], 0), bb, at(w.LuX[k], 0), bb);
    }
  }

  // sub-device blocks and boundary-pair blocks into the point-major outputs
  void scatter(const double2* sub, long sub_stride, int nblk_sub, const Blocks* pairs, double2* out, int nblk_out,
               bool diag) {
    if (!out || !cx.ok()) return;
    const int np = L.npts, P = L.P, T = L.T, b = L.b;
    const long bb = L.bb, ob = (long)nblk_out * bb, go = (long)T * bb;
    auto sc = [&](int q0, int n, int first, int nblk, long dst_blk) {
      if (n <= 0 || nblk <= 0) return;
      cx.chk(launch_scatter_blocks(b, n, nblk, sub + (long)q0 * sub_stride + (long)first * bb, sub_stride,
                                   out + dst_blk * bb, np, go, ob, cx.s));
    };
    const int last = diag ? L.mlast + 1 : L.mlast;   // blocks of the last partition
    sc(0, np, 1, nblk_sub - 1, 0);                                                             // partition 0
    if (P >= 3) sc(np, (P - 2) * np, 0, nblk_sub, T - 1);                                      // middle ones
    sc((P - 1) * np, np, 0, last, (long)(P - 1) * T - 1);                                       // the last one
    if (pairs) cx.chk(launch_scatter_blocks(b, (P - 1) * np, 1, pairs->p, bb, out + (long)(T - 2) * bb, np, go, ob,
                                            cx.s));
  }
};

}  // namespace

extern "C" {

size_t negf_serinv_workspace_bytes(const negf_problem* problem, int32_t partitions, int32_t greater) {
  if (check_problems(problem, 1) != NEGF_OK || problem->n_e < 1) return 0;
  Layout L;
  if (!make_layout(problem->dev.nb, problem->dev.b, problem->n_e, partitions, L)) return 0;
  Carver cv{nullptr, 0};
  carve_serinv(cv, L, greater ? 2 : 1);
  return cv.off + 256;
}

negf_status negf_serinv_lesser_greater(const negf_problem* problem, int32_t partitions, const negf_options* opt,
                                       void* GR_diag, void* GR_upper, void* GR_lower, void* GL_diag, void* GL_upper,
                                       void* GG_diag, void* GG_upper, int32_t* info, void* workspace, size_t ws_bytes,
                                       void* stream) {
  if (check_problems(problem, 1) != NEGF_OK) return NEGF_EINVAL;
  if (!GR_diag || !GR_upper || !GL_diag || !GL_upper || !info || !workspace) return NEGF_EINVAL;
  if ((GG_diag == nullptr) != (GG_upper == nullptr)) return NEGF_EINVAL;
  const void* ps[] = {GR_diag, GR_upper, GR_lower, GL_diag, GL_upper, GG_diag, GG_upper};
  for (const void* p : ps)
    if (p && !aligned16(p)) return NEGF_EINVAL;
  const negf_problem& pr = problem[0];
  if (pr.n_e == 0) return NEGF_OK;
  Layout L;
  if (!make_layout(pr.dev.nb, pr.dev.b, pr.n_e, partitions, L)) return NEGF_EINVAL;
  const int nk = GG_diag ? 2 : 1;
  if (ws_bytes < negf_serinv_workspace_bytes(problem, partitions, nk == 2)) return NEGF_EINVAL;
  Ctx cx;
  cx.s = (hipStream_t)stream;
  cx.o = get_opts(opt);
  Carver cv{align256(workspace), ws_bytes - (size_t)(align256(workspace) - (char*)workspace)};
  SerinvWs w = carve_serinv(cv, L, nk);
  if (cv.overflow) return NEGF_EINVAL;
  cx.chk(launch_fill_int(pr.n_e, info, 0, cx.s));
  // the leads of every point, as for the RGF calls
  Chunk ch;
  ch.nb = pr.dev.nb; ch.b = pr.dev.b; ch.npts = pr.n_e; ch.first_point = 0; ch.out_diag_off = 0; ch.out_off_off = 0;
  ch.segs.push_back(Seg{&pr, 0, pr.n_e, 0});
  ChunkWs cw{};
  cw.pw = w.pw;
  cw.lw = w.lw;
  leads_for_sweeps(cx, ch, cw, info, true);
  Serinv s{cx, pr, L, w, nk, info};
  s.eliminate_interiors();
  s.reduce();
  s.reduced_sweeps();
  s.boundary_terms();
  s.partition_sweeps();
  s.cross_blocks();
  const long bb = L.bb, sD = (long)L.T * bb, sU = (long)(L.T - 1) * bb;
  const int nbk = L.nb;
  s.scatter(w.Gd, sD, L.T, nullptr, (double2*)GR_diag, nbk, true);
  s.scatter(w.Gu, sU, L.T - 1, &w.GuX, (double2*)GR_upper, nbk - 1, false);
  s.scatter(w.Gl, sU, L.T - 1, &w.GlX, (double2*)GR_lower, nbk - 1, false);
  s.scatter(w.Ld[0], sD, L.T, nullptr, (double2*)GL_diag, nbk, true);
  s.scatter(w.Lu[0], sU, L.T - 1, &w.LuX[0], (double2*)GL_upper, nbk - 1, false);
  if (nk == 2) {
    s.scatter(w.Ld[1], sD, L.T, nullptr, (double2*)GG_diag, nbk, true);
    s.scatter(w.Lu[1], sU, L.T - 1, &w.LuX[1], (double2*)GG_upper, nbk - 1, false);
  }
  return to_status(cx.err);
}

}  // extern "C"
