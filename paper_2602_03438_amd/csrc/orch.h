// Host-side orchestration core shared by the C ABI entry points: options,
// workspace carving, point chunks, the launch context (batched product,
// inversion, linear-combination and assembly launches on one stream) and the
// lead decimation.  Internal to the library.
#pragma once
#include "../../include/negf.h"
#include "internal.h"

#include <algorithm>
#include <vector>

namespace negf {
namespace orch {

inline const double2 ONE = {1.0, 0.0};
inline const double2 MONE = {-1.0, 0.0};
inline const double2 ZERO = {0.0, 0.0};

struct Opts {
  double tol = 1e-14;
  int max_iter = 64;
  double accept = 1e-8;
  int batch = 0;
  int inv_nb = 16;
  int xcd = 1;
  int tile = GEMM_TILE_64;
  int tile32 = GEMM_TILE_64;
  int gauss = 0;
  int dense = 0;       // 1: coupling blocks are multiplied as dense blocks
};

inline Opts get_opts(const negf_options* o) {
  Opts r;
  if (!o) return r;
  if (o->sr_tol > 0) r.tol = o->sr_tol;
  if (o->sr_max_iter > 0) r.max_iter = o->sr_max_iter;
  if (o->sr_accept > 0) r.accept = o->sr_accept;
  if (o->batch > 0) r.batch = o->batch;
  if (o->inv_nb == 16 || o->inv_nb == 32) r.inv_nb = o->inv_nb;
  if (o->xcd_remap == 0 || o->xcd_remap == 1) r.xcd = o->xcd_remap;
  if (o->gemm_tile >= GEMM_TILE_64 && o->gemm_tile <= GEMM_TILE_LAST) r.tile = o->gemm_tile;
  if (o->gemm_tile_f32 >= GEMM_TILE_64 && o->gemm_tile_f32 <= GEMM_TILE_LAST) r.tile32 = o->gemm_tile_f32;
  if (o->cmul == 3) r.gauss = 1;
  if (o->cmul == 4) r.gauss = 0;
  if (o->dense_coupling == 1) r.dense = 1;
  return r;
}

// Bump allocator over the caller's workspace; with base == nullptr it only
// measures, which is how negf_workspace_bytes sizes the workspace.
struct Carver {
  char* base;
  size_t cap, off = 0;
  bool overflow = false;
  template <typename T>
  T* take(size_t count) {
    const size_t bytes = (count * sizeof(T) + 255) & ~(size_t)255;
    T* p = base ? (T*)(base + off) : nullptr;
    off += bytes;
    if (base && off > cap) overflow = true;
    return p;
  }
};

struct Seg {
  const negf_problem* pr;
  int e0, n, off;  // energies [e0, e0+n) of problem pr, at chunk-local point index off
};
struct Chunk {
  int nb, b, npts;
  long first_point;           // global index of the first point
  size_t out_diag_off;        // offsets (complex elements) into [points][nb][b][b] outputs
  size_t out_off_off;         // offsets into [points][nb-1][b][b] outputs
  std::vector<Seg> segs;
};

template <typename BatchOf>
std::vector<Chunk> make_chunks_by(const negf_problem* pr, int n_prob, BatchOf batch_of);

inline std::vector<Chunk> make_chunks(const negf_problem* pr, int n_prob, int batch) {
  return make_chunks_by(pr, n_prob, [batch](int, int) { return batch; });
}

template <typename BatchOf>
std::vector<Chunk> make_chunks_by(const negf_problem* pr, int n_prob, BatchOf batch_of) {
  std::vector<Chunk> out;
  long gp = 0;
  size_t od = 0, oo = 0;
  for (int q = 0; q < n_prob; ++q) {
    const int nb = pr[q].dev.nb, b = pr[q].dev.b;
    const int batch = batch_of(nb, b);
    int e = 0;
    while (e < pr[q].n_e) {
      const bool extend = !out.empty() && out.back().nb == nb && out.back().b == b &&
                          (batch <= 0 || out.back().npts < batch);
      if (!extend) {
        Chunk c;
        c.nb = nb; c.b = b; c.npts = 0; c.first_point = gp; c.out_diag_off = od; c.out_off_off = oo;
        out.push_back(c);
      }
      Chunk& c = out.back();
      const int room = batch > 0 ? batch - c.npts : pr[q].n_e - e;
      const int take = std::min(room, pr[q].n_e - e);
      c.segs.push_back(Seg{&pr[q], e, take, c.npts});
      c.npts += take;
      e += take;
      gp += take;
      od += (size_t)take * nb * b * b;
      oo += (size_t)take * (nb - 1) * b * b;
    }
  }
  return out;
}

// ------------------------------------------------------------------ buffers

struct Blocks {   // a batch of b x b blocks, item p at p * stride
  double2* p = nullptr;
  long stride = 0;
  double2* at(int i) const { return p + (long)i * stride; }
};

struct LeadWs {   // per (point, lead) pair scratch of the decimation
  Blocks d, alpha, beta, eps_s, eps, a, c, g, ag, cg, t1, t2;   // eps holds eps - eps_s in the chain
  Blocks dseed;   // d - alpha g~ beta of a seeded solve (carved only where a seed may be given)
  double *a2, *c2, *d2, *r2, *m2, *g2, *part;
  int *active, *iters, *n_active, *accepted, *closed;
  void* inv_scratch;
};

struct PointWs {   // per point persistent data of the sweeps
  Blocks sigL, sigR, gamL, gamR, slL, slR, sgL, sgR;
  double2* X;     // [npts][nb-1] blocks
  double2* Mst;   // [npts][nb] blocks (refinement only)
  Blocks T0, T1, T2, T3, T4, C0, C1;
  void* inv_scratch;
  double* dot;
  unsigned long long* cmask;   // zero-slab maps of the coupling blocks, [nb-1][b/16] (nullable)
};

inline Blocks take_blocks(Carver& cv, int b, int n) {
  Blocks r;
  r.stride = (long)b * b;
  r.p = cv.take<double2>((size_t)n * b * b);
  return r;
}

inline LeadWs carve_leads(Carver& cv, int b, int npairs, bool seeded) {
  LeadWs w;
  Blocks* all[] = {&w.d, &w.alpha, &w.beta, &w.eps_s, &w.eps, &w.a, &w.c, &w.g, &w.ag, &w.cg, &w.t1, &w.t2};
  for (Blocks* x : all) *x = take_blocks(cv, b, npairs);
  w.dseed = seeded ? take_blocks(cv, b, npairs) : Blocks{};
  w.closed = seeded ? cv.take<int>(npairs) : nullptr;
  w.a2 = cv.take<double>(npairs); w.c2 = cv.take<double>(npairs); w.d2 = cv.take<double>(npairs);
  w.r2 = cv.take<double>(npairs); w.m2 = cv.take<double>(npairs); w.g2 = cv.take<double>(npairs);
  w.part = cv.take<double>((size_t)npairs * FROB_SPLIT);
  w.active = cv.take<int>(npairs); w.iters = cv.take<int>(npairs); w.n_active = cv.take<int>(1);
  w.accepted = cv.take<int>(npairs);
  w.inv_scratch = cv.take<char>(inverse_scratch_bytes(b, npairs));
  return w;
}

enum { OPK_OBC = 0, OPK_R = 1, OPK_RL = 2, OPK_T = 3 };

// Lays out the workspace of one chunk.  Lead scratch and sweep temporaries
// live in the same region (the leads finish before the sweeps start).
struct ChunkWs {
  PointWs pw;
  LeadWs lw;
};

inline ChunkWs carve_chunk(Carver& cv, int opk, int nb, int b, int npts, negf_precision prec, int nsides) {
  ChunkWs w{};
  PointWs& p = w.pw;
  if (opk != OPK_OBC) {
    Blocks* pers[] = {&p.sigL, &p.sigR, &p.gamL, &p.gamR, &p.slL, &p.slR, &p.sgL, &p.sgR};
    for (Blocks* x : pers) *x = take_blocks(cv, b, npts);
    p.X = (opk == OPK_T) ? nullptr : cv.take<double2>((size_t)npts * (nb - 1) * b * b);
    p.Mst = (prec == NEGF_FP32_REFINE && opk != OPK_T) ? cv.take<double2>((size_t)npts * nb * b * b) : nullptr;
    p.dot = cv.take<double>(npts);
    p.cmask = (b % 64 == 0 && b <= 1024) ? cv.take<unsigned long long>((size_t)(nb - 1) * (b / 16)) : nullptr;
  }
  // shared region
  Carver sub{cv.base ? cv.base + cv.off : nullptr, cv.base ? cv.cap - std::min(cv.cap, cv.off) : 0};
  w.lw = carve_leads(sub, b, npts * nsides, opk == OPK_OBC);
  size_t lead_bytes = sub.off;
  Carver sub2{cv.base ? cv.base + cv.off : nullptr, cv.base ? cv.cap - std::min(cv.cap, cv.off) : 0};
  if (opk != OPK_OBC) {
    Blocks* tmp[] = {&p.T0, &p.T1, &p.T2, &p.T3, &p.T4, &p.C0, &p.C1};
    for (Blocks* x : tmp) *x = take_blocks(sub2, b, npts);
    p.inv_scratch = sub2.take<char>(inverse_scratch_bytes(b, npts));
  }
  const size_t region = std::max(lead_bytes, sub2.off);
  cv.take<char>(region);
  if (sub.overflow || sub2.overflow) cv.overflow = true;
  return w;
}

// ------------------------------------------------------------------ launch helpers

struct Ctx {
  hipStream_t s;
  Opts o;
  hipError_t err = hipSuccess;
  bool ok() const { return err == hipSuccess; }
  void chk(hipError_t e) { if (err == hipSuccess && e != hipSuccess) err = e; }

  // zero-slab maps of the current chunk's coupling blocks (nullptr: treat them as dense)
  const unsigned long long* cmask = nullptr;
  int cmask_words = 0;
  // map of coupling block i when it enters a product as op(B) = A_{i,i+1} (op 1)
  // or as op(A) = A_{i,i+1}^H (op 2)
  struct KMask { const unsigned long long* m; int op; };
  KMask cpl(int i, int op) const { return cmask ? KMask{cmask + (long)i * cmask_words, op} : KMask{nullptr, 0}; }

  // C = alpha op(A) op(B) + beta Cin over a batch of b x b blocks
  // skew: the product is known to be anti-Hermitian (only its upper triangle is computed).
  // Not used by the sweeps: at the conditioning of these devices the non-anti-Hermitian
  // rounding of a full product (~1e-8 relative) is what the oracle also carries, and
  // mirroring one triangle moves the result that far from it.
  // km: zero-slab map of a coupling-block operand (products skip its zero slabs)
  void gemm(Prec pr, Op oa, Op ob, int b, int batch, double2 alpha, const double2* A, long sA, const double2* B,
            long sB, double2 beta, const double2* Cin, long sCin, double2* C, long sC, const int* active = nullptr,
            bool skew = false, KMask km = KMask{nullptr, 0}) {
    if (!ok()) return;
    GemmDesc g{};
    g.M = b; g.N = b; g.K = b; g.batch = batch;
    g.opA = oa; g.opB = ob;
    g.A = MatRef{A, b, sA};
    g.B = MatRef{B, b, sB};
    g.alpha = alpha; g.beta = beta;
    g.Cin = MatRef{Cin, b, sCin};
    g.C = MatOut{C, b, sC};
    g.active = active;
    g.prec = pr;
    g.xcd_remap = o.xcd;
    g.tile = tile_for_launch(pr == PREC_F32 ? o.tile32 : o.tile, b, b, batch);
    g.prof_class = -1;
    g.gauss = pr == PREC_F64 ? o.gauss : 0;
    g.skew = skew ? 1 : 0;
    g.kmask = km.m;
    g.kmask_op = km.op;
    chk(launch_gemm(g, s));
  }
  void inverse(int b, int batch, double2* M, long sM, double2* out, long sO, void* scratch, int* info, int info_mod,
               const int* active = nullptr) {
    if (!ok()) return;
    InvDesc d{};
    d.n = b; d.batch = batch;
    d.M = M; d.ldm = b; d.sM = sM;
    d.out = out; d.ldo = b; d.sO = sO;
    d.scratch = scratch;
    d.info = info; d.info_mod = info_mod;
    d.active = active;
    d.nb = o.inv_nb;
    d.gauss = o.gauss;
    chk(launch_inverse(d, s));
  }
  void lincomb(int b, int batch, double2 c1, const double2* X, long sX, double2 c2, const double2* Y, long sY,
               double2 g, double2* out, long sOut, const int* active = nullptr) {
    if (!ok()) return;
    chk(launch_lincomb(b, batch, c1, X, sX, c2, Y, sY, g, out, sOut, active, s));
  }
  void assemble(AssembleDesc d) {
    if (!ok()) return;
    chk(launch_assemble(d, s));
  }
};

inline AssembleDesc asm_base(int b, int n, const double* energies, double2* out, long sOut) {
  AssembleDesc d{};
  d.b = b; d.batch = n; d.energies = energies;
  d.eta = 0.0; d.s_coef = 1.0;
  d.h_coef = -1.0;
  d.y_coef = -1.0; d.z_coef = -1.0;
  d.out = out; d.sOut = sOut;
  return d;
}

inline const double2* blk(const void* base, long i, int b) {
  return base ? (const double2*)base + i * (long)b * b : nullptr;
}

struct Outs {
  double2 *GRd, *GRu, *GRl, *GLd, *GLu, *GGd, *GGu;
  int* info;
  double* T;
};

// Both leads of every point of the chunk into w.pw.sigL / sigR, Gamma and (lesser) Sigma^<>.
void leads_for_sweeps(Ctx& cx, const Chunk& ch, ChunkWs& w, int* info, bool lesser);
void run_decimation(Ctx& cx, const Chunk& ch, const int* sides, int nsides, LeadWs& w, const double2* seed,
                    long seed_stride, Blocks sig_out_L, Blocks sig_out_R, int* info_pts, int* iters_out,
                    double* resid_out);
negf_status check_problems(const negf_problem* pr, int n_prob);
long count_points(const negf_problem* pr, int n_prob);
size_t workspace_for(int opk, const negf_problem* pr, int n_prob, negf_precision prec, const Opts& o);
inline bool aligned16(const void* p) { return ((uintptr_t)p & 15) == 0; }
inline char* align256(void* p) { return (char*)(((uintptr_t)p + 255) & ~(uintptr_t)255); }
inline negf_status to_status(hipError_t e) { return e == hipSuccess ? NEGF_OK : NEGF_EHIP; }

}  // namespace orch
}  // namespace negf
