// Internal launch interfaces of the NEGF library (not part of the public ABI).
#pragma once
#include "common.h"

namespace negf {

enum Op { OP_N = 0, OP_C = 1 };          // op(X) = X or X^H
// Output tile shapes of the complex product kernel (see gemm.hip)
enum { GEMM_TILE_DEFAULT = 0, GEMM_TILE_64 = 1, GEMM_TILE_128x64 = 2, GEMM_TILE_128x128 = 3, GEMM_TILE_64_8W = 4,
       GEMM_TILE_128x64_16W = 5, GEMM_TILE_32 = 6, GEMM_TILE_LAST = GEMM_TILE_32 };
enum Prec { PREC_F64 = 0, PREC_F32 = 1 };  // arithmetic of the product

// A batch of b x b (or M x K ...) complex matrices: item p starts at p * stride.
struct MatRef {
  const double2* p;
  long ld;
  long stride;
};
struct MatOut {
  double2* p;
  long ld;
  long stride;
};

// C_p = alpha * op(A_p) op(B_p) + beta * Cin_p  for every batch item p.
struct GemmDesc {
  int M, N, K, batch;
  Op opA, opB;
  MatRef A, B;
  double2 alpha, beta;
  MatRef Cin;          // read only when beta != 0; may alias C
  MatOut C;
  const int* active;   // nullable: item p is skipped when active[p] == 0
  Prec prec;
  int tile;            // 0 = default tile shape; see gemm.hip
  int xcd_remap;       // group the tiles of one batch item on one XCD
  int prof_class;      // -1: by precision
  int gauss;           // double products with three real products per complex one
  int skew;            // the result is anti-Hermitian (M == N): only tiles touching the upper
                       // triangle are computed, the strict lower triangle is then set to -conj
                       // of the upper one
  // Zero-slab map of a sparse operand T (a b x b block stored row-major, shared
  // by all items): kmask[g] bit k is set when T[16k .. 16k+15][16g .. 16g+15]
  // holds a nonzero.  kmask_op 1: op(B) = T (column group g of B); 2:
  // op(A) = T^H (row group g of op(A)).  A tile skips the K-steps in which all
  // its four groups are zero, a wave the products of its fragments that are
  // zero in a K-step: exact zeros either way.  Used by 64 x 64 tiles on
  // whole-tile sizes with K <= 1024; ignored otherwise.
  const unsigned long long* kmask;
  int kmask_op;
  // Columns [skip_lo, skip_hi) of C are computed but not stored (empty when equal).  Inversion
  // updates only (prof_class KC_INV_GEMM): there op(A) may be those very columns of C.
  int skip_lo, skip_hi;
};
hipError_t launch_gemm(const GemmDesc& d, hipStream_t s);
// The tile a library launch of batch x (M x N) outputs uses: `tile`, or 32 x 32 when 64 x 64 tiles
// would give fewer workgroups than two per CU (a few energy points per call).
int tile_for_launch(int tile, int M, int N, long batch);

// Zero-slab maps (see GemmDesc::kmask) of nblk b x b blocks T_i = x H_i + y S_i
// for any x, y: a slab is marked when H_i or S_i (nullable) has a nonzero in
// it.  out: nblk * (b / 16) words; accumulate = 1 ORs into the existing words.
// b must be a multiple of 64 and at most 1024.
hipError_t launch_slab_map(int b, int nblk, const double2* H, const double2* S, unsigned long long* out,
                           int accumulate, hipStream_t s);

// Blocked Gauss-Jordan inversion with partial pivoting of a batch of n x n
// matrices.  M is overwritten; the inverse is written to out (may not alias M).
struct InvDesc {
  int n, batch;
  double2* M;
  long ldm, sM;
  double2* out;
  long ldo, sO;
  void* scratch;        // inverse_scratch_bytes(n, batch)
  int* info;            // nullable; item p reports into info[p % info_mod]
  int info_mod;         // 0: info[p]
  const int* active;    // nullable
  int nb;               // panel width (16 or 32; 0 = default)
  int gauss;            // trailing updates with three real products per complex one
};
size_t inverse_scratch_bytes(int n, int batch);
hipError_t launch_inverse(const InvDesc& d, hipStream_t s);

// ---- element-wise and reduction kernels (elem.hip) ----
// All "blocks" are b x b interleaved complex, batch item p at base + p * stride.

// out_p = zc_p * op(S) + h_coef * op(H) + y_coef * Y + z_coef * Z_p, with
// zc_p = s_coef * (energies[p] + i * eta) and op = identity or conjugate
// transpose (applied to S and H only).  S == nullptr means identity when
// s_identity is set and zero otherwise; H, Y, Z may be null (zero).
// Y is shared by the whole batch; Z_p is per item.
struct AssembleDesc {
  int b, batch;
  const double* energies;   // device, one per item; nullptr => 0
  double eta, s_coef;
  const double2* S;
  int s_identity;
  const double2* H;
  double h_coef;
  int op;                   // 0: as stored, 1: conjugate transpose of S and H
  const double2* Y;
  double y_coef;
  const double2* Z;
  long sZ;
  double z_coef;
  double2* out;
  long sOut;
  const int* active;
  // Items in groups of `inner` (0: no grouping): item p reads energies[p % inner] and the
  // blocks S, H, Y at offset (p / inner) * sHo elements (the same block index in different
  // parts of a device, e.g. one per partition).
  int inner;
  long sHo;
  // Y of item p additionally offset by (inner > 0 ? p % inner : p) * sY elements: one block per
  // energy (energy-dependent scattering self-energies); 0 for a Y shared by every item
  long sY;
};
hipError_t launch_assemble(const AssembleDesc& d, hipStream_t s);
// out_p += c * W_p^H for b x b blocks (out must not alias W)
hipError_t launch_add_adjoint(int b, int batch, double2 c, const double2* W, long sW, double2* out, long sOut,
                              hipStream_t s);
// For item z < nitems and t < nblk: block t of dst_z = block t of src_z, with
// src_z = src + z * sS and dst_z = dst + (z / inner) * sDo + (z % inner) * sDi (elements).
hipError_t launch_scatter_blocks(int b, int nitems, int nblk, const double2* src, long sS, double2* dst, int inner,
                                 long sDo, long sDi, hipStream_t s);

// dst_p = src_p (plain copy of a batch of b x b blocks)
hipError_t launch_copy_blocks(int b, int batch, const double2* src, long sS, double2* dst, long sD, hipStream_t s);
// nrm2[p] = ||X_p - shift I||_F^2 for items with active[p] != 0 (all when active is null);
// part: scratch of batch * FROB_SPLIT doubles.
constexpr int FROB_SPLIT = 16;
hipError_t launch_frob2(int b, int batch, const double2* X, long sX, double shift, const int* active, double* part,
                        double* nrm2, hipStream_t s);
// Decimation convergence update for each item (one per (point, lead) pair).
hipError_t launch_sr_check(int batch, const double* a2, const double* c2, const double* d2, double tol, int iter,
                           int* active, int* iters, int* n_active, hipStream_t s);
// From Sigma^R_p: gamma_p = i (S - S^H), sl_p = i f_p gamma_p, sg_p = -i (1 - f_p) gamma_p,
// f_p = 1/(1+exp((E_p - mu)/kT)).  Any output may be null.
hipError_t launch_gamma_sigma(int b, int batch, const double2* sig, long sS, const double* energies, double mu,
                              double kT, double2* gamma, long sG, double2* sl, long sL, double2* sg, long sGr,
                              hipStream_t s);
// T_p = Re sum_ij P_p[i][j] conj(Q_p[i][j])
hipError_t launch_dot_re(int b, int batch, const double2* P, long sP, const double2* Q, long sQ, double* out,
                         hipStream_t s);
// SR result: resid_p = sqrt(r2) / (sqrt(m2) sqrt(g2)); info_p updated with ENOCONV when
// not converged or resid > accept; NaN -> ENONFINITE.
hipError_t launch_sr_finish(int batch, const double* r2, const double* m2, const double* g2, const int* active,
                            double accept, double* resid_out, int* info, int info_mod, hipStream_t s);
// info_p = ENONFINITE if any entry of X_p is not finite (only if info_p is OK)
hipError_t launch_check_finite(int b, int batch, const double2* X, long sX, int* info, int info_mod, hipStream_t s);
// out_p = c1 X_p + c2 Y_p + g I   (X, Y nullable; out may alias X or Y)
hipError_t launch_lincomb(int b, int batch, double2 c1, const double2* X, long sX, double2 c2, const double2* Y,
                          long sY, double2 g, double2* out, long sOut, const int* active, hipStream_t s);
hipError_t launch_fill_int(int n, int* p, int v, hipStream_t s);
// Seeded decimation: active_p = (flags_p != OK), iters_p = 0
hipError_t launch_seed_flags(int np, const int* flags, int* active, int* iters, hipStream_t s);
// g_p <- g_dec_p for every pair whose seed was rejected (flags_p != OK)
hipError_t launch_seed_select(int b, int np, const int* flags, const double2* g_dec, double2* g, hipStream_t s);
// Seeded closure of the decimation: for every active pair whose closure residual
// sqrt(r2) / (sqrt(m2) sqrt(g2)) is finite and <= accept: closed = 1, active = 0,
// iters = iter, accepted = ST_OK; closed = 0 for every other pair.
hipError_t launch_closure_accept(int np, const double* r2, const double* m2, const double* g2, double accept, int iter,
                                 int* active, int* iters, int* accepted, int* closed, hipStream_t s);

// ---- runtime helpers and profiling (prof.hip) ----
hipError_t rt_copy_d2d(void* dst, const void* src, size_t bytes, hipStream_t s);
// worker streams (default priority), fork/join events, stream capture into one graph
hipError_t rt_stream_create(hipStream_t* s);
hipError_t rt_stream_destroy(hipStream_t s);
hipError_t rt_event_create(hipEvent_t* e);
hipError_t rt_event_destroy(hipEvent_t e);
hipError_t rt_record_wait(hipEvent_t e, hipStream_t from, hipStream_t to);   // `to` waits for `from`
hipError_t rt_capture_begin(hipStream_t s);
hipError_t rt_capture_end(hipStream_t s, void** exec);
hipError_t rt_graph_launch(void* exec, hipStream_t s);
hipError_t rt_graph_destroy(void* exec);
double rt_wallclock_hz();
// *dst = device wall clock (constant-rate counter) when the stream reaches this point
hipError_t launch_stamp(unsigned long long* dst, hipStream_t s);
// point queue: one round's task intake and results for one chunk segment (slots [e0, e0 + n) of a
// problem with n_slots slots; slot_task, info and GRd start at the segment's first slot)
hipError_t launch_queue_pop(double* energies, int e0, int n, int n_slots, const double* task_E, int n_tasks,
                            int* round, int* slot_task, int* info, hipStream_t s);
hipError_t launch_queue_finish(const double2* GRd, int nb, int b, int n, const int* slot_task, const int* info,
                               int* task_info, double* task_dos, unsigned long long* task_stamp, hipStream_t s);
enum KernelClass { KC_GEMM64 = 0, KC_GEMM32 = 1, KC_INV_PANEL = 2, KC_INV_SWAP = 3, KC_INV_PERM = 4, KC_ELEM = 5,
                   KC_INV_GEMM = 6, KC_GEMM_CPL = 7, KC_COUNT = 8 };
void prof_begin(int cls, hipStream_t s);
void prof_end(int cls, hipStream_t s, double flops, double bytes);
// Device counters of executed flops of class cls (PROF_SLOTS of them, a kernel adds to
// slot (wave id) & (PROF_SLOTS - 1)); nullptr when profiling is off or a graph is being
// captured.  negf_profile_read sums them.
constexpr int PROF_SLOTS = 1024;
unsigned long long* prof_flop_slots(int cls);

}  // namespace negf
