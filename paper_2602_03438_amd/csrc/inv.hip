// Batched in-place inversion of complex n x n blocks by blocked Gauss-Jordan
// elimination with partial (row) pivoting.
//
// Block step for the panel J = [j0, j0+nb) of the current matrix A:
//   1. panel kernel (one workgroup per matrix, one thread per row, the n x nb
//      panel in registers): nb unblocked Gauss-Jordan steps restricted to the
//      panel -- pivot = the row r >= j of largest |Re a_rj| + |Im a_rj| (compared
//      to 2^-9 relative, ties to the smaller row), row interchange, scale the
//      pivot row, eliminate the column from every other row with the
//      multipliers stored in place.  The result W = [A_JJ^{-1}; -A_RJ A_JJ^{-1}]
//      (rows in pivoted order) goes to scratch and the panel columns of A are
//      cleared.  The same workgroup composes the nb interchanges into one row
//      map, applies it to the other columns of the current super-panel, copies
//      the pivot rows into U (nb x n, identity in the panel columns), clears
//      those rows, and folds the map into the row orders sigma (whole matrix)
//      and tau (since the start of the super-panel).
//   2. product: A += W U on the matrix cores (one batched complex product,
//      K = nb): pivot rows become A_JJ^{-1} A_JC, the other rows
//      A_RC - A_RJ A_JJ^{-1} A_JC, and W lands in the panel columns.
// Two levels: the panels run inside super-panels of NBO = 128 columns; the
// columns outside a super-panel are brought up to date once per super-panel
// (interchanges through tau, then one product with K = 128).
// After the last panel A holds (P A)^{-1} with (P A)[i] = A[sigma[i]]; the
// inverse A^{-1}[r][c] = (P A)^{-1}[r][sigma^{-1}[c]] is a column gather.
// Arithmetic: 8 n^3 real flops per matrix, all but O(n^2 nb) of them in the
// batched products.
#include "internal.h"

namespace negf {

namespace {

constexpr int MAX_ROWS = 1024;
constexpr int NB_MAX = 32;
constexpr int NBO = 128;   // outer block (super-panel width) of the two-level scheme

struct PanelArgs {
  int n, j0, nbw;
  int c0, c1;               // the current super-panel: columns the interchanges and U cover
  double2* A; long lda, sA;
  double2* W; long sW;      // W_p: n x NB row-major
  double2* U; long sU;      // U_p: NB x n row-major (columns c0..c1 written)
  int* sigma;               // sigma_p[i]: original row now at position i
  int* tau; long sS;        // tau_p[i]: row, at the start of the super-panel, now at position i
  int* info; int info_mod;
  const int* active;
};

// Shared state of one panel workgroup.
template <int NB>
struct PanelLds {
  unsigned red[MAX_ROWS / 64] __attribute__((aligned(16)));
  double2 srow[NB];
  double2 prow[NB];
  int spiv[NB];
  int cont[MAX_ROWS];        // cont[i]: row, at the start of the panel, whose content is now at row i
  double2 qstage[NB][NBO];   // new contents of the interchanged rows below the panel
};

// Maximum of an unsigned value over the 64 lanes of a wavefront: prefix maxima
// inside each row of 16 lanes by DPP row shifts, then the row broadcasts carry
// them to lane 63.
__device__ __forceinline__ unsigned wave_max_u32(unsigned v) {
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, false));  // row_shr:1
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, false));  // row_shr:2
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, false));  // row_shr:4
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, false));  // row_shr:8
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false));  // row_bcast:15
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false));  // row_bcast:31
  return (unsigned)__builtin_amdgcn_readlane((int)v, 63);
}

// Pivot key of row r: the upper 21 bits of the magnitude |Re| + |Im| (a
// non-negative double orders like its bit pattern; a NaN ranks above
// everything so that it is taken and reported) and 2047 - r in the low 11
// bits, so that the unsigned maximum picks the largest magnitude (to 2^-9
// relative) and, among equal keys, the smallest row.
__device__ __forceinline__ unsigned pivot_key(double2 v, int r) {
  const double m = fabs(v.x) + fabs(v.y);
  const unsigned hi = (unsigned)((unsigned long long)__double_as_longlong(m) >> 32);
  return ((m != m) ? 0xFFFFF800u : (hi & 0xFFFFF800u)) | (unsigned)(2047 - r);
}

// One Gauss-Jordan step of the panel, for column j = j0 + jj.  The panel row
// is kept rotated so that the column being eliminated is always x[0]: all
// register indices are compile-time constants while the step loop stays a
// real loop (unrolled steps make a kernel whose straight-line code no longer
// fits the instruction cache, and its fetches then dominate the panel time).
// After step jj, x[c] holds panel column (jj + 1 + c) mod NB.  The pivot row
// in LDS uses the same rotated order.  Two barriers: after the pivot
// reduction, and after the pivot row (scaled by its owner) and the displaced
// row j are published.  PB: pivot-row elements held in registers at a time.
template <int NB, int PB>
__device__ __forceinline__ void panel_step(double2 (&x)[NB], PanelLds<NB>& L, int r, int j, int jj, bool valid,
                                           int& status) {
  const int lane = r & 63, wave = r >> 6;
  unsigned key = (valid && r >= j) ? pivot_key(x[0], r) : 0u;
  key = wave_max_u32(key);
  if (lane == 0) L.red[wave] = key;
  __syncthreads();
  {
    const uint4* rv = reinterpret_cast<const uint4*>(L.red);
#pragma unroll
    for (int q = 0; q < MAX_ROWS / 256; ++q) {
      const uint4 t = rv[q];
      key = max(max(key, t.x), max(t.y, max(t.z, t.w)));
    }
  }
  const int pr = 2047 - (int)(key & 0x7FFu);
  if (r == pr) {
    const double2 d = x[0];
    if (d.x == 0.0 && d.y == 0.0) status = ST_ESINGULAR;
    const double2 dinv = cinv(d);
    if (!(isfinite(dinv.x) && isfinite(dinv.y))) status = status == ST_OK ? ST_ENONFINITE : status;
    L.prow[0] = dinv;
#pragma unroll
    for (int c = 1; c < NB; ++c) L.prow[c] = cmul(x[c], dinv);
  }
  if (r == j) {
    if (pr != j) {
#pragma unroll
      for (int c = 0; c < NB; ++c) L.srow[c] = x[c];
      const int t = L.cont[j];
      L.cont[j] = L.cont[pr];
      L.cont[pr] = t;
    }
    L.spiv[jj] = pr;
  }
  __syncthreads();
  if (r == j) {
#pragma unroll
    for (int c = 0; c < NB; ++c) x[c] = L.prow[c];
  } else if (valid) {
    if (r == pr) {
#pragma unroll
      for (int c = 0; c < NB; ++c) x[c] = L.srow[c];
    }
    // eliminate column j (multiplier stored in place: x[0] becomes -f / pivot)
    const double2 f = x[0];
    x[0] = make_double2(0.0, 0.0);
#pragma unroll
    for (int c = 0; c < NB; ++c) {
      const double2 pc = L.prow[c];
      x[c].x -= f.x * pc.x - f.y * pc.y;
      x[c].y -= f.x * pc.y + f.y * pc.x;
      if ((c % PB) == PB - 1) __builtin_amdgcn_sched_barrier(0);
    }
  }
  // rotate: the next column moves to x[0]
  const double2 t0 = x[0];
#pragma unroll
  for (int c = 0; c + 1 < NB; ++c) x[c] = x[c + 1];
  x[NB - 1] = t0;
}

template <int NB, int MAXT>
__global__ void __launch_bounds__(MAXT) gj_panel_kernel(PanelArgs a) {
  const int p = blockIdx.x;
  if (a.active && a.active[p] == 0) return;
  double2* __restrict__ A = a.A + (long)p * a.sA;
  double2* __restrict__ W = a.W + (long)p * a.sW;
  double2* __restrict__ U = a.U + (long)p * a.sU;
  int* __restrict__ sigma = a.sigma + (long)p * a.sS;
  int* __restrict__ tau = a.tau + (long)p * a.sS;
  const int r = threadIdx.x;
  const int nt = blockDim.x;
  const int n = a.n, j0 = a.j0, nbw = a.nbw;
  const int jend = j0 + nbw;
  const bool valid = r < n;
  __shared__ PanelLds<NB> L;
  if (r < MAX_ROWS / 64) L.red[r] = 0u;   // waves beyond the last never write their slot
  for (int i = r; i < n; i += nt) L.cont[i] = i;

  double2 x[NB];
#pragma unroll
  for (int c = 0; c < NB; ++c)
    x[c] = (valid && c < nbw) ? A[(long)r * a.lda + j0 + c] : make_double2(0.0, 0.0);

  int status = ST_OK;
  constexpr int PB = (NB > 16 || MAXT > 512) ? 4 : 8;
#pragma unroll 1
  for (int jj = 0; jj < nbw; ++jj) panel_step<NB, PB>(x, L, r, j0 + jj, jj, valid, status);

  if (valid) {
    // after nbw rotations x[c] holds panel column (c + nbw) mod NB
#pragma unroll
    for (int c = 0; c < NB; ++c) W[(long)r * NB + (c + nbw) % NB] = x[c];
#pragma unroll
    for (int c = 0; c < NB; ++c)
      if (c < nbw) A[(long)r * a.lda + j0 + c] = make_double2(0.0, 0.0);
  }
  __syncthreads();

  // The nbw interchanges, composed into cont[], act on the rows D = panel rows
  // and the rows below the panel they touched.  Every new row of D is an old
  // row of D, so all reads go first (pivot rows into U, moved rows into LDS),
  // then, after a barrier, the writes.
  const int c0 = a.c0, cnt = a.c1 - a.c0;
  const int tot = nbw * cnt;
  const v2d* __restrict__ Av = reinterpret_cast<const v2d*>(A);
  constexpr int G = (NB > 16 || MAXT > 512) ? 4 : 8;   // loads in flight per thread (register budget)
  for (int base = 0; base < tot; base += G * nt) {
    v2d v[G];
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int e = base + g * nt + r;
      const int s = e / cnt, c = c0 + e % cnt;
      const bool outside = c < j0 || c >= jend;
      v[g] = (e < tot && outside) ? Av[(long)L.cont[j0 + s] * a.lda + c]
                                  : v2d{(e < tot && c - j0 == s) ? 1.0 : 0.0, 0.0};
    }
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int e = base + g * nt + r;
      if (e < tot) reinterpret_cast<v2d*>(U)[(long)(e / cnt) * n + c0 + e % cnt] = v[g];
    }
  }
  for (int base = 0; base < tot; base += G * nt) {
    v2d v[G];
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int e = base + g * nt + r;
      const int s = e / cnt, c = c0 + e % cnt, q = e < tot ? L.spiv[s] : 0;
      const bool take = e < tot && q >= jend && (c < j0 || c >= jend);
      v[g] = take ? Av[(long)L.cont[q] * a.lda + c] : v2d{0.0, 0.0};
    }
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int e = base + g * nt + r;
      const int s = e / cnt, c = c0 + e % cnt, q = e < tot ? L.spiv[s] : 0;
      if (e < tot && q >= jend && (c < j0 || c >= jend)) {
        L.qstage[s][c - c0].x = v[g].x;
        L.qstage[s][c - c0].y = v[g].y;
      }
    }
  }
  // row orders: new entry of a row d of D = old entry of row cont[d]
  int d = -1, sv = 0, tv = 0;
  if (r < 2 * nbw) {
    d = r < nbw ? j0 + r : L.spiv[r - nbw];
    if (r >= nbw && d < jend) d = -1;
    if (d >= 0) {
      const int src = L.cont[d];
      sv = j0 == 0 ? src : sigma[src];
      tv = j0 == c0 ? src : tau[src];
    }
  }
  __syncthreads();
  for (int e = r; e < tot; e += nt) {
    const int s = e / cnt, c = c0 + e % cnt;
    if (c >= j0 && c < jend) continue;
    A[(long)(j0 + s) * a.lda + c] = make_double2(0.0, 0.0);
    const int q = L.spiv[s];
    if (q >= jend) A[(long)q * a.lda + c] = L.qstage[s][c - c0];
  }
  if (j0 == 0) {
    for (int i = r; i < n; i += nt) sigma[i] = L.cont[i];
  } else if (d >= 0) {
    sigma[d] = sv;
  }
  if (j0 == c0) {
    for (int i = r; i < n; i += nt) tau[i] = L.cont[i];
  } else if (d >= 0) {
    tau[d] = tv;
  }
  if (status != ST_OK && a.info) atomicCAS(a.info + (a.info_mod > 0 ? p % a.info_mod : p), ST_OK, status);
}

// out[r][c] = X[r][sigma^{-1}[c]]; one workgroup per (matrix, GATHER_ROWS rows)
constexpr int GATHER_ROWS = 16;

__global__ void __launch_bounds__(256) gj_gather_kernel(int n, const double2* M, long ldm, long sM, double2* out,
                                                        long ldo, long sO, const int* sigma, long sS,
                                                        const int* active) {
  const int p = blockIdx.y;
  if (active && active[p] == 0) return;
  __shared__ int inv[MAX_ROWS];
  const int* sg = sigma + (long)p * sS;
  for (int i = threadIdx.x; i < n; i += blockDim.x) inv[sg[i]] = i;
  __syncthreads();
  const int r0 = blockIdx.x * GATHER_ROWS;
  const double2* Mp = M + (long)p * sM;
  double2* Op = out + (long)p * sO;
  for (int e = threadIdx.x; e < GATHER_ROWS * n; e += blockDim.x) {
    const int rr = r0 + e / n, c = e % n;
    if (rr < n) Op[(long)rr * ldo + c] = Mp[(long)rr * ldm + inv[c]];
  }
}

// Outer step of the two-level blocking for the super-panel J = [J0, J0+mo),
// one workgroup per (matrix, OUTER_COLS columns).  Blocks inside J move their
// columns into Wo (n x mo) and clear them, and write the identity into Uo.
// Blocks outside J apply the super-panel's interchanges (the content map tau)
// to their columns: the pivot rows J0..J0+mo-1 go to Uo (mo x n) and are
// cleared, the rows below J that took part receive their new contents.  All
// reads of a block precede its writes (a barrier between).
constexpr int OUTER_COLS = 16;
constexpr int OUTER_THREADS = 256;

__global__ void __launch_bounds__(OUTER_THREADS) gj_outer_kernel(int n, int J0, int mo, double2* A, long lda,
                                                                 long sA, double2* Wo, long sW, double2* Uo,
                                                                 long sU, const int* tau, long sT,
                                                                 const int* active) {
  const int p = blockIdx.y;
  if (active && active[p] == 0) return;
  double2* __restrict__ Ap = A + (long)p * sA;
  double2* __restrict__ U = Uo + (long)p * sU;
  const int cb = blockIdx.x * OUTER_COLS;
  const int w = min(OUTER_COLS, n - cb);
  const int t = threadIdx.x;
  if (cb >= J0 && cb < J0 + mo) {
    double2* __restrict__ Wp = Wo + (long)p * sW;
    for (int e = t; e < n * OUTER_COLS; e += OUTER_THREADS) {
      const int rr = e / OUTER_COLS, cc = e % OUTER_COLS;
      if (cc >= w) continue;
      const long o = (long)rr * lda + cb + cc;
      Wp[(long)rr * mo + (cb - J0 + cc)] = Ap[o];
      Ap[o] = make_double2(0.0, 0.0);
    }
    for (int e = t; e < mo * OUTER_COLS; e += OUTER_THREADS) {
      const int k = e / OUTER_COLS, cc = e % OUTER_COLS;
      if (cc < w) U[(long)k * n + cb + cc] = make_double2(k == cb - J0 + cc ? 1.0 : 0.0, 0.0);
    }
    return;
  }
  __shared__ int rows[2 * NBO];
  __shared__ int srcs[2 * NBO];
  __shared__ int nq;
  const int* tp = tau + (long)p * sT;
  if (t == 0) nq = 0;
  __syncthreads();
  for (int i = t; i < mo; i += OUTER_THREADS) {
    rows[i] = J0 + i;
    srcs[i] = tp[J0 + i];
  }
  // rows below J whose content changed (at most mo of them)
  for (int i = J0 + mo + t; i < n; i += OUTER_THREADS) {
    const int s = tp[i];
    if (s != i) {
      const int k = atomicAdd(&nq, 1);
      if (mo + k < 2 * NBO) {
        rows[mo + k] = i;
        srcs[mo + k] = s;
      }
    }
  }
  __syncthreads();
  const int tot = min(mo + nq, 2 * NBO) * OUTER_COLS;
  constexpr int G = 2 * NBO * OUTER_COLS / OUTER_THREADS;
  const v2d* __restrict__ Av = reinterpret_cast<const v2d*>(Ap);
  v2d v[G];
#pragma unroll
  for (int g = 0; g < G; ++g) {
    const int e = g * OUTER_THREADS + t, k = e / OUTER_COLS, cc = e % OUTER_COLS;
    v[g] = (e < tot && cc < w) ? Av[(long)srcs[k] * lda + cb + cc] : v2d{0.0, 0.0};
  }
  __syncthreads();
  v2d* __restrict__ Aw = reinterpret_cast<v2d*>(Ap);
#pragma unroll
  for (int g = 0; g < G; ++g) {
    const int e = g * OUTER_THREADS + t, k = e / OUTER_COLS, cc = e % OUTER_COLS;
    if (e < tot && cc < w) {
      if (k < mo) {
        reinterpret_cast<v2d*>(U)[(long)k * n + cb + cc] = v[g];
        Aw[(long)(J0 + k) * lda + cb + cc] = v2d{0.0, 0.0};
      } else {
        Aw[(long)rows[k] * lda + cb + cc] = v[g];
      }
    }
  }
}

struct ScratchLayout {
  size_t per_al;
  size_t off_W, off_U, off_Wo, off_Uo, off_sigma, off_tau;
};

ScratchLayout layout(int n) {
  ScratchLayout L{};
  size_t o = 0;
  L.off_W = o;  o += (size_t)n * NB_MAX * sizeof(double2);
  L.off_U = o;  o += (size_t)NB_MAX * n * sizeof(double2);
  L.off_Wo = o; o += (size_t)n * NBO * sizeof(double2);
  L.off_Uo = o; o += (size_t)NBO * n * sizeof(double2);
  L.off_sigma = o; o += (size_t)n * sizeof(int);
  L.off_tau = o;   o += (size_t)n * sizeof(int);
  L.per_al = (o + 255) & ~(size_t)255;
  return L;
}

GemmDesc update_desc(int M, int N, int K, const double2* Wm, long ldw, long sW, const double2* Um, long ldu, long sU,
                     double2* C, long ldc, long sC, int batch, const int* active, int gauss) {
  GemmDesc g{};
  g.M = M; g.N = N; g.K = K; g.batch = batch;
  g.opA = OP_N; g.opB = OP_N;
  g.A = MatRef{Wm, ldw, sW};
  g.B = MatRef{Um, ldu, sU};
  g.alpha = make_double2(1.0, 0.0);
  g.beta = make_double2(1.0, 0.0);
  g.Cin = MatRef{C, ldc, sC};
  g.C = MatOut{C, ldc, sC};
  g.active = active;
  g.prec = PREC_F64;
  g.xcd_remap = 1;
  g.tile = GEMM_TILE_64;
  g.prof_class = KC_INV_GEMM;
  g.gauss = gauss;
  return g;
}

}  // namespace

size_t inverse_scratch_bytes(int n, int batch) { return layout(n).per_al * batch; }

hipError_t launch_inverse(const InvDesc& d, hipStream_t s) {
  const int n = d.n;
  if (n <= 0 || d.batch <= 0) return hipSuccess;
  if (n > MAX_ROWS) return hipErrorInvalidValue;
  const int NB = (d.nb == 32 && n <= 512) ? 32 : 16;
  const ScratchLayout SL = layout(n);
  const long sItem = (long)(SL.per_al / sizeof(double2));   // per_al is a multiple of 256 bytes
  const long sI = (long)(SL.per_al / sizeof(int));
  char* base = (char*)d.scratch;
  double2* W = (double2*)(base + SL.off_W);
  double2* U = (double2*)(base + SL.off_U);
  double2* Wo = (double2*)(base + SL.off_Wo);
  double2* Uo = (double2*)(base + SL.off_Uo);
  int* sigma = (int*)(base + SL.off_sigma);
  int* tau = (int*)(base + SL.off_tau);
  const int nthr = ((n + 63) / 64) * 64;
  // two levels when the matrix is wider than one super-panel
  const int outer = n > NBO ? NBO : n;
  hipError_t e = hipSuccess;
  for (int J0 = 0; J0 < n; J0 += outer) {
    const int mo = (n - J0 < outer) ? n - J0 : outer;
    for (int j0 = J0; j0 < J0 + mo; j0 += NB) {
      const int nbw = (J0 + mo - j0 < NB) ? J0 + mo - j0 : NB;
      PanelArgs pa{n, j0, nbw, J0, J0 + mo, d.M, d.ldm, d.sM, W, sItem, U, sItem, sigma, tau, sI,
                   d.info, d.info_mod, d.active};
      prof_begin(KC_INV_PANEL, s);
      if (NB == 32) hipLaunchKernelGGL((gj_panel_kernel<32, 512>), dim3(d.batch), dim3(nthr), 0, s, pa);
      else if (n <= 512) hipLaunchKernelGGL((gj_panel_kernel<16, 512>), dim3(d.batch), dim3(nthr), 0, s, pa);
      else hipLaunchKernelGGL((gj_panel_kernel<16, MAX_ROWS>), dim3(d.batch), dim3(nthr), 0, s, pa);
      prof_end(KC_INV_PANEL, s, 8.0 * n * NB * NB * d.batch, 0);
      if ((e = hipGetLastError()) != hipSuccess) return e;
      // update of the super-panel columns: A[:, J] += W U[:, J]
      GemmDesc g = update_desc(n, mo, nbw, W, NB, sItem, U + J0, n, sItem, d.M + J0, d.ldm, d.sM, d.batch, d.active,
                               d.gauss);
      if ((e = launch_gemm(g, s)) != hipSuccess) return e;
    }
    if (mo == n) break;   // one level: the super-panel was the whole matrix
    // outer step: interchanges and pivot rows of the other columns, then A += Wo Uo
    prof_begin(KC_INV_SWAP, s);
    hipLaunchKernelGGL(gj_outer_kernel, dim3((n + OUTER_COLS - 1) / OUTER_COLS, d.batch), dim3(OUTER_THREADS), 0, s,
                       n, J0, mo, d.M, d.ldm, d.sM, Wo, sItem, Uo, sItem, tau, sI, d.active);
    prof_end(KC_INV_SWAP, s, 0, 0);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    GemmDesc g =
        update_desc(n, n, mo, Wo, mo, sItem, Uo, n, sItem, d.M, d.ldm, d.sM, d.batch, d.active, d.gauss);
    if ((e = launch_gemm(g, s)) != hipSuccess) return e;
  }
  prof_begin(KC_INV_PERM, s);
  hipLaunchKernelGGL(gj_gather_kernel, dim3((n + GATHER_ROWS - 1) / GATHER_ROWS, d.batch), dim3(256), 0, s, n, d.M,
                     d.ldm, d.sM, d.out, d.ldo, d.sO, sigma, sI, d.active);
  prof_end(KC_INV_PERM, s, 0, 32.0 * n * n * d.batch);
  return hipGetLastError();
}

}  // namespace negf
