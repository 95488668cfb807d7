// Batched in-place inversion of complex n x n blocks by blocked Gauss-Jordan
// elimination with partial (row) pivoting.
//
// Block step for the panel J = [j0, j0+nb) of the current matrix A:
//   1. panel kernel (one workgroup per matrix, one thread per row, the n x nb
//      panel in registers): nb unblocked Gauss-Jordan steps restricted to the
//      panel -- pivot = argmax_{r >= j} |Re a_rj| + |Im a_rj|, row interchange,
//      scale the pivot row, eliminate the column from every other row with the
//      multipliers stored in place.  The result W = [A_JJ^{-1}; -A_RJ A_JJ^{-1}]
//      (rows in pivoted order) goes to scratch and the panel columns of A are
//      cleared.  The same workgroup then applies the nb interchanges to the
//      other columns, copies the pivot rows into U (nb x n, identity in the
//      panel columns), clears those rows, and appends the interchanges to the
//      row-order array sigma.
//   2. product: A += W U on the matrix cores (one batched complex product,
//      K = nb): pivot rows become A_JJ^{-1} A_JC, the other rows
//      A_RC - A_RJ A_JJ^{-1} A_JC, and W lands in the panel columns.
// After the last panel A holds (P A)^{-1} with (P A)[i] = A[sigma[i]]; the
// inverse A^{-1}[r][c] = (P A)^{-1}[r][sigma^{-1}[c]] is a column gather.
// Arithmetic: 8 n^3 real flops per matrix, all but O(n^2 nb) of them in the
// batched products.
#include "internal.h"

namespace negf {

namespace {

constexpr int MAX_ROWS = 1024;
constexpr int NB_MAX = 32;

struct PanelArgs {
  int n, j0, nbw;
  int c0, c1;               // columns the interchanges and U cover (the current super-panel)
  double2* A; long lda, sA;
  double2* W; long sW;      // W_p: n x NB row-major
  double2* U; long sU;      // U_p: NB x n row-major (columns c0..c1 written)
  int* sigma; long sS;      // sigma_p[i]: original row now at position i
  int* piv;                 // piv_p[j]: row interchanged with row j (same stride as sigma)
  int* info; int info_mod;
  const int* active;
};

// Shared state of one panel workgroup.
template <int NB>
struct PanelLds {
  double red_key[MAX_ROWS / 64];
  int red_idx[MAX_ROWS / 64];
  double2 srow[2][NB];
  double2 prow[NB];
  int spiv[NB];
};

// Gauss-Jordan step JJ of the panel.  JJ is a compile-time index so that the
// panel row x[] stays in registers (a runtime index would move it to scratch).
template <int JJ, int NB>
__device__ __forceinline__ void panel_step(double2 (&x)[NB], PanelLds<NB>& L, int r, int n, int j0, bool valid,
                                           int nwaves, int& status) {
  const int lane = r & 63, wave = r >> 6;
  const int j = j0 + JJ;
  // --- pivot search over rows r >= j (ties -> smallest row index)
  double key = (valid && r >= j) ? fabs(x[JJ].x) + fabs(x[JJ].y) : -1.0;
  if (key != key) key = 1e308;  // a NaN candidate is taken and reported below
  int idx = r;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const double k2 = __shfl_xor(key, off);
    const int i2 = __shfl_xor(idx, off);
    if (k2 > key || (k2 == key && i2 < idx)) { key = k2; idx = i2; }
  }
  if (lane == 0) { L.red_key[wave] = key; L.red_idx[wave] = idx; }
  __syncthreads();
  key = L.red_key[0];
  idx = L.red_idx[0];
  for (int w = 1; w < nwaves; ++w) {
    const double k2 = L.red_key[w];
    const int i2 = L.red_idx[w];
    if (k2 > key || (k2 == key && i2 < idx)) { key = k2; idx = i2; }
  }
  const int pr = idx;
  // --- interchange rows j and pr of the panel
  if (pr != j) {
    if (r == j) {
#pragma unroll
      for (int c = 0; c < NB; ++c) L.srow[0][c] = x[c];
    }
    if (r == pr) {
#pragma unroll
      for (int c = 0; c < NB; ++c) L.srow[1][c] = x[c];
    }
    __syncthreads();
    if (r == j) {
#pragma unroll
      for (int c = 0; c < NB; ++c) x[c] = L.srow[1][c];
    }
    if (r == pr) {
#pragma unroll
      for (int c = 0; c < NB; ++c) x[c] = L.srow[0][c];
    }
  }
  // --- scale the pivot row and publish it
  if (r == j) {
    const double2 d = x[JJ];
    if (d.x == 0.0 && d.y == 0.0) status = ST_ESINGULAR;
    const double2 dinv = cinv(d);
    if (!(isfinite(dinv.x) && isfinite(dinv.y))) status = status == ST_OK ? ST_ENONFINITE : status;
#pragma unroll
    for (int c = 0; c < NB; ++c) x[c] = (c == JJ) ? dinv : cmul(x[c], dinv);
#pragma unroll
    for (int c = 0; c < NB; ++c) L.prow[c] = x[c];
    L.spiv[JJ] = pr;
  }
  __syncthreads();
  // --- eliminate column JJ from every other row (multiplier stored in place)
  if (valid && r != j) {
    const double2 f = x[JJ];
    x[JJ] = make_double2(0.0, 0.0);
#pragma unroll
    for (int c = 0; c < NB; ++c) {
      const double2 pc = L.prow[c];
      x[c].x -= f.x * pc.x - f.y * pc.y;
      x[c].y -= f.x * pc.y + f.y * pc.x;
      // keep the pivot row streaming through a few registers instead of all at once
      if ((c & 7) == 7) __builtin_amdgcn_sched_barrier(0);
    }
  }
}

template <int JJ, int NB>
struct PanelSteps {
  __device__ __forceinline__ static void run(double2 (&x)[NB], PanelLds<NB>& L, int r, int n, int j0, int nbw,
                                             bool valid, int nwaves, int& status) {
    if (JJ < nbw) {
      panel_step<JJ, NB>(x, L, r, n, j0, valid, nwaves, status);
      PanelSteps<JJ + 1, NB>::run(x, L, r, n, j0, nbw, valid, nwaves, status);
    }
  }
};
template <int NB>
struct PanelSteps<NB, NB> {
  __device__ __forceinline__ static void run(double2 (&)[NB], PanelLds<NB>&, int, int, int, int, bool, int, int&) {}
};

template <int NB, int MAXT>
__global__ void __launch_bounds__(MAXT) gj_panel_kernel(PanelArgs a) {
  const int p = blockIdx.x;
  if (a.active && a.active[p] == 0) return;
  double2* __restrict__ A = a.A + (long)p * a.sA;
  double2* __restrict__ W = a.W + (long)p * a.sW;
  double2* __restrict__ U = a.U + (long)p * a.sU;
  int* __restrict__ sigma = a.sigma + (long)p * a.sS;
  const int r = threadIdx.x;
  const int n = a.n, j0 = a.j0, nbw = a.nbw;
  const bool valid = r < n;
  const int nwaves = (blockDim.x + 63) >> 6;
  __shared__ PanelLds<NB> L;

  double2 x[NB];
#pragma unroll
  for (int c = 0; c < NB; ++c)
    x[c] = (valid && c < nbw) ? A[(long)r * a.lda + j0 + c] : make_double2(0.0, 0.0);

  int status = ST_OK;
  PanelSteps<0, NB>::run(x, L, r, n, j0, nbw, valid, nwaves, status);

  if (valid) {
#pragma unroll
    for (int c = 0; c < NB; ++c) W[(long)r * NB + c] = x[c];
#pragma unroll
    for (int c = 0; c < NB; ++c)
      if (c < nbw) A[(long)r * a.lda + j0 + c] = make_double2(0.0, 0.0);
  }
  __syncthreads();
  // --- interchanges on the other columns of [c0, c1), pivot rows into U (identity in the panel columns)
  for (int c = a.c0 + r; c < a.c1; c += blockDim.x) {
    if (c >= j0 && c < j0 + nbw) {
      for (int k = 0; k < nbw; ++k) U[(long)k * n + c] = make_double2(k == c - j0 ? 1.0 : 0.0, 0.0);
      continue;
    }
    for (int k = 0; k < nbw; ++k) {
      const int jr = j0 + k, q = L.spiv[k];
      if (q != jr) {
        const double2 t0 = A[(long)jr * a.lda + c];
        A[(long)jr * a.lda + c] = A[(long)q * a.lda + c];
        A[(long)q * a.lda + c] = t0;
      }
    }
    for (int k = 0; k < nbw; ++k) {
      const long o = (long)(j0 + k) * a.lda + c;
      U[(long)k * n + c] = A[o];
      A[o] = make_double2(0.0, 0.0);
    }
  }
  // --- row order: sigma starts as the identity and takes the interchanges in order
  if (j0 == 0)
    for (int i = r; i < n; i += blockDim.x) sigma[i] = i;
  __syncthreads();
  if (r == 0)
    for (int k = 0; k < nbw; ++k) {
      const int jr = j0 + k, q = L.spiv[k];
      const int t = sigma[jr];
      sigma[jr] = sigma[q];
      sigma[q] = t;
    }
  if (r < nbw) a.piv[(long)p * a.sS + j0 + r] = L.spiv[r];
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

// Outer step of the two-level blocking, for the super-panel J = [J0, J0+mo):
// the mo interchanges recorded by the inner panels are applied to the columns
// outside J, the pivot rows of those columns move into Uo (mo x n, identity in
// the columns of J) and are cleared.  One thread per column.
__global__ void __launch_bounds__(256) gj_outer_swap_kernel(int n, int J0, int mo, double2* A, long lda, long sA,
                                                            double2* Uo, long sU, const int* piv, long sP,
                                                            const int* active) {
  const int p = blockIdx.y;
  if (active && active[p] == 0) return;
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  double2* Ap = A + (long)p * sA;
  double2* U = Uo + (long)p * sU;
  const int* pv = piv + (long)p * sP;
  if (c >= J0 && c < J0 + mo) {
    for (int k = 0; k < mo; ++k) U[(long)k * n + c] = make_double2(k == c - J0 ? 1.0 : 0.0, 0.0);
    return;
  }
  for (int k = 0; k < mo; ++k) {
    const int jr = J0 + k, q = pv[jr];
    if (q != jr) {
      const double2 t0 = Ap[(long)jr * lda + c];
      Ap[(long)jr * lda + c] = Ap[(long)q * lda + c];
      Ap[(long)q * lda + c] = t0;
    }
  }
  for (int k = 0; k < mo; ++k) {
    const long o = (long)(J0 + k) * lda + c;
    U[(long)k * n + c] = Ap[o];
    Ap[o] = make_double2(0.0, 0.0);
  }
}

// Wo (n x mo) <- columns [J0, J0+mo) of A, which are then cleared.
__global__ void __launch_bounds__(256) gj_take_panel_kernel(int n, int J0, int mo, double2* A, long lda, long sA,
                                                            double2* Wo, long sW, const int* active) {
  const int p = blockIdx.y;
  if (active && active[p] == 0) return;
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)n * mo) return;
  const int r = (int)(e / mo), c = (int)(e % mo);
  double2* Ap = A + (long)p * sA;
  Wo[(long)p * sW + e] = Ap[(long)r * lda + J0 + c];
  Ap[(long)r * lda + J0 + c] = make_double2(0.0, 0.0);
}

constexpr int NBO = 128;   // outer block of the two-level scheme

struct ScratchLayout {
  size_t per_al;
  size_t off_W, off_U, off_Wo, off_Uo, off_sigma, off_piv;
};

ScratchLayout layout(int n) {
  ScratchLayout L{};
  size_t o = 0;
  L.off_W = o;  o += (size_t)n * NB_MAX * sizeof(double2);
  L.off_U = o;  o += (size_t)NB_MAX * n * sizeof(double2);
  L.off_Wo = o; o += (size_t)n * NBO * sizeof(double2);
  L.off_Uo = o; o += (size_t)NBO * n * sizeof(double2);
  L.off_sigma = o; o += (size_t)n * sizeof(int);
  L.off_piv = o;   o += (size_t)n * sizeof(int);
  L.per_al = (o + 255) & ~(size_t)255;
  return L;
}

GemmDesc update_desc(int M, int N, int K, const double2* Wm, long ldw, long sW, const double2* Um, long ldu, long sU,
                     double2* C, long ldc, long sC, int batch, const int* active) {
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
  int* piv = (int*)(base + SL.off_piv);
  const int nthr = ((n + 63) / 64) * 64;
  // two levels when the matrix is wider than one super-panel
  const int outer = n > NBO ? NBO : n;
  hipError_t e = hipSuccess;
  for (int J0 = 0; J0 < n; J0 += outer) {
    const int mo = (n - J0 < outer) ? n - J0 : outer;
    for (int j0 = J0; j0 < J0 + mo; j0 += NB) {
      const int nbw = (J0 + mo - j0 < NB) ? J0 + mo - j0 : NB;
      PanelArgs pa{n, j0, nbw, J0, J0 + mo, d.M, d.ldm, d.sM, W, sItem, U, sItem, sigma, sI, piv,
                   d.info, d.info_mod, d.active};
      prof_begin(KC_INV_PANEL, s);
      if (NB == 32) hipLaunchKernelGGL((gj_panel_kernel<32, 512>), dim3(d.batch), dim3(nthr), 0, s, pa);
      else if (n <= 512) hipLaunchKernelGGL((gj_panel_kernel<16, 512>), dim3(d.batch), dim3(nthr), 0, s, pa);
      else hipLaunchKernelGGL((gj_panel_kernel<16, MAX_ROWS>), dim3(d.batch), dim3(nthr), 0, s, pa);
      prof_end(KC_INV_PANEL, s, 8.0 * n * NB * NB * d.batch, 0);
      if ((e = hipGetLastError()) != hipSuccess) return e;
      // update of the super-panel columns: A[:, J] += W U[:, J]
      GemmDesc g = update_desc(n, mo, nbw, W, NB, sItem, U + J0, n, sItem, d.M + J0, d.ldm, d.sM, d.batch, d.active);
      if ((e = launch_gemm(g, s)) != hipSuccess) return e;
    }
    if (mo == n) break;   // one level: the super-panel was the whole matrix
    // outer step: interchanges and pivot rows of the other columns, then A += Wo Uo
    prof_begin(KC_INV_SWAP, s);
    hipLaunchKernelGGL(gj_take_panel_kernel, dim3((unsigned)(((long)n * mo + 255) / 256), d.batch), dim3(256), 0, s,
                       n, J0, mo, d.M, d.ldm, d.sM, Wo, sItem, d.active);
    hipLaunchKernelGGL(gj_outer_swap_kernel, dim3((n + 255) / 256, d.batch), dim3(256), 0, s, n, J0, mo, d.M, d.ldm,
                       d.sM, Uo, sItem, piv, sI, d.active);
    prof_end(KC_INV_SWAP, s, 0, 0);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    GemmDesc g = update_desc(n, n, mo, Wo, mo, sItem, Uo, n, sItem, d.M, d.ldm, d.sM, d.batch, d.active);
    if ((e = launch_gemm(g, s)) != hipSuccess) return e;
  }
  prof_begin(KC_INV_PERM, s);
  hipLaunchKernelGGL(gj_gather_kernel, dim3((n + GATHER_ROWS - 1) / GATHER_ROWS, d.batch), dim3(256), 0, s, n, d.M,
                     d.ldm, d.sM, d.out, d.ldo, d.sO, sigma, sI, d.active);
  prof_end(KC_INV_PERM, s, 0, 32.0 * n * n * d.batch);
  return hipGetLastError();
}

}  // namespace negf
