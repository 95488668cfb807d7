// Batched in-place inversion of complex n x n blocks by blocked Gauss-Jordan
// elimination with partial (row) pivoting.
//
// Block step for the panel J = [j0, j0+nb) of the current matrix A:
//   1. panel kernel: one workgroup per matrix, one thread per row, the n x nb
//      panel in registers.  nb unblocked Gauss-Jordan steps restricted to the
//      panel: pivot = argmax_{r >= j} |Re a_rj| + |Im a_rj|, row swap, scale
//      the pivot row, eliminate the column from every other row, storing the
//      multipliers in place.  The result W = [A_JJ^{-1}; -A_RJ A_JJ^{-1}]
//      (rows in pivoted order) goes to scratch; the panel columns of A are
//      cleared.
//   2. swap kernel: applies the nb row interchanges to the columns outside the
//      panel, copies the pivot rows into U (nb x n) with the identity in the
//      panel columns, and clears those rows in A.
//   3. product: A += W U on the matrix cores (one batched complex product,
//      K = nb).  This updates the pivot rows to A_JJ^{-1} A_JC, the other rows
//      to A_RC - A_RJ A_JJ^{-1} A_JC, and writes W into the panel columns.
// After the last panel A holds (P A)^{-1} for the accumulated row permutation
// P; the inverse A^{-1} = (P A)^{-1} P is obtained by a column gather.
// Arithmetic: 8 n^3 real flops per matrix, all but O(n^2 nb) of them in the
// batched products.
#include "internal.h"

namespace negf {

namespace {

constexpr int MAX_ROWS = 1024;

struct PanelArgs {
  int n, j0, nbw;
  double2* A; long lda, sA;
  double2* W; long sW;      // W_p: n x NB row-major
  int* piv; long sP;        // piv_p[j]: row swapped with row j at step j
  int* info; int info_mod;
  const int* active;
};

template <int NB, int MAXT>
__global__ void __launch_bounds__(MAXT) gj_panel_kernel(PanelArgs a) {
  const int p = blockIdx.x;
  if (a.active && a.active[p] == 0) return;
  double2* __restrict__ A = a.A + (long)p * a.sA;
  double2* __restrict__ W = a.W + (long)p * a.sW;
  int* __restrict__ piv = a.piv + (long)p * a.sP;
  const int r = threadIdx.x;
  const int n = a.n, j0 = a.j0;
  const bool valid = r < n;
  const int lane = r & 63, wave = r >> 6, nwaves = (blockDim.x + 63) >> 6;

  __shared__ double red_key[MAX_ROWS / 64];
  __shared__ int red_idx[MAX_ROWS / 64];
  __shared__ double2 srow[2][NB];
  __shared__ double2 prow[NB];

  double2 x[NB];
#pragma unroll
  for (int c = 0; c < NB; ++c)
    x[c] = (valid && c < a.nbw) ? A[(long)r * a.lda + j0 + c] : make_double2(0.0, 0.0);

  int status = ST_OK;
#pragma unroll
  for (int jj = 0; jj < NB; ++jj) {
    if (jj >= a.nbw) break;
    const int j = j0 + jj;
    // --- pivot search over rows r >= j (ties -> smallest row index)
    double key = (valid && r >= j) ? fabs(x[jj].x) + fabs(x[jj].y) : -1.0;
    if (key != key) key = 1e308;  // a NaN pivot candidate is taken and reported below
    int idx = r;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const double k2 = __shfl_xor(key, off);
      const int i2 = __shfl_xor(idx, off);
      if (k2 > key || (k2 == key && i2 < idx)) { key = k2; idx = i2; }
    }
    if (lane == 0) { red_key[wave] = key; red_idx[wave] = idx; }
    __syncthreads();
    key = red_key[0];
    idx = red_idx[0];
    for (int w = 1; w < nwaves; ++w) {
      const double k2 = red_key[w];
      const int i2 = red_idx[w];
      if (k2 > key || (k2 == key && i2 < idx)) { key = k2; idx = i2; }
    }
    const int pr = idx;
    // --- interchange rows j and pr of the panel
    if (pr != j) {
      if (r == j) {
#pragma unroll
        for (int c = 0; c < NB; ++c) srow[0][c] = x[c];
      }
      if (r == pr) {
#pragma unroll
        for (int c = 0; c < NB; ++c) srow[1][c] = x[c];
      }
      __syncthreads();
      if (r == j) {
#pragma unroll
        for (int c = 0; c < NB; ++c) x[c] = srow[1][c];
      }
      if (r == pr) {
#pragma unroll
        for (int c = 0; c < NB; ++c) x[c] = srow[0][c];
      }
    }
    // --- scale the pivot row and publish it
    if (r == j) {
      const double2 d = x[jj];
      if (d.x == 0.0 && d.y == 0.0) status = ST_ESINGULAR;
      const double2 dinv = cinv(d);
      if (!(isfinite(dinv.x) && isfinite(dinv.y))) status = status == ST_OK ? ST_ENONFINITE : status;
#pragma unroll
      for (int c = 0; c < NB; ++c) x[c] = (c == jj) ? dinv : cmul(x[c], dinv);
#pragma unroll
      for (int c = 0; c < NB; ++c) prow[c] = x[c];
      piv[j] = pr;
    }
    __syncthreads();
    // --- eliminate column jj from every other row (multiplier stored in place)
    if (valid && r != j) {
      const double2 f = x[jj];
      x[jj] = make_double2(0.0, 0.0);
#pragma unroll
      for (int c = 0; c < NB; ++c) {
        const double2 pc = prow[c];
        x[c].x -= f.x * pc.x - f.y * pc.y;
        x[c].y -= f.x * pc.y + f.y * pc.x;
      }
    }
  }
  if (valid) {
#pragma unroll
    for (int c = 0; c < NB; ++c) W[(long)r * NB + c] = x[c];
#pragma unroll
    for (int c = 0; c < NB; ++c)
      if (c < a.nbw) A[(long)r * a.lda + j0 + c] = make_double2(0.0, 0.0);
  }
  if (status != ST_OK && a.info) atomicCAS(a.info + (a.info_mod > 0 ? p % a.info_mod : p), ST_OK, status);
}

struct SwapArgs {
  int n, j0, nbw, NB;
  double2* A; long lda, sA;
  double2* U; long sU;      // U_p: NB x n row-major
  const int* piv; long sP;
  const int* active;
};

__global__ void __launch_bounds__(256) gj_swap_kernel(SwapArgs a) {
  const int p = blockIdx.y;
  if (a.active && a.active[p] == 0) return;
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= a.n) return;
  double2* __restrict__ A = a.A + (long)p * a.sA;
  double2* __restrict__ U = a.U + (long)p * a.sU;
  const int* __restrict__ piv = a.piv + (long)p * a.sP;
  if (c >= a.j0 && c < a.j0 + a.nbw) {
    for (int k = 0; k < a.nbw; ++k) U[(long)k * a.n + c] = make_double2(k == c - a.j0 ? 1.0 : 0.0, 0.0);
    return;
  }
  for (int k = 0; k < a.nbw; ++k) {
    const int j = a.j0 + k, pr = piv[j];
    if (pr != j) {
      const double2 t0 = A[(long)j * a.lda + c];
      A[(long)j * a.lda + c] = A[(long)pr * a.lda + c];
      A[(long)pr * a.lda + c] = t0;
    }
  }
  for (int k = 0; k < a.nbw; ++k) {
    const long o = (long)(a.j0 + k) * a.lda + c;
    U[(long)k * a.n + c] = A[o];
    A[o] = make_double2(0.0, 0.0);
  }
}

// perm_p: column c of the inverse is column perm[c] of (P A)^{-1}.  Applying
// the right factors P_{n-1} ... P_0 in that order swaps perm entries k, piv[k].
__global__ void gj_perm_kernel(int n, const int* piv, long sP, int* perm, long sPerm, int batch, const int* active) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= batch) return;
  if (active && active[p] == 0) return;
  const int* pv = piv + (long)p * sP;
  int* pm = perm + (long)p * sPerm;
  for (int c = 0; c < n; ++c) pm[c] = c;
  for (int k = n - 1; k >= 0; --k) {
    const int q = pv[k];
    const int t = pm[k];
    pm[k] = pm[q];
    pm[q] = t;
  }
}

__global__ void __launch_bounds__(256) gj_gather_kernel(int n, const double2* M, long ldm, long sM, double2* out,
                                                        long ldo, long sO, const int* perm, long sPerm,
                                                        const int* active) {
  const int p = blockIdx.z;
  if (active && active[p] == 0) return;
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (c >= n) return;
  const int src = perm[(long)p * sPerm + c];
  out[(long)p * sO + (long)r * ldo + c] = M[(long)p * sM + (long)r * ldm + src];
}

constexpr int NB_MAX = 32;

}  // namespace

size_t inverse_scratch_bytes(int n, int batch) {
  // W (n x NB_MAX) + U (NB_MAX x n) complex, piv + perm int, per item
  const size_t per = (size_t)2 * n * NB_MAX * sizeof(double2) + (size_t)2 * n * sizeof(int);
  return ((per + 255) & ~(size_t)255) * batch;
}

hipError_t launch_inverse(const InvDesc& d, hipStream_t s) {
  const int n = d.n;
  if (n <= 0 || d.batch <= 0) return hipSuccess;
  if (n > MAX_ROWS) return hipErrorInvalidValue;
  const int NB = (d.nb == 32 && n <= 512) ? 32 : 16;
  const size_t per = (size_t)2 * n * NB_MAX * sizeof(double2) + (size_t)2 * n * sizeof(int);
  const size_t per_al = (per + 255) & ~(size_t)255;
  const long sItem = (long)(per_al / sizeof(double2));  // per_al is a multiple of 256 bytes
  char* base = (char*)d.scratch;
  double2* W = (double2*)base;
  double2* U = (double2*)(base + (size_t)n * NB_MAX * sizeof(double2));
  int* piv = (int*)(base + (size_t)2 * n * NB_MAX * sizeof(double2));
  int* perm = piv + n;
  const long sI = (long)(per_al / sizeof(int));
  const int nthr = ((n + 63) / 64) * 64;
  hipError_t e = hipSuccess;
  for (int j0 = 0; j0 < n; j0 += NB) {
    const int nbw = (n - j0 < NB) ? n - j0 : NB;
    PanelArgs pa{n, j0, nbw, d.M, d.ldm, d.sM, W, sItem, piv, sI, d.info, d.info_mod, d.active};
    prof_begin(KC_INV_PANEL, s);
    if (NB == 32) hipLaunchKernelGGL((gj_panel_kernel<32, 512>), dim3(d.batch), dim3(nthr), 0, s, pa);
    else hipLaunchKernelGGL((gj_panel_kernel<16, MAX_ROWS>), dim3(d.batch), dim3(nthr), 0, s, pa);
    prof_end(KC_INV_PANEL, s, 8.0 * n * NB * NB * d.batch, 0);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    SwapArgs sa{n, j0, nbw, NB, d.M, d.ldm, d.sM, U, sItem, piv, sI, d.active};
    prof_begin(KC_INV_SWAP, s);
    hipLaunchKernelGGL(gj_swap_kernel, dim3((n + 255) / 256, d.batch), dim3(256), 0, s, sa);
    prof_end(KC_INV_SWAP, s, 0, 0);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    GemmDesc g{};
    g.M = n; g.N = n; g.K = nbw; g.batch = d.batch;
    g.opA = OP_N; g.opB = OP_N;
    g.A = MatRef{W, NB, sItem};
    g.B = MatRef{U, n, sItem};
    g.alpha = make_double2(1.0, 0.0);
    g.beta = make_double2(1.0, 0.0);
    g.Cin = MatRef{d.M, d.ldm, d.sM};
    g.C = MatOut{d.M, d.ldm, d.sM};
    g.active = d.active;
    g.prec = PREC_F64;
    g.xcd_remap = 1;
    g.prof_class = KC_INV_GEMM;
    if ((e = launch_gemm(g, s)) != hipSuccess) return e;
  }
  prof_begin(KC_INV_PERM, s);
  hipLaunchKernelGGL(gj_perm_kernel, dim3((d.batch + 63) / 64), dim3(64), 0, s, n, piv, sI, perm, sI, d.batch, d.active);
  hipLaunchKernelGGL(gj_gather_kernel, dim3((n + 255) / 256, n, d.batch), dim3(256), 0, s, n, d.M, d.ldm, d.sM, d.out,
                     d.ldo, d.sO, perm, sI, d.active);
  prof_end(KC_INV_PERM, s, 0, 0);
  return hipGetLastError();
}

}  // namespace negf
