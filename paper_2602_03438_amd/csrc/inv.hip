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
  double2* A; long lda, sA;
  double2* W; long sW;      // W_p: n x NB row-major
  double2* U; long sU;      // U_p: NB x n row-major
  int* sigma; long sS;      // sigma_p[i]: original row now at position i
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
  // --- interchanges on the other columns, pivot rows into U (identity in the panel columns)
  for (int c = r; c < n; c += blockDim.x) {
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

size_t per_item_bytes(int n) {
  const size_t per = (size_t)2 * n * NB_MAX * sizeof(double2) + (size_t)n * sizeof(int);
  return (per + 255) & ~(size_t)255;
}

}  // namespace

size_t inverse_scratch_bytes(int n, int batch) { return per_item_bytes(n) * batch; }

hipError_t launch_inverse(const InvDesc& d, hipStream_t s) {
  const int n = d.n;
  if (n <= 0 || d.batch <= 0) return hipSuccess;
  if (n > MAX_ROWS) return hipErrorInvalidValue;
  const int NB = (d.nb == 32 && n <= 512) ? 32 : 16;
  const size_t per_al = per_item_bytes(n);
  const long sItem = (long)(per_al / sizeof(double2));   // per_al is a multiple of 256 bytes
  const long sI = (long)(per_al / sizeof(int));
  char* base = (char*)d.scratch;
  double2* W = (double2*)base;
  double2* U = (double2*)(base + (size_t)n * NB_MAX * sizeof(double2));
  int* sigma = (int*)(base + (size_t)2 * n * NB_MAX * sizeof(double2));
  const int nthr = ((n + 63) / 64) * 64;
  hipError_t e = hipSuccess;
  for (int j0 = 0; j0 < n; j0 += NB) {
    const int nbw = (n - j0 < NB) ? n - j0 : NB;
    PanelArgs pa{n, j0, nbw, d.M, d.ldm, d.sM, W, sItem, U, sItem, sigma, sI, d.info, d.info_mod, d.active};
    prof_begin(KC_INV_PANEL, s);
    if (NB == 32) hipLaunchKernelGGL((gj_panel_kernel<32, 512>), dim3(d.batch), dim3(nthr), 0, s, pa);
    else if (n <= 512) hipLaunchKernelGGL((gj_panel_kernel<16, 512>), dim3(d.batch), dim3(nthr), 0, s, pa);
    else hipLaunchKernelGGL((gj_panel_kernel<16, MAX_ROWS>), dim3(d.batch), dim3(nthr), 0, s, pa);
    prof_end(KC_INV_PANEL, s, 8.0 * n * NB * NB * d.batch, 0);
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
    g.tile = GEMM_TILE_64;
    g.prof_class = KC_INV_GEMM;
    if ((e = launch_gemm(g, s)) != hipSuccess) return e;
  }
  prof_begin(KC_INV_PERM, s);
  hipLaunchKernelGGL(gj_gather_kernel, dim3((n + GATHER_ROWS - 1) / GATHER_ROWS, d.batch), dim3(256), 0, s, n, d.M,
                     d.ldm, d.sM, d.out, d.ldo, d.sO, sigma, sI, d.active);
  prof_end(KC_INV_PERM, s, 0, 32.0 * n * n * d.batch);
  return hipGetLastError();
}

}  // namespace negf
