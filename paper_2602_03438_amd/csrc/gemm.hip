// Batched complex block products on the CDNA4 matrix cores.
//
// C_p = alpha * op(A_p) op(B_p) + beta * Cin_p with op = identity or conjugate
// transpose, for a batch of interleaved-complex matrices.  The complex product
// is formed from four real products per k-step (re*re, -im*im, re*im, im*re)
// on v_mfma_f64_16x16x4f64 (double) or v_mfma_f32_16x16x4f32 (single: operands
// rounded to complex64 when they are staged, single accumulation, result
// widened to double on store).
//
// Work decomposition: one 256-thread workgroup (4 waves in 2 x 2) per 64 x 64
// output tile; each wave owns a 32 x 32 sub-tile = 2 x 2 MFMA tiles of 16 x 16
// with separate real and imaginary accumulators.  K advances in steps of 16
// complex values through two LDS stages: global loads for step k+1 are issued
// into registers before the MFMAs of step k, and land in the other LDS stage
// afterwards, so there is one barrier per step.
//
// LDS keeps each tile in the layout it has in HBM (no transpose on the store
// path; the MFMA operand reads do the reorientation):
//   "row" layout [64][16+1]: 64 rows (m or n), 16 contiguous k values
//   "col" layout [16][64+1]: 16 k rows, 64 contiguous m or n values
// op(A)=A   (A stored M x K) -> row ; op(A)=A^H (stored K x M) -> col
// op(B)=B   (B stored K x N) -> col ; op(B)=B^H (stored N x K) -> row
// The +1 complex padding keeps a 16-lane group of MFMA operand reads on
// distinct banks in both layouts.
#include "internal.h"

namespace negf {

namespace {

constexpr int BM = 64, BN = 64, BK = 16, NT = 256;
constexpr int LD_ROW = BK + 1;
constexpr int LD_COL = BM + 1;
constexpr int TILE_ELEMS = (BM * LD_ROW > BK * LD_COL) ? BM * LD_ROW : BK * LD_COL;

template <typename T> struct Cx;
template <> struct Cx<double> { typedef double2 type; };
template <> struct Cx<float> { typedef float2 type; };

template <typename T> struct Acc;
template <> struct Acc<double> { typedef v4d type; };
template <> struct Acc<float> { typedef v4f type; };

__device__ __forceinline__ v4d mfma16(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ v4f mfma16(float a, float b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

template <typename T> __device__ __forceinline__ int acc_row(int lk, int v);
template <> __device__ __forceinline__ int acc_row<double>(int lk, int v) { return lk + 4 * v; }
template <> __device__ __forceinline__ int acc_row<float>(int lk, int v) { return 4 * lk + v; }

template <typename T> __device__ __forceinline__ typename Cx<T>::type to_cx(double2 v, bool conj);
template <> __device__ __forceinline__ double2 to_cx<double>(double2 v, bool conj) {
  return conj ? make_double2(v.x, -v.y) : v;
}
template <> __device__ __forceinline__ float2 to_cx<float>(double2 v, bool conj) {
  return make_float2((float)v.x, conj ? -(float)v.y : (float)v.y);
}

struct KArgs {
  int M, N, K, batch;
  const double2* A; long lda, sA;
  const double2* B; long ldb, sB;
  const double2* Cin; long ldci, sCi;
  double2* C; long ldc, sC;
  double2 alpha, beta;
  const int* active;
  int tiles_m, tiles_n, xcd_remap;
};

// Stage one 64 x 16 (row layout) or 16 x 64 (col layout) operand tile into registers.
// rows0/cols0: tile origin in the stored matrix; R/Cn: stored matrix extent.
template <bool ROWL>
__device__ __forceinline__ void load_tile(double2 (&r)[4], const double2* __restrict__ base, long ld, int row0,
                                          int col0, int R, int Cn) {
  const int t = threadIdx.x;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    int rr, cc;
    if (ROWL) { rr = (t >> 4) + 16 * j; cc = t & 15; }
    else      { rr = (t >> 6) + 4 * j;  cc = t & 63; }
    const int gr = row0 + rr, gc = col0 + cc;
    r[j] = (gr < R && gc < Cn) ? base[(long)gr * ld + gc] : make_double2(0.0, 0.0);
  }
}

template <typename T, bool ROWL>
__device__ __forceinline__ void store_tile(typename Cx<T>::type* s, const double2 (&r)[4], bool conj) {
  const int t = threadIdx.x;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    int idx;
    if (ROWL) idx = ((t >> 4) + 16 * j) * LD_ROW + (t & 15);
    else      idx = ((t >> 6) + 4 * j) * LD_COL + (t & 63);
    s[idx] = to_cx<T>(r[j], conj);
  }
}

template <typename T, int OPA, int OPB>
__global__ void __launch_bounds__(NT, 2) zgemm_kernel(KArgs a) {
  typedef typename Cx<T>::type CT;
  typedef typename Acc<T>::type AT;
  constexpr bool A_ROW = (OPA == OP_N);  // A stored M x K
  constexpr bool B_ROW = (OPB == OP_C);  // B stored N x K
  __shared__ CT sA[2][TILE_ELEMS];
  __shared__ CT sB[2][TILE_ELEMS];

  const int per_item = a.tiles_m * a.tiles_n;
  const long total = (long)per_item * a.batch;
  long lid = blockIdx.x;
  if (a.xcd_remap && (total & 7) == 0) lid = (lid & 7) * (total >> 3) + (lid >> 3);
  const int p = (int)(lid / per_item);
  const int tid = (int)(lid - (long)p * per_item);
  if (a.active && a.active[p] == 0) return;
  const int tm = tid / a.tiles_n, tn = tid - tm * a.tiles_n;
  const int m0 = tm * BM, n0 = tn * BN;

  const double2* __restrict__ Ap = a.A + (long)p * a.sA;
  const double2* __restrict__ Bp = a.B + (long)p * a.sB;

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int li = lane & 15, lk = lane >> 4;

  AT accR[2][2], accI[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      accR[i][j] = AT{0, 0, 0, 0};
      accI[i][j] = AT{0, 0, 0, 0};
    }

  double2 ra[4], rb[4];
  auto gload = [&](int k0) {
    if (A_ROW) load_tile<true>(ra, Ap, a.lda, m0, k0, a.M, a.K);
    else       load_tile<false>(ra, Ap, a.lda, k0, m0, a.K, a.M);
    if (B_ROW) load_tile<true>(rb, Bp, a.ldb, n0, k0, a.N, a.K);
    else       load_tile<false>(rb, Bp, a.ldb, k0, n0, a.K, a.N);
  };
  auto lstore = [&](int st) {
    store_tile<T, A_ROW>(sA[st], ra, OPA == OP_C);
    store_tile<T, B_ROW>(sB[st], rb, OPB == OP_C);
  };

  const int nk = (a.K + BK - 1) / BK;
  gload(0);
  lstore(0);
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int st = kt & 1;
    if (kt + 1 < nk) gload((kt + 1) * BK);
    const CT* __restrict__ xA = sA[st];
    const CT* __restrict__ xB = sB[st];
#pragma unroll
    for (int kk = 0; kk < BK / 4; ++kk) {
      const int kq = kk * 4 + lk;
      CT av[2], bv[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const int m = wm * 32 + i * 16 + li;
        av[i] = A_ROW ? xA[m * LD_ROW + kq] : xA[kq * LD_COL + m];
        const int n = wn * 32 + i * 16 + li;
        bv[i] = B_ROW ? xB[n * LD_ROW + kq] : xB[kq * LD_COL + n];
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) accR[i][j] = mfma16(av[i].x, bv[j].x, accR[i][j]);
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) accI[i][j] = mfma16(av[i].x, bv[j].y, accI[i][j]);
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) accR[i][j] = mfma16(-av[i].y, bv[j].y, accR[i][j]);
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) accI[i][j] = mfma16(av[i].y, bv[j].x, accI[i][j]);
    }
    if (kt + 1 < nk) lstore(st ^ 1);
    __syncthreads();
  }

  // Epilogue.  Accumulator element v of a lane sits in column lane%16 of the
  // 16 x 16 tile; its row is 4*(lane/16)+v for the single-precision MFMA and
  // lane/16+4*v for the double-precision one (measured on gfx950).
  double2* __restrict__ Cp = a.C + (long)p * a.sC;
  const double2* __restrict__ Ci = a.Cin ? a.Cin + (long)p * a.sCi : nullptr;
  const bool use_beta = (a.beta.x != 0.0 || a.beta.y != 0.0) && Ci != nullptr;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int col = n0 + wn * 32 + j * 16 + li;
      if (col >= a.N) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = m0 + wm * 32 + i * 16 + acc_row<T>(lk, v);
        if (row >= a.M) continue;
        const double re = (double)accR[i][j][v], im = (double)accI[i][j][v];
        double2 out = make_double2(a.alpha.x * re - a.alpha.y * im, a.alpha.x * im + a.alpha.y * re);
        if (use_beta) {
          const double2 c = Ci[(long)row * a.ldci + col];
          out.x += a.beta.x * c.x - a.beta.y * c.y;
          out.y += a.beta.x * c.y + a.beta.y * c.x;
        }
        Cp[(long)row * a.ldc + col] = out;
      }
    }
}

template <typename T>
hipError_t launch_t(const GemmDesc& d, const KArgs& ka, dim3 grid, hipStream_t s) {
  if (d.opA == OP_N && d.opB == OP_N) hipLaunchKernelGGL((zgemm_kernel<T, OP_N, OP_N>), grid, dim3(NT), 0, s, ka);
  else if (d.opA == OP_C && d.opB == OP_N) hipLaunchKernelGGL((zgemm_kernel<T, OP_C, OP_N>), grid, dim3(NT), 0, s, ka);
  else if (d.opA == OP_N && d.opB == OP_C) hipLaunchKernelGGL((zgemm_kernel<T, OP_N, OP_C>), grid, dim3(NT), 0, s, ka);
  else hipLaunchKernelGGL((zgemm_kernel<T, OP_C, OP_C>), grid, dim3(NT), 0, s, ka);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_gemm(const GemmDesc& d, hipStream_t s) {
  if (d.M <= 0 || d.N <= 0 || d.batch <= 0) return hipSuccess;
  KArgs ka;
  ka.M = d.M; ka.N = d.N; ka.K = d.K; ka.batch = d.batch;
  ka.A = d.A.p; ka.lda = d.A.ld; ka.sA = d.A.stride;
  ka.B = d.B.p; ka.ldb = d.B.ld; ka.sB = d.B.stride;
  ka.Cin = d.Cin.p; ka.ldci = d.Cin.ld; ka.sCi = d.Cin.stride;
  ka.C = d.C.p; ka.ldc = d.C.ld; ka.sC = d.C.stride;
  ka.alpha = d.alpha; ka.beta = d.beta;
  ka.active = d.active;
  ka.tiles_m = (d.M + BM - 1) / BM;
  ka.tiles_n = (d.N + BN - 1) / BN;
  ka.xcd_remap = d.xcd_remap;
  const long total = (long)ka.tiles_m * ka.tiles_n * d.batch;
  dim3 grid((unsigned)total);
  const int cls = d.prof_class >= 0 ? d.prof_class : (d.prec == PREC_F32 ? KC_GEMM32 : KC_GEMM64);
  prof_begin(cls, s);
  hipError_t e = d.prec == PREC_F32 ? launch_t<float>(d, ka, grid, s) : launch_t<double>(d, ka, grid, s);
  prof_end(cls, s, 8.0 * d.M * (double)d.N * d.K * d.batch, 16.0 * d.batch * ((double)d.M * d.K + (double)d.K * d.N + 2.0 * d.M * d.N));
  return e;
}

}  // namespace negf
