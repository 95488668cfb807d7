// Kernels of the learned lead initialiser: a 3-layer perceptron
//   Z1 = X W1 + b1, A1 = tanh(Z1); Z2 = A1 W2 + b2, A2 = tanh(Z2); Y = A2 W3 + b3
// trained in single precision (forward, hand-written backward of the mean
// squared error, Adam) and evaluated in bfloat16 (weights and activations
// rounded to bf16, single-precision accumulation).
//
// All products go through one real GEMM kernel on the matrix cores:
// v_mfma_f32_16x16x4f32 for single precision, v_mfma_f32_16x16x16bf16_1k for
// bfloat16 operands, 64 x 64 output tiles per 256-thread workgroup, 16-deep K
// steps staged through LDS, with the bias / activation / activation-derivative
// applied in the epilogue.  Row-major storage; weights are [fan_in][fan_out].
#include "../../include/negf.h"
#include "internal.h"

namespace negf {
namespace {

typedef short bf16x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ unsigned short f2bf(float f) {
  // round to nearest even
  unsigned int u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (unsigned short)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf2f(unsigned short h) { return __uint_as_float(((unsigned int)h) << 16); }

enum Epi { EPI_STORE = 0, EPI_BIAS = 1, EPI_BIAS_TANH = 2, EPI_DTANH = 3, EPI_ACCUM = 4 };

struct SArgs {
  int M, N, K;
  const void* A; int lda; int transA;   // op(A) is M x K; transA: A stored K x M
  const void* B; int ldb; int transB;   // op(B) is K x N; transB: B stored N x K
  float* C; int ldc;
  const float* bias;                    // EPI_BIAS / EPI_BIAS_TANH
  const float* act; int ldact;          // EPI_DTANH: C = acc * (1 - act^2)
  unsigned short* Cb;                   // optional bf16 copy of the output (inference)
  float alpha, beta;                    // EPI_ACCUM: C = alpha acc + beta C
  int epi;
};

constexpr int SB = 64, SK = 16, SNT = 256;

// T = float: operands read as float; T = unsigned short: operands are bf16 bit patterns
template <typename T>
__device__ __forceinline__ float ldv(const void* p, long i) {
  return ((const float*)p)[i];
}
template <>
__device__ __forceinline__ float ldv<unsigned short>(const void* p, long i) {
  return bf2f(((const unsigned short*)p)[i]);
}

template <typename T, bool BF16MMA>
__global__ void __launch_bounds__(SNT) sgemm_kernel(SArgs a) {
  __shared__ float sA[SK][SB + 1];
  __shared__ float sB[SK][SB + 1];
  const int m0 = blockIdx.y * SB, n0 = blockIdx.x * SB;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int li = lane & 15, lk = lane >> 4;
  v4f acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = v4f{0, 0, 0, 0};
  for (int k0 = 0; k0 < a.K; k0 += SK) {
    // stage op(A)[m0..m0+63][k0..k0+15] and op(B)[k0..k0+15][n0..n0+63] as [k][m], [k][n]
    for (int e = t; e < SK * SB; e += SNT) {
      const int kk = e / SB, mm = e % SB;
      const int gm = m0 + mm, gk = k0 + kk;
      float va = 0.f;
      if (gm < a.M && gk < a.K) va = a.transA ? ldv<T>(a.A, (long)gk * a.lda + gm) : ldv<T>(a.A, (long)gm * a.lda + gk);
      sA[kk][mm] = va;
      const int gn = n0 + mm;
      float vb = 0.f;
      if (gn < a.N && gk < a.K) vb = a.transB ? ldv<T>(a.B, (long)gn * a.ldb + gk) : ldv<T>(a.B, (long)gk * a.ldb + gn);
      sB[kk][mm] = vb;
    }
    __syncthreads();
    if (BF16MMA) {
      // one 16x16x16 bf16 step: lane holds A[row][4*(lane/16)+i], B[4*(lane/16)+i][col]
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          bf16x4 av, bv;
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            av[q] = (short)f2bf(sA[4 * lk + q][wm * 32 + i * 16 + li]);
            bv[q] = (short)f2bf(sB[4 * lk + q][wn * 32 + j * 16 + li]);
          }
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc[i][j], 0, 0, 0);
        }
    } else {
#pragma unroll
      for (int kk = 0; kk < SK / 4; ++kk) {
        const int kq = kk * 4 + lk;
        float av[2], bv[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          av[i] = sA[kq][wm * 32 + i * 16 + li];
          bv[i] = sB[kq][wn * 32 + i * 16 + li];
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[i], bv[j], acc[i][j], 0, 0, 0);
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int col = n0 + wn * 32 + j * 16 + li;
      if (col >= a.N) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = m0 + wm * 32 + i * 16 + 4 * lk + v;
        if (row >= a.M) continue;
        float x = acc[i][j][v];
        const long o = (long)row * a.ldc + col;
        if (a.epi == EPI_BIAS || a.epi == EPI_BIAS_TANH) x += a.bias[col];
        if (a.epi == EPI_BIAS_TANH) x = tanhf(x);
        if (a.epi == EPI_DTANH) {
          const float y = a.act[(long)row * a.ldact + col];
          x *= 1.f - y * y;
        }
        if (a.epi == EPI_ACCUM) x = a.alpha * x + (a.beta != 0.f ? a.beta * a.C[o] : 0.f);
        if (a.C) a.C[o] = x;
        if (a.Cb) a.Cb[o] = f2bf(x);
      }
    }
}

hipError_t sgemm(const SArgs& a, bool bf16_operands, hipStream_t s) {
  if (a.M <= 0 || a.N <= 0) return hipSuccess;
  dim3 grid((a.N + SB - 1) / SB, (a.M + SB - 1) / SB);
  if (bf16_operands) hipLaunchKernelGGL((sgemm_kernel<unsigned short, true>), grid, dim3(SNT), 0, s, a);
  else hipLaunchKernelGGL((sgemm_kernel<float, false>), grid, dim3(SNT), 0, s, a);
  return hipGetLastError();
}

// dY = 2 (Y - T) / (n * out)
__global__ void mse_grad_kernel(long n, const float* Y, const float* T, float scale, float* dY) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    dY[i] = scale * (Y[i] - T[i]);
}

// db[c] = sum_r dZ[r][c]   (one workgroup per column block, deterministic order)
__global__ void __launch_bounds__(256) colsum_kernel(int rows, int cols, const float* dZ, float* db) {
  const int c = blockIdx.x;
  float s = 0.f;
  for (int r = threadIdx.x; r < rows; r += 256) s += dZ[(long)r * cols + c];
  __shared__ float red[4];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) db[c] = red[0] + red[1] + red[2] + red[3];
}

__global__ void adam_kernel(long n, float* p, const float* g, float* m, float* v, float lr, float b1, float b2,
                            float eps, float c1, float c2) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float mh = mi / c1, vh = vi / c2;
    p[i] -= lr * mh / (sqrtf(vh) + eps);
  }
}

__global__ void to_bf16_kernel(long n, const float* src, unsigned short* dst) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    dst[i] = f2bf(src[i]);
}

// ---- data transforms of the learned pipeline ----
constexpr int PART = 64;   // partial sums per column (moments) or in total (squared error)

// part[c * PART + blockIdx.x] = sum over this workgroup's rows of (X[r][c] - shift[c])^pw
// (pw 1 or 2; shift nullable = 0), accumulated in double.  Grid (PART, F).
__global__ void __launch_bounds__(256) colpart_kernel(long n, int F, const float* X, const double* shift, int pw,
                                                      double* part) {
  const int c = blockIdx.y;
  const double sh = shift ? shift[c] : 0.0;
  double acc = 0.0;
  for (long r = (long)blockIdx.x * 256 + threadIdx.x; r < n; r += (long)PART * 256) {
    const double d = (double)X[r * F + c] - sh;
    acc += pw == 1 ? d : d * d;
  }
  __shared__ double red[4];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) part[(long)c * PART + blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// mode 0: mean[c] = sum(part) / n;  mode 1: sd[c] = max(sqrt(sum(part) / (n - 1)), floor)
__global__ void colfinish_kernel(long n, int F, const double* part, int mode, double* mean, float* outf, float floor_) {
  const int c = threadIdx.x;
  if (c >= F) return;
  double s = 0.0;
  for (int j = 0; j < PART; ++j) s += part[(long)c * PART + j];
  if (mode == 0) {
    mean[c] = s / (double)n;
    outf[c] = (float)(s / (double)n);
  } else {
    const double v = n > 1 ? s / (double)(n - 1) : 0.0;
    outf[c] = fmaxf((float)sqrt(v), floor_);
  }
}

__global__ void normalize_kernel(long n, int F, const float* X, const float* mu, const float* sd, float* Xn) {
  const long tot = n * F;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < tot; i += (long)gridDim.x * blockDim.x) {
    const int c = (int)(i % F);
    Xn[i] = (X[i] - mu[c]) / sd[c];
  }
}

// y = sign(x) log(1 + |x|), or its inverse sign(x) (exp(|x|) - 1)
__global__ void signed_log_kernel(long n, const float* x, float* y, int inverse) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const float v = x[i], a = fabsf(v);
    const float m = inverse ? expm1f(a) : log1pf(a);
    y[i] = v < 0.f ? -m : m;
  }
}

// part[blockIdx.x] = sum over this workgroup's elements of (Y - T)^2 (double)
__global__ void __launch_bounds__(256) sqerr_part_kernel(long n, const float* Y, const float* T, double* part) {
  double acc = 0.0;
  for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long)PART * 256) {
    const double d = (double)Y[i] - (double)T[i];
    acc += d * d;
  }
  __shared__ double red[4];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

__global__ void sqerr_finish_kernel(long n, const double* part, double* out) {
  if (threadIdx.x != 0) return;
  double s = 0.0;
  for (int j = 0; j < PART; ++j) s += part[j];
  *out = s / (double)n;
}

// out[p * b + j] = (Re, Im) of T_p[j][j]  (float)
__global__ void mode_diag_kernel(long n, int b, const double2* T, float* out) {
  const long tot = n * b;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < tot; i += (long)gridDim.x * blockDim.x) {
    const long p = i / b;
    const int j = (int)(i - p * b);
    const double2 v = T[(p * b + j) * b + j];
    out[2 * i] = (float)v.x;
    out[2 * i + 1] = (float)v.y;
  }
}

// out_p[r][c] = U[r][c] * (y[p * b + c][0] + i y[p * b + c][1])   (U diag(x_p))
__global__ void mode_scale_kernel(long n, int b, const double2* U, const float* y, double2* out) {
  const long bb = (long)b * b, tot = n * bb;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < tot; i += (long)gridDim.x * blockDim.x) {
    const long p = i / bb;
    const long e = i - p * bb;
    const int c = (int)(e % b);
    const double2 u = U[e];
    const double xr = y[2 * (p * b + c)], xi = y[2 * (p * b + c) + 1];
    out[i] = make_double2(u.x * xr - u.y * xi, u.x * xi + u.y * xr);
  }
}

inline unsigned grid_1d(long n) {
  long g = (n + 255) / 256;
  return (unsigned)(g < 2048 ? (g > 0 ? g : 1) : 2048);
}

SArgs sa(int M, int N, int K, const void* A, int lda, int tA, const void* B, int ldb, int tB, float* C, int ldc,
         int epi) {
  SArgs a{};
  a.M = M; a.N = N; a.K = K;
  a.A = A; a.lda = lda; a.transA = tA;
  a.B = B; a.ldb = ldb; a.transB = tB;
  a.C = C; a.ldc = ldc;
  a.alpha = 1.f; a.beta = 0.f;
  a.epi = epi;
  return a;
}

}  // namespace
}  // namespace negf

using namespace negf;

extern "C" {

negf_status negf_mlp_forward(int32_t n, int32_t F, int32_t H, int32_t O, const float* X, const float* W1,
                             const float* b1, const float* W2, const float* b2, const float* W3, const float* b3,
                             float* A1, float* A2, float* Y, void* stream) {
  if (n < 0 || F <= 0 || H <= 0 || O <= 0) return NEGF_EINVAL;
  if (n == 0) return NEGF_OK;
  if (!X || !W1 || !b1 || !W2 || !b2 || !W3 || !b3 || !A1 || !A2 || !Y) return NEGF_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  SArgs a = sa(n, H, F, X, F, 0, W1, H, 0, A1, H, EPI_BIAS_TANH);
  a.bias = b1;
  if (sgemm(a, false, s) != hipSuccess) return NEGF_EHIP;
  a = sa(n, H, H, A1, H, 0, W2, H, 0, A2, H, EPI_BIAS_TANH);
  a.bias = b2;
  if (sgemm(a, false, s) != hipSuccess) return NEGF_EHIP;
  a = sa(n, O, H, A2, H, 0, W3, O, 0, Y, O, EPI_BIAS);
  a.bias = b3;
  return sgemm(a, false, s) == hipSuccess ? NEGF_OK : NEGF_EHIP;
}

negf_status negf_mlp_backward(int32_t n, int32_t F, int32_t H, int32_t O, const float* X, const float* W2,
                              const float* W3, const float* A1, const float* A2, const float* Y, const float* T,
                              float* dW1, float* db1, float* dW2, float* db2, float* dW3, float* db3, float* dY,
                              float* dZ2, float* dZ1, void* stream) {
  if (n <= 0 || F <= 0 || H <= 0 || O <= 0) return NEGF_EINVAL;
  const void* req[] = {X, W2, W3, A1, A2, Y, T, dW1, db1, dW2, db2, dW3, db3, dY, dZ2, dZ1};
  for (const void* p : req)
    if (!p) return NEGF_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  const long ny = (long)n * O;
  hipLaunchKernelGGL(mse_grad_kernel, dim3(grid_1d(ny)), dim3(256), 0, s, ny, Y, T, 2.f / (float)ny, dY);
  // dW3 = A2^T dY ; db3 = colsum dY
  if (sgemm(sa(H, O, n, A2, H, 1, dY, O, 0, dW3, O, EPI_STORE), false, s) != hipSuccess) return NEGF_EHIP;
  hipLaunchKernelGGL(colsum_kernel, dim3(O), dim3(256), 0, s, n, O, dY, db3);
  // dZ2 = (dY W3^T) * (1 - A2^2)
  SArgs a = sa(n, H, O, dY, O, 0, W3, O, 1, dZ2, H, EPI_DTANH);
  a.act = A2; a.ldact = H;
  if (sgemm(a, false, s) != hipSuccess) return NEGF_EHIP;
  if (sgemm(sa(H, H, n, A1, H, 1, dZ2, H, 0, dW2, H, EPI_STORE), false, s) != hipSuccess) return NEGF_EHIP;
  hipLaunchKernelGGL(colsum_kernel, dim3(H), dim3(256), 0, s, n, H, dZ2, db2);
  // dZ1 = (dZ2 W2^T) * (1 - A1^2)
  a = sa(n, H, H, dZ2, H, 0, W2, H, 1, dZ1, H, EPI_DTANH);
  a.act = A1; a.ldact = H;
  if (sgemm(a, false, s) != hipSuccess) return NEGF_EHIP;
  if (sgemm(sa(F, H, n, X, F, 1, dZ1, H, 0, dW1, H, EPI_STORE), false, s) != hipSuccess) return NEGF_EHIP;
  hipLaunchKernelGGL(colsum_kernel, dim3(H), dim3(256), 0, s, n, H, dZ1, db1);
  return hipGetLastError() == hipSuccess ? NEGF_OK : NEGF_EHIP;
}

negf_status negf_mlp_adam_step(int32_t count, float* param, const float* grad, float* m, float* v, int32_t t,
                               float lr, float beta1, float beta2, float eps, void* stream) {
  if (count < 0 || t < 1) return NEGF_EINVAL;
  if (count == 0) return NEGF_OK;
  if (!param || !grad || !m || !v) return NEGF_EINVAL;
  const float c1 = 1.f - powf(beta1, (float)t), c2 = 1.f - powf(beta2, (float)t);
  hipLaunchKernelGGL(adam_kernel, dim3(grid_1d(count)), dim3(256), 0, (hipStream_t)stream, (long)count, param, grad,
                     m, v, lr, beta1, beta2, eps, c1, c2);
  return hipGetLastError() == hipSuccess ? NEGF_OK : NEGF_EHIP;
}

negf_status negf_mlp_to_bf16(const float* src, uint16_t* dst, int64_t count, void* stream) {
  if (count < 0 || (count > 0 && (!src || !dst))) return NEGF_EINVAL;
  if (count == 0) return NEGF_OK;
  hipLaunchKernelGGL(to_bf16_kernel, dim3(grid_1d(count)), dim3(256), 0, (hipStream_t)stream, (long)count, src,
                     (unsigned short*)dst);
  return hipGetLastError() == hipSuccess ? NEGF_OK : NEGF_EHIP;
}

negf_status negf_mlp_infer_bf16(int32_t n, int32_t F, int32_t H, int32_t O, const uint16_t* Xb, const uint16_t* W1b,
                                const float* b1, const uint16_t* W2b, const float* b2, const uint16_t* W3b,
                                const float* b3, uint16_t* scratch, float* Y, void* stream) {
  if (n < 0 || F <= 0 || H <= 0 || O <= 0) return NEGF_EINVAL;
  if (n == 0) return NEGF_OK;
  if (!Xb || !W1b || !b1 || !W2b || !b2 || !W3b || !b3 || !scratch || !Y) return NEGF_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  unsigned short* A1b = (unsigned short*)scratch;
  unsigned short* A2b = A1b + (size_t)n * H;
  SArgs a = sa(n, H, F, Xb, F, 0, W1b, H, 0, nullptr, H, EPI_BIAS_TANH);
  a.bias = b1; a.Cb = A1b;
  if (sgemm(a, true, s) != hipSuccess) return NEGF_EHIP;
  a = sa(n, H, H, A1b, H, 0, W2b, H, 0, nullptr, H, EPI_BIAS_TANH);
  a.bias = b2; a.Cb = A2b;
  if (sgemm(a, true, s) != hipSuccess) return NEGF_EHIP;
  a = sa(n, O, H, A2b, H, 0, W3b, O, 0, Y, O, EPI_BIAS);
  a.bias = b3;
  return sgemm(a, true, s) == hipSuccess ? NEGF_OK : NEGF_EHIP;
}

negf_status negf_mlp_moments(int64_t n, int32_t F, const float* X, float* mu, float* sd, double* scratch,
                             void* stream) {
  if (n < 1 || F < 1 || F > 1024 || !X || !mu || !sd || !scratch) return NEGF_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  double* part = scratch;
  double* mean = scratch + (size_t)F * PART;
  hipLaunchKernelGGL(colpart_kernel, dim3(PART, F), dim3(256), 0, s, (long)n, F, X, (const double*)nullptr, 1, part);
  hipLaunchKernelGGL(colfinish_kernel, dim3(1), dim3(1024), 0, s, (long)n, F, (const double*)part, 0, mean, mu, 0.f);
  hipLaunchKernelGGL(colpart_kernel, dim3(PART, F), dim3(256), 0, s, (long)n, F, X, (const double*)mean, 2, part);
  hipLaunchKernelGGL(colfinish_kernel, dim3(1), dim3(1024), 0, s, (long)n, F, (const double*)part, 1, mean, sd,
                     1e-6f);
  return hipGetLastError() == hipSuccess ? NEGF_OK : NEGF_EHIP;
}

negf_status negf_mlp_normalize(int64_t n, int32_t F, const float* X, const float* mu, const float* sd, float* Xn,
                               void* stream) {
  if (n < 0 || F < 1 || (n > 0 && (!X || !mu || !sd || !Xn))) return NEGF_EINVAL;
  if (n == 0) return NEGF_OK;
  hipLaunchKernelGGL(normalize_kernel, dim3(grid_1d(n * F)), dim3(256), 0, (hipStream_t)stream, (long)n, F, X, mu,
                     sd, Xn);
  return hipGetLastError() == hipSuccess ? NEGF_OK : NEGF_EHIP;
}

negf_status negf_mlp_signed_log(int64_t count, const float* x, float* y, int32_t inverse, void* stream) {
  if (count < 0 || (count > 0 && (!x || !y))) return NEGF_EINVAL;
  if (count == 0) return NEGF_OK;
  hipLaunchKernelGGL(signed_log_kernel, dim3(grid_1d(count)), dim3(256), 0, (hipStream_t)stream, (long)count, x, y,
                     inverse ? 1 : 0);
  return hipGetLastError() == hipSuccess ? NEGF_OK : NEGF_EHIP;
}

negf_status negf_mlp_mse(int64_t count, const float* Y, const float* T, double* out, double* scratch, void* stream) {
  if (count < 1 || !Y || !T || !out || !scratch) return NEGF_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(sqerr_part_kernel, dim3(PART), dim3(256), 0, s, (long)count, Y, T, scratch);
  hipLaunchKernelGGL(sqerr_finish_kernel, dim3(1), dim3(64), 0, s, (long)count, (const double*)scratch, out);
  return hipGetLastError() == hipSuccess ? NEGF_OK : NEGF_EHIP;
}

negf_status negf_mode_diag(int32_t n, int32_t b, const void* T, float* out, void* stream) {
  if (n < 0 || b < 1 || (n > 0 && (!T || !out))) return NEGF_EINVAL;
  if (n == 0) return NEGF_OK;
  hipLaunchKernelGGL(mode_diag_kernel, dim3(grid_1d((long)n * b)), dim3(256), 0, (hipStream_t)stream, (long)n, b,
                     (const double2*)T, out);
  return hipGetLastError() == hipSuccess ? NEGF_OK : NEGF_EHIP;
}

negf_status negf_mode_scale_columns(int32_t n, int32_t b, const void* U, const float* y, void* out, void* stream) {
  if (n < 0 || b < 1 || (n > 0 && (!U || !y || !out))) return NEGF_EINVAL;
  if (n == 0) return NEGF_OK;
  hipLaunchKernelGGL(mode_scale_kernel, dim3(grid_1d((long)n * b * b)), dim3(256), 0, (hipStream_t)stream, (long)n,
                     b, (const double2*)U, y, (double2*)out);
  return hipGetLastError() == hipSuccess ? NEGF_OK : NEGF_EHIP;
}

}  // extern "C"
