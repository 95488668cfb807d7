// Energy convolution of Eq. (3) by FFT (the paper evaluates it in the time
// domain after a fast Fourier transform, Section II), and the (E; i,j) <->
// (i,j; E) layout change of Fig. 2.
//
//   B[e][x] = scale * sum_{k=0}^{n_w-1} G[e + k0 - k][x] * W[k][x]
//
// for every element x (a matrix entry of the selected blocks) of energy-major
// arrays G [n_e][n_el], W [n_w][n_el], B [n_e][n_el]: a linear convolution
// along the energy axis, element by element.  One workgroup takes a tile of
// TE consecutive elements: it reads their G and W series straight from the
// energy-major layout (the layout change happens on the way into LDS, so
// nothing is transposed through HBM), zero-pads both to L = 2^m >= n_e +
// n_w - 1 (so the circular convolution of the FFT is the linear one on every
// output used), transforms both in LDS (radix-2, decimation in time from
// bit-reversed positions), multiplies the spectra, transforms back
// (decimation in frequency with conjugate twiddles, natural order in,
// bit-reversed out) and writes scale / L times the slice [k0, k0 + n_e) back
// energy-major.  HBM traffic is the algorithmic one (G, W read once, B written
// once) when the tiles that share cache lines run on the same XCD, which the
// tile order arranges.
#include "../../include/negf.h"
#include "internal.h"

namespace negf {
namespace {

constexpr int ENT = 256;   // threads per workgroup

__global__ void twiddle_kernel(int L, double2* tw) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= L / 2) return;
  double s, c;
  sincospi(-2.0 * (double)j / (double)L, &s, &c);
  tw[j] = make_double2(c, s);
}

struct EArgs {
  int n_e, n_w, k0;
  long n_el;
  const double2* G;
  const double2* W;
  double2* B;
  const double2* tw;      // exp(-2 pi i j / L), j < L / 2
  double2 scale;          // already divided by L
  long tiles;
};

__device__ __forceinline__ unsigned brev(unsigned v, int bits) { return __builtin_bitreverse32(v) >> (32 - bits); }

template <int LOG2L, int TE>
__global__ void __launch_bounds__(ENT) econv_kernel(EArgs a) {
  constexpr int L = 1 << LOG2L, H = L / 2;
  __shared__ double2 sG[TE][L];
  __shared__ double2 sW[TE][L];
  // consecutive workgroups go round-robin over the 8 XCDs; give each XCD a contiguous run of tiles so
  // that the tiles whose elements share cache lines meet in one L2
  long tile = blockIdx.x;
  if ((a.tiles & 7) == 0) tile = (tile & 7) * (a.tiles >> 3) + (tile >> 3);
  const long x0 = tile * TE;
  const int t = threadIdx.x;
  // load: element fastest, so that a wavefront reads runs of TE consecutive elements per energy
  for (int i = t; i < TE * L; i += ENT) {
    const int s = i % TE, e = i / TE;
    const long x = x0 + s;
    const bool in = x < a.n_el;
    const unsigned r = brev((unsigned)e, LOG2L);
    sG[s][r] = (in && e < a.n_e) ? a.G[(long)e * a.n_el + x] : make_double2(0.0, 0.0);
    sW[s][r] = (in && e < a.n_w) ? a.W[(long)e * a.n_el + x] : make_double2(0.0, 0.0);
  }
  __syncthreads();
  // forward transforms of both series (decimation in time, bit-reversed in, natural order out)
#pragma unroll 1
  for (int st = 1; st <= LOG2L; ++st) {
    const int half = 1 << (st - 1), shift = LOG2L - st;
    for (int i = t; i < TE * H; i += ENT) {
      const int s = i / H, bf = i % H;
      const int j = bf & (half - 1);
      const int i0 = ((bf >> (st - 1)) << st) + j, i1 = i0 + half;
      const double2 w = a.tw[j << shift];
      double2 u = sG[s][i0], v = cmul(sG[s][i1], w);
      sG[s][i0] = cadd(u, v);
      sG[s][i1] = csub(u, v);
      u = sW[s][i0];
      v = cmul(sW[s][i1], w);
      sW[s][i0] = cadd(u, v);
      sW[s][i1] = csub(u, v);
    }
    __syncthreads();
  }
  for (int i = t; i < TE * L; i += ENT) {
    const int s = i / L, k = i % L;
    sG[s][k] = cmul(sG[s][k], sW[s][k]);
  }
  __syncthreads();
  // inverse transform (decimation in frequency with conjugate twiddles: natural in, bit-reversed out)
#pragma unroll 1
  for (int st = LOG2L; st >= 1; --st) {
    const int half = 1 << (st - 1), shift = LOG2L - st;
    for (int i = t; i < TE * H; i += ENT) {
      const int s = i / H, bf = i % H;
      const int j = bf & (half - 1);
      const int i0 = ((bf >> (st - 1)) << st) + j, i1 = i0 + half;
      const double2 w = cconj(a.tw[j << shift]);
      const double2 u = sG[s][i0], v = sG[s][i1];
      sG[s][i0] = cadd(u, v);
      sG[s][i1] = cmul(csub(u, v), w);
    }
    __syncthreads();
  }
  for (int i = t; i < TE * a.n_e; i += ENT) {
    const int s = i % TE, e = i / TE;
    const long x = x0 + s;
    if (x < a.n_el) a.B[(long)e * a.n_el + x] = cmul(a.scale, sG[s][brev((unsigned)(e + a.k0), LOG2L)]);
  }
}

template <int LOG2L, int TE>
hipError_t launch_econv(EArgs a, hipStream_t s) {
  a.tiles = (a.n_el + TE - 1) / TE;
  hipLaunchKernelGGL((econv_kernel<LOG2L, TE>), dim3((unsigned)a.tiles), dim3(ENT), 0, s, a);
  return hipGetLastError();
}

// TE elements per workgroup: 64 KB of LDS (two workgroups per CU) for L <= 2048, 128 KB at L = 4096
hipError_t dispatch_econv(int log2l, EArgs a, hipStream_t s) {
  switch (log2l) {
    case 4: return launch_econv<4, 8>(a, s);
    case 5: return launch_econv<5, 8>(a, s);
    case 6: return launch_econv<6, 8>(a, s);
    case 7: return launch_econv<7, 8>(a, s);
    case 8: return launch_econv<8, 8>(a, s);
    case 9: return launch_econv<9, 4>(a, s);
    case 10: return launch_econv<10, 2>(a, s);
    case 11: return launch_econv<11, 1>(a, s);
    case 12: return launch_econv<12, 1>(a, s);
    default: return hipErrorInvalidValue;
  }
}

constexpr int MAX_LOG2L = 12;

int log2_len(int n_e, int n_w) {
  const int need = n_e + n_w - 1;
  int m = 4;
  while ((1 << m) < need) ++m;
  return m;
}

// dst[c][r] = src[r][c], complex128, through 32 x 32 LDS tiles
constexpr int TT = 32, TRW = 8;
__global__ void __launch_bounds__(TT * TRW) transpose_kernel(long rows, long cols, long gx, const double2* src,
                                                             double2* dst) {
  __shared__ double2 tile[TT][TT + 1];
  const long bid = blockIdx.x;
  const long r0 = (bid / gx) * TT, c0 = (bid % gx) * TT;
  for (int i = threadIdx.y; i < TT; i += TRW) {
    const long r = r0 + i, c = c0 + threadIdx.x;
    if (r < rows && c < cols) tile[i][threadIdx.x] = src[r * cols + c];
  }
  __syncthreads();
  for (int i = threadIdx.y; i < TT; i += TRW) {
    const long c = c0 + i, r = r0 + threadIdx.x;
    if (r < rows && c < cols) dst[c * rows + r] = tile[threadIdx.x][i];
  }
}

}  // namespace
}  // namespace negf

using namespace negf;

extern "C" {

size_t negf_econv_workspace_bytes(int32_t n_e, int32_t n_w) {
  if (n_e < 1 || n_w < 1) return 0;
  const int m = log2_len(n_e, n_w);
  if (m > MAX_LOG2L) return 0;
  return ((size_t)(1 << m) / 2) * sizeof(double2) + 256;
}

negf_status negf_energy_convolution(int32_t n_e, int64_t n_el, const void* G, int32_t n_w, int32_t k0, const void* W,
                                    const double* scale, void* B, void* workspace, size_t ws_bytes, void* stream) {
  if (n_e < 1 || n_w < 1 || n_el < 0 || k0 < 0 || k0 >= n_w || !scale) return NEGF_EINVAL;
  const int m = log2_len(n_e, n_w);
  if (m > MAX_LOG2L) return NEGF_EINVAL;
  if (n_el == 0) return NEGF_OK;
  if (!G || !W || !B || !workspace || B == G || B == W) return NEGF_EINVAL;
  if (((uintptr_t)G | (uintptr_t)W | (uintptr_t)B) & 15) return NEGF_EINVAL;
  if (ws_bytes < negf_econv_workspace_bytes(n_e, n_w)) return NEGF_EINVAL;
  if (n_el > 0x7fffffffL) return NEGF_EINVAL;   // one workgroup per element tile: the grid's limit
  hipStream_t s = (hipStream_t)stream;
  double2* tw = (double2*)(((uintptr_t)workspace + 255) & ~(uintptr_t)255);
  const int L = 1 << m;
  hipLaunchKernelGGL(twiddle_kernel, dim3((L / 2 + 255) / 256), dim3(256), 0, s, L, tw);
  EArgs a{};
  a.n_e = n_e; a.n_w = n_w; a.k0 = k0; a.n_el = n_el;
  a.G = (const double2*)G; a.W = (const double2*)W; a.B = (double2*)B;
  a.tw = tw;
  a.scale = make_double2(scale[0] / L, scale[1] / L);
  prof_begin(KC_ELEM, s);
  hipError_t e = dispatch_econv(m, a, s);
  prof_end(KC_ELEM, s, 0.0, 16.0 * (double)n_el * (2.0 * n_e + n_w));
  return e == hipSuccess ? NEGF_OK : NEGF_EHIP;
}

negf_status negf_transpose(int64_t rows, int64_t cols, const void* src, void* dst, void* stream) {
  if (rows < 0 || cols < 0) return NEGF_EINVAL;
  if (rows == 0 || cols == 0) return NEGF_OK;
  if (!src || !dst || src == dst || (((uintptr_t)src | (uintptr_t)dst) & 15)) return NEGF_EINVAL;
  const long gx = (cols + TT - 1) / TT, gy = (rows + TT - 1) / TT;
  if (gx * gy > 0x7fffffffL) return NEGF_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  prof_begin(KC_ELEM, s);
  hipLaunchKernelGGL(transpose_kernel, dim3((unsigned)(gx * gy)), dim3(TT, TRW), 0, s, (long)rows, (long)cols, gx,
                     (const double2*)src, (double2*)dst);
  prof_end(KC_ELEM, s, 0.0, 32.0 * (double)rows * cols);
  return hipGetLastError() == hipSuccess ? NEGF_OK : NEGF_EHIP;
}

}  // extern "C"
