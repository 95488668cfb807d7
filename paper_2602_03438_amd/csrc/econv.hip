// Energy convolution of Eq. (3) by FFT (the paper evaluates it in the time
// domain after a fast Fourier transform, Section II), and the (E; i,j) <->
// (i,j; E) layout change of Fig. 2.
//
//   B[e][x] = scale * sum_{k=0}^{n_w-1} G[e + k0 - k][x] * W[k][x]
//
// for every element x (a matrix entry of the selected blocks) of energy-major
// arrays G [n_e][n_el], W [n_w][n_el], B [n_e][n_el]: a linear convolution
// along the energy axis, element by element.  Both series are zero-padded to
// L = 2^m >= n_e + n_w - 1, so the circular convolution of the FFT equals the
// linear one on every output used.
//
// One workgroup takes TE consecutive elements and L / 8 threads per element;
// each thread holds 8 points of a series in registers, the positions
// lt + q L / 8 (q < 8).  That is exactly what a self-sorting (Stockham)
// transform reads in its first pass and writes in its last, so
//   * the loads from the energy-major arrays land in registers directly (the
//     layout change happens on the way in: nothing is transposed through HBM),
//     and lanes next to each other read elements next to each other;
//   * the passes are radix 8 (one radix-2 or radix-4 pass where log2 L is not a
//     multiple of 3), and LDS only carries the exchange between two passes
//     (log2(L)/3 - 1 exchanges per transform instead of one LDS round trip per
//     radix-2 stage) and the twiddle table;
//   * the spectra of G and W meet in the same registers, the product needs no
//     exchange, and the inverse (a forward transform between two complex
//     conjugations) starts from those registers and leaves every thread holding
//     its own output energies, which it writes energy-major.
// HBM traffic is the algorithmic one (G, W read once, B written once) when the
// tiles that share cache lines run on the same XCD, which the tile order
// arranges.
#include "../../include/negf.h"
#include "internal.h"

namespace negf {
namespace {

__global__ void twiddle_kernel(int L, double2* tw) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= L) return;
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
  const double2* tw;      // exp(-2 pi i j / L), j < L
  double2 scale;          // already divided by L
  long tiles;
};

// LDS slot of index i (16-byte slots, element fastest).  With one element per workgroup the
// 16-byte slots of eight neighbouring lanes fall in distinct banks for every pass's write and read
// pattern once bits 3..5 of the index are folded into bits 0..2; with two or more elements the plain
// index has at most two-way conflicts, and keeps each pass's eight stores at constant offsets from
// one address (no per-store address registers held across the three transforms)
template <int TE>
__device__ __forceinline__ int swz(int i) {
  if constexpr (TE == 1) return i ^ ((i >> 3) & 7);
  else return i;
}

__device__ __forceinline__ double2 mul_mi(double2 z) { return make_double2(z.y, -z.x); }   // -i z

// in-place forward DFT of R points, R in {2, 4, 8}
template <int R>
__device__ __forceinline__ void dft(double2* x) {
  if constexpr (R == 2) {
    const double2 a = x[0], b = x[1];
    x[0] = cadd(a, b);
    x[1] = csub(a, b);
  } else if constexpr (R == 4) {
    const double2 s02 = cadd(x[0], x[2]), d02 = csub(x[0], x[2]);
    const double2 s13 = cadd(x[1], x[3]), d13 = mul_mi(csub(x[1], x[3]));
    x[0] = cadd(s02, s13);
    x[2] = csub(s02, s13);
    x[1] = cadd(d02, d13);
    x[3] = csub(d02, d13);
  } else {
    // even outputs: 4-point DFT of v_r + v_{r+4}; odd outputs: of (v_r - v_{r+4}) exp(-i pi r / 4)
    constexpr double h = 0.70710678118654752440;
    double2 e[4], o[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      e[r] = cadd(x[r], x[r + 4]);
      o[r] = csub(x[r], x[r + 4]);
    }
    o[1] = make_double2(h * (o[1].x + o[1].y), h * (o[1].y - o[1].x));
    o[2] = mul_mi(o[2]);
    o[3] = make_double2(h * (o[3].y - o[3].x), -h * (o[3].x + o[3].y));
    dft<4>(e);
    dft<4>(o);
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      x[2 * m] = e[m];
      x[2 * m + 1] = o[m];
    }
  }
}

// One Stockham pass of radix R over sub-transforms of length NS * R (NS = product of the earlier
// radices).  A thread runs C = 8 / R butterflies j = lt + c L/8; butterfly j reads the positions
// j + r L/R (register slot c + C r), twiddles them by exp(-2 pi i k r / (NS R)) with k = j mod NS
// (the table entries k r L / (NS R) for r = 1, 2, 4, all below L / 2; the others are their products),
// and writes its R outputs to (j - k) R + k + m NS.  In the last pass those positions are
// lt + (c + C m) L/8 again, so the outputs stay in the thread's registers.
template <int R, int NS, int L, int TE, bool LAST>
__device__ __forceinline__ void pass(double2 (&v)[8], double2* lds, const double2* tw, int s, int lt) {
  constexpr int C = 8 / R, T = L / 8, STEP = L / (NS * R);
  double2 o[8];
#pragma unroll
  for (int c = 0; c < C; ++c) {
    const int j = lt + c * T;
    const int k = j & (NS - 1);
    double2 x[R];
#pragma unroll
    for (int r = 0; r < R; ++r) x[r] = v[c + C * r];
    if constexpr (NS > 1) {
      const double2 w1 = tw[k * STEP];
      if constexpr (R == 2) {
        x[1] = cmul(x[1], w1);
      } else {
        const double2 w2 = tw[2 * k * STEP];
        x[1] = cmul(x[1], w1);
        x[2] = cmul(x[2], w2);
        x[3] = cmul(x[3], cmul(w2, w1));
        if constexpr (R == 8) {
          const double2 w4 = tw[4 * k * STEP];
          x[4] = cmul(x[4], w4);
          x[5] = cmul(x[5], cmul(w4, w1));
          x[6] = cmul(x[6], cmul(w4, w2));
          x[7] = cmul(x[7], cmul(w4, cmul(w2, w1)));
        }
      }
    }
    dft<R>(x);
    if constexpr (LAST) {
#pragma unroll
      for (int m = 0; m < R; ++m) o[c + C * m] = x[m];
    } else {
      const int base = (j - k) * R + k;
#pragma unroll
      for (int m = 0; m < R; ++m) lds[swz<TE>((base + m * NS) * TE + s)] = x[m];
    }
  }
  if constexpr (LAST) {
#pragma unroll
    for (int q = 0; q < 8; ++q) v[q] = o[q];
  } else {
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 8; ++q) v[q] = lds[swz<TE>((lt + q * T) * TE + s)];
    __syncthreads();   // the next pass (or transform) overwrites the buffer
  }
}

// forward transform of length L from the sub-transform length NS on: radix 8 while at least 16
// points remain per sub-transform, then one pass of what is left (2, 4 or 8)
template <int L, int TE, int NS>
__device__ __forceinline__ void fft_from(double2 (&v)[8], double2* lds, const double2* tw, int s, int lt) {
  constexpr int REM = L / NS;
  if constexpr (REM == 2) {
    pass<2, NS, L, TE, true>(v, lds, tw, s, lt);
  } else if constexpr (REM == 4) {
    pass<4, NS, L, TE, true>(v, lds, tw, s, lt);
  } else if constexpr (REM == 8) {
    pass<8, NS, L, TE, true>(v, lds, tw, s, lt);
  } else {
    pass<8, NS, L, TE, false>(v, lds, tw, s, lt);
    fft_from<L, TE, NS * 8>(v, lds, tw, s, lt);
  }
}

template <int LOG2L, int NT>
__global__ void __launch_bounds__(NT) econv_kernel(EArgs a) {
  constexpr int L = 1 << LOG2L, T = L / 8, TE = NT / T;
  static_assert(TE >= 1 && TE * T == NT, "threads per workgroup must be a multiple of L / 8");
  __shared__ double2 lds[L * TE];
  __shared__ double2 stw[L / 2];
  // consecutive workgroups go round-robin over the 8 XCDs; give each XCD a contiguous run of tiles so
  // that the tiles whose elements share cache lines meet in one L2
  long tile = blockIdx.x;
  if ((a.tiles & 7) == 0) tile = (tile & 7) * (a.tiles >> 3) + (tile >> 3);
  const int t = threadIdx.x, s = t % TE, lt = t / TE;
  const long x = tile * TE + s;
  const bool in = x < a.n_el;
  double2 g[8], w[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int e = lt + q * T;
    g[q] = (in && e < a.n_e) ? a.G[(long)e * a.n_el + x] : make_double2(0.0, 0.0);
    w[q] = (in && e < a.n_w) ? a.W[(long)e * a.n_el + x] : make_double2(0.0, 0.0);
  }
  // the twiddles every pass after the first reads (indices below L / 2) go to LDS: the first pass
  // needs none, and its exchange barrier orders these writes before any read
  for (int i = t; i < L / 2; i += NT) stw[i] = a.tw[i];
  fft_from<L, TE, 1>(g, lds, stw, s, lt);
  fft_from<L, TE, 1>(w, lds, stw, s, lt);
  // inverse transform as conj(F(conj(.))): the product is conjugated here, the result at the store
#pragma unroll
  for (int q = 0; q < 8; ++q) g[q] = cconj(cmul(g[q], w[q]));
  fft_from<L, TE, 1>(g, lds, stw, s, lt);
  if (!in) return;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int e = lt + q * T - a.k0;
    if (e >= 0 && e < a.n_e) a.B[(long)e * a.n_el + x] = cmul(a.scale, cconj(g[q]));
  }
}

template <int LOG2L, int NT>
hipError_t launch_econv(EArgs a, hipStream_t s) {
  constexpr int TE = NT / ((1 << LOG2L) / 8);
  a.tiles = (a.n_el + TE - 1) / TE;
  hipLaunchKernelGGL((econv_kernel<LOG2L, NT>), dim3((unsigned)a.tiles), dim3(NT), 0, s, a);
  return hipGetLastError();
}

// Two elements or more per workgroup (lanes next to each other read 32 contiguous bytes or more of
// one energy row) and room for two workgroups per CU in LDS (exchange buffer and twiddle table:
// 72 KB at L = 1024, 80 KB at L = 2048), so that one workgroup's loads overlap the other's
// transforms; L = 4096 keeps one element per 512 threads (96 KB)
hipError_t dispatch_econv(int log2l, EArgs a, hipStream_t s) {
  switch (log2l) {
    case 4: return launch_econv<4, 256>(a, s);
    case 5: return launch_econv<5, 256>(a, s);
    case 6: return launch_econv<6, 256>(a, s);
    case 7: return launch_econv<7, 256>(a, s);
    case 8: return launch_econv<8, 256>(a, s);
    case 9: return launch_econv<9, 256>(a, s);
    case 10: return launch_econv<10, 512>(a, s);
    case 11: return launch_econv<11, 512>(a, s);
    case 12: return launch_econv<12, 512>(a, s);
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
  return (size_t)(1 << m) * sizeof(double2) + 256;
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
  hipLaunchKernelGGL(twiddle_kernel, dim3((L + 255) / 256), dim3(256), 0, s, L, tw);
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
