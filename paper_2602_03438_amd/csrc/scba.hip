// The self-consistent loop of Fig. 1 around Eq. (1)-(3), with a fixed boson
// bath: solve every energy with its scattering self-energies (the RGF sweeps),
// rebuild the self-energies from G^<> by the energy convolution of Eq. (3),
// measure how far they moved, mix, repeat.
//
// Everything an iteration computes runs on the device: the sweeps, two
// convolutions (lesser, greater) that read the energy-major diagonal blocks
// the sweeps wrote, one streaming pass for the residual and one for the
// mixing.  The host only reads the two sums of the residual to decide whether
// to stop.  Per energy the self-energies are nb b b complex elements; the
// problem handed to the sweeps points at them with sc_stride = nb b b.
#include "../../include/negf.h"
#include "internal.h"

#include <algorithm>
#include <cmath>

namespace negf {
namespace {

constexpr int SB = 256;       // threads per workgroup of the streaming kernels
constexpr int RPARTS = 1024;  // workgroups of the residual's first stage (fixed: the sum's order is fixed)
constexpr long MIX_WG = 8192; // grid cap of the mixing pass (grid-stride beyond)
constexpr int U = 4;          // elements per thread and pass of the streaming kernels

__device__ __forceinline__ double norm2(double2 z) { return z.x * z.x + z.y * z.y; }

// sum over one workgroup of SB threads; every thread gets the total
__device__ __forceinline__ double wg_sum(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int s = SB / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  const double t = red[0];
  __syncthreads();
  return t;
}

// part[2 w]     = sum over workgroup w's elements of |F^< - S^<|^2 + |F^> - S^>|^2
// part[2 w + 1] = sum of |F^<|^2 + |F^>|^2
// Each thread takes U elements SB apart per pass (lanes next to each other read neighbouring elements)
// and issues all of their loads before the arithmetic, so that 4 U independent 16-byte loads are in flight.
__global__ void __launch_bounds__(SB) resid_partial_kernel(long n, const double2* __restrict__ Fl,
                                                           const double2* __restrict__ Fg,
                                                           const double2* __restrict__ Sl,
                                                           const double2* __restrict__ Sg, double* part) {
  __shared__ double red[SB];
  double num = 0.0, den = 0.0;
  for (long x0 = (long)blockIdx.x * SB * U + threadIdx.x; x0 < n; x0 += (long)gridDim.x * SB * U) {
    double2 fl[U], fg[U], sl[U], sg[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const long x = x0 + (long)u * SB;
      const bool in = x < n;
      fl[u] = in ? Fl[x] : make_double2(0.0, 0.0);
      fg[u] = in ? Fg[x] : make_double2(0.0, 0.0);
      sl[u] = in ? Sl[x] : make_double2(0.0, 0.0);
      sg[u] = in ? Sg[x] : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      num += norm2(csub(fl[u], sl[u])) + norm2(csub(fg[u], sg[u]));
      den += norm2(fl[u]) + norm2(fg[u]);
    }
  }
  num = wg_sum(num, red);
  den = wg_sum(den, red);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = num;
    part[2 * blockIdx.x + 1] = den;
  }
}

// out[0], out[1] = the sums of the nparts partial pairs (one workgroup)
__global__ void __launch_bounds__(SB) resid_final_kernel(int nparts, const double* part, double* out) {
  __shared__ double red[SB];
  double num = 0.0, den = 0.0;
  for (int w = threadIdx.x; w < nparts; w += SB) {
    num += part[2 * w];
    den += part[2 * w + 1];
  }
  num = wg_sum(num, red);
  den = wg_sum(den, red);
  if (threadIdx.x == 0) {
    out[0] = num;
    out[1] = den;
  }
}

// with F: S^<> += m (F^<> - S^<>); then S^R = (S^> - S^<) / 2 (without F only the latter).  U elements
// SB apart per thread and pass, all loads first (as in the residual).
__global__ void __launch_bounds__(SB) mix_kernel(long n, double m, const double2* __restrict__ Fl,
                                                 const double2* __restrict__ Fg, double2* __restrict__ Sl,
                                                 double2* __restrict__ Sg, double2* __restrict__ Sr) {
  for (long x0 = (long)blockIdx.x * SB * U + threadIdx.x; x0 < n; x0 += (long)gridDim.x * SB * U) {
    double2 sl[U], sg[U], fl[U], fg[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const long x = x0 + (long)u * SB;
      if (x < n) {
        sl[u] = Sl[x];
        sg[u] = Sg[x];
        if (Fl) {
          fl[u] = Fl[x];
          fg[u] = Fg[x];
        }
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const long x = x0 + (long)u * SB;
      if (x >= n) continue;
      if (Fl) {
        sl[u] = make_double2(sl[u].x + m * (fl[u].x - sl[u].x), sl[u].y + m * (fl[u].y - sl[u].y));
        sg[u] = make_double2(sg[u].x + m * (fg[u].x - sg[u].x), sg[u].y + m * (fg[u].y - sg[u].y));
        Sl[x] = sl[u];
        Sg[x] = sg[u];
      }
      Sr[x] = make_double2(0.5 * (sg[u].x - sl[u].x), 0.5 * (sg[u].y - sl[u].y));
    }
  }
}

inline size_t up256(size_t n) { return (n + 255) & ~(size_t)255; }

struct ScbaLayout {
  size_t rgf, ec, sig, total;   // bytes: sweeps' workspace, convolution's, one [n_e][nb][b][b] array
};

bool scba_layout(const negf_problem* problem, negf_precision prec, const negf_options* opt, int32_t n_w,
                 ScbaLayout& L) {
  if (!problem || n_w < 1) return false;
  const negf_problem& p = *problem;
  if (p.n_e < 1 || p.dev.nb < 2 || p.dev.b < 1) return false;
  L.rgf = negf_workspace_bytes(NEGF_OP_LESSER_GREATER, problem, 1, prec, opt);
  L.ec = negf_econv_workspace_bytes(p.n_e, n_w);
  if (L.rgf == 0 || L.ec == 0) return false;
  L.sig = (size_t)p.n_e * p.dev.nb * p.dev.b * p.dev.b * sizeof(double2);
  L.total = up256(L.rgf) + up256(L.ec) + 2 * up256(L.sig) + up256(2 * RPARTS * sizeof(double)) +
            up256(2 * sizeof(double)) + 256;
  return true;
}

inline bool a16(const void* p) { return ((uintptr_t)p & 15) == 0; }

}  // namespace
}  // namespace negf

using namespace negf;

extern "C" {

size_t negf_scba_workspace_bytes(const negf_problem* problem, negf_precision prec, const negf_options* opt,
                                 int32_t n_w) {
  ScbaLayout L;
  return scba_layout(problem, prec, opt, n_w, L) ? L.total : 0;
}

negf_status negf_scba(const negf_problem* problem, negf_precision prec, const negf_options* opt, int32_t n_w,
                      int32_t k0, const void* W_lesser, const void* W_greater, const double* scale, double mixing,
                      double tol, int32_t max_iter, void* sig_r, void* sig_l, void* sig_g, void* GR_diag,
                      void* GR_upper, void* GR_lower, void* GL_diag, void* GL_upper, void* GG_diag, void* GG_upper,
                      int32_t* info, int32_t* n_iter, double* history, void* workspace, size_t ws_bytes,
                      void* stream) {
  if (!problem || !scale || !n_iter) return NEGF_EINVAL;
  const negf_problem& p0 = *problem;
  const negf_device& d0 = p0.dev;
  if (d0.sig_r_sc || d0.sig_l_sc || d0.sig_g_sc || p0.sc_stride != 0) return NEGF_EINVAL;
  if (k0 < 0 || k0 >= n_w || !(mixing > 0.0 && mixing <= 1.0) || !(tol >= 0.0) || max_iter < 1)
    return NEGF_EINVAL;
  ScbaLayout L;
  if (!scba_layout(problem, prec, opt, n_w, L)) return NEGF_EINVAL;
  const void* req[] = {W_lesser, W_greater, sig_r, sig_l, sig_g, GR_diag, GR_upper, GL_diag, GL_upper, GG_diag,
                       GG_upper, info, workspace};
  for (const void* q : req)
    if (!q || !a16(q)) return NEGF_EINVAL;
  if (GR_lower && !a16(GR_lower)) return NEGF_EINVAL;
  if (sig_r == sig_l || sig_r == sig_g || sig_l == sig_g) return NEGF_EINVAL;
  if (ws_bytes < L.total) return NEGF_EINVAL;

  const long nbb = (long)d0.nb * d0.b * d0.b;
  const long n = (long)p0.n_e * nbb;
  char* base = (char*)(((uintptr_t)workspace + 255) & ~(uintptr_t)255);
  void* ws_rgf = base;
  base += up256(L.rgf);
  void* ws_ec = base;
  base += up256(L.ec);
  double2* Fl = (double2*)base;
  base += up256(L.sig);
  double2* Fg = (double2*)base;
  base += up256(L.sig);
  double* part = (double*)base;
  base += up256(2 * RPARTS * sizeof(double));
  double* sums = (double*)base;

  negf_problem pq = p0;
  pq.dev.sig_r_sc = sig_r;
  pq.dev.sig_l_sc = sig_l;
  pq.dev.sig_g_sc = sig_g;
  pq.sc_stride = nbb;
  hipStream_t s = (hipStream_t)stream;
  double2* Sl = (double2*)sig_l;
  double2* Sg = (double2*)sig_g;
  double2* Sr = (double2*)sig_r;
  const unsigned mix_grid = (unsigned)std::min<long>((n + SB * U - 1) / (SB * U), MIX_WG);
  const unsigned part_grid = (unsigned)std::min<long>((n + SB * U - 1) / (SB * U), RPARTS);
  *n_iter = 0;

  prof_begin(KC_ELEM, s);
  hipLaunchKernelGGL(mix_kernel, dim3(mix_grid), dim3(SB), 0, s, n, 0.0, (const double2*)nullptr,
                     (const double2*)nullptr, Sl, Sg, Sr);
  prof_end(KC_ELEM, s, 0.0, 48.0 * (double)n);
  if (hipGetLastError() != hipSuccess) return NEGF_EHIP;
  for (int it = 0; it < max_iter; ++it) {
    negf_status st = negf_rgf_lesser_greater(&pq, 1, prec, opt, GR_diag, GR_upper, GR_lower, GL_diag, GL_upper,
                                             GG_diag, GG_upper, info, ws_rgf, L.rgf, stream);
    if (st != NEGF_OK) return st;
    st = negf_energy_convolution(p0.n_e, nbb, GL_diag, n_w, k0, W_lesser, scale, Fl, ws_ec, L.ec, stream);
    if (st != NEGF_OK) return st;
    st = negf_energy_convolution(p0.n_e, nbb, GG_diag, n_w, k0, W_greater, scale, Fg, ws_ec, L.ec, stream);
    if (st != NEGF_OK) return st;
    prof_begin(KC_ELEM, s);
    hipLaunchKernelGGL(resid_partial_kernel, dim3(part_grid), dim3(SB), 0, s, n, (const double2*)Fl,
                       (const double2*)Fg, (const double2*)Sl, (const double2*)Sg, part);
    hipLaunchKernelGGL(resid_final_kernel, dim3(1), dim3(SB), 0, s, (int)part_grid, (const double*)part, sums);
    prof_end(KC_ELEM, s, 0.0, 64.0 * (double)n);
    double h[2] = {0.0, 0.0};
    if (hipGetLastError() != hipSuccess || hipMemcpyAsync(h, sums, sizeof(h), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return NEGF_EHIP;
    const double r = h[1] > 0.0 ? std::sqrt(h[0] / h[1]) : (h[0] == 0.0 ? 0.0 : INFINITY);
    if (history) history[it] = r;
    *n_iter = it + 1;
    if (!std::isfinite(r)) return NEGF_ENONFINITE;
    if (r <= tol) return NEGF_OK;
    if (it == max_iter - 1) return NEGF_ENOCONV;
    prof_begin(KC_ELEM, s);
    hipLaunchKernelGGL(mix_kernel, dim3(mix_grid), dim3(SB), 0, s, n, mixing, (const double2*)Fl,
                       (const double2*)Fg, Sl, Sg, Sr);
    prof_end(KC_ELEM, s, 0.0, 112.0 * (double)n);
    if (hipGetLastError() != hipSuccess) return NEGF_EHIP;
  }
  return NEGF_ENOCONV;
}

}  // extern "C"
