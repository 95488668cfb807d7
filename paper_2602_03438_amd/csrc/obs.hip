// Observables of Section III from the outputs of the sweeps: the density of
// states resolved by block, DOS_i(E) = -Im Tr G^R_ii / pi, and the spectral
// current through the interface between blocks i and i+1,
//
//   j_i(E) = -2 Re Tr[A_{i,i+1} G^<_{i+1,i}] = 2 Re sum_{a,b} A_{i,i+1}[a][b] conj(G^<_{i,i+1}[a][b])
//
// (G^<_{i+1,i} = -(G^<_{i,i+1})^H; A_{i,i+1} = E S_{i,i+1} - H_{i,i+1}; e = hbar = 1, one spin), which
// is the same at every interface when the current is conserved (the paper's check of its
// implementation, Fig. 5(b)).  One workgroup per (point, block or interface) streams the b x b blocks
// once, coalesced, and sums in a fixed order.
#include "../../include/negf.h"
#include "internal.h"

namespace negf {
namespace {

constexpr int OB = 256;

__device__ __forceinline__ double wg_sum(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int s = OB / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  return red[0];
}

// dos[p][i] = -Im Tr G^R_ii / pi for the n points of one problem segment; grid (nb, n)
__global__ void __launch_bounds__(OB) dos_kernel(int nb, int b, const double2* GRd, double* dos) {
  __shared__ double red[OB];
  const int i = blockIdx.x, p = blockIdx.y;
  const double2* g = GRd + ((long)p * nb + i) * b * b;
  double acc = 0.0;
  for (int j = threadIdx.x; j < b; j += OB) acc += g[(long)j * b + j].y;
  acc = wg_sum(acc, red);
  if (threadIdx.x == 0) dos[(long)p * nb + i] = -acc / M_PI;
}

// current[p][i] = 2 Re sum A_{i,i+1} (.) conj(G^<_{i,i+1}) with A_{i,i+1} = E_p S_{i,i+1} - H_{i,i+1}
// (S_upper NULL: S_{i,i+1} = 0); grid (nb - 1, n)
__global__ void __launch_bounds__(OB) current_kernel(int nb, int b, const double* energies, const double2* H_upper,
                                                     const double2* S_upper, const double2* GLu, double* current) {
  __shared__ double red[OB];
  const int i = blockIdx.x, p = blockIdx.y;
  const long bb = (long)b * b;
  const double e = energies[p];
  const double2* h = H_upper + i * bb;
  const double2* sv = S_upper ? S_upper + i * bb : nullptr;
  const double2* g = GLu + ((long)p * (nb - 1) + i) * bb;
  double acc = 0.0;
  for (long x = threadIdx.x; x < bb; x += OB) {
    double2 a = make_double2(-h[x].x, -h[x].y);
    if (sv) {
      a.x += e * sv[x].x;
      a.y += e * sv[x].y;
    }
    const double2 q = g[x];
    acc += a.x * q.x + a.y * q.y;   // Re(a conj(q))
  }
  acc = wg_sum(acc, red);
  if (threadIdx.x == 0) current[(long)p * (nb - 1) + i] = 2.0 * acc;
}

}  // namespace
}  // namespace negf

using namespace negf;

extern "C" {

negf_status negf_observables(const negf_problem* problems, int32_t n_prob, const void* GR_diag, const void* GL_upper,
                             double* dos, double* current, void* stream) {
  if (!problems || n_prob <= 0) return NEGF_EINVAL;
  if ((dos && !GR_diag) || (current && !GL_upper)) return NEGF_EINVAL;
  if (((uintptr_t)GR_diag | (uintptr_t)GL_upper) & 15) return NEGF_EINVAL;
  if (((uintptr_t)dos | (uintptr_t)current) & 7) return NEGF_EINVAL;
  for (int q = 0; q < n_prob; ++q) {
    const negf_problem& p = problems[q];
    const negf_device& d = p.dev;
    if (d.nb < 2 || d.b < 1 || d.b > 1024 || p.n_e < 0 || p.n_e > 65535) return NEGF_EINVAL;
    if (p.n_e > 0 && !p.energies) return NEGF_EINVAL;
    if (current && p.n_e > 0 && !d.H_upper) return NEGF_EINVAL;
    if (((uintptr_t)d.H_upper | (uintptr_t)d.S_upper) & 15) return NEGF_EINVAL;
  }
  if (!dos && !current) return NEGF_OK;
  hipStream_t s = (hipStream_t)stream;
  // offsets into the outputs: complex elements of G (diagonal, upper) and entries of dos, current
  long off_d = 0, off_u = 0, off_dos = 0, off_cur = 0;
  prof_begin(KC_ELEM, s);
  double bytes = 0.0;
  for (int q = 0; q < n_prob; ++q) {
    const negf_problem& p = problems[q];
    const negf_device& d = p.dev;
    const long bb = (long)d.b * d.b;
    if (p.n_e > 0) {
      if (dos) {
        hipLaunchKernelGGL(dos_kernel, dim3(d.nb, p.n_e), dim3(OB), 0, s, d.nb, d.b,
                           (const double2*)GR_diag + off_d, dos + off_dos);
        bytes += 16.0 * (double)p.n_e * d.nb * d.b;
      }
      if (current) {
        hipLaunchKernelGGL(current_kernel, dim3(d.nb - 1, p.n_e), dim3(OB), 0, s, d.nb, d.b, p.energies,
                           (const double2*)d.H_upper, (const double2*)d.S_upper, (const double2*)GL_upper + off_u,
                           current + off_cur);
        bytes += 16.0 * (d.S_upper ? 3.0 : 2.0) * (double)p.n_e * (d.nb - 1) * bb;
      }
    }
    off_d += (long)p.n_e * d.nb * bb;
    off_u += (long)p.n_e * (d.nb - 1) * bb;
    off_dos += (long)p.n_e * d.nb;
    off_cur += (long)p.n_e * (d.nb - 1);
  }
  prof_end(KC_ELEM, s, 0.0, bytes);
  return hipGetLastError() == hipSuccess ? NEGF_OK : NEGF_EHIP;
}

}  // extern "C"
