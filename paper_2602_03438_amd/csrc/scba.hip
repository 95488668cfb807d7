// The self-consistent loop of Fig. 1 around Eq. (1)-(3), with a fixed boson
// bath: solve every energy with its scattering self-energies (the RGF sweeps),
// rebuild the self-energies from G^<> by the energy convolution of Eq. (3),
// measure how far they moved, mix, repeat.
//
// One iteration (negf_scba_step) runs entirely on the device and is enqueued
// without any host synchronisation: the sweeps, two convolutions (lesser,
// greater) that read the energy-major diagonal blocks the sweeps wrote, one
// streaming pass for the residual, whose last workgroup also records the
// residual and the loop state in device memory, and the mixing, which reads
// that state and leaves the self-energies alone once the loop has converged
// (so that a fixed number of captured iterations ends on the same self-energies
// and Green's functions as a loop stopped at convergence).  The mixing is one
// linear pass, or Anderson's extrapolation in four launches (history, normal
// equations, their solution in one workgroup, update), its history of
// differences kept in the workspace as a ring of M slots.  negf_scba drives the
// steps from the host and reads the state after each one to stop early.  Per
// energy the self-energies are nb b b complex elements; the problem handed to
// the sweeps points at them with sc_stride = nb b b.
#include "../../include/negf.h"
#include "internal.h"

#include <algorithm>
#include <cmath>
#include <vector>

namespace negf {
namespace {

constexpr int SB = 256;       // threads per workgroup of the streaming kernels
constexpr int RPARTS = 1024;  // workgroups of the residual's first stage (fixed: the sum's order is fixed)
constexpr long MIX_WG = 8192; // grid cap of the mixing pass (grid-stride beyond)
constexpr int U = 4;          // elements per thread and pass of the streaming kernels
constexpr int MAXM = 4;       // longest Anderson memory  (the launch tables below list one kernel per length)
constexpr int NACC = MAXM * (MAXM + 1) / 2 + MAXM;   // accumulators of its normal equations

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

// The residual r = sqrt(sum |F - S|^2 / sum |F|^2) of iteration `it` from the nparts partial pairs (one
// workgroup, fixed order): last[0] = r, history[it] = r (history nullable), and the loop state, while it is
// still running (state[1] == 0): state[0] = it + 1 (solves so far), state[1] = 1 once r <= tol, 2 if r is not
// finite.  A converged or failed loop keeps its state.
__global__ void __launch_bounds__(SB) resid_final_kernel(int nparts, const double* part, double tol, int it,
                                                         double* last, double* history, int* state) {
  __shared__ double red[SB];
  double num = 0.0, den = 0.0;
  for (int w = threadIdx.x; w < nparts; w += SB) {
    num += part[2 * w];
    den += part[2 * w + 1];
  }
  num = wg_sum(num, red);
  den = wg_sum(den, red);
  if (threadIdx.x == 0) {
    const double r = den > 0.0 ? sqrt(num / den) : (num == 0.0 ? 0.0 : INFINITY);
    last[0] = r;
    if (history) history[it] = r;
    if (state[1] == 0) {
      state[0] = it + 1;
      state[1] = !isfinite(r) ? 2 : (r <= tol ? 1 : 0);
    }
  }
}

// state = {0, 0}: a new loop
__global__ void scba_reset_kernel(int* state) {
  if (threadIdx.x == 0) {
    state[0] = 0;
    state[1] = 0;
  }
}

// with F: S^<> += m (F^<> - S^<>); then S^R = (S^> - S^<) / 2 (without F only the latter).  Nothing is
// written once the loop state (nullable) says converged or failed.  U elements SB apart per thread and
// pass, all loads first (as in the residual).
__global__ void __launch_bounds__(SB) mix_kernel(long n, double m, const double2* __restrict__ Fl,
                                                 const double2* __restrict__ Fg, double2* __restrict__ Sl,
                                                 double2* __restrict__ Sg, double2* __restrict__ Sr,
                                                 const int* state) {
  if (state && state[1] != 0) return;
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

// out[x] = (1 / nk) sum_q G[q stride + x]: the average over the k-points (problems) of each energy's
// diagonal blocks, summed in problem order
__global__ void __launch_bounds__(SB) kavg_kernel(long n, int nk, long stride, const double2* __restrict__ G,
                                                  double2* __restrict__ out) {
  const double inv = 1.0 / nk;
  for (long x = (long)blockIdx.x * SB + threadIdx.x; x < n; x += (long)gridDim.x * SB) {
    double2 acc = G[x];
    for (int q = 1; q < nk; ++q) acc = cadd(acc, G[q * stride + x]);
    out[x] = make_double2(acc.x * inv, acc.y * inv);
  }
}

// ---- Anderson (Pulay) mixing: x = (Sigma^<, Sigma^>), f = F - x, both kinds stored one after the other
// (2n complex per vector).  History: the differences dx_j, df_j of consecutive pairs (x, f), M slots used
// as a ring; xp, fp: the previous pair.

// the previous pair's differences into slot `slot` (unless `first`), then the current pair as the previous
__global__ void __launch_bounds__(SB) anderson_hist_kernel(long n, int first, int slot, const double2* Sl,
                                                           const double2* Sg, const double2* Fl, const double2* Fg,
                                                           double2* xp, double2* fp, double2* DX, double2* DF,
                                                           const int* state) {
  if (state[1] != 0) return;
  for (long x = (long)blockIdx.x * SB + threadIdx.x; x < n; x += (long)gridDim.x * SB) {
#pragma unroll
    for (int kind = 0; kind < 2; ++kind) {
      const double2 sv = kind ? Sg[x] : Sl[x];
      const double2 fv = csub(kind ? Fg[x] : Fl[x], sv);
      const long i = kind * n + x;
      if (!first) {
        DX[slot * 2 * n + i] = csub(sv, xp[i]);
        DF[slot * 2 * n + i] = csub(fv, fp[i]);
      }
      xp[i] = sv;
      fp[i] = fv;
    }
  }
}

// per workgroup: A_ij = Re <df_i, df_j> (i <= j < K, packed row by row over MAXM) and r_i = Re <df_i, f>;
// K is a template argument so that every load of an element is issued before its arithmetic
template <int K>
__global__ void __launch_bounds__(SB) anderson_gram_kernel(long n, const double2* Sl, const double2* Sg,
                                                           const double2* Fl, const double2* Fg, const double2* DF,
                                                           double* part, const int* state) {
  if (state[1] != 0) return;
  __shared__ double red[SB];
  double acc[NACC];
#pragma unroll
  for (int a = 0; a < NACC; ++a) acc[a] = 0.0;
  for (long x = (long)blockIdx.x * SB + threadIdx.x; x < n; x += (long)gridDim.x * SB) {
#pragma unroll
    for (int kind = 0; kind < 2; ++kind) {
      const double2 fv = csub(kind ? Fg[x] : Fl[x], kind ? Sg[x] : Sl[x]);
      const long i = kind * n + x;
      double2 d[MAXM];
#pragma unroll
      for (int j = 0; j < MAXM; ++j) d[j] = j < K ? DF[j * 2 * n + i] : make_double2(0.0, 0.0);
      int a = 0;
#pragma unroll
      for (int p = 0; p < MAXM; ++p)
#pragma unroll
        for (int q = p; q < MAXM; ++q) acc[a++] += d[p].x * d[q].x + d[p].y * d[q].y;
#pragma unroll
      for (int p = 0; p < MAXM; ++p) acc[a++] += d[p].x * fv.x + d[p].y * fv.y;
    }
  }
#pragma unroll
  for (int a = 0; a < NACC; ++a) {
    const double t = wg_sum(acc[a], red);
    if (threadIdx.x == 0) part[(long)blockIdx.x * NACC + a] = t;
  }
}

// one workgroup: the partial sums added in a fixed order, then gamma from (A + 1e-12 trace(A) / k I) gamma = r
// by Gaussian elimination with partial pivoting (k <= MAXM)
__global__ void __launch_bounds__(SB) anderson_solve_kernel(int nparts, int k, const double* part, double* gamma,
                                                            const int* state) {
  if (state[1] != 0) return;
  __shared__ double tot[NACC];
  if ((int)threadIdx.x < NACC) {
    double t = 0.0;
    for (int w = 0; w < nparts; ++w) t += part[(long)w * NACC + threadIdx.x];
    tot[threadIdx.x] = t;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  double A[MAXM][MAXM + 1];
  int a = 0;
  for (int p = 0; p < MAXM; ++p)
    for (int q = p; q < MAXM; ++q, ++a) {
      A[p][q] = tot[a];
      A[q][p] = tot[a];
    }
  for (int p = 0; p < MAXM; ++p) A[p][MAXM] = tot[a++];
  double tr = 0.0;
  for (int p = 0; p < k; ++p) tr += A[p][p];
  for (int p = 0; p < k; ++p) A[p][p] += 1e-12 * tr / k;
  for (int c = 0; c < k; ++c) {
    int piv = c;
    for (int r = c + 1; r < k; ++r)
      if (fabs(A[r][c]) > fabs(A[piv][c])) piv = r;
    if (piv != c)
      for (int q = 0; q <= MAXM; ++q) {
        const double t = A[c][q];
        A[c][q] = A[piv][q];
        A[piv][q] = t;
      }
    for (int r = c + 1; r < k; ++r) {
      const double l = A[r][c] / A[c][c];
      for (int q = c; q < k; ++q) A[r][q] -= l * A[c][q];
      A[r][MAXM] -= l * A[c][MAXM];
    }
  }
  for (int c = k - 1; c >= 0; --c) {
    double v = A[c][MAXM];
    for (int q = c + 1; q < k; ++q) v -= A[c][q] * gamma[q];
    gamma[c] = v / A[c][c];
  }
}

// x += m f - sum_j gamma_j (dx_j + m df_j) for both kinds (j < K), then Sigma^R = (Sigma^> - Sigma^<) / 2
template <int K>
__global__ void __launch_bounds__(SB) anderson_update_kernel(long n, double m, const double* __restrict__ gamma,
                                                             double2* __restrict__ Sl, double2* __restrict__ Sg,
                                                             const double2* __restrict__ Fl,
                                                             const double2* __restrict__ Fg,
                                                             const double2* __restrict__ DX,
                                                             const double2* __restrict__ DF, double2* __restrict__ Sr,
                                                             const int* state) {
  if (state[1] != 0) return;
  constexpr int UA = 2;   // elements per thread and pass: all of their loads are issued first
  double g[MAXM];
#pragma unroll
  for (int j = 0; j < MAXM; ++j) g[j] = j < K ? gamma[j] : 0.0;
  for (long x0 = (long)blockIdx.x * SB * UA + threadIdx.x; x0 < n; x0 += (long)gridDim.x * SB * UA) {
    double2 sv[UA][2], fv[UA][2], dx[UA][2][K > 0 ? K : 1], df[UA][2][K > 0 ? K : 1];
#pragma unroll
    for (int u = 0; u < UA; ++u) {
      const long x = x0 + (long)u * SB;
      if (x < n) {
#pragma unroll
        for (int kind = 0; kind < 2; ++kind) {
          const long i = kind * n + x;
          sv[u][kind] = kind ? Sg[x] : Sl[x];
          fv[u][kind] = kind ? Fg[x] : Fl[x];
#pragma unroll
          for (int j = 0; j < K; ++j) {
            dx[u][kind][j] = DX[j * 2 * n + i];
            df[u][kind][j] = DF[j * 2 * n + i];
          }
        }
      }
    }
#pragma unroll
    for (int u = 0; u < UA; ++u) {
      const long x = x0 + (long)u * SB;
      if (x >= n) continue;
      double2 out[2];
#pragma unroll
      for (int kind = 0; kind < 2; ++kind) {
        const double2 f = csub(fv[u][kind], sv[u][kind]);
        double2 v = make_double2(sv[u][kind].x + m * f.x, sv[u][kind].y + m * f.y);
#pragma unroll
        for (int j = 0; j < K; ++j) {
          v.x -= g[j] * (dx[u][kind][j].x + m * df[u][kind][j].x);
          v.y -= g[j] * (dx[u][kind][j].y + m * df[u][kind][j].y);
        }
        out[kind] = v;
      }
      Sl[x] = out[0];
      Sg[x] = out[1];
      Sr[x] = make_double2(0.5 * (out[1].x - out[0].x), 0.5 * (out[1].y - out[0].y));
    }
  }
}

inline size_t up256(size_t n) { return (n + 255) & ~(size_t)255; }

struct ScbaLayout {
  size_t rgf, ec, sig, total;   // bytes: sweeps' workspace, convolution's, one [n_e][nb][b][b] array
  bool kavg;                    // several k-points: one more such array for their average
  int memory;                   // Anderson memory (0: linear mixing)
};

// the problems (k-points) of one loop share the block shape and the energy count
bool scba_layout(const negf_problem* problems, int32_t n_prob, negf_precision prec, const negf_options* opt,
                 int32_t n_w, int32_t memory, ScbaLayout& L) {
  if (!problems || n_prob < 1 || n_w < 1 || memory < 0 || memory > MAXM) return false;
  const negf_problem& p = problems[0];
  if (p.n_e < 1 || p.dev.nb < 2 || p.dev.b < 1) return false;
  for (int q = 1; q < n_prob; ++q)
    if (problems[q].n_e != p.n_e || problems[q].dev.nb != p.dev.nb || problems[q].dev.b != p.dev.b) return false;
  L.rgf = negf_workspace_bytes(NEGF_OP_LESSER_GREATER, problems, n_prob, prec, opt);
  L.ec = negf_econv_workspace_bytes(p.n_e, n_w);
  if (L.rgf == 0 || L.ec == 0) return false;
  L.sig = (size_t)p.n_e * p.dev.nb * p.dev.b * p.dev.b * sizeof(double2);
  L.kavg = n_prob > 1;
  L.memory = memory;
  // Anderson: 2 M difference vectors and the previous pair, each of both kinds (2 arrays), partial sums, gamma
  const size_t anderson = memory > 0 ? (2 * (size_t)memory + 2) * 2 * up256(L.sig) +
                                           up256((size_t)RPARTS * NACC * sizeof(double)) + up256(MAXM * sizeof(double))
                                     : 0;
  L.total = up256(L.rgf) + up256(L.ec) + (L.kavg ? 3 : 2) * up256(L.sig) + up256(2 * RPARTS * sizeof(double)) +
            up256(sizeof(double)) + up256(2 * sizeof(int)) + anderson + 256;
  return true;
}

inline bool a16(const void* p) { return ((uintptr_t)p & 15) == 0; }

}  // namespace
}  // namespace negf

using namespace negf;

namespace negf {
namespace {

struct StepArgs {
  const negf_problem* problem;   // n_prob problems: one per k-point
  int32_t n_prob;
  negf_precision prec;
  const negf_options* opt;
  int32_t n_w, k0;
  const void *W_lesser, *W_greater;
  const double* scale;
  double mixing;
  int32_t memory;
  double tol;
  void *sig_r, *sig_l, *sig_g;
  void *GR_diag, *GR_upper, *GR_lower, *GL_diag, *GL_upper, *GG_diag, *GG_upper;
  int32_t* info;
  void* workspace;
  size_t ws_bytes;
};

// argument checks shared by the step and the driver; fills the layout
negf_status check_step(const StepArgs& a, ScbaLayout& L) {
  if (!a.problem || a.n_prob < 1 || !a.scale) return NEGF_EINVAL;
  for (int q = 0; q < a.n_prob; ++q) {
    const negf_problem& pq = a.problem[q];
    const negf_device& dq = pq.dev;
    if (dq.sig_r_sc || dq.sig_l_sc || dq.sig_g_sc || pq.sc_stride != 0) return NEGF_EINVAL;
  }
  if (a.k0 < 0 || a.k0 >= a.n_w || !(a.mixing > 0.0 && a.mixing <= 1.0) || !(a.tol >= 0.0)) return NEGF_EINVAL;
  if (!scba_layout(a.problem, a.n_prob, a.prec, a.opt, a.n_w, a.memory, L)) return NEGF_EINVAL;
  const void* req[] = {a.W_lesser, a.W_greater, a.sig_r, a.sig_l, a.sig_g, a.GR_diag, a.GR_upper, a.GL_diag,
                       a.GL_upper, a.GG_diag, a.GG_upper, a.info, a.workspace};
  for (const void* q : req)
    if (!q || !a16(q)) return NEGF_EINVAL;
  if (a.GR_lower && !a16(a.GR_lower)) return NEGF_EINVAL;
  if (a.sig_r == a.sig_l || a.sig_r == a.sig_g || a.sig_l == a.sig_g) return NEGF_EINVAL;
  if (a.ws_bytes < L.total) return NEGF_EINVAL;
  return NEGF_OK;
}

struct Carved {
  void *rgf, *ec;
  double2 *Fl, *Fg, *Gk;   // Gk: the k-average (nullptr with one k-point)
  double2 *DX, *DF, *xp, *fp;   // Anderson history (memory > 0)
  double *apart, *gamma;
  double *part, *last;
  int* state;
};

Carved carve(void* workspace, const ScbaLayout& L) {
  Carved c;
  char* base = (char*)(((uintptr_t)workspace + 255) & ~(uintptr_t)255);
  c.rgf = base;
  base += up256(L.rgf);
  c.ec = base;
  base += up256(L.ec);
  c.Fl = (double2*)base;
  base += up256(L.sig);
  c.Fg = (double2*)base;
  base += up256(L.sig);
  c.Gk = nullptr;
  if (L.kavg) {
    c.Gk = (double2*)base;
    base += up256(L.sig);
  }
  c.part = (double*)base;
  base += up256(2 * RPARTS * sizeof(double));
  c.last = (double*)base;
  base += up256(sizeof(double));
  c.state = (int*)base;
  base += up256(2 * sizeof(int));
  c.DX = c.DF = c.xp = c.fp = nullptr;
  c.apart = c.gamma = nullptr;
  if (L.memory > 0) {
    const size_t v = 2 * up256(L.sig);   // one vector of both kinds
    c.DX = (double2*)base;
    base += L.memory * v;
    c.DF = (double2*)base;
    base += L.memory * v;
    c.xp = (double2*)base;
    base += v;
    c.fp = (double2*)base;
    base += v;
    c.apart = (double*)base;
    base += up256((size_t)RPARTS * NACC * sizeof(double));
    c.gamma = (double*)base;
  }
  return c;
}

// iteration `it` of the loop (it = 0 starts one: state reset, Sigma^R formed from Sigma^<, Sigma^>);
// `update` = 0 never mixes (the last iteration of a fixed count)
negf_status step_impl(const StepArgs& a, const ScbaLayout& L, const Carved& c, int it, int update, double* history,
                      int* state, hipStream_t s) {
  const negf_problem& p0 = *a.problem;
  const negf_device& d0 = p0.dev;
  const long nbb = (long)d0.nb * d0.b * d0.b;
  const long n = (long)p0.n_e * nbb;
  double2* Sl = (double2*)a.sig_l;
  double2* Sg = (double2*)a.sig_g;
  double2* Sr = (double2*)a.sig_r;
  const unsigned mix_grid = (unsigned)std::min<long>((n + SB * U - 1) / (SB * U), MIX_WG);
  const unsigned part_grid = (unsigned)std::min<long>((n + SB * U - 1) / (SB * U), RPARTS);
  if (it == 0) {
    prof_begin(KC_ELEM, s);
    hipLaunchKernelGGL(scba_reset_kernel, dim3(1), dim3(64), 0, s, state);
    hipLaunchKernelGGL(mix_kernel, dim3(mix_grid), dim3(SB), 0, s, n, 0.0, (const double2*)nullptr,
                       (const double2*)nullptr, Sl, Sg, Sr, (const int*)nullptr);
    prof_end(KC_ELEM, s, 0.0, 48.0 * (double)n);
    if (hipGetLastError() != hipSuccess) return NEGF_EHIP;
  }
  // every k-point reads the same per-energy self-energies
  std::vector<negf_problem> pq(a.problem, a.problem + a.n_prob);
  for (negf_problem& q : pq) {
    q.dev.sig_r_sc = a.sig_r;
    q.dev.sig_l_sc = a.sig_l;
    q.dev.sig_g_sc = a.sig_g;
    q.sc_stride = nbb;
  }
  negf_status st = negf_rgf_lesser_greater(pq.data(), a.n_prob, a.prec, a.opt, a.GR_diag, a.GR_upper, a.GR_lower,
                                           a.GL_diag, a.GL_upper, a.GG_diag, a.GG_upper, a.info, c.rgf, L.rgf, s);
  if (st != NEGF_OK) return st;
  // the convolution of Eq. (3) on G^<> (averaged over the k-points when there are several)
  const unsigned avg_grid = (unsigned)std::min<long>((n + SB - 1) / SB, MIX_WG);
  const void* Gsrc[2] = {a.GL_diag, a.GG_diag};
  const void* Wk[2] = {a.W_lesser, a.W_greater};
  double2* Fk[2] = {c.Fl, c.Fg};
  for (int kind = 0; kind < 2; ++kind) {
    const void* Gin = Gsrc[kind];
    if (c.Gk) {
      prof_begin(KC_ELEM, s);
      hipLaunchKernelGGL(kavg_kernel, dim3(avg_grid), dim3(SB), 0, s, n, (int)a.n_prob, n, (const double2*)Gin,
                         c.Gk);
      prof_end(KC_ELEM, s, 0.0, 16.0 * (double)n * (a.n_prob + 1));
      Gin = c.Gk;
    }
    st = negf_energy_convolution(p0.n_e, nbb, Gin, a.n_w, a.k0, Wk[kind], a.scale, Fk[kind], c.ec, L.ec, s);
    if (st != NEGF_OK) return st;
  }
  prof_begin(KC_ELEM, s);
  hipLaunchKernelGGL(resid_partial_kernel, dim3(part_grid), dim3(SB), 0, s, n, (const double2*)c.Fl,
                     (const double2*)c.Fg, (const double2*)Sl, (const double2*)Sg, c.part);
  hipLaunchKernelGGL(resid_final_kernel, dim3(1), dim3(SB), 0, s, (int)part_grid, (const double*)c.part, a.tol, it,
                     c.last, history, state);
  if (update && L.memory == 0)
    hipLaunchKernelGGL(mix_kernel, dim3(mix_grid), dim3(SB), 0, s, n, a.mixing, (const double2*)c.Fl,
                       (const double2*)c.Fg, Sl, Sg, Sr, (const int*)state);
  if (update && L.memory > 0) {
    // history vectors hold 2 n complex (Sigma^< then Sigma^>); `it` counts the iterations since the start
    const int k = std::min(it, L.memory);
    const unsigned ag = (unsigned)std::min<long>((n + SB - 1) / SB, RPARTS);
    hipLaunchKernelGGL(anderson_hist_kernel, dim3(mix_grid), dim3(SB), 0, s, n, it == 0 ? 1 : 0,
                       it == 0 ? 0 : (it - 1) % L.memory, (const double2*)Sl, (const double2*)Sg,
                       (const double2*)c.Fl, (const double2*)c.Fg, c.xp, c.fp, c.DX, c.DF, (const int*)state);
    if (k > 0) {
      decltype(&anderson_gram_kernel<1>) gram[MAXM] = {anderson_gram_kernel<1>, anderson_gram_kernel<2>,
                                                        anderson_gram_kernel<3>, anderson_gram_kernel<4>};
      hipLaunchKernelGGL(gram[k - 1], dim3(ag), dim3(SB), 0, s, n, (const double2*)Sl, (const double2*)Sg,
                         (const double2*)c.Fl, (const double2*)c.Fg, (const double2*)c.DF, c.apart,
                         (const int*)state);
      hipLaunchKernelGGL(anderson_solve_kernel, dim3(1), dim3(SB), 0, s, (int)ag, k, (const double*)c.apart,
                         c.gamma, (const int*)state);
    }
    decltype(&anderson_update_kernel<0>) upd[MAXM + 1] = {anderson_update_kernel<0>, anderson_update_kernel<1>,
                                                          anderson_update_kernel<2>, anderson_update_kernel<3>,
                                                          anderson_update_kernel<4>};
    hipLaunchKernelGGL(upd[k], dim3(mix_grid), dim3(SB), 0, s, n, a.mixing,
                       (const double*)c.gamma, Sl, Sg, (const double2*)c.Fl, (const double2*)c.Fg,
                       (const double2*)c.DX, (const double2*)c.DF, Sr, (const int*)state);
  }
  // bytes: the residual reads F and Sigma of both kinds (4 n complex); linear mixing reads them again and
  // writes three arrays; Anderson's passes move 16 n (history; 8 n at the first, which stores no
  // differences) + (4 + 2 k) n (normal equations, none at the first) + (7 + 4 k) n (update) complex
  const int kk = std::min(it, L.memory);
  const double mixc = !update ? 0.0 : L.memory == 0 ? 7.0 : kk == 0 ? 15.0 : 27.0 + 6.0 * kk;
  prof_end(KC_ELEM, s, 0.0, 16.0 * (4.0 + mixc) * (double)n);
  return hipGetLastError() == hipSuccess ? NEGF_OK : NEGF_EHIP;
}

}  // namespace
}  // namespace negf

extern "C" {

size_t negf_scba_workspace_bytes(const negf_problem* problems, int32_t n_prob, negf_precision prec,
                                 const negf_options* opt, int32_t n_w, int32_t memory) {
  ScbaLayout L;
  return scba_layout(problems, n_prob, prec, opt, n_w, memory, L) ? L.total : 0;
}

negf_status negf_scba_step(const negf_problem* problem, int32_t n_prob, negf_precision prec, const negf_options* opt,
                           int32_t n_w, int32_t k0, const void* W_lesser, const void* W_greater,
                           const double* scale, double mixing, int32_t memory, double tol, int32_t it, int32_t update,
                           void* sig_r,
                           void* sig_l, void* sig_g, void* GR_diag, void* GR_upper, void* GR_lower, void* GL_diag,
                           void* GL_upper, void* GG_diag, void* GG_upper, int32_t* info, double* history,
                           int32_t* state, void* workspace, size_t ws_bytes, void* stream) {
  StepArgs a{problem, n_prob,  prec,    opt,      n_w,      k0,      W_lesser, W_greater, scale,
             mixing,  memory,  tol,     sig_r,    sig_l,    sig_g,   GR_diag,  GR_upper,  GR_lower,
             GL_diag, GL_upper, GG_diag, GG_upper, info,   workspace, ws_bytes};
  ScbaLayout L;
  negf_status st = check_step(a, L);
  if (st != NEGF_OK) return st;
  if (it < 0 || !state || !a16(state) || (history && ((uintptr_t)history & 7))) return NEGF_EINVAL;
  return step_impl(a, L, carve(workspace, L), it, update != 0, history, state, (hipStream_t)stream);
}

negf_status negf_scba(const negf_problem* problem, int32_t n_prob, negf_precision prec, const negf_options* opt,
                      int32_t n_w, int32_t k0, const void* W_lesser, const void* W_greater, const double* scale,
                      double mixing, int32_t memory, double tol, int32_t max_iter, void* sig_r, void* sig_l,
                      void* sig_g,
                      void* GR_diag, void* GR_upper, void* GR_lower, void* GL_diag, void* GL_upper, void* GG_diag,
                      void* GG_upper, int32_t* info, int32_t* n_iter, double* history, void* workspace,
                      size_t ws_bytes, void* stream) {
  StepArgs a{problem, n_prob,  prec,    opt,      n_w,      k0,      W_lesser, W_greater, scale,
             mixing,  memory,  tol,     sig_r,    sig_l,    sig_g,   GR_diag,  GR_upper,  GR_lower,
             GL_diag, GL_upper, GG_diag, GG_upper, info,   workspace, ws_bytes};
  if (!n_iter || max_iter < 1) return NEGF_EINVAL;
  ScbaLayout L;
  negf_status st = check_step(a, L);
  if (st != NEGF_OK) return st;
  const Carved c = carve(workspace, L);
  hipStream_t s = (hipStream_t)stream;
  *n_iter = 0;
  for (int it = 0; it < max_iter; ++it) {
    // the last allowed solve does not mix: the outputs then hold Sigma_n and the G it produced
    st = step_impl(a, L, c, it, it < max_iter - 1, nullptr, c.state, s);
    if (st != NEGF_OK) return st;
    struct {
      double r;
      int state[2];
    } h{0.0, {0, 0}};
    if (hipMemcpyAsync(&h.r, c.last, sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(h.state, c.state, 2 * sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return NEGF_EHIP;
    if (history) history[it] = h.r;
    *n_iter = it + 1;
    if (h.state[1] == 2) return NEGF_ENONFINITE;
    if (h.state[1] == 1) return NEGF_OK;
  }
  return NEGF_ENOCONV;
}

}  // extern "C"
