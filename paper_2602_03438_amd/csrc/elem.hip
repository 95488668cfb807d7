// Element-wise and reduction kernels: assembly of the blocks of z S - H - Sigma,
// lead self-energy post-processing, skew updates, norms and traces.
// All of them stream b x b complex blocks through HBM with coalesced 16-byte
// accesses; those that need a conjugate transpose go through 32 x 32 LDS tiles.
#include "internal.h"

namespace negf {

namespace {

constexpr int TD = 32;   // transpose tile edge
constexpr int TR = 8;    // rows per thread pass (block = 32 x 8)

__device__ __forceinline__ double2 ld_or0(const double2* p, long i) { return p ? p[i] : make_double2(0.0, 0.0); }

// out_p = zc_p op(S) + h op(H) + y Y + zc Z_p  (see AssembleDesc)
__global__ void __launch_bounds__(TD * TR) assemble_kernel(AssembleDesc d) {
  const int p = blockIdx.z;
  if (d.active && d.active[p] == 0) return;
  const int b = d.b;
  const long go = d.inner > 0 ? (long)(p / d.inner) * d.sHo : 0;   // block offset of the item's group
  const double e = d.energies ? d.energies[d.inner > 0 ? p % d.inner : p] : 0.0;
  const double2* S = d.S ? d.S + go : nullptr;
  const double2* Hm = d.H ? d.H + go : nullptr;
  const double2* Y = d.Y ? d.Y + go + (long)(d.inner > 0 ? p % d.inner : p) * d.sY : nullptr;
  const double2 zc = make_double2(d.s_coef * e, d.s_coef * d.eta);
  const int i0 = blockIdx.y * TD, j0 = blockIdx.x * TD;
  __shared__ double2 tS[TD][TD + 1];
  __shared__ double2 tH[TD][TD + 1];
  if (d.op == 1) {
    // stage the source tile (rows j0.., cols i0..) of S and H
    for (int rr = threadIdx.y; rr < TD; rr += TR) {
      const int sr = j0 + rr, sc = i0 + threadIdx.x;
      double2 sv = make_double2(0.0, 0.0), hv = make_double2(0.0, 0.0);
      if (sr < b && sc < b) {
        if (S) sv = S[(long)sr * b + sc];
        else if (d.s_identity && sr == sc) sv = make_double2(1.0, 0.0);
        if (Hm) hv = Hm[(long)sr * b + sc];
      }
      tS[rr][threadIdx.x] = sv;
      tH[rr][threadIdx.x] = hv;
    }
    __syncthreads();
  }
  for (int rr = threadIdx.y; rr < TD; rr += TR) {
    const int i = i0 + rr, j = j0 + threadIdx.x;
    if (i >= b || j >= b) continue;
    const long o = (long)i * b + j;
    double2 sv, hv;
    if (d.op == 1) {
      sv = cconj(tS[threadIdx.x][rr]);
      hv = cconj(tH[threadIdx.x][rr]);
    } else {
      sv = S ? S[o] : make_double2((d.s_identity && i == j) ? 1.0 : 0.0, 0.0);
      hv = ld_or0(Hm, o);
    }
    double2 r = cmul(zc, sv);
    r.x += d.h_coef * hv.x;
    r.y += d.h_coef * hv.y;
    if (Y) {
      const double2 y = Y[o];
      r.x += d.y_coef * y.x;
      r.y += d.y_coef * y.y;
    }
    if (d.Z) {
      const double2 z = d.Z[(long)p * d.sZ + o];
      r.x += d.z_coef * z.x;
      r.y += d.z_coef * z.y;
    }
    d.out[(long)p * d.sOut + o] = r;
  }
}

// out_p += c * W_p^H through 32 x 32 LDS tiles (reads and writes coalesced)
__global__ void __launch_bounds__(TD * TR) add_adjoint_kernel(int b, double2 c, const double2* W, long sW,
                                                              double2* out, long sOut) {
  const int p = blockIdx.z;
  const int i0 = blockIdx.y * TD, j0 = blockIdx.x * TD;   // output tile rows i0.., cols j0..
  __shared__ double2 t[TD][TD + 1];
  const double2* w = W + (long)p * sW;
  double2* o = out + (long)p * sOut;
  for (int rr = threadIdx.y; rr < TD; rr += TR) {          // W rows j0.., cols i0..
    const int r = j0 + rr, cidx = i0 + threadIdx.x;
    t[rr][threadIdx.x] = (r < b && cidx < b) ? w[(long)r * b + cidx] : make_double2(0.0, 0.0);
  }
  __syncthreads();
  for (int rr = threadIdx.y; rr < TD; rr += TR) {
    const int i = i0 + rr, j = j0 + threadIdx.x;
    if (i >= b || j >= b) continue;
    const double2 v = cconj(t[threadIdx.x][rr]);           // (W^H)[i][j] = conj(W[j][i])
    o[(long)i * b + j] = cadd(o[(long)i * b + j], cmul(c, v));
  }
}

__global__ void scatter_blocks_kernel(long n, int nblk, const double2* src, long sS, double2* dst, int inner,
                                      long sDo, long sDi) {
  const int z = blockIdx.y;
  const double2* s = src + (long)z * sS;
  double2* d = dst + (long)(z / inner) * sDo + (long)(z % inner) * sDi;
  const long tot = n * nblk;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < tot; i += (long)gridDim.x * blockDim.x) d[i] = s[i];
}

__global__ void copy_kernel(long n, int batch, const double2* src, long sS, double2* dst, long sD) {
  const int p = blockIdx.y;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    dst[(long)p * sD + i] = src[(long)p * sS + i];
}

template <int NT>
__device__ double block_sum(double v) {
  __shared__ double red[NT / 64];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < NT / 64; ++i) s += red[i];
  return s;
}

constexpr int RED_NT = 512;

// Squared Frobenius norm of X_p - shift*I in FROB_SPLIT slices per item (one
// workgroup each), then a fixed-order sum of the slices: the result does not
// depend on scheduling.
__global__ void __launch_bounds__(RED_NT) frob2_part_kernel(int b, const double2* X, long sX, double shift,
                                                            const int* active, double* part) {
  const int p = blockIdx.y, q = blockIdx.x;
  if (active && active[p] == 0) return;
  const double2* x = X + (long)p * sX;
  const long n = (long)b * b;
  const long per = (n + FROB_SPLIT - 1) / FROB_SPLIT;
  const long lo = (long)q * per, hi = lo + per < n ? lo + per : n;
  double s = 0.0;
  for (long i = lo + threadIdx.x; i < hi; i += RED_NT) {
    double2 v = x[i];
    if (shift != 0.0 && (i / b) == (i % b)) v.x -= shift;
    s += v.x * v.x + v.y * v.y;
  }
  s = block_sum<RED_NT>(s);
  if (threadIdx.x == 0) part[(long)p * FROB_SPLIT + q] = s;
}

__global__ void __launch_bounds__(256) frob2_sum_kernel(int batch, const double* part, const int* active,
                                                        double* out) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= batch || (active && active[p] == 0)) return;
  double s = 0.0;
#pragma unroll
  for (int q = 0; q < FROB_SPLIT; ++q) s += part[(long)p * FROB_SPLIT + q];
  out[p] = s;
}

__global__ void __launch_bounds__(RED_NT) dot_re_kernel(int b, const double2* P, long sP, const double2* Q, long sQ,
                                                        double* out) {
  const int p = blockIdx.x;
  const long n = (long)b * b;
  double s = 0.0;
  for (long i = threadIdx.x; i < n; i += RED_NT) {
    const double2 u = P[(long)p * sP + i], v = Q[(long)p * sQ + i];
    s += u.x * v.x + u.y * v.y;
  }
  s = block_sum<RED_NT>(s);
  if (threadIdx.x == 0) out[p] = s;
}

// One workgroup: updates the active flags of every item and counts the survivors.
__global__ void __launch_bounds__(1024) sr_check_kernel(int batch, const double* a2, const double* c2,
                                                        const double* d2, double tol, int iter, int* active,
                                                        int* iters, int* n_active) {
  int cnt = 0;
  for (int p = threadIdx.x; p < batch; p += blockDim.x) {
    if (active[p]) {
      const double lim = tol * tol * d2[p];
      const bool bad = !(a2[p] == a2[p]) || !(c2[p] == c2[p]);
      if ((a2[p] <= lim && c2[p] <= lim) || bad) {
        active[p] = 0;
        iters[p] = bad ? -iter : iter;
      } else {
        iters[p] = iter;
        cnt++;
      }
    }
  }
  __shared__ int red[16];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) cnt += __shfl_xor(cnt, off);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = cnt;
  __syncthreads();
  if (threadIdx.x == 0) {
    int s = 0;
    for (int i = 0; i < (int)((blockDim.x + 63) >> 6); ++i) s += red[i];
    *n_active = s;
  }
}

__global__ void sr_finish_kernel(int batch, const double* r2, const double* m2, const double* g2, const int* active,
                                 double accept, double* resid, int* info, int info_mod) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= batch) return;
  const double r = sqrt(r2[p]) / (sqrt(m2[p]) * sqrt(g2[p]));
  if (resid) resid[p] = r;
  int st = ST_OK;
  if (!(r == r) || !isfinite(r2[p])) st = ST_ENONFINITE;
  else if ((active && active[p]) || r > accept) st = ST_ENOCONV;
  if (st != ST_OK && info) atomicCAS(info + (info_mod > 0 ? p % info_mod : p), ST_OK, st);
}

// gamma = i (S - S^H); sl = i f gamma; sg = -i (1 - f) gamma
__global__ void __launch_bounds__(TD * TR) gamma_sigma_kernel(int b, const double2* sig, long sS,
                                                              const double* energies, double mu, double kT,
                                                              double2* gamma, long sG, double2* sl, long sL,
                                                              double2* sg, long sGr) {
  const int p = blockIdx.z;
  const int i0 = blockIdx.y * TD, j0 = blockIdx.x * TD;
  __shared__ double2 t[TD][TD + 1];
  const double2* S = sig + (long)p * sS;
  for (int rr = threadIdx.y; rr < TD; rr += TR) {
    const int sr = j0 + rr, sc = i0 + threadIdx.x;
    t[rr][threadIdx.x] = (sr < b && sc < b) ? S[(long)sr * b + sc] : make_double2(0.0, 0.0);
  }
  __syncthreads();
  double f = 0.0;
  if (sl || sg) {
    const double x = energies[p] - mu;
    if (kT > 0.0) {
      const double y = x / kT;
      f = y > 0 ? exp(-y) / (1.0 + exp(-y)) : 1.0 / (1.0 + exp(y));
    } else {
      f = x < 0 ? 1.0 : (x == 0 ? 0.5 : 0.0);
    }
  }
  for (int rr = threadIdx.y; rr < TD; rr += TR) {
    const int i = i0 + rr, j = j0 + threadIdx.x;
    if (i >= b || j >= b) continue;
    const long o = (long)i * b + j;
    const double2 s = S[o];
    const double2 sh = cconj(t[threadIdx.x][rr]);   // (S^H)_ij = conj(S_ji)
    const double2 dlt = csub(s, sh);
    const double2 g = make_double2(-dlt.y, dlt.x);  // i * (S - S^H)
    if (gamma) gamma[(long)p * sG + o] = g;
    if (sl) sl[(long)p * sL + o] = make_double2(-f * g.y, f * g.x);                  // i f g
    if (sg) sg[(long)p * sGr + o] = make_double2((1.0 - f) * g.y, -(1.0 - f) * g.x);  // -i (1-f) g
  }
}

__global__ void __launch_bounds__(RED_NT) check_finite_kernel(int b, const double2* X, long sX, int* info,
                                                              int info_mod) {
  const int p = blockIdx.x;
  const long n = (long)b * b;
  int bad = 0;
  for (long i = threadIdx.x; i < n; i += RED_NT) {
    const double2 v = X[(long)p * sX + i];
    if (!isfinite(v.x) || !isfinite(v.y)) bad = 1;
  }
  if (bad) atomicCAS(info + (info_mod > 0 ? p % info_mod : p), ST_OK, ST_ENONFINITE);
}

__global__ void lincomb_kernel(int b, double2 c1, const double2* X, long sX, double2 c2, const double2* Y, long sY,
                               double2 g, double2* out, long sOut, const int* active) {
  const int p = blockIdx.y;
  if (active && active[p] == 0) return;
  const long n = (long)b * b;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    double2 r = make_double2(0.0, 0.0);
    if (X) r = cmul(c1, X[(long)p * sX + i]);
    if (Y) r = cadd(r, cmul(c2, Y[(long)p * sY + i]));
    if ((i / b) == (i % b)) r = cadd(r, g);
    out[(long)p * sOut + i] = r;
  }
}

__global__ void seed_flags_kernel(int np, const int* flags, int* active, int* iters) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= np) return;
  active[p] = flags[p] == ST_OK ? 0 : 1;
  iters[p] = 0;
}

__global__ void seed_select_kernel(long n, const int* flags, const double2* g_dec, double2* g) {
  const int p = blockIdx.y;
  if (flags[p] == ST_OK) return;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    g[(long)p * n + i] = g_dec[(long)p * n + i];
}

__global__ void closure_accept_kernel(int np, const double* r2, const double* m2, const double* g2, double accept,
                                      int iter, int* active, int* iters, int* accepted, int* closed) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= np) return;
  int c = 0;
  if (active[p]) {
    const double r = sqrt(r2[p]) / (sqrt(m2[p]) * sqrt(g2[p]));
    if (r == r && isfinite(r) && r <= accept) {
      c = 1;
      active[p] = 0;
      iters[p] = iter;
      accepted[p] = ST_OK;
    }
  }
  closed[p] = c;
}

__global__ void stamp_kernel(unsigned long long* dst) {
  if (threadIdx.x == 0) *dst = wall_clock64();
}

// One round of a point queue for one chunk segment (slots [e0, e0 + n) of a problem with n_slots
// slots): slot e0 + i takes task r n_slots + e0 + i of the task list (r = the segment's round
// counter), or none past its end (its energy is left as it was and its task index is -1); the
// slots' info is cleared for the round and the counter advanced.  One workgroup.
__global__ void queue_pop_kernel(double* energies, int e0, int n, int n_slots, const double* task_E, int n_tasks,
                                 int* round, int* slot_task, int* info) {
  __shared__ int r;
  if (threadIdx.x == 0) r = *round;
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const long t = (long)r * n_slots + e0 + i;
    if (t < n_tasks) {
      energies[e0 + i] = task_E[t];
      slot_task[i] = (int)t;
    } else {
      slot_task[i] = -1;
    }
    info[i] = 0;
  }
  __syncthreads();
  if (threadIdx.x == 0) *round = r + 1;
}

// Results of one round for one chunk segment: workgroup i takes slot i; if it held a task t, then
// task_info[t] = info[i], task_dos[t] = -Im sum_blocks Tr G^R_kk / pi and task_stamp[t] = the wall
// clock now.
constexpr int QF = 256;
__global__ void __launch_bounds__(QF) queue_finish_kernel(const double2* GRd, int nb, int b, const int* slot_task,
                                                          const int* info, int* task_info, double* task_dos,
                                                          unsigned long long* task_stamp) {
  const int i = blockIdx.x;
  const int t = slot_task[i];
  if (t < 0) return;
  const double2* g = GRd + (long)i * nb * b * b;
  double acc = 0.0;
  for (int k = threadIdx.x; k < nb * b; k += QF) {
    const int blk = k / b, j = k - blk * b;
    acc += g[(long)blk * b * b + (long)j * b + j].y;
  }
  __shared__ double red[QF];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = QF / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    task_info[t] = info[i];
    task_dos[t] = -red[0] / M_PI;
    task_stamp[t] = wall_clock64();
  }
}

__global__ void fill_int_kernel(int n, int* p, int v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

inline unsigned grid_for(long n) {
  long g = (n + 255) / 256;
  return (unsigned)(g < 1024 ? g : 1024);
}

}  // namespace

hipError_t launch_assemble(const AssembleDesc& d, hipStream_t s) {
  if (d.batch <= 0) return hipSuccess;
  const int nt = (d.b + TD - 1) / TD;
  prof_begin(KC_ELEM, s);
  hipLaunchKernelGGL(assemble_kernel, dim3(nt, nt, d.batch), dim3(TD, TR), 0, s, d);
  prof_end(KC_ELEM, s, 0, 16.0 * d.b * d.b * d.batch * 3);
  return hipGetLastError();
}

hipError_t launch_copy_blocks(int b, int batch, const double2* src, long sS, double2* dst, long sD, hipStream_t s) {
  if (batch <= 0) return hipSuccess;
  const long n = (long)b * b;
  hipLaunchKernelGGL(copy_kernel, dim3(grid_for(n), batch), dim3(256), 0, s, n, batch, src, sS, dst, sD);
  return hipGetLastError();
}

hipError_t launch_add_adjoint(int b, int batch, double2 c, const double2* W, long sW, double2* out, long sOut,
                              hipStream_t s) {
  if (batch <= 0 || b <= 0) return hipSuccess;
  const int nt = (b + TD - 1) / TD;
  prof_begin(KC_ELEM, s);
  hipLaunchKernelGGL(add_adjoint_kernel, dim3(nt, nt, batch), dim3(TD, TR), 0, s, b, c, W, sW, out, sOut);
  prof_end(KC_ELEM, s, 0, 48.0 * b * b * batch);
  return hipGetLastError();
}

hipError_t launch_scatter_blocks(int b, int nitems, int nblk, const double2* src, long sS, double2* dst, int inner,
                                 long sDo, long sDi, hipStream_t s) {
  if (nitems <= 0 || nblk <= 0 || b <= 0) return hipSuccess;
  if (inner <= 0) return hipErrorInvalidValue;
  const long n = (long)b * b;
  prof_begin(KC_ELEM, s);
  hipLaunchKernelGGL(scatter_blocks_kernel, dim3(grid_for(n * nblk), nitems), dim3(256), 0, s, n, nblk, src, sS, dst,
                     inner, sDo, sDi);
  prof_end(KC_ELEM, s, 0, 32.0 * n * nblk * nitems);
  return hipGetLastError();
}

hipError_t launch_frob2(int b, int batch, const double2* X, long sX, double shift, const int* active, double* part,
                        double* nrm2, hipStream_t s) {
  if (batch <= 0) return hipSuccess;
  hipLaunchKernelGGL(frob2_part_kernel, dim3(FROB_SPLIT, batch), dim3(RED_NT), 0, s, b, X, sX, shift, active, part);
  hipLaunchKernelGGL(frob2_sum_kernel, dim3((batch + 255) / 256), dim3(256), 0, s, batch, part, active, nrm2);
  return hipGetLastError();
}

hipError_t launch_sr_check(int batch, const double* a2, const double* c2, const double* d2, double tol, int iter,
                           int* active, int* iters, int* n_active, hipStream_t s) {
  hipLaunchKernelGGL(sr_check_kernel, dim3(1), dim3(1024), 0, s, batch, a2, c2, d2, tol, iter, active, iters,
                     n_active);
  return hipGetLastError();
}

hipError_t launch_gamma_sigma(int b, int batch, const double2* sig, long sS, const double* energies, double mu,
                              double kT, double2* gamma, long sG, double2* sl, long sL, double2* sg, long sGr,
                              hipStream_t s) {
  if (batch <= 0) return hipSuccess;
  const int nt = (b + TD - 1) / TD;
  hipLaunchKernelGGL(gamma_sigma_kernel, dim3(nt, nt, batch), dim3(TD, TR), 0, s, b, sig, sS, energies, mu, kT,
                     gamma, sG, sl, sL, sg, sGr);
  return hipGetLastError();
}

hipError_t launch_dot_re(int b, int batch, const double2* P, long sP, const double2* Q, long sQ, double* out,
                         hipStream_t s) {
  if (batch <= 0) return hipSuccess;
  hipLaunchKernelGGL(dot_re_kernel, dim3(batch), dim3(RED_NT), 0, s, b, P, sP, Q, sQ, out);
  return hipGetLastError();
}

hipError_t launch_sr_finish(int batch, const double* r2, const double* m2, const double* g2, const int* active,
                            double accept, double* resid_out, int* info, int info_mod, hipStream_t s) {
  if (batch <= 0) return hipSuccess;
  hipLaunchKernelGGL(sr_finish_kernel, dim3((batch + 255) / 256), dim3(256), 0, s, batch, r2, m2, g2, active, accept,
                     resid_out, info, info_mod);
  return hipGetLastError();
}

hipError_t launch_check_finite(int b, int batch, const double2* X, long sX, int* info, int info_mod, hipStream_t s) {
  if (batch <= 0) return hipSuccess;
  hipLaunchKernelGGL(check_finite_kernel, dim3(batch), dim3(RED_NT), 0, s, b, X, sX, info, info_mod);
  return hipGetLastError();
}

hipError_t launch_lincomb(int b, int batch, double2 c1, const double2* X, long sX, double2 c2, const double2* Y,
                          long sY, double2 g, double2* out, long sOut, const int* active, hipStream_t s) {
  if (batch <= 0) return hipSuccess;
  const long n = (long)b * b;
  prof_begin(KC_ELEM, s);
  hipLaunchKernelGGL(lincomb_kernel, dim3(grid_for(n), batch), dim3(256), 0, s, b, c1, X, sX, c2, Y, sY, g, out, sOut,
                     active);
  prof_end(KC_ELEM, s, 0, 16.0 * n * batch * ((X ? 1 : 0) + (Y ? 1 : 0) + 1));
  return hipGetLastError();
}

hipError_t launch_seed_flags(int np, const int* flags, int* active, int* iters, hipStream_t s) {
  if (np <= 0) return hipSuccess;
  hipLaunchKernelGGL(seed_flags_kernel, dim3((np + 255) / 256), dim3(256), 0, s, np, flags, active, iters);
  return hipGetLastError();
}

hipError_t launch_seed_select(int b, int np, const int* flags, const double2* g_dec, double2* g, hipStream_t s) {
  if (np <= 0) return hipSuccess;
  const long n = (long)b * b;
  hipLaunchKernelGGL(seed_select_kernel, dim3(grid_for(n), np), dim3(256), 0, s, n, flags, g_dec, g);
  return hipGetLastError();
}

hipError_t launch_closure_accept(int np, const double* r2, const double* m2, const double* g2, double accept, int iter,
                                 int* active, int* iters, int* accepted, int* closed, hipStream_t s) {
  if (np <= 0) return hipSuccess;
  hipLaunchKernelGGL(closure_accept_kernel, dim3((np + 255) / 256), dim3(256), 0, s, np, r2, m2, g2, accept, iter,
                     active, iters, accepted, closed);
  return hipGetLastError();
}

hipError_t launch_stamp(unsigned long long* dst, hipStream_t s) {
  hipLaunchKernelGGL(stamp_kernel, dim3(1), dim3(64), 0, s, dst);
  return hipGetLastError();
}

hipError_t launch_queue_pop(double* energies, int e0, int n, int n_slots, const double* task_E, int n_tasks,
                            int* round, int* slot_task, int* info, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(queue_pop_kernel, dim3(1), dim3(256), 0, s, energies, e0, n, n_slots, task_E, n_tasks, round,
                     slot_task, info);
  return hipGetLastError();
}

hipError_t launch_queue_finish(const double2* GRd, int nb, int b, int n, const int* slot_task, const int* info,
                               int* task_info, double* task_dos, unsigned long long* task_stamp, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(queue_finish_kernel, dim3(n), dim3(QF), 0, s, GRd, nb, b, slot_task, info, task_info, task_dos,
                     task_stamp);
  return hipGetLastError();
}

hipError_t launch_fill_int(int n, int* p, int v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_int_kernel, dim3((n + 255) / 256), dim3(256), 0, s, n, p, v);
  return hipGetLastError();
}

}  // namespace negf
