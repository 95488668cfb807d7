// CPU test double of the library's device kernels.
//
// Linked with the library's own host orchestration (csrc/api.hip) into
// libnegf_hostsim.so, this lets the CPU test suite run the complete call
// sequence of the decimation and the RGF sweeps on host memory and compare the
// result with the oracle, without a GPU.  Every launch_* entry point of
// csrc/internal.h is re-implemented here with plain loops and the same
// argument semantics as the HIP kernels (including the active masks, the
// info codes and the in-place conventions), with bounds assertions on every
// batch item it touches.  It is test infrastructure only: the product library
// libnegf.so never contains it.
#include <atomic>
#include "internal.h"

#include <cassert>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <vector>

namespace negf {

typedef std::complex<double> cd;

static inline cd C(double2 v) { return cd(v.x, v.y); }
static inline double2 D(cd v) { double2 r; r.x = v.real(); r.y = v.imag(); return r; }

static bool act(const int* a, int p) { return !a || a[p] != 0; }

// A zero-slab map may only mark slabs of the sparse operand that are zero: the
// device kernel skips the others' K-steps.  Checked here for every item.
static bool kmask_valid(const GemmDesc& d) {
  if (!d.kmask || (d.kmask_op != 1 && d.kmask_op != 2)) return true;
  if (d.M % 64 || d.N % 64 || d.K % 16 || d.K > 1024) return true;   // the kernel ignores the map
  if ((d.kmask_op == 1 && d.opB != OP_N) || (d.kmask_op == 2 && d.opA != OP_C)) return false;
  const MatRef& T = d.kmask_op == 1 ? d.B : d.A;   // stored K x (N or M)
  const int groups = (d.kmask_op == 1 ? d.N : d.M) / 16;
  for (int p = 0; p < d.batch; ++p) {
    if (!act(d.active, p)) continue;
    const double2* Tp = T.p + (long)p * T.stride;
    for (int c = 0; c < groups; ++c)
      for (int k = 0; k < d.K / 16; ++k) {
        if (d.kmask[c] >> k & 1ull) continue;
        for (int r = 16 * k; r < 16 * k + 16; ++r)
          for (int j = 16 * c; j < 16 * c + 16; ++j) {
            const double2 v = Tp[(long)r * T.ld + j];
            if (v.x != 0.0 || v.y != 0.0) return false;
          }
      }
  }
  return true;
}

hipError_t launch_slab_map(int b, int nblk, const double2* H, const double2* S, unsigned long long* out,
                           int accumulate, hipStream_t) {
  if (nblk <= 0) return hipSuccess;
  if (b % 64 != 0 || b > 1024 || !H || !out) return hipErrorInvalidValue;
  for (int i = 0; i < nblk; ++i)
    for (int c = 0; c < b / 16; ++c) {
      unsigned long long w = 0;
      for (int r = 0; r < b; ++r)
        for (int j = 16 * c; j < 16 * c + 16; ++j) {
          const long e = (long)i * b * b + (long)r * b + j;
          const bool nz = H[e].x != 0.0 || H[e].y != 0.0 || (S && (S[e].x != 0.0 || S[e].y != 0.0));
          if (nz) w |= 1ull << (r / 16);
        }
      unsigned long long& o = out[(long)i * (b / 16) + c];
      o = accumulate ? (o | w) : w;
    }
  return hipSuccess;
}

int tile_for_launch(int tile, int, int, long) { return tile; }   // the double computes every tile alike

hipError_t launch_gemm(const GemmDesc& d, hipStream_t) {
  if (d.M <= 0 || d.N <= 0 || d.batch <= 0) return hipSuccess;
  if (!kmask_valid(d)) {
    fprintf(stderr, "hostsim: zero-slab map marks a nonzero slab (op %d, M %d N %d K %d)\n", d.kmask_op, d.M, d.N, d.K);
    return hipErrorInvalidValue;
  }
  const cd alpha = C(d.alpha), beta = C(d.beta);
  const bool use_beta = (d.beta.x != 0.0 || d.beta.y != 0.0) && d.Cin.p;
  std::vector<cd> out((size_t)d.M * d.N);
  for (int p = 0; p < d.batch; ++p) {
    if (!act(d.active, p)) continue;
    const double2* A = d.A.p + (long)p * d.A.stride;
    const double2* B = d.B.p + (long)p * d.B.stride;
    for (int i = 0; i < d.M; ++i)
      for (int j = 0; j < d.N; ++j) {
        cd s = 0;
        for (int k = 0; k < d.K; ++k) {
          cd a = d.opA == OP_N ? C(A[(long)i * d.A.ld + k]) : std::conj(C(A[(long)k * d.A.ld + i]));
          cd b = d.opB == OP_N ? C(B[(long)k * d.B.ld + j]) : std::conj(C(B[(long)j * d.B.ld + k]));
          if (d.prec == PREC_F32) {
            a = cd((float)a.real(), (float)a.imag());
            b = cd((float)b.real(), (float)b.imag());
          }
          s += a * b;
        }
        if (d.prec == PREC_F32) s = cd((float)s.real(), (float)s.imag());
        cd r = alpha * s;
        if (use_beta) r += beta * C(d.Cin.p[(long)p * d.Cin.stride + (long)i * d.Cin.ld + j]);
        out[(size_t)i * d.N + j] = r;
      }
    double2* Cp = d.C.p + (long)p * d.C.stride;
    for (int i = 0; i < d.M; ++i)
      for (int j = 0; j < d.N; ++j) {
        if (j >= d.skip_lo && j < d.skip_hi) continue;   // computed, not stored
        // anti-Hermitian products: the strict lower triangle mirrors the upper one
        const cd v = (d.skew && i > j) ? -std::conj(out[(size_t)j * d.N + i]) : out[(size_t)i * d.N + j];
        Cp[(long)i * d.C.ld + j] = D(v);
      }
  }
  return hipSuccess;
}

size_t inverse_scratch_bytes(int n, int batch) { return (size_t)(2 * n * 32 * 16 + 8 * n + 255) / 256 * 256 * batch; }

// Gauss-Jordan with partial pivoting on a copy; same info semantics as the panel kernel.
hipError_t launch_inverse(const InvDesc& d, hipStream_t) {
  const int n = d.n;
  std::vector<cd> a((size_t)n * n), inv((size_t)n * n);
  for (int p = 0; p < d.batch; ++p) {
    if (!act(d.active, p)) continue;
    double2* M = d.M + (long)p * d.sM;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        a[(size_t)i * n + j] = C(M[(long)i * d.ldm + j]);
        inv[(size_t)i * n + j] = i == j ? 1.0 : 0.0;
      }
    int st = ST_OK;
    for (int j = 0; j < n; ++j) {
      int pr = j;
      double best = -1;
      for (int r = j; r < n; ++r) {
        double k = std::abs(a[(size_t)r * n + j].real()) + std::abs(a[(size_t)r * n + j].imag());
        if (k > best) { best = k; pr = r; }
      }
      if (pr != j)
        for (int c = 0; c < n; ++c) {
          std::swap(a[(size_t)j * n + c], a[(size_t)pr * n + c]);
          std::swap(inv[(size_t)j * n + c], inv[(size_t)pr * n + c]);
        }
      const cd piv = a[(size_t)j * n + j];
      if (piv == cd(0)) st = ST_ESINGULAR;
      const cd ip = 1.0 / piv;
      if (!std::isfinite(ip.real()) || !std::isfinite(ip.imag())) st = st == ST_OK ? ST_ENONFINITE : st;
      for (int c = 0; c < n; ++c) {
        a[(size_t)j * n + c] *= ip;
        inv[(size_t)j * n + c] *= ip;
      }
      for (int r = 0; r < n; ++r) {
        if (r == j) continue;
        const cd f = a[(size_t)r * n + j];
        if (f == cd(0)) continue;
        for (int c = 0; c < n; ++c) {
          a[(size_t)r * n + c] -= f * a[(size_t)j * n + c];
          inv[(size_t)r * n + c] -= f * inv[(size_t)j * n + c];
        }
      }
    }
    double2* O = d.out + (long)p * d.sO;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        O[(long)i * d.ldo + j] = D(inv[(size_t)i * n + j]);
        M[(long)i * d.ldm + j] = D(0.0);   // M is destroyed, as on the device
      }
    if (st != ST_OK && d.info) {
      int* t = d.info + (d.info_mod > 0 ? p % d.info_mod : p);
      if (*t == ST_OK) *t = st;
    }
  }
  return hipSuccess;
}

hipError_t launch_assemble(const AssembleDesc& d, hipStream_t) {
  const int b = d.b;
  for (int p = 0; p < d.batch; ++p) {
    if (!act(d.active, p)) continue;
    const long go = d.inner > 0 ? (long)(p / d.inner) * d.sHo : 0;
    const double2* S = d.S ? d.S + go : nullptr;
    const double2* Hm = d.H ? d.H + go : nullptr;
    const double2* Y = d.Y ? d.Y + go + (long)(d.inner > 0 ? p % d.inner : p) * d.sY : nullptr;
    const double e = d.energies ? d.energies[d.inner > 0 ? p % d.inner : p] : 0.0;
    const cd zc = d.s_coef * cd(e, d.eta);
    for (int i = 0; i < b; ++i)
      for (int j = 0; j < b; ++j) {
        const long o = (long)i * b + j, ot = (long)j * b + i;
        cd sv, hv;
        if (d.op == 1) {
          sv = S ? std::conj(C(S[ot])) : cd((d.s_identity && i == j) ? 1.0 : 0.0);
          hv = Hm ? std::conj(C(Hm[ot])) : cd(0);
        } else {
          sv = S ? C(S[o]) : cd((d.s_identity && i == j) ? 1.0 : 0.0);
          hv = Hm ? C(Hm[o]) : cd(0);
        }
        cd r = zc * sv + d.h_coef * hv;
        if (Y) r += d.y_coef * C(Y[o]);
        if (d.Z) r += d.z_coef * C(d.Z[(long)p * d.sZ + o]);
        d.out[(long)p * d.sOut + o] = D(r);
      }
  }
  return hipSuccess;
}

hipError_t launch_add_adjoint(int b, int batch, double2 c, const double2* W, long sW, double2* out, long sOut,
                              hipStream_t) {
  for (int p = 0; p < batch; ++p)
    for (int i = 0; i < b; ++i)
      for (int j = 0; j < b; ++j) {
        double2& o = out[(long)p * sOut + (long)i * b + j];
        o = D(C(o) + C(c) * std::conj(C(W[(long)p * sW + (long)j * b + i])));
      }
  return hipSuccess;
}

hipError_t launch_scatter_blocks(int b, int nitems, int nblk, const double2* src, long sS, double2* dst, int inner,
                                 long sDo, long sDi, hipStream_t) {
  if (nitems <= 0 || nblk <= 0) return hipSuccess;
  if (inner <= 0) return hipErrorInvalidValue;
  for (int z = 0; z < nitems; ++z)
    std::memmove(dst + (long)(z / inner) * sDo + (long)(z % inner) * sDi, src + (long)z * sS,
                 sizeof(double2) * b * b * nblk);
  return hipSuccess;
}

hipError_t launch_copy_blocks(int b, int batch, const double2* src, long sS, double2* dst, long sD, hipStream_t) {
  for (int p = 0; p < batch; ++p) std::memmove(dst + (long)p * sD, src + (long)p * sS, sizeof(double2) * b * b);
  return hipSuccess;
}

hipError_t launch_frob2(int b, int batch, const double2* X, long sX, double shift, const int* active, double*,
                        double* nrm2, hipStream_t) {
  for (int p = 0; p < batch; ++p) {
    if (active && active[p] == 0) continue;
    double s = 0;
    for (long i = 0; i < (long)b * b; ++i) {
      cd v = C(X[(long)p * sX + i]);
      if (i / b == i % b) v -= shift;
      s += std::norm(v);
    }
    nrm2[p] = s;
  }
  return hipSuccess;
}

hipError_t launch_sr_check(int batch, const double* a2, const double* c2, const double* d2, double tol, int iter,
                           int* active, int* iters, int* n_active, hipStream_t) {
  int cnt = 0;
  for (int p = 0; p < batch; ++p) {
    if (!active[p]) continue;
    const double lim = tol * tol * d2[p];
    const bool bad = std::isnan(a2[p]) || std::isnan(c2[p]);
    if ((a2[p] <= lim && c2[p] <= lim) || bad) {
      active[p] = 0;
      iters[p] = bad ? -iter : iter;
    } else {
      iters[p] = iter;
      cnt++;
    }
  }
  *n_active = cnt;
  return hipSuccess;
}

hipError_t launch_gamma_sigma(int b, int batch, const double2* sig, long sS, const double* energies, double mu,
                              double kT, double2* gamma, long sG, double2* sl, long sL, double2* sg, long sGr,
                              hipStream_t) {
  for (int p = 0; p < batch; ++p) {
    double f = 0;
    if (sl || sg) {
      const double x = energies[p] - mu;
      f = kT > 0 ? 1.0 / (1.0 + std::exp(x / kT)) : (x < 0 ? 1.0 : (x == 0 ? 0.5 : 0.0));
    }
    for (int i = 0; i < b; ++i)
      for (int j = 0; j < b; ++j) {
        const cd s = C(sig[(long)p * sS + (long)i * b + j]);
        const cd sh = std::conj(C(sig[(long)p * sS + (long)j * b + i]));
        const cd g = cd(0, 1) * (s - sh);
        const long o = (long)i * b + j;
        if (gamma) gamma[(long)p * sG + o] = D(g);
        if (sl) sl[(long)p * sL + o] = D(cd(0, 1) * f * g);
        if (sg) sg[(long)p * sGr + o] = D(cd(0, -1) * (1.0 - f) * g);
      }
  }
  return hipSuccess;
}

hipError_t launch_dot_re(int b, int batch, const double2* P, long sP, const double2* Q, long sQ, double* out,
                         hipStream_t) {
  for (int p = 0; p < batch; ++p) {
    double s = 0;
    for (long i = 0; i < (long)b * b; ++i) s += (C(P[(long)p * sP + i]) * std::conj(C(Q[(long)p * sQ + i]))).real();
    out[p] = s;
  }
  return hipSuccess;
}

hipError_t launch_sr_finish(int batch, const double* r2, const double* m2, const double* g2, const int* active,
                            double accept, double* resid, int* info, int info_mod, hipStream_t) {
  for (int p = 0; p < batch; ++p) {
    const double r = std::sqrt(r2[p]) / (std::sqrt(m2[p]) * std::sqrt(g2[p]));
    if (resid) resid[p] = r;
    int st = ST_OK;
    if (std::isnan(r) || !std::isfinite(r2[p])) st = ST_ENONFINITE;
    else if ((active && active[p]) || r > accept) st = ST_ENOCONV;
    if (st != ST_OK && info) {
      int* t = info + (info_mod > 0 ? p % info_mod : p);
      if (*t == ST_OK) *t = st;
    }
  }
  return hipSuccess;
}

hipError_t launch_check_finite(int b, int batch, const double2* X, long sX, int* info, int info_mod, hipStream_t) {
  for (int p = 0; p < batch; ++p)
    for (long i = 0; i < (long)b * b; ++i) {
      const double2 v = X[(long)p * sX + i];
      if (!std::isfinite(v.x) || !std::isfinite(v.y)) {
        int* t = info + (info_mod > 0 ? p % info_mod : p);
        if (*t == ST_OK) *t = ST_ENONFINITE;
        break;
      }
    }
  return hipSuccess;
}

hipError_t launch_lincomb(int b, int batch, double2 c1, const double2* X, long sX, double2 c2, const double2* Y,
                          long sY, double2 g, double2* out, long sOut, const int* active, hipStream_t) {
  for (int p = 0; p < batch; ++p) {
    if (!act(active, p)) continue;
    for (long i = 0; i < (long)b * b; ++i) {
      cd r = 0;
      if (X) r += C(c1) * C(X[(long)p * sX + i]);
      if (Y) r += C(c2) * C(Y[(long)p * sY + i]);
      if (i / b == i % b) r += C(g);
      out[(long)p * sOut + i] = D(r);
    }
  }
  return hipSuccess;
}

hipError_t launch_fill_int(int n, int* p, int v, hipStream_t) {
  for (int i = 0; i < n; ++i) p[i] = v;
  return hipSuccess;
}

hipError_t launch_seed_flags(int np, const int* flags, int* active, int* iters, hipStream_t) {
  for (int p = 0; p < np; ++p) {
    active[p] = flags[p] == ST_OK ? 0 : 1;
    iters[p] = 0;
  }
  return hipSuccess;
}

hipError_t launch_seed_select(int b, int np, const int* flags, const double2* g_dec, double2* g, hipStream_t) {
  const long n = (long)b * b;
  for (int p = 0; p < np; ++p)
    if (flags[p] != ST_OK) std::memcpy(g + p * n, g_dec + p * n, sizeof(double2) * n);
  return hipSuccess;
}

hipError_t launch_closure_accept(int np, const double* r2, const double* m2, const double* g2, double accept, int iter,
                                 int* active, int* iters, int* accepted, int* closed, hipStream_t) {
  for (int p = 0; p < np; ++p) {
    int c = 0;
    if (active[p]) {
      const double r = std::sqrt(r2[p]) / (std::sqrt(m2[p]) * std::sqrt(g2[p]));
      if (r == r && std::isfinite(r) && r <= accept) {
        c = 1;
        active[p] = 0;
        iters[p] = iter;
        accepted[p] = ST_OK;
      }
    }
    closed[p] = c;
  }
  return hipSuccess;
}

hipError_t rt_copy_d2d(void* dst, const void* src, size_t bytes, hipStream_t) {
  std::memmove(dst, src, bytes);
  return hipSuccess;
}

// streams, events and graphs: the simulation runs every launch eagerly in
// issue order, which is one valid schedule of the fork/join plan.
hipError_t rt_stream_create(hipStream_t* s) {
  static int dummy[16];
  static std::atomic<int> next{0};
  *s = (hipStream_t)&dummy[(next++) % 16];
  return hipSuccess;
}
hipError_t rt_stream_destroy(hipStream_t) { return hipSuccess; }
hipError_t rt_event_create(hipEvent_t* e) {
  static int dummy[64];
  static std::atomic<int> next{0};
  *e = (hipEvent_t)&dummy[(next++) % 64];
  return hipSuccess;
}
hipError_t rt_event_destroy(hipEvent_t) { return hipSuccess; }
hipError_t rt_record_wait(hipEvent_t, hipStream_t, hipStream_t) { return hipSuccess; }
hipError_t rt_capture_begin(hipStream_t) { return hipSuccess; }
hipError_t rt_capture_end(hipStream_t, void** exec) {
  *exec = (void*)1;
  return hipSuccess;
}
hipError_t rt_graph_launch(void*, hipStream_t) { return hipSuccess; }
hipError_t rt_graph_destroy(void*) { return hipSuccess; }
double rt_wallclock_hz() { return 1e8; }
hipError_t launch_stamp(unsigned long long* dst, hipStream_t) {
  static std::atomic<unsigned long long> t{0};
  *dst = ++t;
  return hipSuccess;
}

hipError_t launch_queue_pop(double* energies, int e0, int n, int n_slots, const double* task_E, int n_tasks,
                            int* round, int* slot_task, int* info, hipStream_t) {
  const int r = *round;
  for (int i = 0; i < n; ++i) {
    const long t = (long)r * n_slots + e0 + i;
    if (t < n_tasks) {
      energies[e0 + i] = task_E[t];
      slot_task[i] = (int)t;
    } else {
      slot_task[i] = -1;
    }
    info[i] = 0;
  }
  *round = r + 1;
  return hipSuccess;
}

hipError_t launch_queue_finish(const double2* GRd, int nb, int b, int n, const int* slot_task, const int* info,
                               int* task_info, double* task_dos, unsigned long long* task_stamp, hipStream_t s) {
  for (int i = 0; i < n; ++i) {
    const int t = slot_task[i];
    if (t < 0) continue;
    const double2* g = GRd + (long)i * nb * b * b;
    double acc = 0.0;
    for (int k = 0; k < nb * b; ++k) acc += g[(long)(k / b) * b * b + (long)(k % b) * b + (k % b)].y;
    task_info[t] = info[i];
    task_dos[t] = -acc / M_PI;
    launch_stamp(task_stamp + t, s);
  }
  return hipSuccess;
}

void prof_begin(int, hipStream_t) {}
void prof_end(int, hipStream_t, double, double) {}

}  // namespace negf
