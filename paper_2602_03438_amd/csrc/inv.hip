// Batched in-place inversion of complex n x n blocks by blocked Gauss-Jordan
// elimination with partial (row) pivoting.
//
// Block step for the panel J = [j0, j0+nb) of the current matrix A:
//   1. panel kernel (one workgroup per matrix, one thread per row, the n x nb
//      panel in registers): nb unblocked Gauss-Jordan steps restricted to the
//      panel -- pivot = the row r >= j of largest |Re a_rj| + |Im a_rj| (compared
//      to 2^-9 relative, ties to the smaller row), row interchange, scale the
//      pivot row, eliminate the column from every other row with the
//      multipliers stored in place.  The result W = [A_JJ^{-1}; -A_RJ A_JJ^{-1}]
//      (rows in pivoted order) goes back into the panel columns.  The same
//      workgroup composes the nb interchanges into one row map, applies it to
//      the other columns of the current sub-panel, copies the pivot rows into U
//      (nb x n), clears those rows, and folds the map into the row orders sigma
//      (whole matrix), tau (since the start of the super-panel) and rho (since
//      the start of the sub-panel).
//   2. product: A += W U on the matrix cores (one batched complex product,
//      K = nb) over the other columns of the sub-panel: pivot rows become
//      A_JJ^{-1} A_JC, the other rows A_RC - A_RJ A_JJ^{-1} A_JC.  One launch
//      covers the whole sub-panel; the panel's own columns (W, read in place)
//      are computed from stale U columns and not stored.
// Three levels: panels of nb columns inside sub-panels of NBM = 64 columns
// inside super-panels of NBO = 128 columns.  After a sub-panel the other
// columns of its super-panel are brought up to date (interchanges through rho,
// pivot rows to Um, one product with K = 64); after a super-panel the columns
// outside it (interchanges through tau, pivot rows to Uo, one product with
// K = 128).  Each level's W is the block's own columns, read in place.  The
// K = nb products touch only the 64 columns of a sub-panel, which is what
// keeps the HBM traffic of the narrow updates down.
// After the last panel A holds (P A)^{-1} with (P A)[i] = A[sigma[i]]; the
// inverse A^{-1}[r][c] = (P A)^{-1}[r][sigma^{-1}[c]] is a column gather.
// Arithmetic: 8 n^3 real flops per matrix, all but O(n^2 nb) of them in the
// batched products.
#include "internal.h"

namespace negf {

namespace {

constexpr int MAX_ROWS = 1024;
constexpr int NB_MAX = 32;
constexpr int NBM = 64;    // sub-panel width (middle level)
// Super-panel width (outer level).  256 would halve the outer products but
// doubles the forward error of the inverse at n = 512 (CPU emulation of this
// scheme on matrices of condition 1e6 .. 1e12); 128 matches LAPACK's.
constexpr int NBO = 128;

struct PanelArgs {
  int n, j0, nbw;
  int c0, c1;               // the current sub-panel: columns the interchanges and U cover
  int t0;                   // first column of the current super-panel
  double2* A; long lda, sA;
  double2* U; long sU;      // U_p: NB x n row-major (columns of [c0, c1) outside the panel written)
  int* sigma;               // sigma_p[i]: original row now at position i
  int* tau;                 // tau_p[i]: row, at the start of the super-panel, now at position i
  int* rho; long sS;        // rho_p[i]: row, at the start of the sub-panel, now at position i
  int* info; int info_mod;
  const int* active;
  unsigned long long* flop_slots;   // nullable (profiling): executed flops of the panel
};

constexpr int STAGE_ROWS = 128;   // rows per chunk of the panel's load through LDS

// Shared state of one panel workgroup.
template <int NB>
struct PanelLds {
  unsigned red[MAX_ROWS / 64] __attribute__((aligned(16)));
  v2d prow[NB];              // pivot row, unscaled, in the rotated column order
  int spiv[NB];
  int status;                // first failure of the panel (set by the pivot holder of that step)
  int cont[MAX_ROWS];        // cont[i]: row, at the start of the panel, whose content is now at row i
  // first the transposition buffer of the panel load ([STAGE_ROWS][NB + 1]),
  // later the new contents of the interchanged rows below the panel ([NB][NBM])
  static constexpr int BUF = (STAGE_ROWS * (NB + 1) > NB * NBM) ? STAGE_ROWS * (NB + 1) : NB * NBM;
  v2d buf[BUF];
};

// Maximum of an unsigned value over the 64 lanes of a wavefront: prefix maxima
// inside each row of 16 lanes by DPP row shifts, then the row broadcasts carry
// them to lane 63.
__device__ __forceinline__ unsigned wave_max_u32(unsigned v) {
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, false));  // row_shr:1
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, false));  // row_shr:2
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, false));  // row_shr:4
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, false));  // row_shr:8
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false));  // row_bcast:15
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false));  // row_bcast:31
  return (unsigned)__builtin_amdgcn_readlane((int)v, 63);
}

// Pivot key of row r: the upper 21 bits of the magnitude |Re| + |Im| (a
// non-negative double orders like its bit pattern; a NaN ranks above
// everything so that it is taken and reported) and 2047 - r in the low 11
// bits, so that the unsigned maximum picks the largest magnitude (to 2^-9
// relative) and, among equal keys, the smallest row.
__device__ __forceinline__ unsigned pivot_key(v2d v, int r) {
  const double m = fabs(v.x) + fabs(v.y);
  const unsigned hi = (unsigned)((unsigned long long)__double_as_longlong(m) >> 32);
  return ((m != m) ? 0xFFFFF800u : (hi & 0xFFFFF800u)) | (unsigned)(2047 - r);
}

__device__ __forceinline__ v2d vmul(v2d a, v2d b) { return v2d{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }

// 1 / d = conj(d) / |d|^2 with one division: d is first scaled by the power of
// two of its larger component (exact), so |d|^2 neither overflows nor
// underflows.  d = 0 gives a non-finite result.
__device__ __forceinline__ v2d vinv(v2d d) {
  const double m = fmax(fabs(d.x), fabs(d.y));
  const int e = m > 0.0 && m <= 1.7976931348623157e308 ? ilogb(m) : 0;
  const double ax = ldexp(d.x, -e), ay = ldexp(d.y, -e);
  const double q = 1.0 / (ax * ax + ay * ay);
  return v2d{ldexp(ax * q, -e), ldexp(-ay * q, -e)};
}

// x -= f * p (complex), as four fused multiply-adds
__device__ __forceinline__ void csub_mul(v2d& x, v2d f, v2d p) {
  x.x = fma(-f.x, p.x, fma(f.y, p.y, x.x));
  x.y = fma(-f.x, p.y, fma(-f.y, p.x, x.y));
}

// One Gauss-Jordan step of the panel, for column j = j0 + jj.  Each thread
// holds two rows (t and t + NT) as register arrays that are only ever indexed
// by compile-time constants: the step loop advances U columns per iteration
// (the column being eliminated is x[s][KK]) and then rotates the rows by U, so
// the code stays a short loop (straight-line steps over the whole panel are
// tens of KB of code).  Before the loop iteration that starts at
// step jb, x[s][c] holds panel column (jb + c) mod NB; the pivot row in LDS
// uses the same order.  The pivot row is published unscaled and every thread
// forms 1 / pivot itself, so the only serial work between the two barriers is
// the owner's LDS store.
template <int NB, int NT, int KK>
__device__ __forceinline__ void panel_step(v2d (&x)[2][NB], int (&lr)[2], PanelLds<NB>& L, int t, int n, int j,
                                           int jj) {
  const int lane = t & 63, wave = t >> 6;
  unsigned key = 0u;
  if (lr[0] < n && lr[0] >= j) key = pivot_key(x[0][KK], lr[0]);
  if (lr[1] < n && lr[1] >= j) key = max(key, pivot_key(x[1][KK], lr[1]));
  key = wave_max_u32(key);
  if (lane == 0) L.red[wave] = key;
  __syncthreads();
  {
    const uint4* rv = reinterpret_cast<const uint4*>(L.red);
#pragma unroll
    for (int q = 0; q < MAX_ROWS / 256; ++q) {
      const uint4 u = rv[q];
      key = max(max(key, u.x), max(u.y, max(u.z, u.w)));
    }
  }
  const int pr = 2047 - (int)(key & 0x7FFu);
  // The interchange of rows j and pr is only a relabelling: the holder of row pr
  // becomes row j (the pivot row), the holder of row j becomes row pr.
  const bool p0 = lr[0] == pr, p1 = lr[1] == pr;
  if (p0) {
#pragma unroll
    for (int c = 0; c < NB; ++c) L.prow[c] = x[0][c];
  }
  if (p1) {
#pragma unroll
    for (int c = 0; c < NB; ++c) L.prow[c] = x[1][c];
  }
  if (p0 || p1) {
    if (pr != j) {
      const int u = L.cont[j];
      L.cont[j] = L.cont[pr];
      L.cont[pr] = u;
    }
    L.spiv[jj] = pr;
  }
  __syncthreads();
  // the whole pivot row at once: one LDS latency instead of one per column
  v2d pc[NB];
#pragma unroll
  for (int c = 0; c < NB; ++c) pc[c] = L.prow[c];
  const v2d d = pc[KK];
  const v2d dinv = vinv(d);
  if ((p0 || p1) && L.status == ST_OK) {
    if (d.x == 0.0 && d.y == 0.0) L.status = ST_ESINGULAR;
    else if (!(isfinite(dinv.x) && isfinite(dinv.y))) L.status = ST_ENONFINITE;
  }
  if (lr[0] == j) lr[0] = pr;
  if (lr[1] == j) lr[1] = pr;
  if (p0) lr[0] = j;
  if (p1) lr[1] = j;
  // the new pivot row is cleared and then takes the same update as every other
  // row with multiplier -1 / pivot, which leaves pivot row / pivot in it
  if (p0) {
#pragma unroll
    for (int c = 0; c < NB; ++c) x[0][c] = v2d{0.0, 0.0};
  }
  if (p1) {
#pragma unroll
    for (int c = 0; c < NB; ++c) x[1][c] = v2d{0.0, 0.0};
  }
  const v2d f0 = p0 ? -dinv : vmul(x[0][KK], dinv);
  const v2d f1 = p1 ? -dinv : vmul(x[1][KK], dinv);
  // column j of the inverse: -x_rj / pivot in the other rows, 1 / pivot in row j
  x[0][KK] = -f0;
  x[1][KK] = -f1;
#pragma unroll
  for (int c = 0; c < NB; ++c) {
    if (c == KK) continue;
    csub_mul(x[0][c], f0, pc[c]);
    csub_mul(x[1][c], f1, pc[c]);
  }
}

template <int NB, int NT, int KK, int U>
struct PanelGroup {
  __device__ __forceinline__ static void run(v2d (&x)[2][NB], int (&lr)[2], PanelLds<NB>& L, int t, int n, int j0,
                                             int jb, int nbw) {
    if (jb + KK < nbw) {
      panel_step<NB, NT, KK>(x, lr, L, t, n, j0 + jb + KK, jb + KK);
      PanelGroup<NB, NT, KK + 1, U>::run(x, lr, L, t, n, j0, jb, nbw);
    }
  }
};
template <int NB, int NT, int U>
struct PanelGroup<NB, NT, U, U> {
  __device__ __forceinline__ static void run(v2d (&)[2][NB], int (&)[2], PanelLds<NB>&, int, int, int, int, int) {}
};

// Panel kernel: one workgroup of NT threads per matrix, two rows per thread
// (n <= 2 NT).  The panel is read coalesced (consecutive lanes along a row)
// and handed to its row owners through LDS in chunks of STAGE_ROWS rows; the
// result W goes back into the panel columns the same way.
template <int NB, int NT>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(1, 2))) gj_panel_kernel(PanelArgs a) {
  const int p = blockIdx.x;
  if (a.active && a.active[p] == 0) return;
  double2* __restrict__ A = a.A + (long)p * a.sA;
  double2* __restrict__ U = a.U + (long)p * a.sU;
  int* __restrict__ sigma = a.sigma + (long)p * a.sS;
  int* __restrict__ tau = a.tau + (long)p * a.sS;
  int* __restrict__ rho = a.rho + (long)p * a.sS;
  const v2d* __restrict__ Av = reinterpret_cast<const v2d*>(A);
  const int t = threadIdx.x;
  const int n = a.n, j0 = a.j0, nbw = a.nbw;
  const int jend = j0 + nbw;
  const long lda = a.lda;
  __shared__ PanelLds<NB> L;
  if (t < MAX_ROWS / 64) L.red[t] = 0u;   // waves beyond the last never write their slot
  if (t == 0) L.status = ST_OK;
  for (int i = t; i < n; i += NT) L.cont[i] = i;

  // --- panel load: chunk ch covers rows [ch*STAGE_ROWS, (ch+1)*STAGE_ROWS)
  constexpr int CH = 2 * NT / STAGE_ROWS;
  constexpr int PER = STAGE_ROWS * NB / NT;
  static_assert(CH * STAGE_ROWS == 2 * NT && PER * NT == STAGE_ROWS * NB, "panel load must tile evenly");
  v2d x[2][NB];
#pragma unroll
  for (int c = 0; c < NB; ++c) x[0][c] = x[1][c] = v2d{0.0, 0.0};
  v2d ld[PER], nx[PER];
  auto gload = [&](int ch, v2d (&dst)[PER]) {
#pragma unroll
    for (int e = 0; e < PER; ++e) {
      const int idx = e * NT + t, rr = ch * STAGE_ROWS + idx / NB, cc = idx % NB;
      dst[e] = (rr < n && cc < nbw) ? Av[(long)rr * lda + j0 + cc] : v2d{0.0, 0.0};
    }
  };
  gload(0, ld);
  constexpr int CH_UNROLL = CH <= 4 ? CH : 1;   // wider unrolling only adds live address registers
#pragma unroll CH_UNROLL
  for (int ch = 0; ch < CH; ++ch) {
    if (ch + 1 < CH) gload(ch + 1, nx);
#pragma unroll
    for (int e = 0; e < PER; ++e) {
      const int idx = e * NT + t;
      L.buf[(idx / NB) * (NB + 1) + idx % NB] = ld[e];
    }
    __syncthreads();
    const int first = ch * STAGE_ROWS;        // first row of the chunk
    const int tb = first % NT;                // its owner thread
    const bool mine = t >= tb && t < tb + STAGE_ROWS;
    const bool s0 = mine && first < NT, s1 = mine && first >= NT;
    const int li = mine ? t - tb : 0;
#pragma unroll
    for (int c = 0; c < NB; ++c) {
      const v2d v = L.buf[li * (NB + 1) + c];
      x[0][c] = s0 ? v : x[0][c];
      x[1][c] = s1 ? v : x[1][c];
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < PER; ++e) ld[e] = nx[e];
  }

  constexpr int SG = 4;   // steps per loop iteration
  static_assert(NB % SG == 0, "panel width must be a multiple of the step group");
  int rot = 0;
  int lr[2] = {t, t + NT};   // logical row held in each register row
#pragma unroll 1
  for (int jb = 0; jb < nbw; jb += SG) {
    PanelGroup<NB, NT, 0, SG>::run(x, lr, L, t, n, j0, jb, nbw);
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      v2d h[SG];
#pragma unroll
      for (int c = 0; c < SG; ++c) h[c] = x[s][c];
#pragma unroll
      for (int c = 0; c + SG < NB; ++c) x[s][c] = x[s][c + SG];
#pragma unroll
      for (int c = 0; c < SG; ++c) x[s][NB - SG + c] = h[c];
    }
    rot += SG;
  }

  // --- the panel result W = [A_JJ^{-1}; -A_RJ A_JJ^{-1}] back into A's panel columns,
  // through LDS in chunks so that the stores are coalesced; after the rotations
  // x[s][c] holds panel column (c + rot) mod NB
  // (each register row goes to its logical row; both slots are offered to every chunk)
#pragma unroll CH_UNROLL
  for (int ch = 0; ch < CH; ++ch) {
    const int first = ch * STAGE_ROWS;
    if (lr[0] >= first && lr[0] < first + STAGE_ROWS) {
#pragma unroll
      for (int c = 0; c < NB; ++c) L.buf[(lr[0] - first) * (NB + 1) + (c + rot) % NB] = x[0][c];
    }
    if (lr[1] >= first && lr[1] < first + STAGE_ROWS) {
#pragma unroll
      for (int c = 0; c < NB; ++c) L.buf[(lr[1] - first) * (NB + 1) + (c + rot) % NB] = x[1][c];
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < PER; ++e) {
      const int idx = e * NT + t, rr = first + idx / NB, cc = idx % NB;
      if (rr < n && cc < nbw)
        reinterpret_cast<v2d*>(A)[(long)rr * lda + j0 + cc] = L.buf[(idx / NB) * (NB + 1) + cc];
    }
    __syncthreads();
  }

  // The nbw interchanges, composed into cont[], act on the rows D = panel rows
  // and the rows below the panel they touched.  Every new row of D is an old
  // row of D, so all reads go first (pivot rows into U, moved rows into LDS),
  // then, after a barrier, the writes.
  const int c0 = a.c0, cnt = a.c1 - a.c0;
  const int tot = nbw * cnt;
  constexpr int G = (NB > 16 || NT > 256) ? 4 : 8;   // loads in flight per thread and kind
  for (int base = 0; base < tot; base += G * NT) {
    v2d u[G], q[G];
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int e = base + g * NT + t;
      const int s = e / cnt, c = c0 + e % cnt;
      const bool in = e < tot, outside = c < j0 || c >= jend;
      const int qr = in ? L.spiv[s] : 0;
      u[g] = (in && outside) ? Av[(long)L.cont[j0 + s] * lda + c] : v2d{0.0, 0.0};
      q[g] = (in && outside && qr >= jend) ? Av[(long)L.cont[qr] * lda + c] : v2d{0.0, 0.0};
    }
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int e = base + g * NT + t;
      if (e >= tot) continue;
      const int s = e / cnt, c = c0 + e % cnt;
      if (c >= j0 && c < jend) continue;
      reinterpret_cast<v2d*>(U)[(long)s * n + c] = u[g];
      if (L.spiv[s] >= jend) L.buf[s * NBM + (c - c0)] = q[g];
    }
  }
  // row orders: new entry of a row d of D = old entry of row cont[d]
  int d = -1, sv = 0, tv = 0, rv = 0;
  if (t < 2 * nbw) {
    d = t < nbw ? j0 + t : L.spiv[t - nbw];
    if (t >= nbw && d < jend) d = -1;
    if (d >= 0) {
      const int src = L.cont[d];
      sv = j0 == 0 ? src : sigma[src];
      tv = j0 == a.t0 ? src : tau[src];
      rv = j0 == c0 ? src : rho[src];
    }
  }
  __syncthreads();
  for (int e = t; e < tot; e += NT) {
    const int s = e / cnt, c = c0 + e % cnt;
    if (c >= j0 && c < jend) continue;
    A[(long)(j0 + s) * lda + c] = make_double2(0.0, 0.0);
    const int qr = L.spiv[s];
    if (qr >= jend) reinterpret_cast<v2d*>(A)[(long)qr * lda + c] = L.buf[s * NBM + (c - c0)];
  }
  if (j0 == 0) {
    for (int i = t; i < n; i += NT) sigma[i] = L.cont[i];
  } else if (d >= 0) {
    sigma[d] = sv;
  }
  if (j0 == a.t0) {
    for (int i = t; i < n; i += NT) tau[i] = L.cont[i];
  } else if (d >= 0) {
    tau[d] = tv;
  }
  if (j0 == c0) {
    for (int i = t; i < n; i += NT) rho[i] = L.cont[i];
  } else if (d >= 0) {
    rho[d] = rv;
  }
  if (t == 0 && L.status != ST_OK && a.info) atomicCAS(a.info + (a.info_mod > 0 ? p % a.info_mod : p), ST_OK, L.status);
  // nbw elimination steps over n rows and the panel's nbw columns, one complex multiply-add each
  if (t == 0 && a.flop_slots) atomicAdd(a.flop_slots + (p & (PROF_SLOTS - 1)), 8ull * n * nbw * nbw);
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

// Block step of the middle or outer level for the block J = [J0, J0+mo) (a
// sub-panel or a super-panel), one workgroup per (matrix, OUTER_COLS columns)
// of [lo, hi) outside J: the block's interchanges (its content map tau) are
// applied to those columns, the pivot rows J0..J0+mo-1 go to Uo (mo x n) and
// are cleared, and the rows below J that took part receive their new
// contents.  All reads of a block precede its writes (a barrier between).  The
// columns of J already hold their final W.
constexpr int OUTER_COLS = 16;
constexpr int OUTER_THREADS = 256;

__global__ void __launch_bounds__(OUTER_THREADS) gj_outer_kernel(int n, int J0, int mo, int lo, int hi, double2* A,
                                                                 long lda, long sA, double2* Uo, long sU,
                                                                 const int* tau, long sT, const int* active) {
  const int p = blockIdx.y;
  if (active && active[p] == 0) return;
  double2* __restrict__ Ap = A + (long)p * sA;
  double2* __restrict__ U = Uo + (long)p * sU;
  const int cb = lo + blockIdx.x * OUTER_COLS;
  const int w = min(OUTER_COLS, hi - cb);
  const int t = threadIdx.x;
  if (cb >= J0 && cb < J0 + mo) return;
  __shared__ int rows[2 * NBO];
  __shared__ int srcs[2 * NBO];
  __shared__ int nq;
  const int* tp = tau + (long)p * sT;
  if (t == 0) nq = 0;
  __syncthreads();
  for (int i = t; i < mo; i += OUTER_THREADS) {
    rows[i] = J0 + i;
    srcs[i] = tp[J0 + i];
  }
  // rows below J whose content changed (at most mo of them)
  for (int i = J0 + mo + t; i < n; i += OUTER_THREADS) {
    const int s = tp[i];
    if (s != i) {
      const int k = atomicAdd(&nq, 1);
      if (mo + k < 2 * NBO) {
        rows[mo + k] = i;
        srcs[mo + k] = s;
      }
    }
  }
  __syncthreads();
  const int tot = min(mo + nq, 2 * NBO) * OUTER_COLS;
  constexpr int G = 2 * NBO * OUTER_COLS / OUTER_THREADS;
  const v2d* __restrict__ Av = reinterpret_cast<const v2d*>(Ap);
  v2d v[G];
#pragma unroll
  for (int g = 0; g < G; ++g) {
    const int e = g * OUTER_THREADS + t, k = e / OUTER_COLS, cc = e % OUTER_COLS;
    v[g] = (e < tot && cc < w) ? Av[(long)srcs[k] * lda + cb + cc] : v2d{0.0, 0.0};
  }
  __syncthreads();
  v2d* __restrict__ Aw = reinterpret_cast<v2d*>(Ap);
#pragma unroll
  for (int g = 0; g < G; ++g) {
    const int e = g * OUTER_THREADS + t, k = e / OUTER_COLS, cc = e % OUTER_COLS;
    if (e < tot && cc < w) {
      if (k < mo) {
        reinterpret_cast<v2d*>(U)[(long)k * n + cb + cc] = v[g];
        Aw[(long)(J0 + k) * lda + cb + cc] = v2d{0.0, 0.0};
      } else {
        Aw[(long)rows[k] * lda + cb + cc] = v[g];
      }
    }
  }
}

struct ScratchLayout {
  size_t per_al;
  size_t off_U, off_Um, off_Uo, off_sigma, off_tau, off_rho;
};

ScratchLayout layout(int n) {
  ScratchLayout L{};
  size_t o = 0;
  L.off_U = o;  o += (size_t)NB_MAX * n * sizeof(double2);
  L.off_Um = o; o += (size_t)NBM * n * sizeof(double2);
  L.off_Uo = o; o += (size_t)NBO * n * sizeof(double2);
  L.off_sigma = o; o += (size_t)n * sizeof(int);
  L.off_tau = o;   o += (size_t)n * sizeof(int);
  L.off_rho = o;   o += (size_t)n * sizeof(int);
  L.per_al = (o + 255) & ~(size_t)255;
  return L;
}

// Columns [c_lo, c_hi) of every matrix: A[:, c] += A[:, jb:jb+K] U[:, c], the
// first operand being the block's result W read in place (those columns are
// not written by this product).
// A[:, c] += W U[:, c] for the columns c in [c_lo, c_hi) outside [s_lo, s_hi), W = A[:, jb, jb + K)
// read in place (the skipped columns may be W's own: they are computed but not stored).
hipError_t update_cols(const InvDesc& d, int n, int jb, int K, const double2* U, long sU, int c_lo, int c_hi,
                       hipStream_t s, int s_lo = 0, int s_hi = 0) {
  if (c_hi <= c_lo) return hipSuccess;
  if (s_hi > s_lo && s_lo <= c_lo && s_hi >= c_hi) return hipSuccess;   // nothing left to store
  GemmDesc g{};
  g.M = n; g.N = c_hi - c_lo; g.K = K; g.batch = d.batch;
  g.opA = OP_N; g.opB = OP_N;
  g.A = MatRef{d.M + jb, d.ldm, d.sM};
  g.B = MatRef{U + c_lo, n, sU};
  g.alpha = make_double2(1.0, 0.0);
  g.beta = make_double2(1.0, 0.0);
  g.Cin = MatRef{d.M + c_lo, d.ldm, d.sM};
  g.C = MatOut{d.M + c_lo, d.ldm, d.sM};
  g.active = d.active;
  g.prec = PREC_F64;
  g.xcd_remap = 1;
  g.tile = tile_for_launch(GEMM_TILE_64_8W, g.M, g.N, g.batch);
  g.prof_class = KC_INV_GEMM;
  g.gauss = d.gauss;
  if (s_hi > s_lo) {
    g.skip_lo = s_lo - c_lo;
    g.skip_hi = s_hi - c_lo;
  }
  return launch_gemm(g, s);
}

}  // namespace

size_t inverse_scratch_bytes(int n, int batch) { return layout(n).per_al * batch; }

hipError_t launch_inverse(const InvDesc& d, hipStream_t s) {
  const int n = d.n;
  if (n <= 0 || d.batch <= 0) return hipSuccess;
  if (n > MAX_ROWS) return hipErrorInvalidValue;
  const int NB = (d.nb == 32 && n <= 512) ? 32 : 16;
  static_assert(NBM % NB_MAX == 0 && NBO % NBM == 0, "block widths must nest");
  const ScratchLayout SL = layout(n);
  const long sItem = (long)(SL.per_al / sizeof(double2));   // per_al is a multiple of 256 bytes
  const long sI = (long)(SL.per_al / sizeof(int));
  char* base = (char*)d.scratch;
  double2* U = (double2*)(base + SL.off_U);
  double2* Um = (double2*)(base + SL.off_Um);
  double2* Uo = (double2*)(base + SL.off_Uo);
  int* sigma = (int*)(base + SL.off_sigma);
  int* tau = (int*)(base + SL.off_tau);
  int* rho = (int*)(base + SL.off_rho);
  hipError_t e = hipSuccess;
  // interchanges of the block [J0, J0+mo) through its map into the columns [lo, hi) outside it,
  // then A[:, c] += W Ub[:, c] there, W read in place from the block's columns
  auto block_step = [&](int J0, int mo, int lo, int hi, double2* Ub, const int* map) -> hipError_t {
    prof_begin(KC_INV_SWAP, s);
    hipLaunchKernelGGL(gj_outer_kernel, dim3((hi - lo + OUTER_COLS - 1) / OUTER_COLS, d.batch), dim3(OUTER_THREADS),
                       0, s, n, J0, mo, lo, hi, d.M, d.ldm, d.sM, Ub, sItem, map, sI, d.active);
    prof_end(KC_INV_SWAP, s, 0, 0);
    hipError_t r = hipGetLastError();
    if (r != hipSuccess) return r;
    if ((r = update_cols(d, n, J0, mo, Ub, sItem, lo, J0, s)) != hipSuccess) return r;
    return update_cols(d, n, J0, mo, Ub, sItem, J0 + mo, hi, s);
  };
  for (int J0 = 0; J0 < n; J0 += NBO) {
    const int mo = min(NBO, n - J0);
    for (int S0 = J0; S0 < J0 + mo; S0 += NBM) {
      const int ms = min(NBM, J0 + mo - S0);
      for (int j0 = S0; j0 < S0 + ms; j0 += NB) {
        const int nbw = min(NB, S0 + ms - j0);
        PanelArgs pa{n, j0, nbw, S0, S0 + ms, J0, d.M, d.ldm, d.sM, U, sItem, sigma, tau, rho, sI, d.info,
                     d.info_mod, d.active, prof_flop_slots(KC_INV_PANEL)};
        prof_begin(KC_INV_PANEL, s);
        // two rows per thread: 256 threads up to n = 512, 512 up to n = MAX_ROWS
        if (NB == 32) hipLaunchKernelGGL((gj_panel_kernel<32, 256>), dim3(d.batch), dim3(256), 0, s, pa);
        else if (n <= 512) hipLaunchKernelGGL((gj_panel_kernel<16, 256>), dim3(d.batch), dim3(256), 0, s, pa);
        else hipLaunchKernelGGL((gj_panel_kernel<16, MAX_ROWS / 2>), dim3(d.batch), dim3(MAX_ROWS / 2), 0, s, pa);
        prof_end(KC_INV_PANEL, s, 0.0, 0);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        // the other columns of the sub-panel, on both sides of the panel, in one launch:
        // A[:, c] += W U[:, c], W read in place from the panel columns (which are not stored)
        if ((e = update_cols(d, n, j0, nbw, U, sItem, S0, S0 + ms, s, j0, j0 + nbw)) != hipSuccess) return e;
      }
      // middle level: the other columns of the super-panel
      if (ms < mo && (e = block_step(S0, ms, J0, J0 + mo, Um, rho)) != hipSuccess) return e;
    }
    // outer level: the columns outside the super-panel
    if (mo < n && (e = block_step(J0, mo, 0, n, Uo, tau)) != hipSuccess) return e;
  }
  prof_begin(KC_INV_PERM, s);
  hipLaunchKernelGGL(gj_gather_kernel, dim3((n + GATHER_ROWS - 1) / GATHER_ROWS, d.batch), dim3(256), 0, s, n, d.M,
                     d.ldm, d.sM, d.out, d.ldo, d.sO, sigma, sI, d.active);
  prof_end(KC_INV_PERM, s, 0, 32.0 * n * n * d.batch);
  return hipGetLastError();
}

}  // namespace negf
