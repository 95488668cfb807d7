// Batched complex block products on the CDNA4 matrix cores.
//
// C_p = alpha * op(A_p) op(B_p) + beta * Cin_p with op = identity or conjugate
// transpose, for a batch of interleaved-complex matrices.  The complex product
// is formed from four real products per k-step (re*re, -im*im, re*im, im*re)
// on v_mfma_f64_16x16x4f64 (double) or v_mfma_f32_16x16x4f32 (single: operands
// rounded to complex64 when they are staged, single accumulation, result
// widened to double on store).  The double kernel can instead use three real
// products (Gauss's method): P1 = Re A Re B, P2 = Im A Im B,
// P3 = (Re A + Im A)(Re B + Im B), Re C = P1 - P2, Im C = P3 - P1 - P2; the
// operand sums are formed from the staged tiles, so the matrix cores do 3/4
// of the work.  Its error is bounded normwise by a small multiple of the
// four-product one (the imaginary part is not componentwise accurate when it
// cancels).
//
// Work decomposition: one workgroup of WM x WN waves per BM x BN output tile
// (64x64 with 2x2 or 4x2 waves, 128x64 with 4x2 or 8x2, 128x128 with 4x2); each wave owns
// a (BM/WM) x (BN/WN) sub-tile of 16 x 16 MFMA tiles with separate real and
// imaginary accumulators.  K advances in steps of 16 complex values through
// two LDS stages: global loads for step k+1 are issued into registers before
// the MFMAs of step k and land in the other LDS stage afterwards, so there is
// one barrier per step.  Consecutive workgroup ids are dealt round-robin over
// the 8 XCDs; with xcd_remap the tiles of one batch item are renumbered so
// that they land on the same XCD and share its L2.
//
// LDS keeps each tile in the layout it has in HBM (no transpose on the store
// path; the MFMA operand reads do the reorientation):
//   "row" layout [BM][16+1]: BM rows (m or n), 16 contiguous k values
//   "col" layout [16][BM+1]: 16 k rows, BM contiguous m or n values
// op(A)=A   (A stored M x K) -> row ; op(A)=A^H (stored K x M) -> col
// op(B)=B   (B stored K x N) -> col ; op(B)=B^H (stored N x K) -> row
// The +1 complex padding keeps a 16-lane group of MFMA operand reads on
// distinct banks in both layouts.
#include "internal.h"

namespace negf {

namespace {

constexpr int BK = 16;

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

// Row of accumulator element v of a lane (column = lane % 16) in the 16 x 16
// output tile: 4*(lane/16)+v for the single-precision MFMA, lane/16+4*v for
// the double-precision one (measured on gfx950).
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
  int upper;   // skip tiles that lie entirely below the diagonal
  const unsigned long long* kmask;   // zero-slab map of a sparse operand (64 x 64 tiles only)
  int kmask_op;                      // 1: indexed by the column tile, 2: by the row tile
  int skip_lo, skip_hi;              // columns of C not stored (inversion updates, tag 1)
  unsigned long long* flop_slots;    // nullable (profiling): each wave adds the flops of the matrix
                                     // instructions it issued to one of PROF_SLOTS counters
};

template <int BM_, int BN_, int WM_, int WN_>
struct Cfg {
  static constexpr int BM = BM_, BN = BN_, WM = WM_, WN = WN_;
  static constexpr int NT = 64 * WM * WN;
  static constexpr int TM = BM / WM, TN = BN / WN;   // wave sub-tile
  static constexpr int FM = TM / 16, FN = TN / 16;   // MFMA tiles per wave
  static constexpr int LA = BM * BK / NT, LB = BN * BK / NT;  // staged elements per thread
  static constexpr int LD_ROW = BK + 1;
  static constexpr int LDA_COL = BM + 1, LDB_COL = BN + 1;
  static constexpr int A_ELEMS = (BM * LD_ROW > BK * LDA_COL) ? BM * LD_ROW : BK * LDA_COL;
  static constexpr int B_ELEMS = (BN * LD_ROW > BK * LDB_COL) ? BN * LD_ROW : BK * LDB_COL;
  static_assert(LA * NT == BM * BK && LB * NT == BN * BK, "tile must split evenly over the threads");
  static_assert(FM >= 1 && FN >= 1 && TM % 16 == 0 && TN % 16 == 0, "wave tile must be 16-aligned");
};

// Stage an R x 16 (row layout) or 16 x R (col layout) operand tile into registers.
// row0/col0: tile origin in the stored matrix; nR/nC: stored matrix extent.
template <int R, int NT, int L, bool ROWL>
__device__ __forceinline__ void load_tile(double2 (&r)[L], const double2* __restrict__ base, long ld, int row0,
                                          int col0, int nR, int nC) {
  const int t = threadIdx.x;
#pragma unroll
  for (int j = 0; j < L; ++j) {
    const int e = t + NT * j;
    const int rr = ROWL ? e / BK : e / R;
    const int cc = ROWL ? e % BK : e % R;
    const int gr = row0 + rr, gc = col0 + cc;
    r[j] = (gr < nR && gc < nC) ? base[(long)gr * ld + gc] : make_double2(0.0, 0.0);
  }
}

template <typename T, int R, int NT, int L, bool ROWL>
__device__ __forceinline__ void store_tile(typename Cx<T>::type* s, const double2 (&r)[L], bool conj) {
  const int t = threadIdx.x;
#pragma unroll
  for (int j = 0; j < L; ++j) {
    const int e = t + NT * j;
    const int idx = ROWL ? (e / BK) * (BK + 1) + (e % BK) : (e / R) * (R + 1) + (e % R);
    s[idx] = to_cx<T>(r[j], conj);
  }
}

// Full tiles (the tile lies inside the matrix): no bounds tests, native vectors.
template <int R, int NT, int L, bool ROWL>
__device__ __forceinline__ void load_tile_full(v2d (&r)[L], const double2* __restrict__ base, long ld, int row0,
                                               int col0) {
  const int t = threadIdx.x;
#pragma unroll
  for (int j = 0; j < L; ++j) {
    const int e = t + NT * j;
    const int rr = ROWL ? e / BK : e / R;
    const int cc = ROWL ? e % BK : e % R;
    r[j] = *reinterpret_cast<const v2d*>(base + (long)(row0 + rr) * ld + col0 + cc);
  }
}

template <typename T, int R, int NT, int L, bool ROWL>
__device__ __forceinline__ void store_tile_v(typename Cx<T>::type* s, const v2d (&r)[L], bool conj) {
  const int t = threadIdx.x;
#pragma unroll
  for (int j = 0; j < L; ++j) {
    const int e = t + NT * j;
    const int idx = ROWL ? (e / BK) * (BK + 1) + (e % BK) : (e / R) * (R + 1) + (e % R);
    s[idx] = to_cx<T>(make_double2(r[j].x, r[j].y), conj);
  }
}

// TAG only separates symbols in profiles (0: sweep products, 1: inversion
// updates, 2: products with a sparse coupling operand); the code is the same.  FULL: M, N and K are multiples
// of the tile and of the K-step, so no operand or result access needs a bounds
// test; operand tiles are then fetched two K-steps ahead (two register sets)
// instead of one.
template <typename T, int OPA, int OPB, typename CF, int TAG = 0, bool GAUSS = false, bool FULL = false>
__global__ void __launch_bounds__(CF::NT, CF::NT >= 1024 ? 1 : 2) zgemm_kernel(KArgs a) {
  typedef typename Cx<T>::type CT;
  typedef typename Acc<T>::type AT;
  constexpr int BM = CF::BM, BN = CF::BN, NT = CF::NT, FM = CF::FM, FN = CF::FN;
  constexpr bool A_ROW = (OPA == OP_N);  // A stored M x K
  constexpr bool B_ROW = (OPB == OP_C);  // B stored N x K
  __shared__ CT sA[2][CF::A_ELEMS];
  __shared__ CT sB[2][CF::B_ELEMS];

  const int per_item = a.tiles_m * a.tiles_n;
  const long total = (long)per_item * a.batch;
  long lid = blockIdx.x;
  if (a.xcd_remap && (total & 7) == 0) lid = (lid & 7) * (total >> 3) + (lid >> 3);
  const int p = (int)(lid / per_item);
  const int tid = (int)(lid - (long)p * per_item);
  if (a.active && a.active[p] == 0) return;
  const int tm = tid / a.tiles_n, tn = tid - tm * a.tiles_n;
  const int m0 = tm * BM, n0 = tn * BN;
  if (a.upper && n0 + BN <= m0) return;

  const double2* __restrict__ Ap = a.A + (long)p * a.sA;
  const double2* __restrict__ Bp = a.B + (long)p * a.sB;

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave / CF::WN, wn = wave % CF::WN;
  const int li = lane & 15, lk = lane >> 4;

  // four products: accR = Re C, accI = Im C; Gauss: accR = P1, accI = P2, accS = P3
  constexpr int NS = GAUSS ? FM : 1;
  AT accR[FM][FN], accI[FM][FN], accS[NS][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      accR[i][j] = AT{0, 0, 0, 0};
      accI[i][j] = AT{0, 0, 0, 0};
    }
#pragma unroll
  for (int i = 0; i < NS; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) accS[i][j] = AT{0, 0, 0, 0};

  const int nk = (a.K + BK - 1) / BK;
  // one K-step of MFMAs on the LDS stage (xA, xB); bit i*FN+j of `on` enables the
  // products of the wave's row fragment i with its column fragment j (all of them
  // unless a sparse operand's fragment is zero in this K-step)
  constexpr unsigned ALL_ON = (1u << (FM * FN)) - 1u;
  // only the products with a sparse operand (tag 2, 64 x 64 tiles) read a zero-slab map
  constexpr bool SPARSE_OK = TAG == 2 && BM == 64 && BN == 64;
  // (for the dense kernels the guard folds to true at compile time)
  auto on_ij = [&](unsigned on, int i, int j) { return !SPARSE_OK || ((on >> (i * FN + j)) & 1u) != 0u; };
  // profiling: the flops of the fragment products a wave issued ((GAUSS ? 3 : 4) real products of
  // BK / 4 matrix instructions each, 2 * 16 * 16 * 4 flop per instruction), striped over the slots
  auto prof_count = [&](unsigned long long* slots, unsigned fr) {
    if (slots && (threadIdx.x & 63) == 0) {
      const unsigned long long fl = (unsigned long long)fr * (GAUSS ? 3u : 4u) * (BK / 4) * 2048ull;
      atomicAdd(slots + ((blockIdx.x * (CF::NT / 64) + (threadIdx.x >> 6)) & (PROF_SLOTS - 1)), fl);
    }
  };
  auto mac = [&](const CT* __restrict__ xA, const CT* __restrict__ xB, unsigned on) {
#pragma unroll
    for (int kk = 0; kk < BK / 4; ++kk) {
      const int kq = kk * 4 + lk;
      CT av[FM], bv[FN];
#pragma unroll
      for (int i = 0; i < FM; ++i) {
        const int m = wm * CF::TM + i * 16 + li;
        av[i] = A_ROW ? xA[m * CF::LD_ROW + kq] : xA[kq * CF::LDA_COL + m];
      }
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        const int n = wn * CF::TN + j * 16 + li;
        bv[j] = B_ROW ? xB[n * CF::LD_ROW + kq] : xB[kq * CF::LDB_COL + n];
      }
      if constexpr (GAUSS) {
        T as[FM], bs[FN];
#pragma unroll
        for (int i = 0; i < FM; ++i) as[i] = av[i].x + av[i].y;
#pragma unroll
        for (int j = 0; j < FN; ++j) bs[j] = bv[j].x + bv[j].y;
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j)
            if (on_ij(on, i, j)) accR[i][j] = mfma16(av[i].x, bv[j].x, accR[i][j]);
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j)
            if (on_ij(on, i, j)) accI[i][j] = mfma16(av[i].y, bv[j].y, accI[i][j]);
#pragma unroll
        for (int i = 0; i < NS; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j)
            if (on_ij(on, i, j)) accS[i][j] = mfma16(as[i], bs[j], accS[i][j]);
      } else {
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j)
            if (on_ij(on, i, j)) accR[i][j] = mfma16(av[i].x, bv[j].x, accR[i][j]);
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j)
            if (on_ij(on, i, j)) accI[i][j] = mfma16(av[i].x, bv[j].y, accI[i][j]);
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j)
            if (on_ij(on, i, j)) accR[i][j] = mfma16(-av[i].y, bv[j].y, accR[i][j]);
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j)
            if (on_ij(on, i, j)) accI[i][j] = mfma16(av[i].y, bv[j].x, accI[i][j]);
      }
    }
  };
  if constexpr (FULL) {
    v2d qa[2][CF::LA], qb[2][CF::LB];
    auto gl = [&](v2d (&ra)[CF::LA], v2d (&rb)[CF::LB], int k0) {
      if (A_ROW) load_tile_full<BM, NT, CF::LA, true>(ra, Ap, a.lda, m0, k0);
      else       load_tile_full<BM, NT, CF::LA, false>(ra, Ap, a.lda, k0, m0);
      if (B_ROW) load_tile_full<BN, NT, CF::LB, true>(rb, Bp, a.ldb, n0, k0);
      else       load_tile_full<BN, NT, CF::LB, false>(rb, Bp, a.ldb, k0, n0);
    };
    auto ls = [&](const v2d (&ra)[CF::LA], const v2d (&rb)[CF::LB], int st) {
      store_tile_v<T, BM, NT, CF::LA, A_ROW>(sA[st], ra, OPA == OP_C);
      store_tile_v<T, BN, NT, CF::LB, B_ROW>(sB[st], rb, OPB == OP_C);
    };
    // The K-steps that contribute are taken in ascending order, the j-th of
    // them in LDS stage j & 1 through register set j & 1: every step 0..nk-1
    // for a dense product, otherwise (nk <= 64) the bit set `rem` of the steps
    // a zero-slab map of the sparse operand leaves.
    unsigned long long rem = nk >= 64 ? ~0ull : (1ull << nk) - 1;
    // per wave: K-steps in which each of its row (op 2) or column (op 1) fragments is nonzero
    unsigned long long fm[CF::FM > CF::FN ? CF::FM : CF::FN];
    const bool sparse = SPARSE_OK && a.kmask && nk <= 64;
    if (sparse) {
      const unsigned long long* w4 = a.kmask + (a.kmask_op == 1 ? 4 * tn : 4 * tm);
      rem &= w4[0] | w4[1] | w4[2] | w4[3];
      const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
      const int g0 = a.kmask_op == 1 ? (wv % CF::WN) * CF::TN / 16 : (wv / CF::WN) * CF::TM / 16;
#pragma unroll
      for (int f = 0; f < (a.kmask_op == 1 ? FN : FM); ++f) fm[f] = w4[g0 + f];
    }
    auto enables = [&](int k) -> unsigned {
      if (!sparse) return ALL_ON;
      unsigned on = 0u;
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) {
          const unsigned long long w = a.kmask_op == 1 ? fm[j] : fm[i];
          on |= (unsigned)((w >> k) & 1ull) << (i * FN + j);
        }
      return on;
    };
    const int nact = sparse ? __popcll(rem) : nk;
    unsigned frags = 0u;   // fragment products issued by this wave (K-step x enabled (i, j))
    int kseq = 0;
    auto next_k = [&]() {
      if (!sparse) return kseq++;
      const int k = __builtin_ctzll(rem);
      rem &= rem - 1;
      return k;
    };
    // K-step index held by register set 0/1 and by LDS stage 0/1
    int kset0 = 0, kset1 = 0, kst0 = 0, kst1 = 0;
    if (nact > 0) {
      kset0 = next_k();
      gl(qa[0], qb[0], kset0 * BK);
      if (nact > 1) {
        kset1 = next_k();
        gl(qa[1], qb[1], kset1 * BK);
      }
      ls(qa[0], qb[0], 0);
      kst0 = kset0;
    }
    __syncthreads();
    for (int j = 0; j < nact; j += 2) {
      if (j + 2 < nact) {
        kset0 = next_k();
        gl(qa[0], qb[0], kset0 * BK);
      }
      {
        const unsigned on0 = enables(kst0);
        frags += __popc(on0);
        mac(sA[0], sB[0], on0);
      }
      if (j + 1 < nact) {
        ls(qa[1], qb[1], 1);
        kst1 = kset1;
      }
      __syncthreads();
      if (j + 1 < nact) {
        if (j + 3 < nact) {
          kset1 = next_k();
          gl(qa[1], qb[1], kset1 * BK);
        }
        const unsigned on1 = enables(kst1);
        frags += __popc(on1);
        mac(sA[1], sB[1], on1);
        if (j + 2 < nact) {
          ls(qa[0], qb[0], 0);
          kst0 = kset0;
        }
        __syncthreads();
      }
    }
    prof_count(a.flop_slots, frags);
  } else {
    double2 ra[CF::LA], rb[CF::LB];
    auto gload = [&](int k0) {
      if (A_ROW) load_tile<BM, NT, CF::LA, true>(ra, Ap, a.lda, m0, k0, a.M, a.K);
      else       load_tile<BM, NT, CF::LA, false>(ra, Ap, a.lda, k0, m0, a.K, a.M);
      if (B_ROW) load_tile<BN, NT, CF::LB, true>(rb, Bp, a.ldb, n0, k0, a.N, a.K);
      else       load_tile<BN, NT, CF::LB, false>(rb, Bp, a.ldb, k0, n0, a.K, a.N);
    };
    auto lstore = [&](int st) {
      store_tile<T, BM, NT, CF::LA, A_ROW>(sA[st], ra, OPA == OP_C);
      store_tile<T, BN, NT, CF::LB, B_ROW>(sB[st], rb, OPB == OP_C);
    };

    gload(0);
    lstore(0);
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
      const int st = kt & 1;
      if (kt + 1 < nk) gload((kt + 1) * BK);
      mac(sA[st], sB[st], ALL_ON);
      if (kt + 1 < nk) lstore(st ^ 1);
      __syncthreads();
    }
    prof_count(a.flop_slots, (unsigned)nk * FM * FN);
  }

  double2* __restrict__ Cp = a.C + (long)p * a.sC;
  const double2* __restrict__ Ci = a.Cin ? a.Cin + (long)p * a.sCi : nullptr;
  const bool use_beta = (a.beta.x != 0.0 || a.beta.y != 0.0) && Ci != nullptr;
  // Per row of MFMA tiles: all Cin reads are issued before any result is
  // stored (C may alias Cin, so the compiler would otherwise wait on each
  // read in turn); values stay in registers as native vectors.
#pragma unroll
  for (int i = 0; i < FM; ++i) {
    v2d cin[FN][4];
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      const int col = n0 + wn * CF::TN + j * 16 + li;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = m0 + wm * CF::TM + i * 16 + acc_row<T>(lk, v);
        const bool ok = use_beta && (FULL || (col < a.N && row < a.M));
        cin[j][v] = ok ? *reinterpret_cast<const v2d*>(Ci + (long)row * a.ldci + col) : v2d{0.0, 0.0};
      }
    }
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      const int col = n0 + wn * CF::TN + j * 16 + li;
      if (!FULL && col >= a.N) continue;
      if constexpr (TAG == 1) {
        if (col >= a.skip_lo && col < a.skip_hi) continue;
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = m0 + wm * CF::TM + i * 16 + acc_row<T>(lk, v);
        if (!FULL && row >= a.M) continue;
        double re, im;
        if constexpr (GAUSS) {
          const double p1 = (double)accR[i][j][v], p2 = (double)accI[i][j][v];
          re = p1 - p2;
          im = (double)accS[i < NS ? i : 0][j][v] - p1 - p2;
        } else {
          re = (double)accR[i][j][v];
          im = (double)accI[i][j][v];
        }
        const v2d c = cin[j][v];
        v2d out;
        out.x = a.alpha.x * re - a.alpha.y * im + (a.beta.x * c.x - a.beta.y * c.y);
        out.y = a.alpha.x * im + a.alpha.y * re + (a.beta.x * c.y + a.beta.y * c.x);
        *reinterpret_cast<v2d*>(Cp + (long)row * a.ldc + col) = out;
      }
    }
  }
}

typedef Cfg<64, 64, 2, 2> Cfg64;
typedef Cfg<128, 64, 4, 2> Cfg128x64;
typedef Cfg<128, 128, 4, 2> Cfg128;
typedef Cfg<64, 64, 4, 2> Cfg64w8;   // 8 waves of 16 x 32: fewer registers per wave, more waves per SIMD
typedef Cfg<128, 64, 8, 2> Cfg128x64w16;   // 16 waves of 16 x 32
typedef Cfg<32, 32, 2, 2> Cfg32;           // small batches: four times the workgroups of a 64 x 64 tile

// A launch whose 64 x 64 tiles would give fewer workgroups than two per CU (a few energy points
// per call: one b = 512 product is 64 tiles) is better off on 32 x 32 tiles, so that the whole chip
// takes part; it gives up the zero-slab skipping of coupling operands (64 x 64 tiles only).
constexpr long SMALL_LAUNCH_TILES = 512;

template <typename T, typename CF, bool GAUSS, bool FULL>
void launch_ops(const GemmDesc& d, const KArgs& ka, dim3 grid, hipStream_t s) {
  const dim3 block(CF::NT);
  // products that skip the zero slabs of a coupling operand: a symbol of their own (tag 2)
  if constexpr (FULL && CF::BM == 64 && CF::BN == 64) {
    if (ka.kmask && ka.kmask_op == 1 && d.opA == OP_N && d.opB == OP_N) {
      hipLaunchKernelGGL((zgemm_kernel<T, OP_N, OP_N, CF, 2, GAUSS, FULL>), grid, block, 0, s, ka);
      return;
    }
    if (ka.kmask && ka.kmask_op == 2 && d.opA == OP_C && d.opB == OP_N) {
      hipLaunchKernelGGL((zgemm_kernel<T, OP_C, OP_N, CF, 2, GAUSS, FULL>), grid, block, 0, s, ka);
      return;
    }
  }
  if (d.prof_class == KC_INV_GEMM && d.opA == OP_N && d.opB == OP_N)
    hipLaunchKernelGGL((zgemm_kernel<T, OP_N, OP_N, CF, 1, GAUSS, FULL>), grid, block, 0, s, ka);
  else if (d.prof_class == KC_INV_GEMM && d.opA == OP_C && d.opB == OP_N)
    hipLaunchKernelGGL((zgemm_kernel<T, OP_C, OP_N, CF, 1, GAUSS, FULL>), grid, block, 0, s, ka);
  else if (d.opA == OP_N && d.opB == OP_N)
    hipLaunchKernelGGL((zgemm_kernel<T, OP_N, OP_N, CF, 0, GAUSS, FULL>), grid, block, 0, s, ka);
  else if (d.opA == OP_C && d.opB == OP_N)
    hipLaunchKernelGGL((zgemm_kernel<T, OP_C, OP_N, CF, 0, GAUSS, FULL>), grid, block, 0, s, ka);
  else if (d.opA == OP_N && d.opB == OP_C)
    hipLaunchKernelGGL((zgemm_kernel<T, OP_N, OP_C, CF, 0, GAUSS, FULL>), grid, block, 0, s, ka);
  else hipLaunchKernelGGL((zgemm_kernel<T, OP_C, OP_C, CF, 0, GAUSS, FULL>), grid, block, 0, s, ka);
}

template <typename T, typename CF, bool GAUSS>
hipError_t launch_cfg(const GemmDesc& d, KArgs ka, hipStream_t s) {
  ka.tiles_m = (d.M + CF::BM - 1) / CF::BM;
  ka.tiles_n = (d.N + CF::BN - 1) / CF::BN;
  const long total = (long)ka.tiles_m * ka.tiles_n * d.batch;
  const dim3 grid((unsigned)total);
  // the 128 x 128 tile has no registers left for a second operand set
  constexpr bool kFullOk = !(CF::BM == 128 && CF::BN == 128);
  const bool full = kFullOk && d.M % CF::BM == 0 && d.N % CF::BN == 0 && d.K % BK == 0 && d.K >= BK;
  if constexpr (kFullOk) {
    if (full) {
      launch_ops<T, CF, GAUSS, true>(d, ka, grid, s);
      return hipGetLastError();
    }
  }
  launch_ops<T, CF, GAUSS, false>(d, ka, grid, s);
  return hipGetLastError();
}

// The three-product form keeps a third accumulator set; with 128x128 tiles
// that no longer fits the register file, so it runs on 128x64 tiles there.
template <typename T, bool GAUSS>
hipError_t launch_t(const GemmDesc& d, const KArgs& ka, int tile, hipStream_t s) {
  if (GAUSS && tile == GEMM_TILE_128x128) tile = GEMM_TILE_128x64;
  switch (tile) {
    case GEMM_TILE_32: return launch_cfg<T, Cfg32, GAUSS>(d, ka, s);
    case GEMM_TILE_128x64: return launch_cfg<T, Cfg128x64, GAUSS>(d, ka, s);
    case GEMM_TILE_64_8W: return launch_cfg<T, Cfg64w8, GAUSS>(d, ka, s);
    case GEMM_TILE_128x64_16W: return launch_cfg<T, Cfg128x64w16, GAUSS>(d, ka, s);
    case GEMM_TILE_128x128:
      if constexpr (!GAUSS) return launch_cfg<T, Cfg128, GAUSS>(d, ka, s);
      [[fallthrough]];
    default: return launch_cfg<T, Cfg64, GAUSS>(d, ka, s);
  }
}

}  // namespace

int tile_for_launch(int tile, int M, int N, long batch) {
  const long tiles64 = (long)((M + 63) / 64) * ((N + 63) / 64) * batch;
  return (tiles64 < SMALL_LAUNCH_TILES && M >= 32 && N >= 32) ? GEMM_TILE_32 : tile;
}

namespace {

// Strict lower triangle of each n x n item from its upper triangle,
// C[r][c] = -conj(C[c][r]) for r > c: 32 x 32 tiles on or below the diagonal,
// each transposed through LDS so that reads and writes are coalesced.
constexpr int MIR = 32;

__global__ void __launch_bounds__(256) skew_mirror_kernel(int n, double2* C, long ldc, long sC, const int* active) {
  const int p = blockIdx.z;
  if (active && active[p] == 0) return;
  const int tr = blockIdx.y, tc = blockIdx.x;   // destination tile (rows tr, columns tc)
  if (tr < tc) return;
  __shared__ double2 S[MIR][MIR + 1];
  double2* Cp = C + (long)p * sC;
  const int r0 = tr * MIR, c0 = tc * MIR;
  // source: rows c0.., columns r0.. (upper side)
  for (int e = threadIdx.x; e < MIR * MIR; e += blockDim.x) {
    const int i = e / MIR, j = e % MIR;
    const int sr = c0 + i, sc = r0 + j;
    if (sr < n && sc < n) S[i][j] = Cp[(long)sr * ldc + sc];
  }
  __syncthreads();
  for (int e = threadIdx.x; e < MIR * MIR; e += blockDim.x) {
    const int i = e / MIR, j = e % MIR;
    const int r = r0 + i, c = c0 + j;
    if (r < n && c < n && r > c) {
      const double2 v = S[j][i];
      Cp[(long)r * ldc + c] = make_double2(-v.x, v.y);
    }
  }
}

// Zero-slab map: one workgroup per (block, 64-column tile), one word per
// 16-column group of the tile; bit k marks a nonzero in rows [16k, 16k+16) of
// the group's columns, in H or S.
__global__ void __launch_bounds__(256) slab_map_kernel(int b, const double2* H, const double2* S,
                                                       unsigned long long* out, int accumulate) {
  const int c = blockIdx.x, i = blockIdx.y, t = threadIdx.x;
  const long off = (long)i * b * b + 64 * c;
  __shared__ unsigned long long word[4];
  if (t < 4) word[t] = 0ull;
  __syncthreads();
  unsigned long long w[4] = {0ull, 0ull, 0ull, 0ull};
  for (int e = t; e < b * 64; e += 256) {
    const int r = e >> 6, cc = e & 63;
    const double2 h = H[off + (long)r * b + cc];
    bool nz = h.x != 0.0 || h.y != 0.0;
    if (S) {
      const double2 v = S[off + (long)r * b + cc];
      nz = nz || v.x != 0.0 || v.y != 0.0;
    }
    // a thread's columns stay in one group: e advances by 256 = 4 rows
    if (nz) w[cc >> 4] |= 1ull << (r >> 4);
  }
#pragma unroll
  for (int g = 0; g < 4; ++g)
    if (w[g]) atomicOr(&word[g], w[g]);
  __syncthreads();
  if (t < 4) {
    unsigned long long* o = out + (long)i * (b / 16) + 4 * c + t;
    *o = accumulate ? (*o | word[t]) : word[t];
  }
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
  ka.xcd_remap = d.xcd_remap;
  ka.tiles_m = ka.tiles_n = 0;
  ka.kmask = (d.kmask_op == 1 || d.kmask_op == 2) ? d.kmask : nullptr;
  ka.kmask_op = d.kmask_op;
  ka.flop_slots = nullptr;
  if (d.skew && d.M != d.N) return hipErrorInvalidValue;
  ka.upper = d.skew ? 1 : 0;
  // only the inversion-update symbols (tag 1: NN or CN with class KC_INV_GEMM) honour a skip range
  if (d.skip_hi > d.skip_lo &&
      (d.prof_class != KC_INV_GEMM || d.opB != OP_N || d.skew || d.skip_lo < 0 || d.skip_hi > d.N))
    return hipErrorInvalidValue;
  ka.skip_lo = d.skip_lo;
  ka.skip_hi = d.skip_hi;
  int tile = d.tile;
  if (tile == GEMM_TILE_DEFAULT) tile = GEMM_TILE_64;
  const bool gauss = d.prec != PREC_F32 && d.gauss;
  const bool coupling = ka.kmask && (ka.kmask_op == 1 || ka.kmask_op == 2);
  const int cls = d.prof_class >= 0 ? d.prof_class
                  : coupling        ? KC_GEMM_CPL
                                    : (d.prec == PREC_F32 ? KC_GEMM32 : KC_GEMM64);
  ka.flop_slots = prof_flop_slots(cls);
  prof_begin(cls, s);
  hipError_t e = d.prec == PREC_F32 ? launch_t<float, false>(d, ka, tile, s)
                 : gauss            ? launch_t<double, true>(d, ka, tile, s)
                                    : launch_t<double, false>(d, ka, tile, s);
  // flops are counted on the device (only the items, tiles and K-steps that run); bytes: A and B
  // read, C read and written
  prof_end(cls, s, 0.0, 16.0 * d.batch * ((double)d.M * d.K + (double)d.K * d.N + 2.0 * d.M * d.N));
  if (e == hipSuccess && d.skew) {
    const int nt = (d.M + MIR - 1) / MIR;
    hipLaunchKernelGGL(skew_mirror_kernel, dim3(nt, nt, d.batch), dim3(256), 0, s, d.M, d.C.p, d.C.ld, d.C.stride,
                       d.active);
    e = hipGetLastError();
  }
  return e;
}

hipError_t launch_slab_map(int b, int nblk, const double2* H, const double2* S, unsigned long long* out,
                           int accumulate, hipStream_t s) {
  if (nblk <= 0) return hipSuccess;
  if (b % 64 != 0 || b > 1024 || !H || !out) return hipErrorInvalidValue;
  hipLaunchKernelGGL(slab_map_kernel, dim3(b / 64, nblk), dim3(256), 0, s, b, H, S, out, accumulate);
  return hipGetLastError();
}

}  // namespace negf
