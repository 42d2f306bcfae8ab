// Grouped, batched FP64 MFMA GEMM over 64 x 64 output tiles:
//   Cout = beta * Cin + alpha * sum_seg sum_k A(m,k) B(c,k)
// with either operand stored k-contiguous or m-contiguous, k ranges clipped
// to the nonzero part of a triangular operand, and lower-triangle or
// lower-plus-mirror stores for symmetric results.  Used by the selected
// inversion for its products with the inverses of the diagonal factor blocks
// (TRMM/LAUUM/TRTRI steps) and the two GEMMs of each backward step.
#include <algorithm>
#include <cmath>
#include <type_traits>

#include <vector>

#include "bta_device.hpp"
#include "bta_internal.hpp"
#include "bta_testing.h"

namespace bta {

// Tile configuration: a workgroup of 4 waves (2 x 2) computes a
// (32*WM) x (32*WN) tile; each wave WM x WN MFMA blocks of 16 x 16; k is staged
// through LDS in chunks of BK (row stride BK + 2 doubles: consecutive rows
// shift by 4 banks and rows stay 16-byte aligned).
template <int WM, int WN, int BK>
struct GemmCfg {
  static constexpr int TM = 32 * WM, TN = 32 * WN, LD = BK + 2;
  static constexpr int EA = TM * BK / NT, EB = TN * BK / NT;  // doubles staged per thread
  static_assert(EA == 16 && EB == 16, "staging assumes 16 doubles per thread per operand");
};

template <int TM, int BK>
struct Chunk {
  double v[16];
};

// Load one TM x BK operand chunk (element (m, k) = trans ? p[k*ld + m] : p[m*ld + k];
// zero outside mext x kext) into registers.
template <int TM, int BK>
__device__ __forceinline__ void chunk_load(Chunk<TM, BK>& c, const double* p, int64_t ld, int trans, int mext, int kext,
                                           int tid) {
  if (!trans) {
    constexpr int TPR = BK / 16;  // threads per row
    const int m = tid / TPR, k0 = (tid % TPR) * 16;
    const double* src = p + (int64_t)m * ld + k0;
    const bool row_ok = m < mext;
    if (row_ok && k0 + 16 <= kext && ((ld & 1) == 0) && ((((uintptr_t)src) & 15) == 0)) {
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        d2v x = *reinterpret_cast<const d2v*>(src + 2 * j);
        c.v[2 * j] = x[0];
        c.v[2 * j + 1] = x[1];
      }
    } else {
#pragma unroll
      for (int j = 0; j < 16; ++j) c.v[j] = (row_ok && k0 + j < kext) ? src[j] : 0.0;
    }
  } else {
    constexpr int TPK = TM / 16;  // threads per k row
    const int k = tid / TPK, m0 = (tid % TPK) * 16;
    const double* src = p + (int64_t)k * ld + m0;
    const bool k_ok = k < kext;
    if (k_ok && m0 + 16 <= mext && ((ld & 1) == 0) && ((((uintptr_t)src) & 15) == 0)) {
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        d2v x = *reinterpret_cast<const d2v*>(src + 2 * j);
        c.v[2 * j] = x[0];
        c.v[2 * j + 1] = x[1];
      }
    } else {
#pragma unroll
      for (int j = 0; j < 16; ++j) c.v[j] = (k_ok && m0 + j < mext) ? src[j] : 0.0;
    }
  }
}

template <int TM, int BK>
__device__ __forceinline__ void chunk_store(const Chunk<TM, BK>& c, double* lds, int trans, int tid) {
  constexpr int LD = BK + 2;
  if (!trans) {
    constexpr int TPR = BK / 16;
    const int m = tid / TPR, k0 = (tid % TPR) * 16;
    double* dst = lds + m * LD + k0;
#pragma unroll
    for (int j = 0; j < 8; ++j) *reinterpret_cast<d2v*>(dst + 2 * j) = d2v{c.v[2 * j], c.v[2 * j + 1]};
  } else {
    constexpr int TPK = TM / 16;
    const int k = tid / TPK, m0 = (tid % TPK) * 16;
#pragma unroll
    for (int j = 0; j < 16; ++j) lds[(m0 + j) * LD + k] = c.v[j];
  }
}

template <int WM, int WN>
struct AccT {
  d4 v[WM][WN];
};

// acc += A_lds B_lds^T over one BK chunk (k permuted within each 16-wide group
// so that every lane reads 4 consecutive k with two 16-byte LDS reads).
template <int WM, int WN, int BK>
__device__ __forceinline__ void chunk_mma(AccT<WM, WN>& acc, const double* As, const double* Bs, int tid) {
  constexpr int LD = BK + 2;
  const int w = tid >> 6, lane = tid & 63;
  const int r0 = 16 * WM * (w >> 1) + (lane & 15);
  const int c0 = 16 * WN * (w & 1) + (lane & 15);
  const int kl = (lane >> 4) * 4;
#pragma unroll
  for (int kg = 0; kg < BK / 16; ++kg) {
    d4 a[WM], b[WN];
#pragma unroll
    for (int i = 0; i < WM; ++i) {
      const double* pa = As + (r0 + 16 * i) * LD + kg * 16 + kl;
      const d2v x0 = *reinterpret_cast<const d2v*>(pa);
      const d2v x1 = *reinterpret_cast<const d2v*>(pa + 2);
      a[i] = d4{x0[0], x0[1], x1[0], x1[1]};
    }
#pragma unroll
    for (int j = 0; j < WN; ++j) {
      const double* pb = Bs + (c0 + 16 * j) * LD + kg * 16 + kl;
      const d2v x0 = *reinterpret_cast<const d2v*>(pb);
      const d2v x1 = *reinterpret_cast<const d2v*>(pb + 2);
      b[j] = d4{x0[0], x0[1], x1[0], x1[1]};
    }
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int i = 0; i < WM; ++i)
#pragma unroll
        for (int j = 0; j < WN; ++j) acc.v[i][j] = mfma16(a[i][s], b[j][s], acc.v[i][j]);
  }
}

template <int WM, int WN, int BK>
__device__ __forceinline__ void gemm_tile_body(const GProb& P, long long local, int tid, double* As, double* Bs) {
  using C = GemmCfg<WM, WN, BK>;
  constexpr int TM = C::TM, TN = C::TN;
  const int batch = (int)(local / P.tiles_per_batch);
  const int tile = (int)(local - (long long)batch * P.tiles_per_batch);
  const int b0 = batch / P.nb1, b1 = batch - b0 * P.nb1;
  int tm, tn;
  if (P.lower_tiles) {
    // tile -> (tm, tn) over the tiles that touch the lower triangle, row by row:
    // row tm holds tiles tn = 0 .. floor((tm*TM + TM - 1) / TN)
    tm = 0;
    int rem = tile;
    for (;;) {
      const int w = min(P.ntn, (tm * TM + TM - 1) / TN + 1);
      if (rem < w) break;
      rem -= w;
      ++tm;
    }
    tn = rem;
  } else {
    tm = tile / P.ntn;
    tn = tile - tm * P.ntn;
  }
  const int m0 = tm * TM, n0 = tn * TN;
  const int mext = min(TM, P.M - m0), next = min(TN, P.N - n0);

  // k ranges of the segments (triangular operands clip them)
  int kbeg[2] = {0, 0}, kend[2] = {0, 0}, nk[2] = {0, 0};
  const double* Ab[2] = {nullptr, nullptr};
  const double* Bb[2] = {nullptr, nullptr};
  for (int s = 0; s < P.nseg; ++s) {
    const GSeg& g = P.seg[s];
    int k0 = 0, k1 = g.K;
    switch (g.tri) {
      case TRI_K_GE_COL: k0 = n0; break;
      case TRI_K_GE_ROW: k0 = m0; break;
      case TRI_K_LE_ROW: k1 = min(g.K, m0 + TM); break;
      case TRI_K_LE_COL: k1 = min(g.K, n0 + TN); break;
      default: break;
    }
    k0 = (k0 / BK) * BK;
    if (k0 > k1) k0 = k1;
    kbeg[s] = k0;
    kend[s] = k1;
    nk[s] = (k1 - k0 + BK - 1) / BK;
    Ab[s] = g.A + b0 * g.sA0 + b1 * g.sA1;
    Bb[s] = g.B + b0 * g.sB0 + b1 * g.sB1;
  }
  const int total = nk[0] + nk[1];

  AccT<WM, WN> acc;
#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int jj = 0; jj < WN; ++jj) acc.v[i][jj] = d4{0.0, 0.0, 0.0, 0.0};
  Chunk<TM, BK> ra;
  Chunk<TN, BK> rb;
  auto load = [&](int kk) {
    const int s = kk < nk[0] ? 0 : 1;
    const int q = s == 0 ? kk : kk - nk[0];
    const int k = kbeg[s] + q * BK;
    const int kext = min(BK, kend[s] - k);
    const GSeg& g = P.seg[s];
    const double* pa = g.at ? Ab[s] + (int64_t)k * g.lda + m0 : Ab[s] + (int64_t)m0 * g.lda + k;
    const double* pb = g.bt ? Bb[s] + (int64_t)k * g.ldb + n0 : Bb[s] + (int64_t)n0 * g.ldb + k;
    chunk_load<TM, BK>(ra, pa, g.lda, g.at, mext, kext, tid);
    chunk_load<TN, BK>(rb, pb, g.ldb, g.bt, next, kext, tid);
  };
  if (total > 0) load(0);
  for (int kk = 0; kk < total; ++kk) {
    const int s = kk < nk[0] ? 0 : 1;
    __syncthreads();
    chunk_store<TM, BK>(ra, As, P.seg[s].at, tid);
    chunk_store<TN, BK>(rb, Bs, P.seg[s].bt, tid);
    __syncthreads();
    if (kk + 1 < total) load(kk + 1);
    chunk_mma<WM, WN, BK>(acc, As, Bs, tid);
  }

  // epilogue: final values first (Cin may alias Cout), then the stores
  const int w = tid >> 6, lane = tid & 63;
  const int rw = 16 * WM * (w >> 1), cw = 16 * WN * (w & 1);
  const int64_t coff = b0 * P.sC0 + b1 * P.sC1;
  double* Cb = P.Cout + coff;
  const double* Cib = P.Cin ? P.Cin + coff : nullptr;
#pragma unroll
  for (int bi = 0; bi < WM; ++bi)
#pragma unroll
    for (int bj = 0; bj < WN; ++bj)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int r = rw + 16 * bi + acc_row(lane, e), c = cw + 16 * bj + acc_col(lane);
        const int gr = m0 + r, gc = n0 + c;
        double v = P.alpha * acc.v[bi][bj][e];
        const bool live = r < mext && c < next && !(P.store != ST_FULL && gc > gr);
        if (live && P.beta != 0.0) v += P.beta * Cib[(int64_t)gr * P.ldc + gc];
        acc.v[bi][bj][e] = v;
      }
#pragma unroll
  for (int bi = 0; bi < WM; ++bi)
#pragma unroll
    for (int bj = 0; bj < WN; ++bj)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int r = rw + 16 * bi + acc_row(lane, e), c = cw + 16 * bj + acc_col(lane);
        const int gr = m0 + r, gc = n0 + c;
        if (r >= mext || c >= next) continue;
        if (P.store != ST_FULL && gc > gr) continue;
        Cb[(int64_t)gr * P.ldc + gc] = acc.v[bi][bj][e];
        if (P.store == ST_LOWER_MIRROR && gc < gr) Cb[(int64_t)gc * P.ldc + gr] = acc.v[bi][bj][e];
      }
}

// ---------------------------------------------------------------- direct-to-LDS tile body
// The same product with operands moved from global memory straight into LDS
// (global_load_lds_dwordx4: each lane moves one 16-byte piece, the pieces of a
// wave instruction land contiguously), two LDS stages of BK = 16, one barrier
// per stage and no register staging.  Piece placement within a stage:
//   k-contiguous operand (N): slot m*8 + (p ^ swzN(m)) holds k = 2p, 2p+1 of row m;
//   m-contiguous operand (T): slot k*(TM/2) + (q ^ swzT(k)) holds m = 2q, 2q+1 of row k.
// Both swizzles make the MFMA operand reads (16-byte reads of rows m for N,
// 8-byte reads of 16 consecutive m for T) free of LDS bank conflicts.
// Requirements (checked on the host by dl_ok): 16-byte aligned operand bases,
// even leading dimensions and batch strides, even K, and even M (N) for a
// transposed A (B), so that no piece straddles the edge of an operand.
__device__ __align__(16) double g_zero_piece[2] = {0.0, 0.0};

__device__ __forceinline__ int swzN(int m) { return (m ^ (m >> 3)) & 7; }
__device__ __forceinline__ int swzT(int k) { return ((k >> 2) & 1) << 3; }

__device__ __forceinline__ void load_piece_lds(const double* src, double* lds_wave) {
  __builtin_amdgcn_global_load_lds(static_cast<const void*>(src),
                                   (__attribute__((address_space(3))) void*)(lds_wave), 16, 0, 0);
}

template <int WM, int WN>
struct DLCfg {
  static constexpr int TM = 32 * WM, TN = 32 * WN, BK = 16;
  static constexpr int SA = TM * BK, SB = TN * BK;          // doubles per stage and operand
  static constexpr int IA = SA / 2 / NT, IB = SB / 2 / NT;  // pieces per thread per stage
  static constexpr int STAGE = SA + SB;
  static_assert(IA >= 1 && IB >= 1, "tile too small for the direct-load stage");
};

// One operand's pieces of stage (k .. k+kext) for the tile at row r0 (mext rows).
template <int TR, int NI>
__device__ __forceinline__ void stage_operand(const double* base, int64_t ld, int trans, int r0, int rext, int k,
                                              int kext, double* dst, int wave, int lane) {
#pragma unroll
  for (int j = 0; j < NI; ++j) {
    const int slot = (wave * NI + j) * 64 + lane;
    const double* src = g_zero_piece;
    if (!trans) {
      const int m = slot >> 3, p = (slot & 7) ^ swzN(slot >> 3);
      if (m < rext && 2 * p < kext) src = base + (int64_t)(r0 + m) * ld + k + 2 * p;
    } else {
      constexpr int PR = TR / 2;
      const int kk = slot / PR, q = (slot % PR) ^ swzT(slot / PR);
      if (kk < kext && 2 * q < rext) src = base + (int64_t)(k + kk) * ld + r0 + 2 * q;
    }
    load_piece_lds(src, dst + (wave * NI + j) * 128);
  }
}

// Operand values of one stage for MFMA blocks i = 0..W-1 at rows r0 + 16 i + lane%16,
// v[i][s] = X(row, 4*(lane/16) + s).
template <int TR, int W>
__device__ __forceinline__ void stage_read(double (&v)[W][4], const double* st, int trans, int r0, int lane) {
  const int g = lane >> 4;
#pragma unroll
  for (int i = 0; i < W; ++i) {
    const int m = r0 + 16 * i + (lane & 15);
    if (!trans) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const d2v x = *reinterpret_cast<const d2v*>(st + 2 * (m * 8 + ((2 * g + h) ^ swzN(m))));
        v[i][2 * h] = x[0];
        v[i][2 * h + 1] = x[1];
      }
    } else {
      constexpr int PR = TR / 2;
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int k = 4 * g + s;
        v[i][s] = st[2 * (k * PR + ((m >> 1) ^ swzT(k))) + (m & 1)];
      }
    }
  }
}

// Tile (tm, tn) of batch entry `local` of problem P; full-tile problems are
// walked in groups of 4 tile rows, column by column, so that consecutive tiles
// (which share an XCD, see xcd_tile) reuse A and B panels in that XCD's L2.
template <int TM, int TN>
__device__ __forceinline__ void tile_coords(const GProb& P, int tile, int& tm, int& tn) {
  if (P.lower_tiles) {
    tm = 0;
    int rem = tile;
    for (;;) {
      const int w = min(P.ntn, (tm * TM + TM - 1) / TN + 1);
      if (rem < w) break;
      rem -= w;
      ++tm;
    }
    tn = rem;
  } else {
    constexpr int G = 4;
    const int grp = tile / (G * P.ntn);
    const int rows = min(G, P.ntm - grp * G);
    const int rem = tile - grp * G * P.ntn;
    tm = grp * G + rem % rows;
    tn = rem / rows;
  }
}

// L0: layout of every problem's first segment as at * 2 + bt when the launch
// shares one (its k loop then has no layout branch), 4 when it does not.
template <int WM, int WN, int L0>
__device__ __forceinline__ void gemm_tile_dl(const GProb& P, long long local, int tid, double* lds) {
  using C = DLCfg<WM, WN>;
  constexpr int TM = C::TM, TN = C::TN, BK = C::BK;
  const int batch = (int)(local / P.tiles_per_batch);
  const int tile = (int)(local - (long long)batch * P.tiles_per_batch);
  const int b0 = batch / P.nb1, b1 = batch - b0 * P.nb1;
  int tm, tn;
  tile_coords<TM, TN>(P, tile, tm, tn);
  const int m0 = tm * TM, n0 = tn * TN;
  const int mext = min(TM, P.M - m0), next = min(TN, P.N - n0);
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;

  // k ranges of the two segments (triangular operands clip them); plain
  // scalars and selects, so that nothing is indexed by a run-time segment number
  auto krange = [&](const GSeg& g, int& k0, int& k1) {
    k0 = 0;
    k1 = g.K;
    switch (g.tri) {
      case TRI_K_GE_COL: k0 = n0; break;
      case TRI_K_GE_ROW: k0 = m0; break;
      case TRI_K_LE_ROW: k1 = min(g.K, m0 + TM); break;
      case TRI_K_LE_COL: k1 = min(g.K, n0 + TN); break;
      default: break;
    }
    k0 = (k0 / BK) * BK;
    if (k0 > k1) k0 = k1;
  };
  int kb0, ke0, kb1 = 0, ke1 = 0;
  krange(P.seg[0], kb0, ke0);
  if (P.nseg > 1) krange(P.seg[1], kb1, ke1);
  const int nk0 = (ke0 - kb0 + BK - 1) / BK;
  const int total = nk0 + (ke1 - kb1 + BK - 1) / BK;
  const double* A0 = P.seg[0].A + b0 * P.seg[0].sA0 + b1 * P.seg[0].sA1;
  const double* B0 = P.seg[0].B + b0 * P.seg[0].sB0 + b1 * P.seg[0].sB1;
  const double* A1 = P.seg[1].A + b0 * P.seg[1].sA0 + b1 * P.seg[1].sA1;
  const double* B1 = P.seg[1].B + b0 * P.seg[1].sB0 + b1 * P.seg[1].sB1;
  // the segments' layouts and strides, read once into scalar registers (a
  // reload inside the k loop costs a scalar load and a full wait per stage)
  const int at0 = __builtin_amdgcn_readfirstlane(P.seg[0].at), bt0 = __builtin_amdgcn_readfirstlane(P.seg[0].bt);
  const int at1 = __builtin_amdgcn_readfirstlane(P.seg[1].at), bt1 = __builtin_amdgcn_readfirstlane(P.seg[1].bt);
  const int64_t lda0 = P.seg[0].lda, lda1 = P.seg[1].lda, ldb0 = P.seg[0].ldb, ldb1 = P.seg[1].ldb;

  auto issue = [&](int kk) {
    const bool first = kk < nk0;
    const int k = first ? kb0 + kk * BK : kb1 + (kk - nk0) * BK;
    const int kext = min(BK, (first ? ke0 : ke1) - k);
    double* st = lds + (kk & 1) * C::STAGE;
    stage_operand<TM, C::IA>(first ? A0 : A1, first ? lda0 : lda1, first ? at0 : at1, m0, mext, k, kext, st, wave, lane);
    stage_operand<TN, C::IB>(first ? B0 : B1, first ? ldb0 : ldb1, first ? bt0 : bt1, n0, next, k, kext, st + C::SA,
                             wave, lane);
  };

  AccT<WM, WN> acc;
#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int jj = 0; jj < WN; ++jj) acc.v[i][jj] = d4{0.0, 0.0, 0.0, 0.0};
  const int rw = 16 * WM * (wave >> 1), cw = 16 * WN * (wave & 1);
  // MFMA blocks with no element inside the tile's extent, or (lower stores)
  // entirely above the diagonal, are not computed
  bool live[WM][WN];
#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int jj = 0; jj < WN; ++jj)
      live[i][jj] = (rw + 16 * i < mext) && (cw + 16 * jj < next) &&
                    (P.store == ST_FULL || n0 + cw + 16 * jj <= m0 + rw + 16 * i + 15);
  bool all_live = true;
#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int jj = 0; jj < WN; ++jj) all_live = all_live && live[i][jj];
  if (total > 0) issue(0);
  // stages [k0, k1); layout code LC < 4 fixes both operand layouts at compile time
  auto kloop = [&](auto checked, auto lc, int k0, int k1) {
    constexpr bool CK = decltype(checked)::value;
    constexpr int LC = decltype(lc)::value;
    for (int kk = k0; kk < k1; ++kk) {
      // stage kk has landed for every wave, and every wave is done with stage kk-1
      __syncthreads();
      const bool first = kk < nk0;
      const double* st = lds + (kk & 1) * C::STAGE;
      // the next stage's loads first (its buffer was last read before the
      // barrier), then this stage's operands
      if (kk + 1 < total) issue(kk + 1);
      double a[WM][4], b[WN][4];
      stage_read<TM, WM>(a, st, LC < 4 ? (LC >> 1) : (first ? at0 : at1), rw, lane);
      stage_read<TN, WN>(b, st + C::SA, LC < 4 ? (LC & 1) : (first ? bt0 : bt1), cw, lane);
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int i = 0; i < WM; ++i)
#pragma unroll
          for (int jj = 0; jj < WN; ++jj)
            if (!CK || live[i][jj]) acc.v[i][jj] = mfma16(a[i][q], b[jj][q], acc.v[i][jj]);
    }
  };
  using LFix = std::integral_constant<int, L0>;
  using LRun = std::integral_constant<int, 4>;
  if (__builtin_amdgcn_readfirstlane((int)all_live)) {
    kloop(std::false_type{}, LFix{}, 0, L0 < 4 ? nk0 : total);
    if (L0 < 4) kloop(std::false_type{}, LRun{}, nk0, total);
  } else {
    kloop(std::true_type{}, LFix{}, 0, L0 < 4 ? nk0 : total);
    if (L0 < 4) kloop(std::true_type{}, LRun{}, nk0, total);
  }

  const int64_t coff = b0 * P.sC0 + b1 * P.sC1;
  double* Cb = P.Cout + coff;
  const double* Cib = P.Cin ? P.Cin + coff : nullptr;
#pragma unroll
  for (int bi = 0; bi < WM; ++bi)
#pragma unroll
    for (int bj = 0; bj < WN; ++bj)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int r = rw + 16 * bi + acc_row(lane, e), c = cw + 16 * bj + acc_col(lane);
        const int gr = m0 + r, gc = n0 + c;
        double v = P.alpha * acc.v[bi][bj][e];
        const bool live = r < mext && c < next && !(P.store != ST_FULL && gc > gr);
        if (live && P.beta != 0.0) v += P.beta * Cib[(int64_t)gr * P.ldc + gc];
        acc.v[bi][bj][e] = v;
      }
#pragma unroll
  for (int bi = 0; bi < WM; ++bi)
#pragma unroll
    for (int bj = 0; bj < WN; ++bj)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int r = rw + 16 * bi + acc_row(lane, e), c = cw + 16 * bj + acc_col(lane);
        const int gr = m0 + r, gc = n0 + c;
        if (r >= mext || c >= next) continue;
        if (P.store != ST_FULL && gc > gr) continue;
        Cb[(int64_t)gr * P.ldc + gc] = acc.v[bi][bj][e];
        if (P.store == ST_LOWER_MIRROR && gc < gr) Cb[(int64_t)gc * P.ldc + gr] = acc.v[bi][bj][e];
      }
}

// ---------------------------------------------------------------- lean direct-to-LDS tile body
// Waves WR x WC, each (16 BI) x (16 BJ) of the (16 BI WR) x (16 BJ WC) tile;
// stages of BK = 16 as in gemm_tile_dl (same piece layouts).  The source of
// each of a thread's pieces is resolved once per segment (pointer, validity,
// k position); a stage only advances the pointers.
template <int WR, int WC, int BI, int BJ>
struct DL2 {
  static constexpr int NW = WR * WC, NTH = NW * 64, TM = 16 * BI * WR, TN = 16 * BJ * WC, BK = 16;
  static constexpr int SA = TM * BK, SB = TN * BK, STAGE = SA + SB;
  static constexpr int PA = TM * BK / 2, PB = TN * BK / 2, PER_T = (PA + PB) / NTH;
  static_assert((PA + PB) % NTH == 0 && PA % 64 == 0, "stage pieces per thread");
};

// Wait until at most N of this thread's vector memory loads are outstanding,
// then meet the workgroup at a barrier; the statement's memory clobber keeps
// the compiler from moving LDS accesses or direct-to-LDS loads across it.
// (Unlike __syncthreads, whose release fence waits for every outstanding
// direct-to-LDS load, this leaves the newer stages' loads in flight.)
template <int N>
__device__ __forceinline__ void wait_vm_barrier();
template <>
__device__ __forceinline__ void wait_vm_barrier<0>() { asm volatile("s_waitcnt vmcnt(0)\n\ts_barrier" ::: "memory"); }
template <>
__device__ __forceinline__ void wait_vm_barrier<4>() { asm volatile("s_waitcnt vmcnt(4)\n\ts_barrier" ::: "memory"); }
template <>
__device__ __forceinline__ void wait_vm_barrier<8>() { asm volatile("s_waitcnt vmcnt(8)\n\ts_barrier" ::: "memory"); }

// LDS stages of the 64 x 64 list kernel (the batched products): 4, or 2 under
// the measurement override BTA_LIST_STAGES=2.  (The single-problem 64 x 64
// kernel keeps two stages: four measured no better there, where two stages
// leave room for more workgroups per CU: n=128, b=2048 199.2 against 199.8 ms,
// autograd 61.9 against 61.7 ms, the wide arrowhead 288.2 against 286.2 ms.)
static int list_stages() {
  static const int ns = [] {
    long long v = 0;
    return (env_int("BTA_LIST_STAGES", 2, 4, &v) && v == 2) ? 2 : 4;
  }();
  return ns;
}

// NS: LDS stages of the k loop.  2: the next stage's loads overlap this
// stage's products.  NS > 2: NS - 1 stages in flight, each iteration waiting
// only for its own stage's loads (vector memory loads complete in order) --
// for tiles whose per-stage products are too short to cover a load's latency.
template <int WR, int WC, int BI, int BJ, int L0, int NS = 2>
__device__ __forceinline__ void gemm_tile_dl2(const GProb& P, long long local, int tid, double* lds) {
  using C = DL2<WR, WC, BI, BJ>;
  static_assert(NS == 2 || (NS == 4 && C::PER_T == 4), "the deep pipeline's wait counts assume 4 pieces per thread");
  constexpr int TM = C::TM, TN = C::TN, BK = C::BK, PER = C::PER_T;
  const int batch = (int)(local / P.tiles_per_batch);
  const int tile = (int)(local - (long long)batch * P.tiles_per_batch);
  const int b0 = batch / P.nb1, b1 = batch - b0 * P.nb1;
  int tm, tn;
  tile_coords<TM, TN>(P, tile, tm, tn);
  const int m0 = tm * TM, n0 = tn * TN;
  const int mext = min(TM, P.M - m0), next = min(TN, P.N - n0);
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;

  auto krange = [&](const GSeg& g, int& k0, int& k1) {
    k0 = 0;
    k1 = g.K;
    switch (g.tri) {
      case TRI_K_GE_COL: k0 = n0; break;
      case TRI_K_GE_ROW: k0 = m0; break;
      case TRI_K_LE_ROW: k1 = min(g.K, m0 + TM); break;
      case TRI_K_LE_COL: k1 = min(g.K, n0 + TN); break;
      default: break;
    }
    k0 = (k0 / BK) * BK;
    if (k0 > k1) k0 = k1;
  };
  int kb0, ke0, kb1 = 0, ke1 = 0;
  krange(P.seg[0], kb0, ke0);
  if (P.nseg > 1) krange(P.seg[1], kb1, ke1);
  const int nk0 = (ke0 - kb0 + BK - 1) / BK;
  const int total = nk0 + (ke1 - kb1 + BK - 1) / BK;

  // per piece: source pointer at the segment's first stage, its advance per
  // stage, the piece's k offset within a stage, and whether it is inside M / N
  const double* src[PER];
  int64_t inc[PER];
  int kpos[PER];
  bool inb[PER];
  int seg_klen = 0;
  auto setup = [&](int sidx) {
    const GSeg& g = P.seg[sidx];
    const int kb = sidx == 0 ? kb0 : kb1;
    seg_klen = (sidx == 0 ? ke0 : ke1) - kb;
    const double* Ab = g.A + b0 * g.sA0 + b1 * g.sA1;
    const double* Bb = g.B + b0 * g.sB0 + b1 * g.sB1;
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      const int slot = (wave * PER + j) * 64 + lane;
      const bool isA = slot < C::PA;
      const int sl = isA ? slot : slot - C::PA;
      const int R = isA ? TM : TN;
      const int r0 = isA ? m0 : n0, rext = isA ? mext : next;
      const double* base = isA ? Ab : Bb;
      const int64_t ld = isA ? g.lda : g.ldb;
      const int tr = isA ? g.at : g.bt;
      if (!tr) {
        const int m = sl >> 3, pc = (sl & 7) ^ swzN(m);
        src[j] = base + (int64_t)(r0 + m) * ld + kb + 2 * pc;
        inc[j] = BK;
        kpos[j] = 2 * pc;
        inb[j] = m < rext;
      } else {
        const int PRT = R / 2;
        const int kr = sl / PRT, qc = (sl - kr * PRT) ^ swzT(kr);
        src[j] = base + (int64_t)(kb + kr) * ld + r0 + 2 * qc;
        inc[j] = (int64_t)BK * ld;
        kpos[j] = kr;
        inb[j] = 2 * qc < rext;
      }
    }
  };
  int stage_in_seg = 0;
  auto issue = [&](int kk) {
    if (kk == 0) { setup(0); stage_in_seg = 0; }
    if (kk == nk0) { setup(1); stage_in_seg = 0; }
    double* st = lds + (kk % NS) * C::STAGE;
    const int krel = stage_in_seg * BK;
    const bool full = krel + BK <= seg_klen;
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      const bool ok = inb[j] && (full || krel + kpos[j] < seg_klen);
      load_piece_lds(ok ? src[j] : g_zero_piece, st + (wave * PER + j) * 128);
      src[j] += inc[j];
    }
    ++stage_in_seg;
  };

  AccT<BI, BJ> acc;
#pragma unroll
  for (int i = 0; i < BI; ++i)
#pragma unroll
    for (int jj = 0; jj < BJ; ++jj) acc.v[i][jj] = d4{0.0, 0.0, 0.0, 0.0};
  const int rw = 16 * BI * (wave / WC), cw = 16 * BJ * (wave % WC);
  bool live[BI][BJ];
#pragma unroll
  for (int i = 0; i < BI; ++i)
#pragma unroll
    for (int jj = 0; jj < BJ; ++jj)
      live[i][jj] = (rw + 16 * i < mext) && (cw + 16 * jj < next) &&
                    (P.store == ST_FULL || n0 + cw + 16 * jj <= m0 + rw + 16 * i + 15);
  bool all_live = true;
#pragma unroll
  for (int i = 0; i < BI; ++i)
#pragma unroll
    for (int jj = 0; jj < BJ; ++jj) all_live = all_live && live[i][jj];
  if (total > 0) issue(0);
  if (NS > 2)
    for (int q = 1; q < NS - 1 && q < total; ++q) issue(q);
  // the segments' layouts, read once into scalar registers (a reload inside
  // the k loop costs a scalar load and a full wait per stage)
  const int at0 = __builtin_amdgcn_readfirstlane(P.seg[0].at), bt0 = __builtin_amdgcn_readfirstlane(P.seg[0].bt);
  const int at1 = __builtin_amdgcn_readfirstlane(P.seg[1].at), bt1 = __builtin_amdgcn_readfirstlane(P.seg[1].bt);
  // the k loop, with the per-block checks only where a block can be dead
  // stages [k0, k1); layout code LC < 4 fixes both operand layouts at compile time
  auto kloop = [&](auto checked, auto lc, int k0, int k1) {
    constexpr bool CK = decltype(checked)::value;
    constexpr int LC = decltype(lc)::value;
    for (int kk = k0; kk < k1; ++kk) {
      if constexpr (NS == 2) {
        __syncthreads();
      } else {  // stages kk + 1 .. kk + NS - 2 may stay in flight
        if (kk + 2 < total) wait_vm_barrier<2 * C::PER_T>();
        else if (kk + 1 < total) wait_vm_barrier<C::PER_T>();
        else wait_vm_barrier<0>();
      }
      const bool first = kk < nk0;
      const double* st = lds + (kk % NS) * C::STAGE;
      // the next stage's loads first (its buffer was last read before the
      // barrier), then this stage's operands
      if (kk + NS - 1 < total) issue(kk + NS - 1);
      double a[BI][4], b[BJ][4];
      stage_read<TM, BI>(a, st, LC < 4 ? (LC >> 1) : (first ? at0 : at1), rw, lane);
      stage_read<TN, BJ>(b, st + C::SA, LC < 4 ? (LC & 1) : (first ? bt0 : bt1), cw, lane);
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int i = 0; i < BI; ++i)
#pragma unroll
          for (int jj = 0; jj < BJ; ++jj)
            if (!CK || live[i][jj]) acc.v[i][jj] = mfma16(a[i][q], b[jj][q], acc.v[i][jj]);
    }
  };
  using LFix = std::integral_constant<int, L0>;
  using LRun = std::integral_constant<int, 4>;
  if (__builtin_amdgcn_readfirstlane((int)all_live)) {
    kloop(std::false_type{}, LFix{}, 0, L0 < 4 ? nk0 : total);
    if (L0 < 4) kloop(std::false_type{}, LRun{}, nk0, total);
  } else {
    kloop(std::true_type{}, LFix{}, 0, L0 < 4 ? nk0 : total);
    if (L0 < 4) kloop(std::true_type{}, LRun{}, nk0, total);
  }

  const int64_t coff = b0 * P.sC0 + b1 * P.sC1;
  double* Cb = P.Cout + coff;
  const double* Cib = P.Cin ? P.Cin + coff : nullptr;
#pragma unroll
  for (int bi = 0; bi < BI; ++bi)
#pragma unroll
    for (int bj = 0; bj < BJ; ++bj)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int r = rw + 16 * bi + acc_row(lane, e), c = cw + 16 * bj + acc_col(lane);
        const int gr = m0 + r, gc = n0 + c;
        double v = P.alpha * acc.v[bi][bj][e];
        const bool lv = r < mext && c < next && !(P.store != ST_FULL && gc > gr);
        if (lv && P.beta != 0.0) v += P.beta * Cib[(int64_t)gr * P.ldc + gc];
        acc.v[bi][bj][e] = v;
      }
#pragma unroll
  for (int bi = 0; bi < BI; ++bi)
#pragma unroll
    for (int bj = 0; bj < BJ; ++bj)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int r = rw + 16 * bi + acc_row(lane, e), c = cw + 16 * bj + acc_col(lane);
        const int gr = m0 + r, gc = n0 + c;
        if (r >= mext || c >= next) continue;
        if (P.store != ST_FULL && gc > gr) continue;
        Cb[(int64_t)gr * P.ldc + gc] = acc.v[bi][bj][e];
        if (P.store == ST_LOWER_MIRROR && gc < gr) Cb[(int64_t)gc * P.ldc + gr] = acc.v[bi][bj][e];
      }
}

// Workgroups are dealt to the 8 XCDs round robin (workgroup i runs on XCD
// i % 8); renumber them so that each XCD receives a contiguous range of tiles.
__device__ __forceinline__ long long xcd_tile(long long bid, long long nblocks) {
  constexpr int NX = 8;
  const long long q = nblocks / NX, r = nblocks % NX;
  const long long x = bid % NX, j = bid / NX;
  return x * q + (x < r ? x : r) + j;
}

__device__ __forceinline__ int find_prob(const GemmArgs& args, long long t) {
  int j = 0;
  while (j + 1 < args.nprob && t >= args.p[j + 1].tile_begin) ++j;
  return j;
}

__global__ __launch_bounds__(NT, 2) void gemm_kernel(GemmArgs args) {
  __shared__ double As[64 * 66];
  __shared__ double Bs[64 * 66];
  const int j = find_prob(args, blockIdx.x);
  gemm_tile_body<2, 2, 64>(args.p[j], blockIdx.x - args.p[j].tile_begin, threadIdx.x, As, Bs);
}

__global__ __launch_bounds__(NT, 1) void gemm128_kernel(GemmArgs args) {
  __shared__ double As[128 * 34];
  __shared__ double Bs[128 * 34];
  const int j = find_prob(args, blockIdx.x);
  gemm_tile_body<4, 4, 32>(args.p[j], blockIdx.x - args.p[j].tile_begin, threadIdx.x, As, Bs);
}

template <int L0>
__global__ __launch_bounds__(NT, 2) void gemm_dl128_kernel(GemmArgs args) {
  __shared__ __align__(16) double lds[2 * DLCfg<4, 4>::STAGE];
  const long long t = xcd_tile(blockIdx.x, gridDim.x);
  const int j = find_prob(args, t);
  gemm_tile_dl<4, 4, L0>(args.p[j], t - args.p[j].tile_begin, threadIdx.x, lds);
}

template <int L0>
__global__ __launch_bounds__(NT, 4) void gemm_dl64_kernel(GemmArgs args) {
  __shared__ __align__(16) double lds[2 * DLCfg<2, 2>::STAGE];
  const long long t = xcd_tile(blockIdx.x, gridDim.x);
  const int j = find_prob(args, t);
  gemm_tile_dl<2, 2, L0>(args.p[j], t - args.p[j].tile_begin, threadIdx.x, lds);
}

template <int L0>
__global__ __launch_bounds__(256, 2) void gemm_l64_kernel(GemmArgs args) {
  __shared__ __align__(16) double lds[2 * DL2<2, 2, 2, 2>::STAGE];
  const long long t = xcd_tile(blockIdx.x, gridDim.x);
  const int j = find_prob(args, t);
  gemm_tile_dl2<2, 2, 2, 2, L0>(args.p[j], t - args.p[j].tile_begin, threadIdx.x, lds);
}

template <int L0>
__global__ __launch_bounds__(512, 3) void gemm_l128x64_kernel(GemmArgs args) {
  __shared__ __align__(16) double lds[2 * DL2<4, 2, 2, 2>::STAGE];
  const long long t = xcd_tile(blockIdx.x, gridDim.x);
  const int j = find_prob(args, t);
  gemm_tile_dl2<4, 2, 2, 2, L0>(args.p[j], t - args.p[j].tile_begin, threadIdx.x, lds);
}

// 128 x 128 tiles: four LDS stages, three in flight (one workgroup per CU:
// the deeper pipeline covers the loads that a second workgroup covered with
// two stages; n=128, b=2048 selected inversion 118.7 -> 118.2 ms, n=256,
// b=4096 1600.6 -> 1590.5 ms); two stages under BTA_L128_STAGES=2.
template <int L0>
__global__ __launch_bounds__(512, 1) void gemm_l128_kernel(GemmArgs args) {
  __shared__ __align__(16) double lds[4 * DL2<4, 2, 2, 4>::STAGE];
  const long long t = xcd_tile(blockIdx.x, gridDim.x);
  const int j = find_prob(args, t);
  gemm_tile_dl2<4, 2, 2, 4, L0, 4>(args.p[j], t - args.p[j].tile_begin, threadIdx.x, lds);
}
template <int L0>
__global__ __launch_bounds__(512, 2) void gemm_l128s2_kernel(GemmArgs args) {
  __shared__ __align__(16) double lds[2 * DL2<4, 2, 2, 4>::STAGE];
  const long long t = xcd_tile(blockIdx.x, gridDim.x);
  const int j = find_prob(args, t);
  gemm_tile_dl2<4, 2, 2, 4, L0>(args.p[j], t - args.p[j].tile_begin, threadIdx.x, lds);
}
static int l128_stages() {
  static const int ns = [] {
    long long v = 0;
    return (env_int("BTA_L128_STAGES", 2, 4, &v) && v == 2) ? 2 : 4;
  }();
  return ns;
}

// Whether the direct-to-LDS bodies can take a problem: 16-byte aligned
// operands, even leading dimensions, strides and k extents (their loads move
// pairs of doubles).
__host__ __device__ inline bool dl_ok(const GProb& p) {
  auto al = [](const double* q) { return q == nullptr || (reinterpret_cast<uintptr_t>(q) & 15) == 0; };
  for (int s = 0; s < p.nseg; ++s) {
    const GSeg& g = p.seg[s];
    if (!al(g.A) || !al(g.B)) return false;
    if ((g.lda | g.ldb | g.sA0 | g.sA1 | g.sB0 | g.sB1) & 1) return false;
    if (g.K & 1) return false;
    if (g.at && (p.M & 1)) return false;
    if (g.bt && (p.N & 1)) return false;
  }
  return true;
}

// The same tile bodies over a problem list in device memory (batched launches):
// tile_begin[] holds the first tile of every problem.
__device__ __forceinline__ int find_prob_list(const long long* tile_begin, int nprob, long long t) {
  int lo = 0, hi = nprob - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (tile_begin[mid] <= t) lo = mid; else hi = mid - 1;
  }
  return __builtin_amdgcn_readfirstlane(lo);
}

// 64 x 64 tiles: the lean direct-to-LDS body where the problem allows it
// (a workgroup-uniform test), with four LDS stages (three in flight: the
// batched products have short k loops whose loads a single stage of products
// cannot cover), the register-staged body otherwise.
constexpr int LIST64_LDS = 2 * 64 * 66 > 4 * DL2<2, 2, 2, 2>::STAGE ? 2 * 64 * 66 : 4 * DL2<2, 2, 2, 2>::STAGE;
template <int NS>
__global__ __launch_bounds__(NT, 2) void gemm_list_kernel(const GProb* probs, const long long* tile_begin, int nprob) {
  __shared__ __align__(16) double lds[LIST64_LDS];
  const int j = find_prob_list(tile_begin, nprob, blockIdx.x);
  const GProb& P = probs[j];  // read in place: a private copy would live in scratch
  const long long local = blockIdx.x - tile_begin[j];
  if (dl_ok(P)) gemm_tile_dl2<2, 2, 2, 2, 4, NS>(P, local, threadIdx.x, lds);
  else gemm_tile_body<2, 2, 64>(P, local, threadIdx.x, lds, lds + 64 * 66);
}

// 128 x 128 tiles, likewise (the first direct-to-LDS body: 256 threads).
constexpr int LIST128_LDS = 2 * 128 * 34 > 2 * DLCfg<4, 4>::STAGE ? 2 * 128 * 34 : 2 * DLCfg<4, 4>::STAGE;
__global__ __launch_bounds__(NT, 1) void gemm128_list_kernel(const GProb* probs, const long long* tile_begin, int nprob) {
  __shared__ __align__(16) double lds[LIST128_LDS];
  const int j = find_prob_list(tile_begin, nprob, blockIdx.x);
  const GProb& P = probs[j];  // read in place: a private copy would live in scratch
  const long long local = blockIdx.x - tile_begin[j];
  if (dl_ok(P)) gemm_tile_dl<4, 4, 4>(P, local, threadIdx.x, lds);
  else gemm_tile_body<4, 4, 32>(P, local, threadIdx.x, lds, lds + 128 * 34);
}

// Skinny products: at most SK_M rows of C, every segment with plain k ranges
// (TRI_NONE), A read along its rows (at == 0) and B along its k rows
// (bt == 1), one batch entry, a full store.  The selected inversion's arrow
// rows are such products (a rows): with 64 x 64 tiles most of every tile's
// MFMA work and k-loop latency would go to rows that do not exist.  One
// workgroup per 64 columns of one problem: each thread owns a column and a
// k residue mod 4 and keeps SK_M row sums; A is staged through LDS in chunks
// of SK_KC k values (one broadcast read per k and row), B streams from memory
// (coalesced rows of 64 doubles; a chunk's loads of A and B are all issued
// before any is used: the kernel is bound by reading B).  The four k residues are added in a fixed order:
// deterministic.
constexpr int SK_M = 16, SK_KC = 128;

bool gemm_skinny_ok(const GProb& p) {
  if (p.M > SK_M || p.M <= 0 || p.nb0 != 1 || p.nb1 != 1 || p.store != ST_FULL || p.lower_tiles) return false;
  for (int s = 0; s < p.nseg; ++s)
    if (p.seg[s].tri != TRI_NONE || p.seg[s].at != 0 || p.seg[s].bt != 1) return false;
  return true;
}

__global__ __launch_bounds__(256) void gemm_skinny_list_kernel(const GProb* probs, const long long* tile_begin, int nprob) {
  __shared__ double As[SK_M * SK_KC];
  __shared__ double red[4 * SK_M * 64];
  const int j = find_prob_list(tile_begin, nprob, blockIdx.x);
  const GProb& P = probs[j];
  const int tid = threadIdx.x, c = tid & 63;
  const int ks = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int M = P.M, N = P.N;
  const int M4 = (M + 3) & ~3;  // rows in groups of four (rows M .. M4-1 of As are zero)
  const int c0 = (int)(blockIdx.x - tile_begin[j]) * 64;
  const int gc = c0 + c;
  const int ar = tid >> 7, ak = tid & (SK_KC - 1);  // A staging: rows ar + 2q, column ak of the chunk
  double acc[SK_M];
#pragma unroll
  for (int m = 0; m < SK_M; ++m) acc[m] = 0.0;
  for (int s = 0; s < P.nseg; ++s) {
    const GSeg& g = P.seg[s];
    for (int k0 = 0; k0 < g.K; k0 += SK_KC) {
      const int kc = min(SK_KC, g.K - k0);
      // every load of the chunk in flight at once: the A chunk (coalesced
      // along k) and this thread's 32 values of B (k = ks + 4u)
      double areg[SK_M / 2];
#pragma unroll
      for (int q = 0; q < SK_M / 2; ++q) {
        const int m = ar + 2 * q;
        areg[q] = (m < M && ak < kc) ? g.A[(int64_t)m * g.lda + k0 + ak] : 0.0;
      }
      const double* Bk = g.B + (int64_t)k0 * g.ldb + (gc < N ? gc : 0);
      double bv[SK_KC / 4];
#pragma unroll
      for (int u = 0; u < SK_KC / 4; ++u) {
        const int k = ks + 4 * u;
        bv[u] = (k < kc && gc < N) ? Bk[(int64_t)k * g.ldb] : 0.0;
      }
      __syncthreads();  // the previous chunk's reads of As are done
#pragma unroll
      for (int q = 0; q < SK_M / 2; ++q)
        if (ar + 2 * q < M4) As[(ar + 2 * q) * SK_KC + ak] = areg[q];
      __syncthreads();
#pragma unroll
      for (int u = 0; u < SK_KC / 4; ++u) {
        const int k = ks + 4 * u;
#pragma unroll
        for (int mg = 0; mg < SK_M / 4; ++mg) {
          if (4 * mg >= M4) break;  // workgroup-uniform
#pragma unroll
          for (int r = 0; r < 4; ++r) acc[4 * mg + r] = fma(As[(4 * mg + r) * SK_KC + k], bv[u], acc[4 * mg + r]);
        }
      }
    }
  }
#pragma unroll
  for (int m = 0; m < SK_M; ++m) red[(ks * SK_M + m) * 64 + c] = acc[m];
  __syncthreads();
  for (int e = tid; e < M * 64; e += 256) {
    const int m = e >> 6, cc = e & 63, col = c0 + cc;
    if (col >= N) continue;
    double v = red[(0 * SK_M + m) * 64 + cc] + red[(1 * SK_M + m) * 64 + cc];
    v += red[(2 * SK_M + m) * 64 + cc];
    v += red[(3 * SK_M + m) * 64 + cc];
    v *= P.alpha;
    if (P.beta != 0.0) v += P.beta * P.Cin[(int64_t)m * P.ldc + col];
    P.Cout[(int64_t)m * P.ldc + col] = v;
  }
}

// A list of skinny problems (gemm_skinny_ok): tile_begin[] as for 64 x 64
// tiles (one tile per 64 columns: the problems have one row of tiles).
hipError_t gemm_skinny_list_launch(const GProb* d_probs, const long long* d_tile_begin, int nprob, long long ntiles,
                                   hipStream_t stream) {
  if (ntiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(gemm_skinny_list_kernel, dim3((unsigned)ntiles), dim3(256), 0, stream, d_probs, d_tile_begin, nprob);
  return hipGetLastError();
}

hipError_t gemm_list_launch(const GProb* d_probs, const long long* d_tile_begin, int nprob, long long ntiles, int big,
                            hipStream_t stream) {
  if (ntiles <= 0) return hipSuccess;
  if (big)
    hipLaunchKernelGGL(gemm128_list_kernel, dim3((unsigned)ntiles), dim3(NT), 0, stream, d_probs, d_tile_begin, nprob);
  else if (list_stages() == 2)
    hipLaunchKernelGGL(gemm_list_kernel<2>, dim3((unsigned)ntiles), dim3(NT), 0, stream, d_probs, d_tile_begin, nprob);
  else
    hipLaunchKernelGGL(gemm_list_kernel<4>, dim3((unsigned)ntiles), dim3(NT), 0, stream, d_probs, d_tile_begin, nprob);
  return hipGetLastError();
}

long long gemm_prob_tiles(GProb& p, int tile) {
  p.ntm = (p.M + tile - 1) / tile;
  p.ntn = (p.N + tile - 1) / tile;
  if (p.lower_tiles) {
    long long cnt = 0;
    for (int tm = 0; tm < p.ntm; ++tm) cnt += std::min(p.ntn, (tm * tile + tile - 1) / tile + 1);
    p.tiles_per_batch = (int)cnt;
  } else {
    p.tiles_per_batch = p.ntm * p.ntn;
  }
  return (long long)p.tiles_per_batch * p.nb0 * p.nb1;
}

thread_local DryRecorder* g_dry = nullptr;
thread_local StageRecorder* g_rec = nullptr;

// ---------------------------------------------------------------- kernel timer
namespace {
struct KernelTimer {
  unsigned mask = 0;  // kinds recorded: bit k for kind k (KT_FACTOR, KT_GEMM, ...)
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  std::vector<std::pair<int, std::pair<size_t, size_t>>> spans;  // (kind, (start event, stop event))
  size_t open_start[KT_COUNT] = {0, 0, 0, 0};
};
KernelTimer g_timer;
}  // namespace

bool timing_on() { return g_timer.mask != 0; }

void timing_mark(int kind, bool start, hipStream_t stream) {
  if (!((g_timer.mask >> kind) & 1u) || g_timer.used >= g_timer.pool.size()) return;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(stream, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone) return;
  const size_t e = g_timer.used++;
  (void)hipEventRecord(g_timer.pool[e], stream);
  if (start) g_timer.open_start[kind] = e;
  else g_timer.spans.push_back({kind, {g_timer.open_start[kind], e}});
}

static void record_gemm(const GProb& p) {
  for (int b0 = 0; b0 < p.nb0; ++b0)
    for (int b1 = 0; b1 < p.nb1; ++b1) {
      for (int s = 0; s < p.nseg; ++s) {
        const GSeg& g = p.seg[s];
        if (g.K <= 0) continue;
        const double* A = g.A + b0 * g.sA0 + b1 * g.sA1;
        const double* B = g.B + b0 * g.sB0 + b1 * g.sB1;
        if (g.at) g_dry->add(A, g.K, p.M, g.lda, false); else g_dry->add(A, p.M, g.K, g.lda, false);
        if (g.bt) g_dry->add(B, g.K, p.N, g.ldb, false); else g_dry->add(B, p.N, g.K, g.ldb, false);
      }
      const int64_t off = b0 * p.sC0 + b1 * p.sC1;
      if (p.beta != 0.0) g_dry->add(p.Cin + off, p.M, p.N, p.ldc, false);
      g_dry->add(p.Cout + off, p.M, p.N, p.ldc, true);
      if (p.store == ST_LOWER_MIRROR) g_dry->add(p.Cout + off, p.N, p.M, p.ldc, true);
    }
}

static long long plan_tiles(GemmArgs& args, GProb* probs, int nprob, int TM, int TN) {
  args.nprob = 0;
  long long total = 0;
  for (int i = 0; i < nprob; ++i) {
    GProb p = probs[i];
    if (p.M <= 0 || p.N <= 0 || p.nb0 <= 0 || p.nb1 <= 0) continue;
    p.ntm = (p.M + TM - 1) / TM;
    p.ntn = (p.N + TN - 1) / TN;
    if (p.lower_tiles) {
      long long cnt = 0;
      for (int tm = 0; tm < p.ntm; ++tm) cnt += std::min(p.ntn, (tm * TM + TM - 1) / TN + 1);
      p.tiles_per_batch = (int)cnt;
    } else {
      p.tiles_per_batch = p.ntm * p.ntn;
    }
    p.tile_begin = total;
    total += (long long)p.tiles_per_batch * p.nb0 * p.nb1;
    args.p[args.nprob++] = p;
    if (args.nprob == GEMM_MAX_PROBS) break;
  }
  args.ntiles = total;
  return total;
}

// Operands the direct-to-LDS body can move in 16-byte pieces.

// 0: choose per launch; 1: register-staged kernels only; 2: direct-to-LDS
// kernels wherever the operands allow; 3 / 4: first direct-to-LDS body with 64
// / 128 tiles; 5 / 6 / 7: lean body with 64 x 64 / 128 x 64 / 128 x 128 tiles
// (tests run every path through this).
static int g_gemm_mode = 0;

// Sum over the tiles of a planned launch of the fraction of MFMA blocks a
// tile computes (ragged edges and lower-store tiles compute fewer).
static double tile_weight(const GemmArgs& a, int TM, int TN) {
  double w = 0.0;
  for (int pi = 0; pi < a.nprob; ++pi) {
    const GProb& p = a.p[pi];
    double per = 0.0;
    for (int tm = 0; tm < p.ntm; ++tm) {
      const int rows = std::min(TM, p.M - tm * TM);
      const int tn_end = p.lower_tiles ? std::min(p.ntn, (tm * TM + TM - 1) / TN + 1) : p.ntn;
      for (int tn = 0; tn < tn_end; ++tn) {
        const int cols = std::min(TN, p.N - tn * TN);
        double f = (double)((rows + 15) / 16 * 16) * ((cols + 15) / 16 * 16) / ((double)TM * TN);
        if (p.store != ST_FULL && tn * TN + TN > tm * TM) f *= 0.6;  // diagonal tile of a lower store
        per += f;
      }
    }
    w += per * p.nb0 * p.nb1;
  }
  return w;
}

hipError_t gemm_launch(GProb* probs, int nprob, hipStream_t stream) {
  if (g_rec) {
    for (int i = 0; i < nprob; ++i)
      if (probs[i].M > 0 && probs[i].N > 0 && probs[i].nb0 > 0 && probs[i].nb1 > 0) g_rec->gemm(probs[i]);
    return hipSuccess;
  }
  if (g_dry) {
    ++g_dry->op;
    for (int i = 0; i < nprob; ++i)
      if (probs[i].M > 0 && probs[i].N > 0) record_gemm(probs[i]);
    return hipSuccess;
  }
  bool dl = g_gemm_mode != 1;
  for (int i = 0; i < nprob; ++i) dl = dl && dl_ok(probs[i]);
  GemmArgs big{}, small{}, mid{};
  const long long t128 = plan_tiles(big, probs, nprob, 128, 128);
  const long long t64 = plan_tiles(small, probs, nprob, 64, 64);
  const long long t12864 = plan_tiles(mid, probs, nprob, 128, 64);
  if (t64 == 0) return hipSuccess;
  if (dl) {
    int kind = g_gemm_mode >= 3 ? g_gemm_mode : 0;
    if (kind == 0) {
      // 128 x 128 tiles (the most efficient per flop) when they fill the CUs
      // in whole rounds (at least 3/4 of the last round) and are mostly full
      // (ragged tiles cost nearly a whole tile of loads); otherwise 64 x 64
      // tiles, with the first direct-to-LDS body for lower-triangle stores
      // (fewer, unevenly sized tiles).
      const double cus = std::max(1, device_cu_count());
      const double rounds = std::ceil((double)t128 / cus);
      const bool fill = (double)t128 >= 0.75 * rounds * cus;
      const bool full = tile_weight(big, 128, 128) >= 0.85 * (double)t128;
      bool lower_only = true;
      for (int i = 0; i < nprob; ++i) lower_only = lower_only && probs[i].lower_tiles;
      kind = (fill && full) ? 7 : (lower_only ? 3 : 5);
    }
    // the first segment's layout when every problem of the launch shares it
    int L0 = small.p[0].seg[0].at * 2 + small.p[0].seg[0].bt;
    for (int i = 1; i < small.nprob; ++i)
      if (small.p[i].seg[0].at * 2 + small.p[i].seg[0].bt != L0) L0 = 4;
#define BTA_LAUNCH_L0(KER, GRID, BLOCK, ARGS)                                                  \
  switch (L0) {                                                                                \
    case 0: hipLaunchKernelGGL((KER<0>), dim3((unsigned)(GRID)), dim3(BLOCK), 0, stream, ARGS); break; \
    case 1: hipLaunchKernelGGL((KER<1>), dim3((unsigned)(GRID)), dim3(BLOCK), 0, stream, ARGS); break; \
    case 2: hipLaunchKernelGGL((KER<2>), dim3((unsigned)(GRID)), dim3(BLOCK), 0, stream, ARGS); break; \
    case 3: hipLaunchKernelGGL((KER<3>), dim3((unsigned)(GRID)), dim3(BLOCK), 0, stream, ARGS); break; \
    default: hipLaunchKernelGGL((KER<4>), dim3((unsigned)(GRID)), dim3(BLOCK), 0, stream, ARGS); break; \
  }
    timing_mark(KT_GEMM, true, stream);
    switch (kind) {
      case 3: BTA_LAUNCH_L0(gemm_dl64_kernel, t64, NT, small); break;
      case 4: BTA_LAUNCH_L0(gemm_dl128_kernel, t128, NT, big); break;
      case 5: BTA_LAUNCH_L0(gemm_l64_kernel, t64, 256, small); break;
      case 7:
        if (l128_stages() == 2) BTA_LAUNCH_L0(gemm_l128s2_kernel, t128, 512, big)
        else BTA_LAUNCH_L0(gemm_l128_kernel, t128, 512, big)
        break;
      default: BTA_LAUNCH_L0(gemm_l128x64_kernel, t12864, 512, mid); break;
    }
#undef BTA_LAUNCH_L0
    timing_mark(KT_GEMM, false, stream);
    return hipGetLastError();
  }
  // 128 x 128 tiles when they alone give at least ~one tile per CU and every
  // problem is at least 128 on both sides; 64 x 64 tiles otherwise.
  bool use_big = t128 >= 200;
  for (int i = 0; i < big.nprob; ++i)
    if (big.p[i].M < 128 && big.p[i].N < 128) use_big = false;
  timing_mark(KT_GEMM, true, stream);
  if (use_big)
    hipLaunchKernelGGL(gemm128_kernel, dim3((unsigned)t128), dim3(NT), 0, stream, big);
  else
    hipLaunchKernelGGL(gemm_kernel, dim3((unsigned)t64), dim3(NT), 0, stream, small);
  timing_mark(KT_GEMM, false, stream);
  return hipGetLastError();
}

// ---------------------------------------------------------------- split-k
// C = beta*Cin + alpha*sum_s P_s over the partial products of a split launch
// (summed in split order: deterministic), with the problem's store mode.
// Block (x, r) covers columns 512x .. 512x + 511 of row r, two per thread
// (16-byte loads when N is even); blocks entirely above the diagonal of a
// lower store exit at once.
__global__ __launch_bounds__(256) void splitk_reduce_kernel(const double* P, int S, int M, int N, const double* Cin,
                                                            double* C, int64_t ldc, double alpha, double beta, int store) {
  const int r = blockIdx.y;
  const int c0 = blockIdx.x * 512;
  if (store != ST_FULL && c0 > r) return;
  const int64_t MN = (int64_t)M * N;
  const int c = c0 + 2 * threadIdx.x;
  if (c >= N) return;
  const int64_t e = (int64_t)r * N + c;
  const bool pair = (N % 2 == 0) && (c + 1 < N);
  double v0 = 0.0, v1 = 0.0;
  if (pair) {
    for (int q = 0; q < S; ++q) {
      const d2v x = *reinterpret_cast<const d2v*>(P + q * MN + e);
      v0 += x[0];
      v1 += x[1];
    }
  } else {
    for (int q = 0; q < S; ++q) {
      v0 += P[q * MN + e];
      if (c + 1 < N) v1 += P[q * MN + e + 1];
    }
  }
  for (int h = 0; h < 2; ++h) {
    const int cc = c + h;
    if (cc >= N || (store != ST_FULL && cc > r)) continue;
    double v = alpha * (h ? v1 : v0);
    if (beta != 0.0) v += beta * Cin[(int64_t)r * ldc + cc];
    C[(int64_t)r * ldc + cc] = v;
    if (store == ST_LOWER_MIRROR && cc < r) C[(int64_t)cc * ldc + r] = v;
  }
}

int splitk_factor(const GProb& p, size_t ws_doubles, int smax) {
  if (p.nb0 != 1 || p.nb1 != 1 || p.nseg < 1 || p.M <= 0 || p.N <= 0) return 1;
  for (int q = 0; q < p.nseg; ++q)
    if (p.seg[q].tri != TRI_NONE) return 1;
  const int K0 = p.seg[0].K;
  GemmArgs tmp{};
  GProb c = p;
  const long long t64 = plan_tiles(tmp, &c, 1, 64, 64);
  int cus = device_cu_count();
  if (cus <= 0 && g_dry) cus = 256;  // host dry run: plan for the full chip
  cus = std::max(1, cus);
  if (t64 <= 0 || 2 * t64 > cus) return 1;
  int S = (int)std::min<long long>(std::min(smax, GEMM_MAX_PROBS), cus / t64);
  S = std::min(S, K0 / 128);  // at least 128 of k per split
  while (S > 1 && (size_t)S * p.M * p.N > ws_doubles) --S;
  return S >= 2 ? S : 1;
}

hipError_t gemm_launch_split(GProb* probs, int nprob, hipStream_t stream, double* ws, size_t ws_doubles, int smax) {
  if (g_rec || nprob != 1 || ws == nullptr) return gemm_launch(probs, nprob, stream);
  const GProb& p = probs[0];
  const int S = splitk_factor(p, ws_doubles, smax);
  if (S < 2) return gemm_launch(probs, nprob, stream);
  const int K0 = p.seg[0].K;
  // split boundaries on multiples of 64 (16-byte aligned operand rows stay aligned)
  const int chunk = ((K0 + S - 1) / S + 63) / 64 * 64;
  GProb sub[GEMM_MAX_PROBS];
  int ns = 0;
  for (int q = 0; q < S; ++q) {
    const int k0 = q * chunk, k1 = std::min(K0, k0 + chunk);
    if (k1 <= k0 && q > 0) break;
    GProb t = p;
    GSeg g = p.seg[0];
    g.A = g.at ? g.A + (int64_t)k0 * g.lda : g.A + k0;
    g.B = g.bt ? g.B + (int64_t)k0 * g.ldb : g.B + k0;
    g.K = k1 - k0;
    t.seg[0] = g;
    t.nseg = q == 0 ? p.nseg : 1;  // the short second segment goes with the first split
    t.Cin = nullptr;
    t.Cout = ws + (int64_t)q * p.M * p.N;
    t.ldc = p.N; t.sC0 = 0; t.sC1 = 0;
    t.alpha = 1.0; t.beta = 0.0;
    t.store = p.store == ST_FULL ? ST_FULL : ST_LOWER;
    sub[ns++] = t;
  }
  hipError_t e = gemm_launch(sub, ns, stream);
  if (e != hipSuccess) return e;
  if (g_dry) {
    ++g_dry->op;
    for (int q = 0; q < ns; ++q) g_dry->add(ws + (int64_t)q * p.M * p.N, p.M, p.N, p.N, false);
    if (p.beta != 0.0) g_dry->add(p.Cin, p.M, p.N, p.ldc, false);
    g_dry->add(p.Cout, p.M, p.N, p.ldc, true);
    if (p.store == ST_LOWER_MIRROR) g_dry->add(p.Cout, p.N, p.M, p.ldc, true);
    return hipSuccess;
  }
  const dim3 grid((unsigned)((p.N + 511) / 512), (unsigned)p.M);
  timing_mark(KT_GEMM, true, stream);
  hipLaunchKernelGGL(splitk_reduce_kernel, grid, dim3(256), 0, stream, ws, ns, p.M, p.N, p.Cin, p.Cout, p.ldc,
                     p.alpha, p.beta, p.store);
  timing_mark(KT_GEMM, false, stream);
  return hipGetLastError();
}

// ---------------------------------------------------------------- small kernels

__global__ __launch_bounds__(NT) void trinv_diag_tiles_kernel(const double* L, int64_t ldL, int64_t sL, double* W,
                                                              int64_t ldW, int64_t sW, int m, int T) {
  __shared__ double S[TS * LDS_LD];
  const int tid = threadIdx.x;
  const int blk = blockIdx.x / T, t = blockIdx.x - (blockIdx.x / T) * T;
  const int ext = min(64, m - t * 64);
  const double* Lt = L + blk * sL + (int64_t)t * 64 * ldL + t * 64;
  for (int e = tid; e < 64 * 64; e += NT) {
    const int rr = e >> 6, cc = e & 63;
    double v;
    if (rr < ext && cc < ext) v = (cc <= rr) ? Lt[(int64_t)rr * ldL + cc] : 0.0;
    else v = (rr == cc) ? 1.0 : 0.0;
    S[rr * LDS_LD + cc] = v;
  }
  __syncthreads();
  double w[16];
  trinv_tile(S, w, tid);
  const int r = tid & 63, q = tid >> 6;
  double* Wt = W + blk * sW + (int64_t)t * 64 * ldW + t * 64;
  if (r < ext) {
#pragma unroll
    for (int mm = 0; mm < 16; ++mm) {
      const int c = 16 * q + mm;
      if (c < ext) Wt[(int64_t)r * ldW + c] = (c <= r) ? w[mm] : 0.0;
    }
  }
}

hipError_t trinv_diag_tiles_launch(const double* L, int64_t ldL, int64_t sL, double* W, int64_t ldW, int64_t sW,
                                   int m, int nblk, hipStream_t stream) {
  const int T = (m + 63) / 64;
  if (T == 0 || nblk == 0) return hipSuccess;
  if (g_rec) {
    g_rec->trinv(TrinvOp{L, ldL, sL, W, ldW, sW, m, nblk});
    return hipSuccess;
  }
  if (g_dry) {
    ++g_dry->op;
    for (int blk = 0; blk < nblk; ++blk) {
      g_dry->add(L + blk * sL, m, m, ldL, false);
      g_dry->add(W + blk * sW, m, m, ldW, true);
    }
    return hipSuccess;
  }
  timing_mark(KT_TRINV, true, stream);
  hipLaunchKernelGGL(trinv_diag_tiles_kernel, dim3((unsigned)(T * nblk)), dim3(NT), 0, stream, L, ldL, sL, W, ldW, sW, m, T);
  timing_mark(KT_TRINV, false, stream);
  return hipGetLastError();
}

__global__ void fill_zero_kernel(double* p, size_t count) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x) p[i] = 0.0;
}

hipError_t fill_zero_launch(double* p, size_t count, hipStream_t stream) {
  if (count == 0) return hipSuccess;
  if (g_rec) {
    g_rec->fill(FillOp{p, (long long)count});
    return hipSuccess;
  }
  if (g_dry) {
    ++g_dry->op;
    g_dry->add(p, 1, (int64_t)count, (int64_t)count, true);
    return hipSuccess;
  }
  const unsigned grid = (unsigned)std::min<size_t>(4096, (count + 255) / 256);
  hipLaunchKernelGGL(fill_zero_kernel, dim3(grid), dim3(256), 0, stream, p, count);
  return hipGetLastError();
}

__global__ void copy2d_kernel(const double* src, int64_t lds, int64_t ss, double* dst, int64_t ldd, int64_t sd,
                              int rows, int cols) {
  const int blk = blockIdx.y;
  const double* s = src + blk * ss;
  double* d = dst + blk * sd;
  const long long stride = (long long)gridDim.x * blockDim.x;
  const bool pairs = ((cols | lds | ldd) & 1) == 0 && ((reinterpret_cast<uintptr_t>(s) | reinterpret_cast<uintptr_t>(d)) & 15) == 0;
  if (pairs) {  // 16-byte moves
    const int hc = cols >> 1;
    const long long total = (long long)rows * hc;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride) {
      const int r = (int)(e / hc), c = 2 * (int)(e - (long long)r * hc);
      *reinterpret_cast<double2*>(d + (int64_t)r * ldd + c) = *reinterpret_cast<const double2*>(s + (int64_t)r * lds + c);
    }
    return;
  }
  const long long total = (long long)rows * cols;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride) {
    const int r = (int)(e / cols), c = (int)(e - (long long)r * cols);
    d[(int64_t)r * ldd + c] = s[(int64_t)r * lds + c];
  }
}

hipError_t copy2d_launch(const double* src, int64_t lds, int64_t ss, double* dst, int64_t ldd, int64_t sd,
                         int rows, int cols, int nb, hipStream_t stream) {
  if (rows <= 0 || cols <= 0 || nb <= 0) return hipSuccess;
  if (g_rec) {
    g_rec->copy(CopyOp{src, lds, ss, dst, ldd, sd, rows, cols, nb});
    return hipSuccess;
  }
  if (g_dry) {
    ++g_dry->op;
    for (int b = 0; b < nb; ++b) {
      g_dry->add(src + b * ss, rows, cols, lds, false);
      g_dry->add(dst + b * sd, rows, cols, ldd, true);
    }
    return hipSuccess;
  }
  const long long total = (long long)rows * cols;
  const unsigned gx = (unsigned)std::min<long long>(2048, (total + 255) / 256);
  hipLaunchKernelGGL(copy2d_kernel, dim3(gx, (unsigned)nb), dim3(256), 0, stream, src, lds, ss, dst, ldd, sd, rows, cols);
  return hipGetLastError();
}

int device_cu_count() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  return cus;
}

}  // namespace bta

// Internal timing controls (not part of the public header): enable the kinds
// in `kinds` (bit k for kind k; 0 turns timing off) with a pool of event
// pairs, read back per-kind total milliseconds and launch counts.  Every
// recorded launch adds two event records to its stream, so a measurement of a
// launch-heavy sequence enables only the kinds it reads.
BTA_TESTING_API int bta_internal_timing(int kinds, int max_launches) {
  using namespace bta;
  for (hipEvent_t e : g_timer.pool) (void)hipEventDestroy(e);
  g_timer.pool.clear();
  g_timer.spans.clear();
  g_timer.used = 0;
  g_timer.mask = 0;
  if (!kinds) return 0;
  g_timer.pool.resize((size_t)2 * max_launches);
  for (auto& e : g_timer.pool)
    if (hipEventCreate(&e) != hipSuccess) return 1;
  g_timer.mask = (unsigned)kinds & ((1u << KT_COUNT) - 1u);
  return 0;
}

// Internal GEMM kernel selection (see g_gemm_mode); returns the previous mode.
BTA_TESTING_API int bta_internal_gemm_mode(int mode) {
  const int prev = bta::g_gemm_mode;
  if (mode >= 0 && mode <= 7) bta::g_gemm_mode = mode;
  return prev;
}

// Internal: one product through the grouped GEMM (tests and measurements):
// C = beta * Cin + alpha * sum_k A(m,k) B(c,k), operand layouts and k range as
// in the selected inversion's problems.  Returns a HIP error code.
BTA_TESTING_API int bta_internal_gemm(
    int M, int N, int K, const double* A, int64_t lda, int at, const double* B, int64_t ldb, int bt, int tri,
    const double* Cin, double* C, int64_t ldc, double alpha, double beta, int store, int lower_tiles, hipStream_t s) {
  bta::GProb p{};
  p.seg[0].A = A; p.seg[0].B = B; p.seg[0].lda = lda; p.seg[0].ldb = ldb; p.seg[0].K = K;
  p.seg[0].at = at; p.seg[0].bt = bt; p.seg[0].tri = tri;
  p.nseg = 1;
  p.Cin = Cin; p.Cout = C; p.ldc = ldc;
  p.M = M; p.N = N; p.nb0 = 1; p.nb1 = 1;
  p.alpha = alpha; p.beta = beta; p.store = store; p.lower_tiles = lower_tiles;
  return (int)bta::gemm_launch(&p, 1, s);
}

// The same kind of product through the skinny list kernel, as two segments
// (k in [0, K1) and [K1, K)) to exercise the segment loop: dlist is device
// memory of at least 512 bytes for the one-problem list.  Returns -1 when the
// product is not skinny (more than 16 rows), else the HIP status.
BTA_TESTING_API int bta_internal_gemm_skinny(int M, int N, int K, int K1, const double* A, int64_t lda, const double* B,
                                             int64_t ldb, const double* Cin, double* C, int64_t ldc, double alpha,
                                             double beta, void* dlist, hipStream_t s) {
  if (K1 < 0 || K1 > K) return -1;
  bta::GProb p{};
  p.seg[0].A = A; p.seg[0].B = B; p.seg[0].lda = lda; p.seg[0].ldb = ldb; p.seg[0].K = K1;
  p.seg[1].A = A + K1; p.seg[1].B = B + (int64_t)K1 * ldb; p.seg[1].lda = lda; p.seg[1].ldb = ldb; p.seg[1].K = K - K1;
  for (int q = 0; q < 2; ++q) { p.seg[q].at = 0; p.seg[q].bt = 1; p.seg[q].tri = bta::TRI_NONE; }
  p.nseg = 2;
  p.Cin = Cin; p.Cout = C; p.ldc = ldc;
  p.M = M; p.N = N; p.nb0 = 1; p.nb1 = 1;
  p.alpha = alpha; p.beta = beta; p.store = bta::ST_FULL; p.lower_tiles = 0;
  if (!bta::gemm_skinny_ok(p)) return -1;
  const long long tiles = bta::gemm_prob_tiles(p, 64);
  const long long begin = 0;
  char* d = static_cast<char*>(dlist);
  hipError_t e = hipMemcpyAsync(d, &p, sizeof(p), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(d + 256, &begin, sizeof(begin), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = bta::gemm_skinny_list_launch(reinterpret_cast<const bta::GProb*>(d), reinterpret_cast<const long long*>(d + 256), 1, tiles, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);  // the host copies are read before returning
  return (int)e;
}

// A list of `nprob` copies of one product (problem q reads A + q*strideA,
// B + q*strideB and writes C + q*strideC) through the 64 x 64 list kernel
// (four LDS stages) or, with big, the 128 x 128 one; dlist is device memory of
// at least 512 * (nprob + 1) bytes.  Returns the HIP status (synchronizes `s`).
BTA_TESTING_API int bta_internal_gemm_list(int M, int N, int K, const double* A, int64_t lda, int at, const double* B,
                                           int64_t ldb, int bt, int tri, const double* Cin, double* C, int64_t ldc,
                                           double alpha, double beta, int store, int lower_tiles, int nprob,
                                           int64_t strideA, int64_t strideB, int64_t strideC, int big, void* dlist,
                                           hipStream_t s) {
  if (nprob < 1 || nprob > 64) return -1;
  std::vector<bta::GProb> ps(nprob);
  std::vector<long long> begin(nprob);
  long long tiles = 0;
  for (int q = 0; q < nprob; ++q) {
    bta::GProb& p = ps[q];
    p = bta::GProb{};
    p.seg[0].A = A + q * strideA; p.seg[0].B = B + q * strideB; p.seg[0].lda = lda; p.seg[0].ldb = ldb; p.seg[0].K = K;
    p.seg[0].at = at; p.seg[0].bt = bt; p.seg[0].tri = tri;
    p.nseg = 1;
    p.Cin = Cin ? Cin + q * strideC : nullptr; p.Cout = C + q * strideC; p.ldc = ldc;
    p.M = M; p.N = N; p.nb0 = 1; p.nb1 = 1;
    p.alpha = alpha; p.beta = beta; p.store = store; p.lower_tiles = lower_tiles;
    begin[q] = tiles;
    tiles += bta::gemm_prob_tiles(p, big ? 128 : 64);
  }
  char* d = static_cast<char*>(dlist);
  const size_t off = ((sizeof(bta::GProb) * nprob + 255) / 256) * 256;
  hipError_t e = hipMemcpyAsync(d, ps.data(), sizeof(bta::GProb) * nprob, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(d + off, begin.data(), sizeof(long long) * nprob, hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = bta::gemm_list_launch(reinterpret_cast<const bta::GProb*>(d), reinterpret_cast<const long long*>(d + off), nprob,
                              tiles, big, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);  // the host copies are read before returning
  return (int)e;
}

// The same product through the split-k path (ws: S*M*N doubles of partials;
// *splits receives the split count used, 1 = none).
BTA_TESTING_API int bta_internal_gemm_split(
    int M, int N, int K, const double* A, int64_t lda, int at, const double* B, int64_t ldb, int bt, const double* Cin,
    double* C, int64_t ldc, double alpha, double beta, int store, int lower_tiles, double* ws, size_t ws_doubles,
    int* splits, hipStream_t s) {
  bta::GProb p{};
  p.seg[0].A = A; p.seg[0].B = B; p.seg[0].lda = lda; p.seg[0].ldb = ldb; p.seg[0].K = K;
  p.seg[0].at = at; p.seg[0].bt = bt; p.seg[0].tri = bta::TRI_NONE;
  p.nseg = 1;
  p.Cin = Cin; p.Cout = C; p.ldc = ldc;
  p.M = M; p.N = N; p.nb0 = 1; p.nb1 = 1;
  p.alpha = alpha; p.beta = beta; p.store = store; p.lower_tiles = lower_tiles;
  if (splits) *splits = bta::splitk_factor(p, ws_doubles);
  return (int)bta::gemm_launch_split(&p, 1, s, ws, ws_doubles);
}

namespace bta {
// Register-only FP64 MFMA loop: every wave runs `iters` rounds of CH
// independent v_mfma_f64_16x16x4_f64 chains with no memory traffic inside the
// loop, so the launch measures the sustained FP64 matrix rate of the device
// (2048 flops per instruction).  Each thread stores one sum, which keeps the
// chains live.
template <int CH>
__global__ __launch_bounds__(256) void mfma_probe_kernel(double* out, int iters) {
  const int lane = threadIdx.x & 63;
  const double a = 1.0 + 1e-3 * lane, b = 1.0 - 1e-3 * lane;
  d4 c[CH];
#pragma unroll
  for (int j = 0; j < CH; ++j) c[j] = d4{0.0, 0.0, 0.0, 0.0};
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int j = 0; j < CH; ++j) c[j] = mfma16(a, b, c[j]);
  }
  double s = 0.0;
#pragma unroll
  for (int j = 0; j < CH; ++j) s += c[j][0] + c[j][1] + c[j][2] + c[j][3];
  out[(size_t)blockIdx.x * 256 + threadIdx.x] = s;
}
}  // namespace bta

// Internal: launch the MFMA rate probe with `grid` workgroups of 256 threads
// on `s` (chains: 4, 8 or 16 independent MFMA chains per wave); d_out holds
// grid * 256 doubles.  Flops = grid * 4 * iters * chains * 2048.
BTA_TESTING_API int bta_internal_mfma_probe(double* d_out, int grid, int iters, int chains, hipStream_t s) {
  if (!d_out || grid < 1 || iters < 1 || (chains != 4 && chains != 8 && chains != 16)) return (int)hipErrorInvalidValue;
  if (chains == 4)
    hipLaunchKernelGGL(bta::mfma_probe_kernel<4>, dim3((unsigned)grid), dim3(256), 0, s, d_out, iters);
  else if (chains == 8)
    hipLaunchKernelGGL(bta::mfma_probe_kernel<8>, dim3((unsigned)grid), dim3(256), 0, s, d_out, iters);
  else
    hipLaunchKernelGGL(bta::mfma_probe_kernel<16>, dim3((unsigned)grid), dim3(256), 0, s, d_out, iters);
  return (int)hipGetLastError();
}

BTA_TESTING_API int bta_internal_timing_read(double* ms, long long* launches) {
  using namespace bta;
  for (int k = 0; k < KT_COUNT; ++k) { ms[k] = 0.0; launches[k] = 0; }
  for (auto& sp : g_timer.spans) {
    if (hipEventSynchronize(g_timer.pool[sp.second.second]) != hipSuccess) return 1;
    float t = 0.f;
    if (hipEventElapsedTime(&t, g_timer.pool[sp.second.first], g_timer.pool[sp.second.second]) != hipSuccess) return 2;
    ms[sp.first] += t;
    launches[sp.first] += 1;
  }
  return g_timer.used >= g_timer.pool.size() ? 3 : 0;  // 3: pool exhausted, spans incomplete
}
