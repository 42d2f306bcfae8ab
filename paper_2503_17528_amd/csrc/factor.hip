// POBTAF (Algorithm 1) on gfx950 as one persistent kernel over a tile DAG.
//
// The BTA factorization is run as a left-looking tile Cholesky of the band:
// every 64 x 64 tile of L is one task, executed by one workgroup, that
// accumulates all updates it needs (in the order of the k tiles) and then
// finishes the tile:
//
//   DIAG (i,c)   L_ii(c,c)   = chol( A_ii(c,c) - sum L(c,k) L(c,k)^T ), W = its inverse
//   OFFD (i,r,c) L_ii(r,c)   = ( A_ii(r,c) - sum L(r,k) L(c,k)^T ) W(c,c)^T      (r > c)
//   SUB  (i,r,c) L_{i+1,i}   = ( A_{i+1,i}(r,c) - sum ... ) W(c,c)^T
//   ARW  (i,r,c) L_{n,i}     = ( A_{n,i}(r,c)  - sum ... ) W(c,c)^T
//   TUPD (i,r,c) P_i(r,c)    = sum_k L_{n,i}(r,k) L_{n,i}(c,k)^T   (tip update of one step)
//   TIPD/TIPO    L_nn tiles from A_nn - sum_i P_i (in step order) - sum ...
//
// The sums over the previous block column (A_{i,i} -= L_{i,i-1} L_{i,i-1}^T and
// A_{n,i} -= L_{n,i-1} L_{i,i-1}^T, the Schur updates of Algorithm 1) are folded
// into the tasks of block column i, so a tile of block i+1 starts accumulating
// as soon as the tiles of block i it needs are final: there is no barrier
// between the steps of the sweep.  The triangular solves of Algorithm 1 are
// products with the inverse W of the 64 x 64 diagonal factor tile, so all the
// arithmetic outside the diagonal tiles runs on FP64 MFMA.
//
// The diagonal tiles form the critical path (each needs the one before it).
// The tile just left of a diagonal tile in the band, L(g, g-1) (L_ii(c,c-1),
// or L_{i,i-1}(0,T-1) at c = 0), is the last input of the diagonal tile, so
// the two are produced together: one k loop accumulates both (they share
// their left operands) up to k = g-2, then L(g, g-1) = (...) W(g-1)^T is
// formed and its product added, and the diagonal tile is factored, all by
// one DIAG task.
//
// Workgroups take task tickets from an atomic counter in a fixed topological
// order (column by column across the whole band), so a task only ever waits
// for tasks with smaller tickets, which are owned by running workgroups: the
// schedule cannot deadlock whatever the number of resident workgroups.  Every
// wait is bounded; a stuck wait raises an abort flag that releases all waits.
#include <algorithm>
#include <vector>

#include "bta_device.hpp"
#include "bta_internal.hpp"
#include "bta_testing.h"

namespace bta {

enum : int { T_DIAG = 0, T_OFFD = 1, T_SUB = 2, T_ARW = 3, T_TUPD = 4, T_TIPD = 5, T_TIPO = 6 };

// Control words of a launch (ints at p.ctl): the ticket counter at 0, the
// abort flag raised by a wait that timed out on a line of its own (128 bytes
// further), which every polling workgroup reads.
constexpr int CTL_ABORT = 32;

struct FactorParams {
  int n, b, a;
  int T;   // tiles per block edge: ceil(b/64)
  int TA;  // tiles per tip edge: ceil(a/64)
  const double* D; const double* B; const double* R; const double* Tt;
  double* LD; double* LB; double* LR; double* LT;
  double* Wd;      // [n][T] 64x64 inverses of the diagonal factor tiles
  double* Wt;      // [TA] inverses of the tip diagonal factor tiles
  double* P;       // [n][TA][TA] 64x64 per-step tip updates
  int* flags;      // completion flags
  int* ctl;        // [0..1] 64-bit ticket counter, [2] abort flag
  int64_t* info;   // caller's info
  long long ntasks;
  long long step_full, step_last;  // tasks per step (with / without SUB)
  int look;                        // DIAG lookahead: DIAG(i,c) is dispatched with column c - look of its step
  int sub_delay;                   // SUB(i,r,c) is dispatched with column c + sub_delay of its step (after
                                   // the last column for c + sub_delay >= T)
  int cached;                      // 1: k-loop operand tiles are read through the L2 (line-aligned tiles only)
  int fast;                        // 1: every k-loop operand tile takes the direct 16-byte path, device
                                   // coherent (b and a even, L arrays 16-byte aligned, cached == 0)
  long long spin_limit;
  unsigned long long* trace;  // optional: 8 words per ticket (start, k loop done, end, type | workgroup << 8,
                              // W ready (DIAG: of g-1), L(g,g-1) published (DIAG), tile factored (DIAG),
                              // end of the last blocking wait in the k loop)
};

struct Task {
  int type, i, r, c;
};

__host__ __device__ inline int64_t fl_D(const FactorParams& p, int i, int r, int c) {
  return (int64_t)i * (2LL * p.T * p.T + (int64_t)p.TA * p.T + (int64_t)p.TA * p.TA) + (int64_t)r * p.T + c;
}
__host__ __device__ inline int64_t fl_B(const FactorParams& p, int i, int r, int c) {
  return fl_D(p, i, 0, 0) + (int64_t)p.T * p.T + (int64_t)r * p.T + c;
}
__host__ __device__ inline int64_t fl_R(const FactorParams& p, int i, int r, int c) {
  return fl_D(p, i, 0, 0) + 2LL * p.T * p.T + (int64_t)r * p.T + c;
}
__host__ __device__ inline int64_t fl_U(const FactorParams& p, int i, int r, int c) {
  return fl_D(p, i, 0, 0) + 2LL * p.T * p.T + (int64_t)p.TA * p.T + (int64_t)r * p.TA + c;
}
__host__ __device__ inline int64_t fl_tip(const FactorParams& p, int r, int c) {
  return fl_D(p, p.n, 0, 0) + (int64_t)r * p.TA + c;
}

__host__ __device__ __forceinline__ Task decode(const FactorParams& p, long long t) {
  Task k{-1, 0, 0, 0};
  const int T = p.T, TA = p.TA;
  long long rem;
  bool has_sub;
  const long long full_total = (long long)(p.n - 1) * p.step_full;
  if (t < full_total) {
    k.i = (int)(t / p.step_full);
    rem = t - (long long)k.i * p.step_full;
    has_sub = true;
  } else if (t - full_total < p.step_last) {
    k.i = p.n - 1;
    rem = t - full_total;
    has_sub = false;
  } else {
    rem = t - full_total - p.step_last;
    for (int c = 0; c < TA; ++c) {
      const int g = TA - c;
      if (rem < g) {
        k.type = rem == 0 ? T_TIPD : T_TIPO;
        k.r = c + (int)rem;
        k.c = c;
        return k;
      }
      rem -= g;
    }
    return k;
  }
  // column c: DIAG tasks (DIAG(0 .. L) at c = 0, DIAG(c + L) after, L = look:
  // a diagonal task starts its long k loop L columns ahead of the chain), OFFD
  // rows c+2 .. T-1 (row c+1 is fused into the next DIAG), the SUB tasks of
  // column c - S (S = sub_delay; rows 0 .. T-1, not row 0 of the last column:
  // fused into the next step's first DIAG), ARW rows 0 .. TA-1; then the SUB
  // tasks of the last S columns.  Every task still waits only on smaller
  // tickets (a SUB tile's sources are SUB tiles of earlier columns and D-block
  // tiles), apart from the DIAG lookahead.
  const int L = p.look, S = has_sub ? p.sub_delay : 0;
  for (int c = 0; c < T + S; ++c) {
    const bool col = c < T;
    const int cs = c - S;
    const int ndg = !col ? 0 : (c == 0) ? L + 1 : ((c + L <= T - 1) ? 1 : 0);
    const int no = (col && c <= T - 2) ? T - c - 2 : 0;
    const int ns = (has_sub && cs >= 0) ? (cs == T - 1 ? T - 1 : T) : 0;
    const int na = col ? TA : 0;
    const int g = ndg + no + ns + na;
    if (rem < g) {
      if (rem < ndg) {
        k.type = T_DIAG;
        k.c = (c == 0) ? (int)rem : c + L;
        k.r = k.c;
      } else if (rem - ndg < no) {
        k.type = T_OFFD;
        k.c = c;
        k.r = c + 2 + (int)(rem - ndg);
      } else if (rem - ndg - no < ns) {
        k.type = T_SUB;
        k.c = cs;
        k.r = (int)(rem - ndg - no) + (cs == T - 1 ? 1 : 0);
      } else {
        k.type = T_ARW;
        k.c = c;
        k.r = (int)(rem - ndg - no - ns);
      }
      return k;
    }
    rem -= g;
  }
  // tip updates of this step (lower tiles, column by column)
  for (int c = 0; c < TA; ++c) {
    const int g = TA - c;
    if (rem < g) {
      k.type = T_TUPD;
      k.r = c + (int)rem;
      k.c = c;
      return k;
    }
    rem -= g;
  }
  return k;
}

// Tile views of the block arrays.
__host__ __device__ inline int ext(int total, int t) { int e = total - 64 * t; return e < 64 ? e : 64; }

struct alignas(256) Shared {
  // the small arrays first: their LDS addresses fit the 16-bit offset of the
  // LDS instructions, so the panel loop of the diagonal tiles reads them
  // without address arithmetic
  double pan[64 * 17];  // diagonal tile factorization workspace
  double rinv[64];
  long long ticket;
  int fail;
  int ok;    // result of wait_ready
  int upto;  // end of the run of final k tiles (k loop)
  union alignas(256) {
    double stage[2][2][PT];  // k loop: pieced operand tiles, double buffered (direct loads)
    struct {
      double As[TS * LDS_LD];
      double Bs[TS * LDS_LD];
    } f;  // finishing a tile: row-major padded tiles
  } u;
};

// One k step of a left-looking task: operand tiles and their completion flags.
struct KSrc {
  OpTile a, b;
  const int* fa;
  const int* fb;
};

// Enumerate the k sources of a task.  Returns the number of k tiles and fills
// src for index kk when kk >= 0.
__host__ __device__ __forceinline__ int ksources(const FactorParams& p, const Task& t, int kk, KSrc* src) {
  const int T = p.T, b = p.b, a = p.a;
  const int64_t bb = (int64_t)b * b, ab = (int64_t)a * b;
  const int nprev = (t.i > 0) ? T : 0;  // previous block column (cross-step update)
  switch (t.type) {
    case T_DIAG:
    case T_OFFD: {
      const int cnt = nprev + t.c;
      if (kk < 0) return cnt;
      if (kk < nprev) {
        const double* Lb = p.LB + (int64_t)(t.i - 1) * bb;
        src->a = OpTile{Lb + (int64_t)t.r * 64 * b + kk * 64, b, ext(b, t.r), ext(b, kk), false};
        src->b = OpTile{Lb + (int64_t)t.c * 64 * b + kk * 64, b, ext(b, t.c), ext(b, kk), false};
        src->fa = p.flags + fl_B(p, t.i - 1, t.r, kk);
        src->fb = p.flags + fl_B(p, t.i - 1, t.c, kk);
      } else {
        const int k = kk - nprev;
        const double* Ld = p.LD + (int64_t)t.i * bb;
        src->a = OpTile{Ld + (int64_t)t.r * 64 * b + k * 64, b, ext(b, t.r), ext(b, k), false};
        src->b = OpTile{Ld + (int64_t)t.c * 64 * b + k * 64, b, ext(b, t.c), ext(b, k), false};
        src->fa = p.flags + fl_D(p, t.i, t.r, k);
        src->fb = p.flags + fl_D(p, t.i, t.c, k);
      }
      return cnt;
    }
    case T_SUB: {
      const int cnt = t.c;
      if (kk < 0) return cnt;
      const double* Lb = p.LB + (int64_t)t.i * bb;
      const double* Ld = p.LD + (int64_t)t.i * bb;
      src->a = OpTile{Lb + (int64_t)t.r * 64 * b + kk * 64, b, ext(b, t.r), ext(b, kk), false};
      src->b = OpTile{Ld + (int64_t)t.c * 64 * b + kk * 64, b, ext(b, t.c), ext(b, kk), false};
      src->fa = p.flags + fl_B(p, t.i, t.r, kk);
      src->fb = p.flags + fl_D(p, t.i, t.c, kk);
      return cnt;
    }
    case T_ARW: {
      const int cnt = nprev + t.c;
      if (kk < 0) return cnt;
      if (kk < nprev) {
        const double* Lr = p.LR + (int64_t)(t.i - 1) * ab;
        const double* Lb = p.LB + (int64_t)(t.i - 1) * bb;
        src->a = OpTile{Lr + (int64_t)t.r * 64 * b + kk * 64, b, ext(a, t.r), ext(b, kk), false};
        src->b = OpTile{Lb + (int64_t)t.c * 64 * b + kk * 64, b, ext(b, t.c), ext(b, kk), false};
        src->fa = p.flags + fl_R(p, t.i - 1, t.r, kk);
        src->fb = p.flags + fl_B(p, t.i - 1, t.c, kk);
      } else {
        const int k = kk - nprev;
        const double* Lr = p.LR + (int64_t)t.i * ab;
        const double* Ld = p.LD + (int64_t)t.i * bb;
        src->a = OpTile{Lr + (int64_t)t.r * 64 * b + k * 64, b, ext(a, t.r), ext(b, k), false};
        src->b = OpTile{Ld + (int64_t)t.c * 64 * b + k * 64, b, ext(b, t.c), ext(b, k), false};
        src->fa = p.flags + fl_R(p, t.i, t.r, k);
        src->fb = p.flags + fl_D(p, t.i, t.c, k);
      }
      return cnt;
    }
    case T_TUPD: {
      const int cnt = T;
      if (kk < 0) return cnt;
      const double* Lr = p.LR + (int64_t)t.i * ab;
      src->a = OpTile{Lr + (int64_t)t.r * 64 * b + kk * 64, b, ext(a, t.r), ext(b, kk), false};
      src->b = OpTile{Lr + (int64_t)t.c * 64 * b + kk * 64, b, ext(a, t.c), ext(b, kk), false};
      src->fa = p.flags + fl_R(p, t.i, t.r, kk);
      src->fb = p.flags + fl_R(p, t.i, t.c, kk);
      return cnt;
    }
    case T_TIPD:
    case T_TIPO: {
      const int cnt = t.c;
      if (kk < 0) return cnt;
      src->a = OpTile{p.LT + (int64_t)t.r * 64 * a + kk * 64, a, ext(a, t.r), ext(a, kk), false};
      src->b = OpTile{p.LT + (int64_t)t.c * 64 * a + kk * 64, a, ext(a, t.c), ext(a, kk), false};
      src->fa = p.flags + fl_tip(p, t.r, kk);
      src->fb = p.flags + fl_tip(p, t.c, kk);
      return cnt;
    }
  }
  return 0;
}

__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ long long uni64(long long v) {
  const int lo = __builtin_amdgcn_readfirstlane((int)(unsigned)(v & 0xffffffffLL));
  const int hi = __builtin_amdgcn_readfirstlane((int)(v >> 32));
  return (long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

// One k-loop operand tile into LDS: the direct path without its test when the
// launch's tiles all take it (F), else the general loader.
template <bool F>
__device__ __forceinline__ void load_k(const FactorParams& p, double* dst, const OpTile& t, int tid) {
  if constexpr (F) tile_load_lds_fast(dst, t, tid);
  else tile_load_lds_dev(dst, t, tid, p.cached != 0);
}

// Block until flags are set (thread 0 polls); returns false on abort.
__device__ __forceinline__ bool wait_ready(const FactorParams& p, const int* f1, const int* f2, Shared& sh, int tid) {
  if (tid == 0) {
    bool ok = spin_wait(f1, p.ctl + CTL_ABORT, p.spin_limit);
    if (ok && f2 != f1) ok = spin_wait(f2, p.ctl + CTL_ABORT, p.spin_limit);
    acquire_fence();
    sh.ok = ok ? 1 : 0;
  }
  __syncthreads();
  return uni(sh.ok) != 0;
}

// Wave 0: extend the run of consecutive final k tiles starting at `from`
// without blocking.  Lane l polls the flags of k tile from + l, so one round
// trip covers up to 64 tiles; one acquire fence covers every tile added.
__device__ __forceinline__ int extend_ready(const FactorParams& p, const Task& t, int from, int nk, int lane) {
  const int kk = from + lane;
  bool ready = false;
  if (kk < nk) {
    KSrc s2;
    ksources(p, t, kk, &s2);
    ready = flag_set(s2.fa) && flag_set(s2.fb);
  }
  const unsigned long long m = __builtin_amdgcn_ballot_w64(ready);
  const int run = (~m == 0ULL) ? 64 : __builtin_ctzll(~m);
  const int upto = from + run;
  if (upto > from) acquire_fence();
  return upto;
}

// Publish a finished tile: every wave's stores are complete in L2 before the
// barrier; one agent-scope release then writes the XCD's L2 back and sets the flag.
__device__ __forceinline__ void publish(int* flag, int tid) {
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (tid == 0) __hip_atomic_store(flag, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// Diagonal tile g = (block i, tile column c) and the tile left of it, L(g, g-1).
// One k loop over the k < g-1 shared by both accumulates
//   acc1 = -(A(g,g) - sum_k L(g,k) L(g,k)^T),  acc2 = -(A(g,g-1) - sum_k L(g,k) L(g-1,k)^T)
// (a padded diagonal tile gets -1 on the padded diagonal).
template <bool F>
__device__ __forceinline__ void diag_partials(const FactorParams& p, const Task& t, Shared& sh, int tid, Acc& acc1,
                                              Acc& acc2, unsigned long long* rec) {
  const int T = p.T, b = p.b;
  const int64_t bb = (int64_t)b * b;
  const int rows = ext(b, t.c);
  const double* in = p.D + t.i * bb + (int64_t)t.c * 64 * b + t.c * 64;

  // the tile left of the diagonal tile, described by the task that would produce it alone
  const bool has_pre = t.c > 0 || t.i > 0;
  Task pt{T_OFFD, t.i, t.c, t.c - 1};
  const double* pin = nullptr;
  int prows = 0, pcols = 0;
  if (t.c > 0) {
    pin = p.D + t.i * bb + (int64_t)t.c * 64 * b + (t.c - 1) * 64;
    prows = rows;
    pcols = ext(b, t.c - 1);
  } else if (t.i > 0) {
    pt = Task{T_SUB, t.i - 1, 0, T - 1};
    pin = p.B + (t.i - 1) * bb + (T - 1) * 64;
    prows = ext(b, 0);
    pcols = ext(b, T - 1);
  }

  acc_load(acc1, in, b, rows, rows, -1.0, tid);
  if (rows < 64) {
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
      for (int bj = 0; bj < 2; ++bj)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int rr = tile_row(tid, bi, j), cc = tile_col(tid, bj);
          if (rr == cc && rr >= rows) acc1.v[bi][bj][j] = -1.0;
        }
  }
  if (has_pre) acc_load(acc2, pin, b, prows, pcols, -1.0, tid);
  else acc_zero(acc2);

  // shared k loop (software pipelined like run_task's)
  const int nk = has_pre ? uni(ksources(p, pt, -1, nullptr)) : 0;
  bool aborted = false;
  if (nk > 0) {
      int upto = 0;
      KSrc s0;
      ksources(p, pt, 0, &s0);
      if (!wait_ready(p, s0.fa, s0.fb, sh, tid)) aborted = true;
      upto = 1;
      load_k<F>(p, sh.u.stage[0][0], s0.a, tid);
      load_k<F>(p, sh.u.stage[0][1], s0.b, tid);
      for (int kk = 0; kk < nk && !aborted; ++kk) {
        if (tid < 64) {
          const int u = (kk + 1 < nk && kk + 1 >= upto) ? extend_ready(p, pt, kk + 1, nk, tid) : upto;
          if (tid == 0) sh.upto = u;
        }
        __builtin_amdgcn_s_waitcnt(0);  // this wave's loads of k tile kk have landed
        __syncthreads();                // everyone's; and stage (kk+1)&1 is no longer read
        const int u = uni(sh.upto);
        upto = u > upto ? u : upto;
        if (kk + 1 < nk) {
          KSrc sn;
          ksources(p, pt, kk + 1, &sn);
          if (kk + 1 >= upto) {
            if (!wait_ready(p, sn.fa, sn.fb, sh, tid)) aborted = true;
            if (rec && tid == 0) rec[7] = __builtin_amdgcn_s_memrealtime();
            upto = kk + 2;
          }
          load_k<F>(p, sh.u.stage[(kk + 1) & 1][0], sn.a, tid);
          load_k<F>(p, sh.u.stage[(kk + 1) & 1][1], sn.b, tid);
        }
        mma_ptile2(acc1, acc2, sh.u.stage[kk & 1][0], sh.u.stage[kk & 1][1], tid);
      }
  }
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
}

// Four consecutive k of LDS row `row`, from k group kg (the k permutation of mma_tile).
__device__ __forceinline__ d4 lds_k4(const double* S, int row, int kg, int kl) {
  const double* q = S + row * LDS_LD + kg * 16 + kl;
  const d2v lo = *reinterpret_cast<const d2v*>(q);
  const d2v hi = *reinterpret_cast<const d2v*>(q + 2);
  return d4{lo[0], lo[1], hi[0], hi[1]};
}

// x = As Bs^T with Bs lower triangular (the inverse W of a diagonal tile), so
// that 16-column block J of x only takes the k groups K <= J.  Wave w holds
// rows 32*(w&1) .. +32 and the column blocks {J0, J1} = {0, 3} or {1, 2}:
// ten of the sixteen k groups per wave instead of sixteen.
template <int J0, int J1>
__device__ __forceinline__ void mma_lower_rhs(d4 (&x)[2][2], const double* As, const double* Bs, int rb, int lane) {
  const int m = lane & 15, kl = (lane >> 4) * 4;
#pragma unroll
  for (int i = 0; i < 2; ++i) x[i][0] = x[i][1] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int kg = 0; kg <= J1; ++kg) {
    d4 a[2], b0 = d4{0.0, 0.0, 0.0, 0.0}, b1;
#pragma unroll
    for (int i = 0; i < 2; ++i) a[i] = lds_k4(As, 16 * (rb + i) + m, kg, kl);
    if (kg <= J0) b0 = lds_k4(Bs, 16 * J0 + m, kg, kl);
    b1 = lds_k4(Bs, 16 * J1 + m, kg, kl);
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        if (kg <= J0) x[i][0] = mfma16(a[i][q], b0[q], x[i][0]);
        x[i][1] = mfma16(a[i][q], b1[q], x[i][1]);
      }
  }
}

// S(I,J) -= X(I,:) X(J,:)^T for one 16-block of the lower triangle (the part
// the Cholesky reads).
template <int I, int J>
__device__ __forceinline__ void syrk_block(double* S, const double* X, int lane) {
  const int m = lane & 15, kl = (lane >> 4) * 4;
  d4 t = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int kg = 0; kg < 4; ++kg) {
    const d4 a = lds_k4(X, 16 * I + m, kg, kl);
    const d4 b = lds_k4(X, 16 * J + m, kg, kl);
#pragma unroll
    for (int q = 0; q < 4; ++q) t = mfma16(a[q], b[q], t);
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) S[(16 * I + acc_row(lane, j)) * LDS_LD + 16 * J + acc_col(lane)] -= t[j];
}

// The ten lower 16-blocks over the four waves: three, three, two and two.
__device__ __forceinline__ void syrk_lower(double* S, const double* X, int tid) {
  const int lane = tid & 63;
  switch (tid >> 6) {
    case 0: syrk_block<0, 0>(S, X, lane); syrk_block<1, 0>(S, X, lane); syrk_block<3, 3>(S, X, lane); break;
    case 1: syrk_block<1, 1>(S, X, lane); syrk_block<2, 0>(S, X, lane); syrk_block<3, 2>(S, X, lane); break;
    case 2: syrk_block<2, 1>(S, X, lane); syrk_block<2, 2>(S, X, lane); break;
    default: syrk_block<3, 0>(S, X, lane); syrk_block<3, 1>(S, X, lane); break;
  }
}

// The rest of diagonal tile g = (i, c) from its partial sums: L(g,g-1) =
// -acc2 W(g-1)^T is stored and published, acc1 += L(g,g-1) L(g,g-1)^T, and the
// diagonal tile is factored and inverted (L and W stored, flag published).
// W(g-1) is loaded once its flag is set.
// rec (optional): [0] W(g-1) ready, [1] L(g,g-1) published, [2] tile factored.
__device__ __forceinline__ void diag_finish(const FactorParams& p, int i, int c, Shared& sh, int tid, Acc& acc1,
                                            Acc& acc2, unsigned long long* rec) {
  const int T = p.T, b = p.b;
  const int64_t bb = (int64_t)b * b;
  const int rows = ext(b, c);
  double* out = p.LD + i * bb + (int64_t)c * 64 * b + c * 64;
  const bool has_pre = c > 0 || i > 0;
  double* pout = nullptr;
  int prows = 0, pcols = 0;
  int* pflag = nullptr;
  const double* Wp = nullptr;
  const int* fWp = nullptr;
  if (c > 0) {
    pout = p.LD + i * bb + (int64_t)c * 64 * b + (c - 1) * 64;
    prows = rows;
    pcols = ext(b, c - 1);
    pflag = p.flags + fl_D(p, i, c, c - 1);
    Wp = p.Wd + ((int64_t)i * T + c - 1) * 4096;
    fWp = p.flags + fl_D(p, i, c - 1, c - 1);
  } else if (i > 0) {
    pout = p.LB + (i - 1) * bb + (T - 1) * 64;
    prows = ext(b, 0);
    pcols = ext(b, T - 1);
    pflag = p.flags + fl_B(p, i - 1, 0, T - 1);
    Wp = p.Wd + ((int64_t)(i - 1) * T + T - 1) * 4096;
    fWp = p.flags + fl_D(p, i - 1, T - 1, T - 1);
  }
  // the rest of this tile is the critical path of the factorization: let its
  // waves win the issue arbitration against another workgroup on this CU
  __builtin_amdgcn_s_setprio(3);

  if (has_pre) {
    wait_ready(p, fWp, fWp, sh, tid);
    if (rec && tid == 0) rec[0] = __builtin_amdgcn_s_memrealtime();
    Stage rw;
    stage_load_dev(rw, OpTile{Wp, 64, 64, 64, false}, tid);
    acc_to_lds(acc2, sh.u.f.As, tid);
    stage_store(rw, sh.u.f.Bs, tid);
    __syncthreads();
    // x = -L(g,g-1) = acc2 W(g-1)^T, W lower triangular
    const int w = tid >> 6, lane = tid & 63, rb = 2 * (w & 1);
    d4 x[2][2];
    if (w < 2) mma_lower_rhs<0, 3>(x, sh.u.f.As, sh.u.f.Bs, rb, lane);
    else mma_lower_rhs<1, 2>(x, sh.u.f.As, sh.u.f.Bs, rb, lane);
    const int jb0 = w < 2 ? 0 : 1, jb1 = w < 2 ? 3 : 2;
#pragma unroll
    for (int ii = 0; ii < 2; ++ii)
#pragma unroll
      for (int jj = 0; jj < 2; ++jj)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int r = 16 * (rb + ii) + acc_row(lane, j), q = 16 * (jj ? jb1 : jb0) + acc_col(lane);
          if (r < prows && q < pcols) st_dev(pout + (int64_t)r * b + q, -x[ii][jj][j]);
        }
    __syncthreads();  // As and Bs are read
#pragma unroll
    for (int ii = 0; ii < 2; ++ii)
#pragma unroll
      for (int jj = 0; jj < 2; ++jj)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          sh.u.f.Bs[(16 * (rb + ii) + acc_row(lane, j)) * LDS_LD + 16 * (jj ? jb1 : jb0) + acc_col(lane)] = x[ii][jj][j];
  }

  // A(g,g) - sum over k < g-1 (acc1 holds its negative) into As
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int j = 0; j < 4; ++j) sh.u.f.As[tile_row(tid, bi, j) * LDS_LD + tile_col(tid, bj)] = -acc1.v[bi][bj][j];
  __syncthreads();
  if (has_pre) {
    // minus L(g,g-1) L(g,g-1)^T = x x^T on the lower triangle, then publish L(g,g-1)
    // (its barrier also orders these LDS updates before the factorization)
    syrk_lower(sh.u.f.As, sh.u.f.Bs, tid);
    __syncthreads();  // the updates are in LDS before the factorization reads them
    if (rec && tid == 0) rec[1] = __builtin_amdgcn_s_memrealtime();
  }

  // factor and invert A(g,g) - sum over all k < g; L(g,g-1)'s flag is published
  // after the first panel (its stores had that long to complete), and W goes
  // to global memory as its rows become final
  double* Wout = p.Wd + ((int64_t)i * T + c) * 4096;
  const int f = uni(chol_inv_tile_mfma_pub(sh.u.f.As, sh.u.f.Bs, sh.rinv, sh.pan, &sh.fail, tid, has_pre ? pflag : nullptr,
                                           Wout));
  if (rec && tid == 0) rec[2] = __builtin_amdgcn_s_memrealtime();
  if (f != 0 && f <= rows && tid == 0) {
    const long long row0 = (long long)i * b + (long long)c * 64;
    atomicMin((unsigned long long*)p.info, (unsigned long long)(row0 + f));
  }
  // the flag covers W only: no task reads a diagonal tile of L (every solve
  // uses W), so L(g,g) is stored after the publication, off the chain
  publish(p.flags + fl_D(p, i, c, c), tid);
  tile_store_lower_dev(sh.u.f.As, out, b, rows, tid);
  __builtin_amdgcn_s_setprio(0);
  // exact zeros in the mirrored upper tile of the diagonal block (no task reads them)
  if (c > 0) {
    double* up = p.LD + i * bb + (int64_t)(c - 1) * 64 * b + c * 64;
    for (int e = tid; e < 64 * 64; e += NT) {
      const int rr = e >> 6, cc = e & 63;
      if (rr < pcols && cc < prows) up[(int64_t)rr * b + cc] = 0.0;
    }
  }
}

template <bool F>
__device__ __forceinline__ void run_diag(const FactorParams& p, const Task& t, Shared& sh, int tid,
                                         unsigned long long& tr1, unsigned long long* rec) {
  Acc acc1, acc2;
  diag_partials<F>(p, t, sh, tid, acc1, acc2, rec);
  if (rec && tid == 0) tr1 = __builtin_amdgcn_s_memrealtime();
  diag_finish(p, t.i, t.c, sh, tid, acc1, acc2, rec ? rec + 4 : nullptr);
}

// One task of one matrix: accumulate, finish, publish.
template <bool F>
__device__ __forceinline__ void run_task(const FactorParams& p, long long tk, Shared& sh, int tid) {
  {
    Task t = decode(p, tk);
    t.type = uni(t.type); t.i = uni(t.i); t.r = uni(t.r); t.c = uni(t.c);
    unsigned long long tr0 = 0, tr1 = 0;
    if (p.trace && tid == 0) tr0 = __builtin_amdgcn_s_memrealtime();
    if (t.type == T_DIAG) {
      unsigned long long* rec = p.trace ? p.trace + 8 * tk : nullptr;
      run_diag<F>(p, t, sh, tid, tr1, rec);
      if (rec && tid == 0) {
        rec[0] = tr0;
        rec[1] = tr1;
        rec[2] = __builtin_amdgcn_s_memrealtime();
        rec[3] = (unsigned long long)t.type | ((unsigned long long)(blockIdx.x & 0xffff) << 8) |
               ((unsigned long long)(t.r & 0xffff) << 24) | ((unsigned long long)(t.c & 0xfff) << 40) |
               ((unsigned long long)(t.i & 0xfff) << 52);
      }
      return;
    }
    const int T = p.T, b = p.b, a = p.a;
    const int64_t bb = (int64_t)b * b, ab = (int64_t)a * b;

    // ---- output tile and its input
    const double* in;
    double* out;
    int64_t ld;
    int rows, cols;
    int* my_flag;
    switch (t.type) {
      case T_DIAG:
      case T_OFFD:
        in = p.D + t.i * bb + (int64_t)t.r * 64 * b + t.c * 64;
        out = p.LD + t.i * bb + (int64_t)t.r * 64 * b + t.c * 64;
        ld = b; rows = ext(b, t.r); cols = ext(b, t.c);
        my_flag = p.flags + fl_D(p, t.i, t.r, t.c);
        break;
      case T_SUB:
        in = p.B + t.i * bb + (int64_t)t.r * 64 * b + t.c * 64;
        out = p.LB + t.i * bb + (int64_t)t.r * 64 * b + t.c * 64;
        ld = b; rows = ext(b, t.r); cols = ext(b, t.c);
        my_flag = p.flags + fl_B(p, t.i, t.r, t.c);
        break;
      case T_ARW:
        in = p.R + t.i * ab + (int64_t)t.r * 64 * b + t.c * 64;
        out = p.LR + t.i * ab + (int64_t)t.r * 64 * b + t.c * 64;
        ld = b; rows = ext(a, t.r); cols = ext(b, t.c);
        my_flag = p.flags + fl_R(p, t.i, t.r, t.c);
        break;
      case T_TUPD:
        in = nullptr;
        out = p.P + ((int64_t)t.i * p.TA * p.TA + (int64_t)t.r * p.TA + t.c) * 4096;
        ld = 64; rows = 64; cols = 64;
        my_flag = p.flags + fl_U(p, t.i, t.r, t.c);
        break;
      default:  // tip
        in = p.Tt + (int64_t)t.r * 64 * a + t.c * 64;
        out = p.LT + (int64_t)t.r * 64 * a + t.c * 64;
        ld = a; rows = ext(a, t.r); cols = ext(a, t.c);
        my_flag = p.flags + fl_tip(p, t.r, t.c);
        break;
    }
    const bool is_diag = (t.type == T_TIPD);  // DIAG tasks run in run_diag

    // ---- accumulator = -(input tile); a padded diagonal tile gets -1 on the padded diagonal
    Acc acc;
    if (in) {
      acc_load(acc, in, ld, rows, cols, -1.0, tid);
      if (is_diag && rows < 64) {
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
          for (int bj = 0; bj < 2; ++bj)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
              const int rr = tile_row(tid, bi, j), cc = tile_col(tid, bj);
              if (rr == cc && rr >= rows) acc.v[bi][bj][j] = -1.0;
            }
      }
    } else {
      acc_zero(acc);
    }

    // tip tiles: subtract the per-step updates in step order
    if (t.type == T_TIPD || t.type == T_TIPO) {
      for (int i = 0; i < p.n; ++i) {
        if (!wait_ready(p, p.flags + fl_U(p, i, t.r, t.c), p.flags + fl_U(p, i, t.r, t.c), sh, tid)) break;
        const double* Pi = p.P + ((int64_t)i * p.TA * p.TA + (int64_t)t.r * p.TA + t.c) * 4096;
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
          for (int bj = 0; bj < 2; ++bj)
#pragma unroll
            for (int j = 0; j < 4; ++j)
              acc.v[bi][bj][j] += ld_dev(Pi + tile_row(tid, bi, j) * 64 + tile_col(tid, bj));
      }
    }

    // ---- left-looking accumulation, software pipelined: the next k tiles are
    // moved into the other LDS stage while the MFMAs of the current ones run.
    const int nk = uni(ksources(p, t, -1, nullptr));
    bool aborted = false;
    if (nk > 0) {
        int upto = 0;
        KSrc s0;
        ksources(p, t, 0, &s0);
        if (!wait_ready(p, s0.fa, s0.fb, sh, tid)) aborted = true;
        upto = 1;
        load_k<F>(p, sh.u.stage[0][0], s0.a, tid);
        load_k<F>(p, sh.u.stage[0][1], s0.b, tid);
        for (int kk = 0; kk < nk && !aborted; ++kk) {
          if (tid < 64) {
            const int u = (kk + 1 < nk && kk + 1 >= upto) ? extend_ready(p, t, kk + 1, nk, tid) : upto;
            if (tid == 0) sh.upto = u;
          }
          __builtin_amdgcn_s_waitcnt(0);  // this wave's loads of k tile kk have landed
          __syncthreads();                // everyone's; and stage (kk+1)&1 is no longer read
          const int u = uni(sh.upto);
          upto = u > upto ? u : upto;
          if (kk + 1 < nk) {
            KSrc sn;
            ksources(p, t, kk + 1, &sn);
            if (kk + 1 >= upto) {  // not final yet: block (rare once the pipeline is primed)
              if (!wait_ready(p, sn.fa, sn.fb, sh, tid)) { aborted = true; }
              if (p.trace && tid == 0) p.trace[8 * tk + 7] = __builtin_amdgcn_s_memrealtime();
              upto = kk + 2;
            }
            load_k<F>(p, sh.u.stage[(kk + 1) & 1][0], sn.a, tid);
            load_k<F>(p, sh.u.stage[(kk + 1) & 1][1], sn.b, tid);
          }
          mma_ptile(acc, sh.u.stage[kk & 1][0], sh.u.stage[kk & 1][1], tid);
        }
    }
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (p.trace && tid == 0) tr1 = __builtin_amdgcn_s_memrealtime();

    // ---- finish the tile
    if (t.type == T_TUPD) {
      acc_store_dev(acc, out, 64, 64, 64, 1.0, tid);
    } else if (is_diag) {
      // LDS: As <- A - sum (the accumulator holds its negative); factor + invert in place
#pragma unroll
      for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
          for (int j = 0; j < 4; ++j) sh.u.f.As[tile_row(tid, bi, j) * LDS_LD + tile_col(tid, bj)] = -acc.v[bi][bj][j];
      __syncthreads();
      const int f = uni(chol_inv_tile_mfma(sh.u.f.As, sh.u.f.Bs, sh.rinv, sh.pan, &sh.fail, tid));
      if (f != 0 && f <= rows && tid == 0) {
        const long long row0 = (long long)p.n * b + (long long)t.c * 64;
        atomicMin((unsigned long long*)p.info, (unsigned long long)(row0 + f));
      }
      double* Wout = p.Wt + (int64_t)t.c * 4096;
      tile_store_dev(sh.u.f.Bs, Wout, 64, 64, 64, tid);
      tile_store_lower_dev(sh.u.f.As, out, ld, rows, tid);  // (rows == cols: the tile is diagonal)
    } else {
      // X = (A - sum) W(c,c)^T
      const double* Wc = (t.type == T_TIPO) ? p.Wt + (int64_t)t.c * 4096
                                            : p.Wd + ((int64_t)t.i * T + t.c) * 4096;
      const int* fdiag = (t.type == T_TIPO) ? p.flags + fl_tip(p, t.c, t.c) : p.flags + fl_D(p, t.i, t.c, t.c);
      wait_ready(p, fdiag, fdiag, sh, tid);
      if (p.trace && tid == 0) p.trace[8 * tk + 4] = __builtin_amdgcn_s_memrealtime();
      Stage rw;
      stage_load_dev(rw, OpTile{Wc, 64, 64, 64, false}, tid);
      acc_to_lds(acc, sh.u.f.As, tid);
      stage_store(rw, sh.u.f.Bs, tid);
      __syncthreads();
      Acc x;
      acc_zero(x);
      mma_tile(x, sh.u.f.As, sh.u.f.Bs, tid);
      acc_store_dev(x, out, ld, rows, cols, -1.0, tid);
      // exact zeros in the mirrored (upper) tile of a diagonal block / the tip
      if (t.type == T_OFFD || t.type == T_TIPO) {
        double* up = (t.type == T_OFFD) ? p.LD + t.i * bb + (int64_t)t.c * 64 * b + t.r * 64
                                        : p.LT + (int64_t)t.c * 64 * a + t.r * 64;
        const int ur = cols, uc = rows;
        for (int e = tid; e < 64 * 64; e += NT) {
          const int rr = e >> 6, cc = e & 63;
          if (rr < ur && cc < uc) up[(int64_t)rr * ld + cc] = 0.0;
        }
      }
    }
    publish(my_flag, tid);
    if (p.trace && tid == 0) {
      unsigned long long* rec = p.trace + 8 * tk;
      rec[0] = tr0;
      rec[1] = tr1;
      rec[2] = __builtin_amdgcn_s_memrealtime();
      rec[3] = (unsigned long long)t.type | ((unsigned long long)(blockIdx.x & 0xffff) << 8) |
               ((unsigned long long)(t.r & 0xffff) << 24) | ((unsigned long long)(t.c & 0xfff) << 40) |
               ((unsigned long long)(t.i & 0xfff) << 52);
    }
  }
}

// Persistent workers: take tickets until the task list is exhausted.
template <bool F>
__device__ __forceinline__ void factor_worker(const FactorParams& p, Shared& sh) {
  const int tid = threadIdx.x;
  for (;;) {
    if (tid == 0) sh.ticket = (long long)atomicAdd((unsigned long long*)p.ctl, 1ULL);
    __syncthreads();
    const long long tk = uni64(sh.ticket);
    if (tk >= p.ntasks) break;
    run_task<F>(p, tk, sh, tid);
  }
}

// One workgroup per CU (the static LDS is more than half of a CU's): the
// kernel is launched with no extra dynamic LDS (SOLO_LDS_PAD = 0).  The diagonal
// tiles (the critical path) then do not share their SIMDs with the MFMA work
// of another task, and every task has the CU's full register file.
constexpr size_t SOLO_LDS_PAD = 0;
static_assert(sizeof(Shared) > 80 * 1024, "one workgroup per CU relies on the LDS footprint");
// F: every k-loop operand tile of the launch takes the direct load path
// (FactorParams::fast), so the k loops carry no per-tile path test.
template <bool F>
__global__ __launch_bounds__(NT, 1) void factor_kernel(FactorParams p) {
  __shared__ Shared sh;
  factor_worker<F>(p, sh);
}

// ---------------------------------------------------------------------------
// Many independent BTA matrices in one persistent launch.  Tickets run over a
// segment table that interleaves the matrices step by step (segment = the
// tasks of one block step of one matrix, the last step of a matrix carries its
// tip tasks); inside a matrix the order is the single-matrix topological order,
// and matrices do not depend on each other, so the schedule stays deadlock free.
struct BatchSeg {
  long long t0;      // first global ticket of the segment
  long long local0;  // first ticket of the segment inside its matrix
  int mat;
  int pad;
};

struct FactorBatchArgs {
  const FactorParams* mats;
  const BatchSeg* segs;
  int nseg;
  long long ntasks;
  int* ctl;
};

template <bool F>
__global__ __launch_bounds__(NT, 1) void factor_batched_kernel(FactorBatchArgs args) {
  __shared__ Shared sh;
  const int tid = threadIdx.x;
  for (;;) {
    if (tid == 0) sh.ticket = (long long)atomicAdd((unsigned long long*)args.ctl, 1ULL);
    __syncthreads();
    const long long tk = uni64(sh.ticket);
    if (tk >= args.ntasks) break;
    int lo = 0, hi = args.nseg - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (args.segs[mid].t0 <= tk) lo = mid; else hi = mid - 1;
    }
    lo = uni(lo);
    const long long local = uni64(args.segs[lo].local0 + (tk - args.segs[lo].t0));
    const FactorParams p = args.mats[uni(args.segs[lo].mat)];
    run_task<F>(p, local, sh, tid);
  }
}

__global__ void factor_batched_reset_kernel(int* flags, long long nflags, int* ctl, const FactorParams* mats, int count) {
  const long long i0 = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  for (long long i = i0; i < nflags; i += (long long)gridDim.x * blockDim.x) flags[i] = 0;
  if (i0 < 4) ctl[i0] = 0;
  if (i0 == 0) ctl[CTL_ABORT] = 0;
  for (long long m = i0; m < count; m += (long long)gridDim.x * blockDim.x) *mats[m].info = 0x7fffffffffffffffLL;
}

__global__ void factor_batched_finish_kernel(const int* ctl, const FactorParams* mats, int count) {
  for (int m = blockIdx.x * blockDim.x + threadIdx.x; m < count; m += gridDim.x * blockDim.x) {
    int64_t* info = mats[m].info;
    if (ctl[CTL_ABORT] != 0) *info = -1;
    else if (*info == 0x7fffffffffffffffLL) *info = 0;
  }
}

// Clear the flags, the ticket counter and the abort flag, and zero info.
__global__ void factor_reset_kernel(int* flags, long long nflags, int* ctl, int64_t* info) {
  const long long i0 = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  for (long long i = i0; i < nflags; i += (long long)gridDim.x * blockDim.x) flags[i] = 0;
  if (i0 < 4) ctl[i0] = 0;
  if (i0 == 0) ctl[CTL_ABORT] = 0;
  if (i0 == 0) *info = 0x7fffffffffffffffLL;
}

// info: "no failure" is kept as INT64_MAX during the run; map to 0, and an
// aborted run (watchdog) to -1.
__global__ void factor_finish_kernel(const int* ctl, int64_t* info) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    if (ctl[CTL_ABORT] != 0) *info = -1;
    else if (*info == 0x7fffffffffffffffLL) *info = 0;
  }
}

// ---------------------------------------------------------------------------
// DIAG lookahead in columns: internal override for measurements (0 = none).
static int g_factor_look = 0;
// DIAG lookahead of the batched kernel: with many matrices in flight a longer
// lookahead only holds more workgroups on waiting tiles (measured on the 64-matrix
// workload in lockstep order: 23.2, 22.5, 23.2, 23.6 and 23.9 ms for 1, 2, 3, 4
// and 8 columns; in proportional order 19.1, 18.4-18.9, 19.1, 19.5 ms for 1-4).
constexpr int BATCH_LOOKAHEAD = 2;
// SUB delay of the batched kernel (columns): SUB tasks dispatched one column
// after their own no longer hold workgroups waiting on the column's diagonal
// tile (64-matrix workload, proportional order: 18.4-18.9 ms undelayed, 16.8 ms
// with 1, 17.2 ms with 2).
constexpr int BATCH_SUB_DELAY = 1;
// Upper bound on the factor kernel's workgroups (internal, for measurements; 0: one per CU).
static int g_factor_max_grid = 0;
// k-loop operands through the L2 where the tiles are line-aligned: internal
// override for measurements (-1 = none).
static int g_factor_cached = -1;

// The DIAG lookahead for blocks of b with an arrow of a: the internal
// override, else BTA_FACTOR_LOOKAHEAD, else the tuning table, else the default.
static int factor_lookahead(int64_t b, int64_t a) {
  if (g_factor_look > 0) return g_factor_look;
  long long v = 0;
  if (env_int("BTA_FACTOR_LOOKAHEAD", 1, 64, &v)) return (int)v;
  if (tune_get(tune_key("factor", b, a, "look"), &v) && v >= 1 && v <= 64) return (int)v;
  return FACTOR_LOOKAHEAD;
}

// SUB dispatch delay in columns for blocks of b with an arrow of a:
// BTA_FACTOR_SUB_DELAY, else the tuning table ("factor", "sub_delay"), else
// min(8, T/4).  A SUB tile's last source is the SUB tile to its left, which
// is final only once the diagonal chain has passed its column; dispatched with
// its own column, a SUB task holds its workgroup waiting for it.  Measured
// (factor ms for delays 0, 1, 2, 4, 8, 16): n=128, b=2048, a=8: 105.6, 98.6,
// 95.0, 86.6, 84.3, 87.9; n=48, b=4096, a=16: 218.4, 194.9, 189.1, 187.4,
// 187.5, 188.2; no change at b=512 (n=256) and b=1024 (n=512, a=256).
static int factor_sub_delay(int64_t b, int64_t a) {
  long long v = 0;
  if (env_int("BTA_FACTOR_SUB_DELAY", 0, 64, &v)) return (int)v;
  if (tune_get(tune_key("factor", b, a, "sub_delay"), &v) && v >= 0 && v <= 64) return (int)v;
  const int64_t T = (b + 63) / 64;
  return (int)std::min<int64_t>(8, T / 4);
}

// Whether the k loops read through the L2 (same order of sources; default off).
static bool factor_cached_loads(int64_t b, int64_t a) {
  if (g_factor_cached >= 0) return g_factor_cached != 0;
  long long v = 0;
  if (env_int("BTA_FACTOR_CACHED", 0, 1, &v)) return v != 0;
  if (tune_get(tune_key("factor", b, a, "cached"), &v)) return v != 0;
  return false;
}

// Whether every operand tile of a factorization starts its rows on 128-byte
// cache lines: the L arrays 128-byte aligned and their leading dimensions
// (b, and a for the tip) multiples of 16 doubles.
static bool factor_lines_aligned(int64_t b, int64_t a, const double* LD, const double* LB, const double* LR,
                                 const double* LT) {
  auto al = [](const void* q) { return q == nullptr || (reinterpret_cast<uintptr_t>(q) & 127) == 0; };
  return b % 16 == 0 && (a == 0 || a % 16 == 0) && al(LD) && al(LB) && al(LR) && al(LT);
}

// Whether every k-loop operand tile of a factorization takes the direct
// 16-byte load path: even b and a (even leading dimensions and column counts)
// and 16-byte aligned L arrays.
static bool factor_ops_direct(int64_t b, int64_t a, const double* LD, const double* LB, const double* LR,
                              const double* LT) {
  auto al = [](const void* q) { return q == nullptr || (reinterpret_cast<uintptr_t>(q) & 15) == 0; };
  return b % 2 == 0 && a % 2 == 0 && al(LD) && al(LB) && al(LR) && al(LT);
}

FactorPlan factor_plan(int64_t n, int64_t b, int64_t a) {
  FactorPlan fp{};
  const int64_t T = (b + 63) / 64, TA = (a + 63) / 64;
  fp.T = (int)T;
  fp.TA = (int)TA;
  fp.nflags = n * (2 * T * T + TA * T + TA * TA) + TA * TA;  // per step D, B, R and tip-update tiles; tip tiles
  // per step: DIAG + OFFD tasks T(T-1)/2 + 1 (the T-1 tiles L_ii(c+1,c) are
  // computed by DIAG tasks), SUB T*T - 1 (L_{i+1,i}(0,T-1) likewise), ARW, TUPD
  fp.step_full = T * (T - 1) / 2 + 1 + T * T - 1 + T * TA + TA * (TA + 1) / 2;
  fp.step_last = T * (T - 1) / 2 + 1 + T * TA + TA * (TA + 1) / 2;
  fp.ntasks = (n - 1) * fp.step_full + fp.step_last + TA * (TA + 1) / 2;
  fp.look = (int)std::min<int64_t>(factor_lookahead(b, a), T - 1);
  fp.sub_delay = (int)std::min<int64_t>(factor_sub_delay(b, a), T);
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off += (bytes + 255) & ~size_t(255); return o; };
  fp.off_ctl = take(256);  // ticket counter, abort flag at CTL_ABORT
  fp.off_flags = take(sizeof(int) * (size_t)fp.nflags);
  fp.off_Wd = take(sizeof(double) * 4096 * (size_t)(n * T));
  fp.off_Wt = take(sizeof(double) * 4096 * (size_t)(TA > 0 ? TA : 1));
  fp.off_P = take(sizeof(double) * 4096 * (size_t)(n * TA * TA > 0 ? n * TA * TA : 1));
  fp.bytes = off;
  return fp;
}

hipError_t factor_launch(const FactorPlan& fp, int64_t n, int64_t b, int64_t a,
                         const double* D, const double* B, const double* R, const double* T,
                         double* LD, double* LB, double* LR, double* LT,
                         void* work, int64_t* info, hipStream_t stream, int num_cus, unsigned long long* trace) {
  char* w = static_cast<char*>(work);
  FactorParams p;
  p.n = (int)n; p.b = (int)b; p.a = (int)a; p.T = fp.T; p.TA = fp.TA;
  p.D = D; p.B = B; p.R = R; p.Tt = T;
  p.LD = LD; p.LB = LB; p.LR = LR; p.LT = LT;
  p.Wd = reinterpret_cast<double*>(w + fp.off_Wd);
  p.Wt = reinterpret_cast<double*>(w + fp.off_Wt);
  p.P = reinterpret_cast<double*>(w + fp.off_P);
  p.flags = reinterpret_cast<int*>(w + fp.off_flags);
  p.ctl = reinterpret_cast<int*>(w + fp.off_ctl);
  p.info = info;
  p.ntasks = fp.ntasks;
  p.step_full = fp.step_full;
  p.step_last = fp.step_last;
  p.look = fp.look;
  p.sub_delay = fp.sub_delay;
  p.cached = (factor_cached_loads(b, a) && factor_lines_aligned(b, a, LD, LB, LR, LT)) ? 1 : 0;
  p.fast = (!p.cached && factor_ops_direct(b, a, LD, LB, LR, LT)) ? 1 : 0;
  p.trace = trace;
  p.spin_limit = 1LL << 22;  // a few seconds of polling without progress before the watchdog fires
  const int rgrid = (int)std::min<long long>(1024, (fp.nflags + 255) / 256 + 1);
  hipLaunchKernelGGL(factor_reset_kernel, dim3(rgrid), dim3(256), 0, stream, p.flags, fp.nflags, p.ctl, info);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  long long cap = num_cus;
  if (g_factor_max_grid > 0) cap = std::min<long long>(cap, g_factor_max_grid);
  const long long grid = std::min<long long>(fp.ntasks, cap);
  if (grid < fp.ntasks && grid <= fp.look + 1) return hipErrorInvalidConfiguration;  // lookahead needs more workers
  timing_mark(KT_FACTOR, true, stream);
  if (p.fast)
    hipLaunchKernelGGL(factor_kernel<true>, dim3((unsigned)grid), dim3(NT), SOLO_LDS_PAD, stream, p);
  else
    hipLaunchKernelGGL(factor_kernel<false>, dim3((unsigned)grid), dim3(NT), SOLO_LDS_PAD, stream, p);
  timing_mark(KT_FACTOR, false, stream);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(factor_finish_kernel, dim3(1), dim3(64), 0, stream, p.ctl, info);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Band-column interleaving of the matrices of a batch.  Segment (m, i, c)
// holds the tasks of column group c of block step i of matrix m, as decode()
// lays them out (the step's tip updates go with its last group, the final tip
// tasks with the last group of the last step).  A group's position on its
// matrix's chain of diagonal tiles is i*T_m + c (the delayed SUB groups after
// the last column stay at the last column); segments are ordered by that
// position scaled by the longest chain over the matrix's own, so that each
// matrix's columns are dispatched at the pace of its own chain and spread
// over the longest chain's time, rather than in lockstep with wider matrices;
// equal positions go longest chain first.  Per matrix the local ticket order
// is kept.  *total receives the number of tickets.
static std::vector<BatchSeg> batch_segments(const FactorBatchPlan& bp, const int64_t* n, long long* total) {
  struct Col {
    long long key, chain, local0, len;
    int m;
  };
  std::vector<Col> cols;
  cols.reserve((size_t)bp.nseg);
  for (int m = 0; m < bp.count; ++m) {
    const FactorPlan& fp = bp.plans[m];
    const int T = fp.T, TA = fp.TA, L = fp.look;
    long long local = 0;
    for (int64_t i = 0; i < n[m]; ++i) {
      const bool has_sub = i < n[m] - 1;
      const int S = has_sub ? fp.sub_delay : 0;
      for (int c = 0; c < T + S; ++c) {
        // the column group of decode(): DIAG tasks, OFFD, the SUB tasks of
        // column c - S and ARW rows; the last S groups hold SUB tasks only
        const bool col = c < T;
        const int cs = c - S;
        const int ndg = !col ? 0 : (c == 0) ? L + 1 : ((c + L <= T - 1) ? 1 : 0);
        const int no = (col && c <= T - 2) ? T - c - 2 : 0;
        const int ns = (has_sub && cs >= 0) ? (cs == T - 1 ? T - 1 : T) : 0;
        long long len = ndg + no + ns + (col ? TA : 0);
        if (c == T + S - 1) {
          len += (long long)TA * (TA + 1) / 2;               // the step's tip updates
          if (!has_sub) len += (long long)TA * (TA + 1) / 2;  // the tip itself
        }
        // position on the chain; the delayed SUB groups stay at the step's
        // last column so that the key never decreases within a matrix
        const long long key = i * T + std::min(c, T - 1);
        if (len > 0) cols.push_back(Col{key, n[m] * (long long)T, local, len, m});  // no segment for an empty group
        local += len;
      }
    }
  }
  // proportional order (the default): by the fraction of its chain scaled to
  // the longest chain, so that every matrix's columns are spread over the
  // longest chain's time instead of crowding its start; lockstep: by chain
  // position
  long long cmax = 1;
  for (const Col& c : cols) cmax = std::max(cmax, c.chain);
  std::vector<double> pos(cols.size());
  for (size_t q = 0; q < cols.size(); ++q) {
    const Col& c = cols[q];
    pos[q] = bp.order == 1 ? (double)c.key * (double)cmax / (double)c.chain : (double)c.key;
  }
  std::vector<size_t> idx(cols.size());
  for (size_t q = 0; q < idx.size(); ++q) idx[q] = q;
  std::stable_sort(idx.begin(), idx.end(), [&](size_t qx, size_t qy) {
    const Col &x = cols[qx], &y = cols[qy];
    if (pos[qx] != pos[qy]) return pos[qx] < pos[qy];
    if (x.chain != y.chain) return x.chain > y.chain;
    return x.m < y.m;
  });
  std::vector<BatchSeg> segs;
  segs.reserve(cols.size());
  long long t = 0;
  for (size_t q : idx) {
    const Col& c = cols[q];
    segs.push_back(BatchSeg{t, c.local0, c.m, 0});
    t += c.len;
  }
  *total = t;
  return segs;
}

// Bound on the batch's dispatched tasks that wait on a larger ticket.  Only
// DIAG tasks dispatched ahead of their column do: DIAG(d), dispatched with
// column d - L, waits on tasks of columns up to d - 2 of its step, so between
// two segments of its matrix at most max(0, L - 2) of them are pending, and
// inside the segment being dispatched at most L + 1 (none without lookahead).
static long long batch_ahead_bound(const std::vector<FactorPlan>& plans, int cap) {
  long long s = 0;
  int inside = 0;
  for (const FactorPlan& fp : plans) {
    const int L = std::min(fp.look, cap);
    s += std::max(0, L - 2);
    if (L > 0) inside = std::max(inside, L + 1);
  }
  return s + inside;
}
static long long batch_ahead_bound(const FactorBatchPlan& bp) { return batch_ahead_bound(bp.plans, 1 << 30); }

// Batched host plan.  num_cus (0: not known) caps the DIAG lookahead so that
// the whole batch's forward waits stay below the number of workgroups.
FactorBatchPlan factor_batch_plan(int count, const int64_t* n, const int64_t* b, const int64_t* a, int num_cus) {
  FactorBatchPlan bp;
  bp.count = count;
  bp.plans.resize(count);
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off += (bytes + 255) & ~size_t(255); return o; };
  bp.off_ctl = take(256);  // ticket counter, abort flag at CTL_ABORT
  bp.off_mats = take(sizeof(FactorParams) * (size_t)count);
  long long nflags = 0;
  bp.flag_off.resize(count);
  bp.ws_off.resize(count);
  // segment order, DIAG lookahead and SUB delay of the batch: measurement
  // overrides BTA_BATCH_ORDER (0 lockstep, 1 proportional),
  // BTA_BATCH_LOOKAHEAD and BTA_BATCH_SUB_DELAY
  long long v = 0;
  bp.order = env_int("BTA_BATCH_ORDER", 0, 1, &v) ? (int)v : 1;
  const int look = env_int("BTA_BATCH_LOOKAHEAD", 0, 64, &v) ? (int)v : BATCH_LOOKAHEAD;
  const int sub_delay = env_int("BTA_BATCH_SUB_DELAY", 0, 64, &v) ? (int)v : BATCH_SUB_DELAY;
  int64_t nseg = 0;  // segments: one per column group of every step
  for (int m = 0; m < count; ++m) {
    bp.plans[m] = factor_plan(n[m], b[m], a[m]);
    bp.plans[m].look = std::min(bp.plans[m].look, look);
    bp.plans[m].sub_delay = std::min(sub_delay, bp.plans[m].T);
    nseg += n[m] * bp.plans[m].T + (n[m] - 1) * bp.plans[m].sub_delay;
    bp.flag_off[m] = nflags;
    nflags += bp.plans[m].nflags;
  }
  bp.nseg = nseg;
  bp.off_segs = take(sizeof(BatchSeg) * (size_t)nseg);
  bp.nflags = nflags;
  bp.off_flags = take(sizeof(int) * (size_t)std::max<long long>(nflags, 1));
  for (int m = 0; m < count; ++m) {
    const FactorPlan& fp = bp.plans[m];
    bp.ws_off[m][0] = take(fp.off_P - fp.off_Wd);          // Wd + Wt
    bp.ws_off[m][1] = take(fp.bytes - fp.off_P);           // P
  }
  bp.bytes = off;
  long long t = 0;
  for (int m = 0; m < count; ++m) t += bp.plans[m].ntasks;
  bp.ntasks = t;
  if (num_cus > 0 && num_cus < t) {
    // the largest common lookahead cap that keeps the forward waits below the grid
    int cap = FACTOR_LOOKAHEAD;
    while (cap > 0 && batch_ahead_bound(bp.plans, cap) > num_cus - 1) --cap;
    for (int m = 0; m < count; ++m) bp.plans[m].look = std::min(bp.plans[m].look, cap);
  }
  return bp;
}

hipError_t factor_batch_launch(const FactorBatchPlan& bp, const BatchMatrix* mats, void* work, hipStream_t stream,
                               int num_cus) {
  char* w = static_cast<char*>(work);
  int* ctl = reinterpret_cast<int*>(w + bp.off_ctl);
  int* flags = reinterpret_cast<int*>(w + bp.off_flags);
  std::vector<FactorParams> hp(bp.count);
  for (int m = 0; m < bp.count; ++m) {
    const FactorPlan& fp = bp.plans[m];
    FactorParams& p = hp[m];
    p = FactorParams{};
    p.n = (int)mats[m].n; p.b = (int)mats[m].b; p.a = (int)mats[m].a; p.T = fp.T; p.TA = fp.TA;
    p.D = mats[m].D; p.B = mats[m].B; p.R = mats[m].R; p.Tt = mats[m].T;
    p.LD = mats[m].LD; p.LB = mats[m].LB; p.LR = mats[m].LR; p.LT = mats[m].LT;
    char* wd = w + bp.ws_off[m][0];
    p.Wd = reinterpret_cast<double*>(wd);
    p.Wt = reinterpret_cast<double*>(wd + (fp.off_Wt - fp.off_Wd));
    p.P = reinterpret_cast<double*>(w + bp.ws_off[m][1]);
    p.flags = flags + bp.flag_off[m];
    p.ctl = ctl;
    p.info = mats[m].info;
    p.ntasks = fp.ntasks;
    p.step_full = fp.step_full;
    p.step_last = fp.step_last;
    p.look = fp.look;
    p.sub_delay = fp.sub_delay;
    p.spin_limit = 1LL << 22;
    p.cached = (factor_cached_loads(p.b, p.a) && factor_lines_aligned(p.b, p.a, p.LD, p.LB, p.LR, p.LT)) ? 1 : 0;
    p.fast = (!p.cached && factor_ops_direct(p.b, p.a, p.LD, p.LB, p.LR, p.LT)) ? 1 : 0;
    p.trace = nullptr;
  }
  std::vector<int64_t> ns(bp.count);
  for (int m = 0; m < bp.count; ++m) ns[m] = mats[m].n;
  long long t = 0;
  const std::vector<BatchSeg> segs = batch_segments(bp, ns.data(), &t);
  hipError_t e = hipMemcpyAsync(w + bp.off_mats, hp.data(), sizeof(FactorParams) * hp.size(), hipMemcpyHostToDevice, stream);
  if (e != hipSuccess) return e;
  e = hipMemcpyAsync(w + bp.off_segs, segs.data(), sizeof(BatchSeg) * segs.size(), hipMemcpyHostToDevice, stream);
  if (e != hipSuccess) return e;
  const FactorParams* dmats = reinterpret_cast<const FactorParams*>(w + bp.off_mats);
  const int rgrid = (int)std::min<long long>(1024, (bp.nflags + 255) / 256 + 1);
  hipLaunchKernelGGL(factor_batched_reset_kernel, dim3(rgrid), dim3(256), 0, stream, flags, bp.nflags, ctl, dmats, bp.count);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  FactorBatchArgs args;
  args.mats = dmats;
  args.segs = reinterpret_cast<const BatchSeg*>(w + bp.off_segs);
  args.nseg = (int)segs.size();
  args.ntasks = t;
  args.ctl = ctl;
  const long long grid = std::min<long long>(t, (long long)num_cus);
  if (grid < t && grid <= batch_ahead_bound(bp)) return hipErrorInvalidConfiguration;  // lookahead needs more workers
  timing_mark(KT_FACTOR, true, stream);
  bool all_fast = true;
  for (const FactorParams& q : hp) all_fast = all_fast && q.fast != 0;
  if (all_fast)
    hipLaunchKernelGGL(factor_batched_kernel<true>, dim3((unsigned)grid), dim3(NT), SOLO_LDS_PAD, stream, args);
  else
    hipLaunchKernelGGL(factor_batched_kernel<false>, dim3((unsigned)grid), dim3(NT), SOLO_LDS_PAD, stream, args);
  timing_mark(KT_FACTOR, false, stream);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(factor_batched_finish_kernel, dim3((bp.count + 255) / 256), dim3(256), 0, stream, ctl, dmats, bp.count);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Host replay of the task schedule: every ticket decodes to a distinct tile,
// every flag a task waits on belongs to a task with a smaller ticket (so the
// in-order ticket dispatch cannot deadlock), and every operand window lies
// inside its array.  counts[] receives the number of tiles of each kind (a
// DIAG task also produces the tile left of its diagonal tile, counted under
// OFFD or SUB).  Returns 0 when the schedule is valid, else an error code.
// `look` and `sub_delay` are the DIAG lookahead and SUB delay to replay (the
// plan's own when negative); maxdep_out (optional) receives, per ticket, the
// largest ticket it waits on.
int factor_schedule_replay(int64_t n, int64_t b, int64_t a, int look, long long* counts /* [7] or null */,
                           std::vector<long long>* maxdep_out, int sub_delay = -1) {
  FactorPlan fp = factor_plan(n, b, a);
  if (look >= 0) fp.look = std::min<int>(look, fp.T - 1);
  if (sub_delay >= 0) fp.sub_delay = std::min<int>(sub_delay, fp.T);
  FactorParams p{};
  p.n = (int)n; p.b = (int)b; p.a = (int)a; p.T = fp.T; p.TA = fp.TA;
  const uintptr_t G = uintptr_t(1) << 40;
  p.LD = reinterpret_cast<double*>(1 * G);
  p.LB = reinterpret_cast<double*>(2 * G);
  p.LR = reinterpret_cast<double*>(3 * G);
  p.LT = reinterpret_cast<double*>(4 * G);
  p.flags = reinterpret_cast<int*>(5 * G);
  p.ntasks = fp.ntasks; p.step_full = fp.step_full; p.step_last = fp.step_last; p.look = fp.look;
  p.sub_delay = fp.sub_delay;
  const size_t lim[4] = {(size_t)(n * b * b), (size_t)((n - 1) * b * b), (size_t)(n * a * b), (size_t)(a * a)};
  auto inside = [&](const OpTile& o) -> bool {
    if (o.rows <= 0 || o.cols <= 0) return false;
    const uintptr_t addr = reinterpret_cast<uintptr_t>(o.p);
    const int arr = (int)(addr / G) - 1;
    if (arr < 0 || arr > 3) return false;
    const size_t off = (addr - (arr + 1) * G) / sizeof(double);
    const size_t last = off + (size_t)(o.rows - 1) * o.ld + (o.cols - 1);
    return last < lim[arr] && (size_t)o.cols <= (size_t)o.ld;
  };
  // rank of a task: the global band column it belongs to (tip tasks after all columns)
  auto rank_of = [&](const Task& t) -> long long {
    switch (t.type) {
      case T_TUPD: return (long long)t.i * p.T + p.T - 1;
      case T_TIPD: case T_TIPO: return (long long)p.n * p.T;
      default: return (long long)t.i * p.T + t.c;
    }
  };
  // pass 1: every ticket decodes to a task, every flag has exactly one owner
  std::vector<long long> owner((size_t)fp.nflags, -1);
  std::vector<long long> rank((size_t)fp.ntasks);
  long long cnt[7] = {0, 0, 0, 0, 0, 0, 0};
  for (long long tk = 0; tk < fp.ntasks; ++tk) {
    const Task t = decode(p, tk);
    if (t.type < 0 || t.type > 6) return 1;
    cnt[t.type]++;
    rank[(size_t)tk] = rank_of(t);
    int64_t f;
    switch (t.type) {
      case T_DIAG: case T_OFFD: f = fl_D(p, t.i, t.r, t.c); if (t.r < t.c || t.r >= p.T) return 2; break;
      case T_SUB: f = fl_B(p, t.i, t.r, t.c); if (t.i >= n - 1) return 2; break;
      case T_ARW: f = fl_R(p, t.i, t.r, t.c); break;
      case T_TUPD: f = fl_U(p, t.i, t.r, t.c); break;
      default: f = fl_tip(p, t.r, t.c); break;
    }
    if (f < 0 || f >= fp.nflags || owner[(size_t)f] != -1) return 3;
    owner[(size_t)f] = tk;
    if (t.type == T_DIAG && (t.c > 0 || t.i > 0)) {
      const int64_t pf = t.c > 0 ? fl_D(p, t.i, t.c, t.c - 1) : fl_B(p, t.i - 1, 0, p.T - 1);
      if (pf < 0 || pf >= fp.nflags || owner[(size_t)pf] != -1) return 3;
      owner[(size_t)pf] = tk;
      cnt[t.c > 0 ? T_OFFD : T_SUB]++;
    }
  }
  // pass 2: dependencies.  A task other than DIAG waits only on tasks with
  // smaller tickets; a DIAG task (dispatched up to `look` columns early) waits
  // only on tasks of smaller rank.  Together with the bound on the number of
  // DIAG tasks ahead of the in-order frontier (checked below) this keeps the
  // schedule deadlock free whenever more workgroups than that bound are resident.
  std::vector<long long> maxdep((size_t)fp.ntasks, -1);  // largest ticket a task waits on
  auto dep_ok = [&](int64_t flag, long long tk, bool diag) -> int {
    if (flag < 0 || flag >= fp.nflags) return 4;
    const long long o = owner[(size_t)flag];
    if (o < 0) return 5;
    if (diag ? !(rank[(size_t)o] < rank[(size_t)tk]) : !(o < tk)) return 5;
    maxdep[(size_t)tk] = std::max(maxdep[(size_t)tk], o);
    return 0;
  };
  for (long long tk = 0; tk < fp.ntasks; ++tk) {
    const Task t = decode(p, tk);
    int e;
    if (t.type == T_DIAG && (t.c > 0 || t.i > 0)) {
      const Task pt = t.c > 0 ? Task{T_OFFD, t.i, t.c, t.c - 1} : Task{T_SUB, t.i - 1, 0, p.T - 1};
      const int64_t pf = t.c > 0 ? fl_D(p, t.i, t.c, t.c - 1) : fl_B(p, t.i - 1, 0, p.T - 1);
      const int64_t wf = t.c > 0 ? fl_D(p, t.i, t.c - 1, t.c - 1) : fl_D(p, t.i - 1, p.T - 1, p.T - 1);
      const int pnk = ksources(p, pt, -1, nullptr);
      if (pnk != ksources(p, t, -1, nullptr) - 1) return 10;
      for (int kk = 0; kk < pnk; ++kk) {
        KSrc s, sd;
        ksources(p, pt, kk, &s);
        ksources(p, t, kk, &sd);
        if (s.a.p != sd.a.p || s.fa != sd.fa) return 10;  // shared left operand
        if ((e = dep_ok(s.fa - p.flags, tk, true)) || (e = dep_ok(s.fb - p.flags, tk, true))) return e;
        if (!inside(s.a) || !inside(s.b)) return 6;
      }
      KSrc last;
      ksources(p, t, pnk, &last);  // the diagonal tile's last k source is the fused tile
      if (last.fa - p.flags != pf || last.fb - p.flags != pf) return 10;
      if (dep_ok(wf, tk, true)) return 7;
      continue;
    }
    const bool diag = t.type == T_DIAG;
    const int nk = ksources(p, t, -1, nullptr);
    for (int kk = 0; kk < nk; ++kk) {
      KSrc s;
      ksources(p, t, kk, &s);
      if ((e = dep_ok(s.fa - p.flags, tk, diag)) || (e = dep_ok(s.fb - p.flags, tk, diag))) return e;
      if (!inside(s.a) || !inside(s.b)) return 6;
    }
    if (t.type == T_OFFD || t.type == T_SUB || t.type == T_ARW) {
      if (dep_ok(fl_D(p, t.i, t.c, t.c), tk, false)) return 7;
    }
    if (t.type == T_TIPO && dep_ok(fl_tip(p, t.c, t.c), tk, false)) return 7;
    if (t.type == T_TIPD || t.type == T_TIPO) {
      for (int i = 0; i < p.n; ++i)
        if (dep_ok(fl_U(p, i, t.r, t.c), tk, false)) return 8;
    }
  }
  // at any point of the dispatch order, at most look + 1 dispatched tasks still
  // wait on a task with a larger ticket
  long long ahead_max = 0;
  std::vector<long long> open;  // max dependency tickets of dispatched tasks that wait ahead
  for (long long tk = 0; tk < fp.ntasks; ++tk) {
    if (maxdep[(size_t)tk] > tk) open.push_back(maxdep[(size_t)tk]);
    open.erase(std::remove_if(open.begin(), open.end(), [&](long long m) { return m <= tk; }), open.end());
    ahead_max = std::max<long long>(ahead_max, (long long)open.size());
  }
  if (ahead_max > fp.look + 1) return 11;
  if (maxdep_out) *maxdep_out = std::move(maxdep);
  const long long T = fp.T, TA = fp.TA;
  const long long expect[7] = {n * T, n * T * (T - 1) / 2, (n - 1) * T * T, n * T * TA, n * TA * (TA + 1) / 2, TA,
                               TA * (TA - 1) / 2};
  for (int k = 0; k < 7; ++k) {
    if (counts) counts[k] = cnt[k];
    if (cnt[k] != expect[k]) return 9;
  }
  return 0;
}

int factor_schedule_check(int64_t n, int64_t b, int64_t a, long long* counts /* [7] or null */) {
  return factor_schedule_replay(n, b, a, -1, counts, nullptr);
}

}  // namespace bta

// Internal: DIAG lookahead in columns for later factorizations (1..64);
// returns the previous value (any other argument only queries).
BTA_TESTING_API int bta_internal_factor_lookahead(int look) {
  const int prev = bta::g_factor_look;
  if (look >= 1 && look <= 64) bta::g_factor_look = look;
  else if (look == 0) bta::g_factor_look = 0;
  return prev;
}

// Internal: the DIAG lookahead and the k-loop load path a factorization of
// (n, b, a) would use now (overrides, environment, tuning table, default).
BTA_TESTING_API int bta_internal_factor_plan_knobs(int64_t n, int64_t b, int64_t a, int* look, int* cached) {
  if (look) *look = bta::factor_plan(n, b, a).look;
  if (cached) *cached = bta::factor_cached_loads(b, a) ? 1 : 0;
  return 0;
}

// Internal: 1 reads the k-loop operand tiles through the L2 where they are
// line-aligned, 0 with device-coherent loads, -1 removes the override (the
// environment, the tuning table or the default decide); returns the previous
// override (any other argument only queries).
BTA_TESTING_API int bta_internal_factor_cached_loads(int on) {
  const int prev = bta::g_factor_cached;
  if (on >= -1 && on <= 1) bta::g_factor_cached = on;
  return prev;
}

// Internal: cap on the single-matrix factor kernel's workgroups (0 = one per
// CU); returns the previous value (a negative argument only queries).
BTA_TESTING_API int bta_internal_factor_max_grid(int g) {
  const int prev = bta::g_factor_max_grid;
  if (g >= 0) bta::g_factor_max_grid = g;
  return prev;
}

// bta_factor with a trace buffer of 8 words per record (device memory): one
// record per ticket; the number of records is returned through *ntasks when
// the pointer is set.
BTA_TESTING_API int bta_internal_factor_traced(
    int64_t n, int64_t b, int64_t a, const double* D, const double* B, const double* R, const double* T, double* LD,
    double* LB, double* LR, double* LT, void* work, int64_t* info, unsigned long long* trace, long long* ntasks,
    hipStream_t stream) {
  const bta::FactorPlan fp = bta::factor_plan(n, b, a);
  if (ntasks) *ntasks = fp.ntasks;
  if (!trace) return 0;
  return bta::factor_launch(fp, n, b, a, D, B, R, T, LD, LB, LR, LT, work, info, stream, bta::device_cu_count(), trace) ==
                 hipSuccess
             ? 0
             : 1;
}

// Host check of the batch interleaving for a launch with `num_cus` workgroups:
// every ticket maps (by the kernel's binary search) to a matrix and a local
// ticket, per matrix the local tickets come out as 0, 1, ... ntasks-1 in
// order, every segment holds exactly the tasks of its band column, and a
// replay of the whole dispatch order with every matrix's dependencies never
// has more dispatched tasks waiting on a larger ticket than the launch's bound
// (itself below the number of workgroups).  *ahead (optional) receives the
// replay's maximum.  Returns 0 or an error code.
BTA_TESTING_API int bta_internal_factor_batch_check(int count, const int64_t* n,
                                                                                       const int64_t* b, const int64_t* a,
                                                                                       int num_cus, long long* ahead) {
  const bta::FactorBatchPlan bp = bta::factor_batch_plan(count, n, b, a, num_cus);
  long long total = 0;
  const std::vector<bta::BatchSeg> segs = bta::batch_segments(bp, n, &total);
  if (total != bp.ntasks || (long long)segs.size() > bp.nseg) return 1;
  std::vector<std::vector<long long>> maxdep(count), global(count);
  std::vector<bta::FactorParams> ps(count);
  for (int m = 0; m < count; ++m) {
    if (bta::factor_schedule_replay(n[m], b[m], a[m], bp.plans[m].look, nullptr, &maxdep[m], bp.plans[m].sub_delay) != 0)
      return 5;
    global[m].assign((size_t)bp.plans[m].ntasks, -1);
    bta::FactorParams& p = ps[m];
    p.n = (int)n[m]; p.b = (int)b[m]; p.a = (int)a[m]; p.T = bp.plans[m].T; p.TA = bp.plans[m].TA;
    p.ntasks = bp.plans[m].ntasks; p.step_full = bp.plans[m].step_full; p.step_last = bp.plans[m].step_last;
    p.look = bp.plans[m].look;
    p.sub_delay = bp.plans[m].sub_delay;
  }
  std::vector<long long> next(count, 0);
  std::vector<int> seg_of(total > 0 ? (size_t)total : 1);
  for (long long tk = 0; tk < total; ++tk) {
    int lo = 0, hi = (int)segs.size() - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (segs[mid].t0 <= tk) lo = mid; else hi = mid - 1;
    }
    const int m = segs[lo].mat;
    const long long local = segs[lo].local0 + (tk - segs[lo].t0);
    if (m < 0 || m >= count || local != next[m]) return 2;
    ++next[m];
    global[m][(size_t)local] = tk;
    seg_of[(size_t)tk] = lo;
  }
  for (int m = 0; m < count; ++m)
    if (next[m] != bp.plans[m].ntasks) return 3;
  // segment contents: the column group a task is dispatched with (DIAG
  // tasks L columns early, SUB tasks S columns late, tip work with the last
  // group) is the segment's group
  {
    std::vector<long long> first_key(count, -1);
    for (size_t q = 0; q < segs.size(); ++q) {
      const long long len = (q + 1 < segs.size() ? segs[q + 1].t0 : total) - segs[q].t0;
      const int m = segs[q].mat;
      const bta::FactorParams& p = ps[m];
      const long long G = p.T + p.sub_delay;  // groups per step (at most)
      long long key = -1;
      for (long long e = 0; e < len; ++e) {
        const bta::Task t = bta::decode(p, segs[q].local0 + e);
        long long k;
        if (t.type == bta::T_TIPD || t.type == bta::T_TIPO) k = (long long)(p.n - 1) * G + p.T - 1;
        else if (t.type == bta::T_TUPD) k = (long long)t.i * G + (t.i < p.n - 1 ? G : p.T) - 1;
        else if (t.type == bta::T_DIAG) k = (long long)t.i * G + (t.c <= p.look ? 0 : t.c - p.look);
        else if (t.type == bta::T_SUB) k = (long long)t.i * G + t.c + p.sub_delay;
        else k = (long long)t.i * G + t.c;
        if (key < 0) key = k;
        if (k != key) return 4;
      }
      if (key <= first_key[m]) return 4;  // columns of a matrix in order, each once
      first_key[m] = key;
    }
  }
  // replay: dispatched tasks that wait on a larger ticket
  long long amax = 0;
  std::vector<long long> open;
  for (long long tk = 0; tk < total; ++tk) {
    const bta::BatchSeg& sg = segs[(size_t)seg_of[(size_t)tk]];
    const long long local = sg.local0 + (tk - sg.t0);
    const long long md = maxdep[sg.mat][(size_t)local];
    if (md >= 0) {
      const long long g = global[sg.mat][(size_t)md];
      if (g > tk) open.push_back(g);
    }
    open.erase(std::remove_if(open.begin(), open.end(), [&](long long x) { return x <= tk; }), open.end());
    amax = std::max<long long>(amax, (long long)open.size());
  }
  if (ahead) *ahead = amax;
  if (amax > bta::batch_ahead_bound(bp)) return 6;
  if (num_cus > 0 && std::min<long long>(total, num_cus) < total && bta::batch_ahead_bound(bp) >= num_cus) return 7;
  return 0;
}

BTA_TESTING_API int bta_internal_factor_schedule_check(int64_t n, int64_t b, int64_t a,
                                                                                          long long* counts) {
  return bta::factor_schedule_check(n, b, a, counts);
}

namespace bta {
// rsqrt_refined applied elementwise (the pivot reciprocal square root of the
// diagonal-tile Cholesky), for the error-bound test.
__global__ __launch_bounds__(256) void rsqrt_probe_kernel(const double* in, double* out, int64_t count) {
  for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < count; k += (int64_t)gridDim.x * 256)
    out[k] = rsqrt_refined(in[k]);
}
}  // namespace bta

BTA_TESTING_API int bta_internal_rsqrt(const double* d_in, double* d_out, int64_t count, hipStream_t s) {
  if (!d_in || !d_out || count < 1) return (int)hipErrorInvalidValue;
  const unsigned grid = (unsigned)std::min<int64_t>(4096, (count + 255) / 256);
  hipLaunchKernelGGL(bta::rsqrt_probe_kernel, dim3(grid), dim3(256), 0, s, d_in, d_out, count);
  return (int)hipGetLastError();
}

namespace bta {
// Latency of the diagonal-tile Cholesky + inverse (the link of the factor's
// critical path) in isolation: one workgroup factors the same 64 x 64 SPD tile
// `iters` times from LDS; ticks[0] receives the summed s_memrealtime ticks
// (100 MHz) of the calls, ticks[1] the failure column, ticks[2..11] the summed
// phase durations (panels and trailing updates, W, levels), L and W the last
// call's factor and inverse.  var selects the panel variant.
template <int VAR>
__device__ void diag_link_probe_body(const double* A, double* Lout, double* Wout, long long* ticks, int iters) {
  __shared__ Shared sh;
  __shared__ long long ts[16];
  const int tid = threadIdx.x;
  double v[16];
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    const int idx = tid + 256 * e;
    v[e] = A[idx];
  }
  long long total = 0, ph[14] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  int f = 0;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int idx = tid + 256 * e;
      sh.u.f.As[(idx >> 6) * LDS_LD + (idx & 63)] = v[e];
    }
    __syncthreads();
    const long long t0 = __builtin_amdgcn_s_memrealtime();
    f = chol_inv_tile_mfma_t<VAR, true>(sh.u.f.As, sh.u.f.Bs, sh.rinv, sh.pan, &sh.fail, tid, ts);
    __syncthreads();
    const long long t1 = __builtin_amdgcn_s_memrealtime();
    total += t1 - t0;
    if (tid == 0) {
      for (int k = 0; k < 10; ++k) ph[k] += ts[k + 1] - ts[k];
      ph[10] += ts[11] - ts[7];  // inside the diagonal-block inverses (wave 0): the pivot check,
      ph[11] += ts[12] - ts[11];  // the substitution,
      ph[12] += ts[13] - ts[12];  // the stores of the block row,
      ph[13] += ts[8] - ts[13];   // and the wait at the barrier
    }
  }
  for (int e = tid; e < 4096; e += NT) {
    const int rr = e >> 6, cc = e & 63;
    Lout[e] = cc <= rr ? sh.u.f.As[rr * LDS_LD + cc] : 0.0;
    Wout[e] = sh.u.f.Bs[rr * LDS_LD + cc];
  }
  if (tid == 0) {
    ticks[0] = total;
    ticks[1] = f;
    for (int k = 0; k < 14; ++k) ticks[2 + k] = ph[k];
  }
}
__global__ __launch_bounds__(NT, 1) void diag_link_probe_kernel0(const double* A, double* L, double* W, long long* t, int it) {
  diag_link_probe_body<0>(A, L, W, t, it);
}
__global__ __launch_bounds__(NT, 1) void diag_link_probe_kernel1(const double* A, double* L, double* W, long long* t, int it) {
  diag_link_probe_body<1>(A, L, W, t, it);
}
}  // namespace bta

BTA_TESTING_API int bta_internal_diag_link_probe(const double* d_A, double* d_L, double* d_W, long long* d_ticks,
                                                 int iters, int var, hipStream_t s) {
  if (!d_A || !d_L || !d_W || !d_ticks || iters < 1) return (int)hipErrorInvalidValue;
  if (var == 0)
    hipLaunchKernelGGL(bta::diag_link_probe_kernel0, dim3(1), dim3(bta::NT), 0, s, d_A, d_L, d_W, d_ticks, iters);
  else if (var == 1)
    hipLaunchKernelGGL(bta::diag_link_probe_kernel1, dim3(1), dim3(bta::NT), 0, s, d_A, d_L, d_W, d_ticks, iters);
  else
    return (int)hipErrorInvalidValue;
  return (int)hipGetLastError();
}

namespace bta {
// Round-trip latency of the cross-workgroup flag hand-off: workgroup 0 and the
// last workgroup of the grid (another XCD) pass a token `iters` times.  mode 0:
// release store / relaxed polls + acquire fence (the factor's protocol);
// mode 1: relaxed device-coherent store after a wait for the wave's stores,
// relaxed polls, no fences.  ticks[0]: summed 100 MHz ticks of the round
// trips measured by workgroup 0.
__global__ __launch_bounds__(64) void flag_pingpong_kernel(int* flags, long long* ticks, int iters, int mode) {
  const bool a = blockIdx.x == 0, b = blockIdx.x == gridDim.x - 1;
  if (!(a || b) || threadIdx.x != 0) return;
  int* mine = flags + (a ? 0 : 64);
  int* other = flags + (a ? 64 : 0);
  const long long t0 = __builtin_amdgcn_s_memrealtime();
  for (int it = 1; it <= iters; ++it) {
    if (b) {
      long long polls = 0;
      while (__hip_atomic_load(other, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < it && ++polls < (1LL << 22)) {
      }
      if (mode == 0) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    if (mode == 0) {
      __hip_atomic_store(mine, it, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      __builtin_amdgcn_s_waitcnt(0);
      __hip_atomic_store(mine, it, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (a) {
      long long polls = 0;
      while (__hip_atomic_load(other, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < it && ++polls < (1LL << 22)) {
      }
      if (mode == 0) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
  }
  if (a) ticks[0] = __builtin_amdgcn_s_memrealtime() - t0;
}
}  // namespace bta

BTA_TESTING_API int bta_internal_flag_pingpong(int* d_flags, long long* d_ticks, int iters, int mode, int grid,
                                               hipStream_t s) {
  if (!d_flags || !d_ticks || iters < 1 || grid < 2) return (int)hipErrorInvalidValue;
  hipLaunchKernelGGL(bta::flag_pingpong_kernel, dim3((unsigned)grid), dim3(64), 0, s, d_flags, d_ticks, iters, mode);
  return (int)hipGetLastError();
}

namespace bta {
// Throughput of the factor's k loop in isolation: every workgroup runs `steps`
// k steps (two 64 x 64 operand tiles into the double-buffered pieced LDS
// stages, then the MFMA product of the previous stage), the tiles taken from a
// row-major matrix of `rows` x `ld` doubles at pseudo-random tile positions
// inside the first `span_rows` rows (a small span stays in the caches).  mode 0:
// device-coherent direct loads (the factor's), 1: no loads (MFMA + barriers
// only), 2: direct loads through the L2, 3: loads into registers two steps
// ahead (plain loads), written to the pieced LDS stage after the MFMAs, 4: as
// 3 with device-coherent buffer loads.  ticks[blockIdx.x]: the workgroup's ticks.
__device__ __forceinline__ void tile_load_regs(d2v (&r)[8], const OpTile& t, int tid, bool coherent) {
  const int w = tid >> 6, lane = tid & 63;
  __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(const_cast<double*>(t.p), (short)0, 0x7fffffff, 0x00020000);
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int slot = (w * 8 + j) * 64 + lane;
    const int m = slot >> 5, pc = (slot & 31) ^ (m & 15);
    const int off = (int)(((int64_t)m * t.ld + 2 * pc) * 8);
    if (coherent) {
      r[j] = __builtin_bit_cast(d2v, __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 16));
    } else {
      r[j] = *reinterpret_cast<const d2v*>(t.p + (int64_t)m * t.ld + 2 * pc);
    }
  }
}
__device__ __forceinline__ void tile_regs_to_lds(double* dst, const d2v (&r)[8], int tid) {
  const int w = tid >> 6, lane = tid & 63;
#pragma unroll
  for (int j = 0; j < 8; ++j) *reinterpret_cast<d2v*>(dst + 2 * ((w * 8 + j) * 64 + lane)) = r[j];
}

__global__ __launch_bounds__(NT, 1) void kloop_probe_kernel(const double* M, int64_t ld, int64_t span_rows, int steps,
                                                            int mode, long long* ticks, double* out) {
  __shared__ Shared sh;
  const int tid = threadIdx.x;
  Acc acc;
  acc_zero(acc);
  // tile rows and columns as powers of two (masks instead of divisions, so the
  // index arithmetic per step is a few instructions, as in the factor)
  unsigned trm = 1, tcm = 1;
  while (2 * trm <= (unsigned)(span_rows / 64)) trm *= 2;
  while (2 * tcm <= (unsigned)(ld / 64)) tcm *= 2;
  auto tile_at = [&](int kk, int which) {
    const unsigned h = blockIdx.x * 2654435761u + (unsigned)kk * 40503u + (unsigned)which * 977u;
    const int64_t tr = (int64_t)(h & (trm - 1)), tc = (int64_t)((h >> 11) & (tcm - 1));
    return OpTile{M + tr * 64 * ld + tc * 64, ld, 64, 64, false};
  };
  long long t0 = 0;
  if (mode >= 3) {
    const bool coh = mode == 4;
    d2v ra[2][8], rb[2][8];
    tile_load_regs(ra[0], tile_at(0, 0), tid, coh);
    tile_load_regs(rb[0], tile_at(0, 1), tid, coh);
    tile_load_regs(ra[1], tile_at(1, 0), tid, coh);
    tile_load_regs(rb[1], tile_at(1, 1), tid, coh);
    __builtin_amdgcn_s_waitcnt(0);
    tile_regs_to_lds(sh.u.stage[0][0], ra[0], tid);
    tile_regs_to_lds(sh.u.stage[0][1], rb[0], tid);
    __syncthreads();
    t0 = __builtin_amdgcn_s_memrealtime();
    // two steps per trip: the register buffers are indexed by constants
#define BTA_KSTEP(C, KK)                                                  \
  do {                                                                    \
    if ((KK) + 2 < steps) {                                               \
      tile_load_regs(ra[C], tile_at((KK) + 2, 0), tid, coh);              \
      tile_load_regs(rb[C], tile_at((KK) + 2, 1), tid, coh);              \
    }                                                                     \
    mma_ptile(acc, sh.u.stage[C][0], sh.u.stage[C][1], tid);              \
    if ((KK) + 1 < steps) {                                               \
      tile_regs_to_lds(sh.u.stage[1 - (C)][0], ra[1 - (C)], tid);         \
      tile_regs_to_lds(sh.u.stage[1 - (C)][1], rb[1 - (C)], tid);         \
    }                                                                     \
    __syncthreads();                                                      \
  } while (0)
    for (int kk = 0; kk < steps; kk += 2) {
      BTA_KSTEP(0, kk);
      if (kk + 1 < steps) BTA_KSTEP(1, kk + 1);
    }
#undef BTA_KSTEP
  } else {
    if (mode != 1) {
      tile_load_lds_dev(sh.u.stage[0][0], tile_at(0, 0), tid, mode == 2);
      tile_load_lds_dev(sh.u.stage[0][1], tile_at(0, 1), tid, mode == 2);
    } else {
      for (int e = tid; e < 2 * PT; e += NT) sh.u.stage[0][0][e] = 1e-3 * (e & 7);
    }
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    t0 = __builtin_amdgcn_s_memrealtime();
    for (int kk = 0; kk < steps; ++kk) {
      const int cur = mode == 1 ? 0 : (kk & 1);
      if (mode != 1 && kk + 1 < steps) {
        tile_load_lds_dev(sh.u.stage[(kk + 1) & 1][0], tile_at(kk + 1, 0), tid, mode == 2);
        tile_load_lds_dev(sh.u.stage[(kk + 1) & 1][1], tile_at(kk + 1, 1), tid, mode == 2);
      }
      mma_ptile(acc, sh.u.stage[cur][0], sh.u.stage[cur][1], tid);
      __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
    }
  }
  const long long t1 = __builtin_amdgcn_s_memrealtime();
  if (tid == 0) ticks[blockIdx.x] = t1 - t0;
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) s += acc.v[i][j][0] + acc.v[i][j][1] + acc.v[i][j][2] + acc.v[i][j][3];
  out[(int64_t)blockIdx.x * NT + tid] = s;
}
}  // namespace bta

BTA_TESTING_API int bta_internal_kloop_probe(const double* d_M, int64_t ld, int64_t span_rows, int steps, int mode,
                                             int grid, long long* d_ticks, double* d_out, hipStream_t s) {
  if (!d_M || !d_ticks || !d_out || steps < 1 || grid < 1 || ld < 64 || ld % 64 || span_rows < 64) return (int)hipErrorInvalidValue;
  hipLaunchKernelGGL(bta::kloop_probe_kernel, dim3((unsigned)grid), dim3(bta::NT), 0, s, d_M, ld, span_rows, steps, mode,
                     d_ticks, d_out);
  return (int)hipGetLastError();
}
