// Device building blocks shared by the gfx950 kernels: FP64 MFMA tile engine
// over 64 x 64 output tiles staged through LDS, the in-LDS Cholesky of a
// diagonal tile fused with the inverse of its factor, and the cross-workgroup
// flag protocol of the persistent tile-task kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bta {

typedef double d4 __attribute__((ext_vector_type(4)));

typedef double d2v __attribute__((ext_vector_type(2)));

constexpr int TS = 64;        // output tile edge
constexpr int NT = 256;       // threads per workgroup (4 waves of 64)
constexpr int LDS_LD = 66;    // LDS row stride in doubles: rows shift by 4 banks, keeps 16-byte alignment

// ---------------------------------------------------------------------------
// v_mfma_f64_16x16x4_f64.  Operand layout (lane l): A supplies (row l%16, k l/16),
// B supplies (k l/16, col l%16).  The 4 accumulator values of lane l hold
// rows 4*j + l/16 (j = 0..3) of column l%16.
// A 16-byte aligned pair of zeros: the source of loads whose element lies outside a tile.
__device__ __align__(16) static const double k_zero_pair[2] = {0.0, 0.0};

__device__ __forceinline__ d4 mfma16(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ int acc_row(int lane, int j) { return 4 * j + (lane >> 4); }
__device__ __forceinline__ int acc_col(int lane) { return lane & 15; }

// A 64 x 64 accumulator tile spread over the 4 waves of a workgroup: wave w
// owns rows 32*(w>>1) .. +32 and cols 32*(w&1) .. +32 as 2 x 2 MFMA blocks.
struct Acc {
  d4 v[2][2];
};

__device__ __forceinline__ void acc_zero(Acc& c) {
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) c.v[i][j] = d4{0.0, 0.0, 0.0, 0.0};
}

// (row, col) inside the 64 x 64 tile of accumulator element (bi, bj, j) of this thread
__device__ __forceinline__ int tile_row(int tid, int bi, int j) {
  const int w = tid >> 6, lane = tid & 63;
  return 32 * (w >> 1) + 16 * bi + acc_row(lane, j);
}
__device__ __forceinline__ int tile_col(int tid, int bj) {
  const int w = tid >> 6, lane = tid & 63;
  return 32 * (w & 1) + 16 * bj + acc_col(lane);
}

// ---------------------------------------------------------------------------
// Operand tile: element (m, k) of a rows x cols window, m < 64, k < 64;
// trans == false: p[m*ld + k]  (k contiguous);  trans == true: p[k*ld + m].
// Elements outside the window read as zero.
struct OpTile {
  const double* p;
  int64_t ld;
  int rows;
  int cols;
  bool trans;
};

// Per-thread register staging of one 64 x 64 operand tile (16 doubles).
struct Stage {
  double v[16];
};

// Device-coherent (agent scope, sc1) element access for data exchanged between
// workgroups of one persistent kernel: such loads and stores do not depend on
// the per-XCD L2 being written back or invalidated.
__device__ __forceinline__ double ld_dev(const double* p) {
  const unsigned long long v =
      __hip_atomic_load(reinterpret_cast<const unsigned long long*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return __builtin_bit_cast(double, v);
}
__device__ __forceinline__ void st_dev(double* p, double v) {
  __hip_atomic_store(reinterpret_cast<unsigned long long*>(p), __builtin_bit_cast(unsigned long long, v), __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
}

// stage_load for tiles produced by other workgroups of the same kernel
// Staging layout: thread tid holds rows 8 j + tid / 32 (j = 0..7), columns
// 2 (tid % 32) and 2 (tid % 32) + 1, so that the 64 lanes of a wave cover two
// whole rows (eight 128-byte lines) per load instruction.  Device-coherent
// 8-byte accesses; elements past a ragged edge read as zero.
__device__ __forceinline__ void stage_load_dev(Stage& s, const OpTile& t, int tid) {
  const int c2 = (tid & 31) * 2, r0 = tid >> 5;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int row = 8 * j + r0;
    const double* src = t.p + (int64_t)row * t.ld + c2;
    s.v[2 * j] = (row < t.rows && c2 < t.cols) ? ld_dev(src) : 0.0;
    s.v[2 * j + 1] = (row < t.rows && c2 + 1 < t.cols) ? ld_dev(src + 1) : 0.0;
  }
}
__device__ __forceinline__ void stage_store(const Stage& s, double* lds, int tid) {
  const int c2 = (tid & 31) * 2, r0 = tid >> 5;
#pragma unroll
  for (int j = 0; j < 8; ++j) *reinterpret_cast<d2v*>(lds + (8 * j + r0) * LDS_LD + c2) = d2v{s.v[2 * j], s.v[2 * j + 1]};
}
// ---------------------------------------------------------------- pieced LDS tiles (direct loads)
// A 64 x 64 operand tile moved from global memory straight into LDS in 16-byte
// pieces (global_load_lds_dwordx4, device coherent).  Row m's piece p (columns
// 2p, 2p+1) sits at slot m*32 + (p ^ (m & 15)): a wave instruction fills two
// whole rows, and the xor spreads the 16 rows that one MFMA operand read
// touches over all LDS banks.
constexpr int PT = 4096;  // doubles per pieced tile
__device__ __forceinline__ int pslot(int m, int p) { return m * 32 + (p ^ (m & 15)); }


__device__ __forceinline__ void lds_dma16_dev(const double* src, double* lds_wave_base) {
  __builtin_amdgcn_global_load_lds(static_cast<const void*>(src),
                                   (__attribute__((address_space(3))) void*)(lds_wave_base), 16, 0, 16 /* sc1 */);
}
// The same 16-byte piece through the caches (no scope bits): allowed only for
// data that is final before its first read on this XCD and whose cache lines
// hold nothing else that changes during the kernel (see tile_load_lds_dev).
__device__ __forceinline__ void lds_dma16_cached(const double* src, double* lds_wave_base) {
  __builtin_amdgcn_global_load_lds(static_cast<const void*>(src),
                                   (__attribute__((address_space(3))) void*)(lds_wave_base), 16, 0, 0);
}

// Issue the loads of tile t into the pieced LDS image dst (elements outside
// t.rows x t.cols read as zero).  Wave w, instruction j fills rows 16w + 2j and
// 16w + 2j + 1.  The caller waits (vmcnt) and synchronizes before reading dst.
// cached (workgroup-uniform): read through the L2 instead of device-coherent
// loads.  Valid for a published (write-once) tile whose rows start on 128-byte
// cache lines and whose leading dimension is a multiple of 16 doubles: no line
// of it can then have entered this XCD's L2 before the tile was final (it is
// only read after its flag), and the consumer's acquire invalidates the CU's L1.
__device__ __forceinline__ void tile_load_lds_dev(double* dst, const OpTile& t, int tid, bool cached = false) {
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  const bool fast = ((t.ld & 1) == 0) && ((t.cols & 1) == 0) && ((reinterpret_cast<uintptr_t>(t.p) & 15) == 0);
  if (fast && cached) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int slot = (w * 8 + j) * 64 + lane;
      const int m = slot >> 5, pc = (slot & 31) ^ (m & 15);
      const double* src = (m < t.rows && 2 * pc < t.cols) ? t.p + (int64_t)m * t.ld + 2 * pc : k_zero_pair;
      lds_dma16_cached(src, dst + (w * 8 + j) * 128);
    }
  } else if (fast) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int slot = (w * 8 + j) * 64 + lane;
      const int m = slot >> 5, pc = (slot & 31) ^ (m & 15);
      const double* src = (m < t.rows && 2 * pc < t.cols) ? t.p + (int64_t)m * t.ld + 2 * pc : k_zero_pair;
      lds_dma16_dev(src, dst + (w * 8 + j) * 128);
    }
  } else {
    // odd extents or leading dimension: element loads through registers
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int slot = (w * 8 + j) * 64 + lane;
      const int m = slot >> 5, pc = (slot & 31) ^ (m & 15);
      const double* src = t.p + (int64_t)m * t.ld + 2 * pc;
      const double x0 = (m < t.rows && 2 * pc < t.cols) ? ld_dev(src) : 0.0;
      const double x1 = (m < t.rows && 2 * pc + 1 < t.cols) ? ld_dev(src + 1) : 0.0;
      *reinterpret_cast<d2v*>(dst + 2 * slot) = d2v{x0, x1};
    }
  }
}

// tile_load_lds_dev for a tile known to take the direct path (even leading
// dimension and column count, 16-byte aligned start; device coherent): the
// same loads without the test, written so that the compiler emits straight
// code.  Instruction j of wave w fills rows m = 16w + 2j + lane/32, piece
// pc = (lane%32) ^ (m%16); every address is formed with plain adds from one
// per-lane row base, and pieces outside rows x cols take the zero pair by a
// select (no branch, no per-load multiply).
__device__ __forceinline__ void tile_load_lds_fast(double* dst, const OpTile& t, int tid) {
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  int lane = tid & 63;
  // the lane terms are recomputed at every call instead of being kept live
  // across the caller's k loop (the factor kernel has no registers to spare)
  asm volatile("" : "+v"(lane));
  const int m0 = 16 * w + (lane >> 5);
  const double* rowbase = t.p + (int64_t)m0 * t.ld;
  const int64_t step = 2 * t.ld;  // two rows per instruction
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int m = m0 + 2 * j;
    const int pc = (lane & 31) ^ (m & 15);
    const double* q = rowbase + j * step + 2 * pc;
    const bool ok = (m < t.rows) & (2 * pc < t.cols);
    lds_dma16_dev(ok ? q : k_zero_pair, dst + (w * 8 + j) * 128);
  }
}

// The four consecutive k values 16*kg + 4*g .. +3 of row m of a pieced tile.
__device__ __forceinline__ d4 ptile_row4(const double* T, int m, int kg, int g) {
  const int p0 = 8 * kg + 2 * g;
  const d2v x0 = *reinterpret_cast<const d2v*>(T + 2 * pslot(m, p0));
  const d2v x1 = *reinterpret_cast<const d2v*>(T + 2 * pslot(m, p0 + 1));
  return d4{x0[0], x0[1], x1[0], x1[1]};
}

// c += A B^T (64 x 64 x 64) from pieced tiles; wave w owns the 32 x 32 block
// (32 (w >> 1), 32 (w & 1)) as 2 x 2 MFMA blocks (same layout as mma_tile).
__device__ __forceinline__ void mma_ptile(Acc& c, const double* A, const double* B, int tid) {
  const int w = tid >> 6, lane = tid & 63;
  const int r0 = 32 * (w >> 1) + (lane & 15), c0 = 32 * (w & 1) + (lane & 15), g = lane >> 4;
#pragma unroll
  for (int kg = 0; kg < 4; ++kg) {
    d4 a[2], b[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      a[i] = ptile_row4(A, r0 + 16 * i, kg, g);
      b[i] = ptile_row4(B, c0 + 16 * i, kg, g);
    }
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) c.v[i][j] = mfma16(a[i][s], b[j][s], c.v[i][j]);
  }
}

// c1 += A A^T and c2 += A B^T from pieced tiles (the two share their left operand).
__device__ __forceinline__ void mma_ptile2(Acc& c1, Acc& c2, const double* A, const double* B, int tid) {
  const int w = tid >> 6, lane = tid & 63;
  const int r0 = 32 * (w >> 1) + (lane & 15), c0 = 32 * (w & 1) + (lane & 15), g = lane >> 4;
#pragma unroll
  for (int kg = 0; kg < 4; ++kg) {
    d4 ar[2], ac[2], bc[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      ar[i] = ptile_row4(A, r0 + 16 * i, kg, g);
      ac[i] = ptile_row4(A, c0 + 16 * i, kg, g);
      bc[i] = ptile_row4(B, c0 + 16 * i, kg, g);
    }
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          c1.v[i][j] = mfma16(ar[i][s], ac[j][s], c1.v[i][j]);
          c2.v[i][j] = mfma16(ar[i][s], bc[j][s], c2.v[i][j]);
        }
    __builtin_amdgcn_sched_barrier(0);
  }
}

// Device-coherent store of the rows x cols corner of a 64 x 64 LDS tile.
__device__ __forceinline__ void tile_store_dev(const double* lds, double* out, int64_t ld, int rows, int cols, int tid) {
  const int c2 = (tid & 31) * 2, r0 = tid >> 5;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int row = 8 * j + r0;
    if (row < rows && c2 < cols) st_dev(out + (int64_t)row * ld + c2, lds[row * LDS_LD + c2]);
    if (row < rows && c2 + 1 < cols) st_dev(out + (int64_t)row * ld + c2 + 1, lds[row * LDS_LD + c2 + 1]);
  }
}

// Rows r0 .. r0 + nrows - 1 (nrows a multiple of 8) of a 64-column LDS tile to
// global memory (device-coherent stores).
__device__ __forceinline__ void tile_store_rows_dev(const double* lds, double* out, int64_t ld, int r0, int nrows, int tid) {
  const int c2 = (tid & 31) * 2, rr = tid >> 5;
  for (int j = 0; 8 * j < nrows; ++j) {
    const int row = r0 + 8 * j + rr;
    st_dev(out + (int64_t)row * ld + c2, lds[row * LDS_LD + c2]);
    st_dev(out + (int64_t)row * ld + c2 + 1, lds[row * LDS_LD + c2 + 1]);
  }
}

// tile_store_dev of a lower-triangular tile whose LDS image holds stale values
// above the diagonal: exact zeros are stored there instead.
__device__ __forceinline__ void tile_store_lower_dev(const double* lds, double* out, int64_t ld, int rows, int tid) {
  const int c2 = (tid & 31) * 2, r0 = tid >> 5;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int row = 8 * j + r0;
    if (row < rows && c2 < rows) st_dev(out + (int64_t)row * ld + c2, c2 <= row ? lds[row * LDS_LD + c2] : 0.0);
    if (row < rows && c2 + 1 < rows)
      st_dev(out + (int64_t)row * ld + c2 + 1, c2 + 1 <= row ? lds[row * LDS_LD + c2 + 1] : 0.0);
  }
}

// acc += A_lds * B_lds^T over one 64-wide k tile: A_lds rows are output rows,
// B_lds rows are output columns, both k-contiguous with stride LDS_LD.
// The 16 k values of each MFMA group are permuted so that every lane reads 4
// consecutive k (two 16-byte LDS reads) per operand per group.
__device__ __forceinline__ void mma_tile(Acc& c, const double* As, const double* Bs, int tid) {
  const int w = tid >> 6, lane = tid & 63;
  const int r0 = 32 * (w >> 1) + (lane & 15);
  const int c0 = 32 * (w & 1) + (lane & 15);
  const int kl = (lane >> 4) * 4;
#pragma unroll
  for (int kg = 0; kg < 4; ++kg) {
    d4 a[2], b[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const double* pa = As + (r0 + 16 * i) * LDS_LD + kg * 16 + kl;
      const double* pb = Bs + (c0 + 16 * i) * LDS_LD + kg * 16 + kl;
      d2v a01 = *reinterpret_cast<const d2v*>(pa);
      d2v a23 = *reinterpret_cast<const d2v*>(pa + 2);
      d2v b01 = *reinterpret_cast<const d2v*>(pb);
      d2v b23 = *reinterpret_cast<const d2v*>(pb + 2);
      a[i] = d4{a01[0], a01[1], a23[0], a23[1]};
      b[i] = d4{b01[0], b01[1], b23[0], b23[1]};
    }
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) c.v[i][j] = mfma16(a[i][s], b[j][s], c.v[i][j]);
  }
}

// Write the accumulator tile into LDS as a row-major 64 x 64 image (stride LDS_LD).
__device__ __forceinline__ void acc_to_lds(const Acc& c, double* lds, int tid) {
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int j = 0; j < 4; ++j) lds[tile_row(tid, bi, j) * LDS_LD + tile_col(tid, bj)] = c.v[bi][bj][j];
}

// Load a rows x cols window of a row-major global tile into the accumulator
// layout (zeros outside the window), scaled by `scale`.
__device__ __forceinline__ void acc_load(Acc& c, const double* p, int64_t ld, int rows, int cols, double scale, int tid) {
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int r = tile_row(tid, bi, j), q = tile_col(tid, bj);
        const bool ok = r < rows && q < cols;
        // unconditional load from a valid address: all sixteen loads are in flight together
        const double v = *(ok ? p + (int64_t)r * ld + q : &k_zero_pair[0]);
        c.v[bi][bj][j] = ok ? scale * v : 0.0;
      }
}

// acc_store with device-coherent stores (tiles read by other workgroups of
// the same kernel)
__device__ __forceinline__ void acc_store_dev(const Acc& c, double* p, int64_t ld, int rows, int cols, double scale, int tid) {
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int r = tile_row(tid, bi, j), q = tile_col(tid, bj);
        if (r < rows && q < cols) st_dev(p + (int64_t)r * ld + q, scale * c.v[bi][bj][j]);
      }
}

// ---------------------------------------------------------------------------
// Cross-lane read: lane `lane`'s value of x, broadcast to the whole wave.
__device__ __forceinline__ double rd_lane(double x, int lane) {
  int lo = __builtin_amdgcn_readlane(__double2loint(x), lane);
  int hi = __builtin_amdgcn_readlane(__double2hiint(x), lane);
  return __hiloint2double(hi, lo);
}

// 1/sqrt(d) from the hardware estimate y (relative error below 2^-24,
// measured) refined by one third-order step: with e = 1 - d y^2,
// 1/sqrt(d) = y (1 - e)^(-1/2) = y (1 + e/2 + 3e^2/8 + O(e^3)), so the step
// leaves an O(2^-72) truncation and about one ulp of rounding, in four
// dependent operations (two Newton steps take eight) on the pivot chain.
// sqrt(d) = d * rsqrt(d); the pivot of a positive definite tile is a normal
// positive number, everything else is reported as a failed pivot.
__device__ __forceinline__ double rsqrt_refined(double d) {
  const double y = __builtin_amdgcn_rsq(d);
  const double t = d * y;
  const double e = __builtin_fma(-t, y, 1.0);
  const double c = __builtin_fma(e, 0.375, 0.5);
  const double u = y * e;
  return __builtin_fma(u, c, y);
}

// ---------------------------------------------------------------- 64 x 64 Cholesky + inverse, MFMA-blocked
// c += sgn * A B^T for 16 x 16 blocks over 16 k, operands in LDS:
// A(m,k) = A[m*lda + k]; B(n,k) = B[n*ldb + k] (bt false) or B[k*ldb + n] (bt true).
// Lane l supplies row/col l%16 and k = 4*(l/16) + s for MFMA s (A rows 16-byte aligned).
__device__ __forceinline__ void mma16x16(d4& c, const double* A, int lda, const double* B, int ldb, bool bt, double sgn,
                                         int lane) {
  const int mn = lane & 15, g = lane >> 4;
  const double* pa = A + mn * lda + 4 * g;
  const d2v a01 = *reinterpret_cast<const d2v*>(pa);
  const d2v a23 = *reinterpret_cast<const d2v*>(pa + 2);
  double b0, b1, b2, b3;
  if (!bt) {
    const double* pb = B + mn * ldb + 4 * g;
    const d2v b01 = *reinterpret_cast<const d2v*>(pb);
    const d2v b23 = *reinterpret_cast<const d2v*>(pb + 2);
    b0 = b01[0]; b1 = b01[1]; b2 = b23[0]; b3 = b23[1];
  } else {
    const double* pb = B + (4 * g) * ldb + mn;
    b0 = pb[0]; b1 = pb[ldb]; b2 = pb[2 * ldb]; b3 = pb[3 * ldb];
  }
  c = mfma16(sgn * a01[0], b0, c);
  c = mfma16(sgn * a01[1], b1, c);
  c = mfma16(sgn * a23[0], b2, c);
  c = mfma16(sgn * a23[1], b3, c);
}

__device__ __forceinline__ void blk_load(d4& c, const double* X, int ld, int lane) {
#pragma unroll
  for (int j = 0; j < 4; ++j) c[j] = X[acc_row(lane, j) * ld + acc_col(lane)];
}
__device__ __forceinline__ void blk_store(const d4& c, double* X, int ld, int lane) {
#pragma unroll
  for (int j = 0; j < 4; ++j) X[acc_row(lane, j) * ld + acc_col(lane)] = c[j];
}

// Cholesky factor and inverse of the SPD tile S (64 x 64, LDS row stride
// LDS_LD; only its lower triangle is read).  On return the lower triangle of S
// holds L (the values above it are stale: store it with tile_store_lower_dev)
// and Wl holds W = L^{-1} (zeros above the diagonal).  Returns 0,
// or the 1-based column of the first pivot that is not a positive finite
// number.  Right-looking by 16-column panels: wave p factors panel p alone
// (lane r holds row r; pivots broadcast across the wave, no barrier), the
// trailing lower blocks get the rank-16 update on MFMA.  W follows blockwise:
// the four 16 x 16 diagonal inverses by column substitution (one lane per
// column, reusing the pivots' reciprocal square roots), then the 2 x 2 block
// recursion W21 = -W22 L21 W11, at 16 and at 32, on MFMA.
// Scratch: rinv[64], tmp[4 * 16 * 17].
// VAR 0: the pivot of column k+1 is broadcast from its updated column entry;
// VAR 1: lane k+1 forms the next pivot from its own L(k+1,k) (one FMA), so
// the cross-lane read of L(k+1,k) leaves the pivot chain.  TIMED: thread 0
// writes s_memrealtime stamps of the phase ends into ts[0..10], and of wave 0's
// steps inside the diagonal-block inverses into ts[11..13].
// early_flag (optional): a flag published (agent-scope release, value 1) once
// panel 0 is done and every wave's earlier global stores are complete, so that
// stores issued before the call are published off the critical path.
// Wg (optional): W is also stored to global memory (device coherent, row
// stride 64): rows 0..31 while the 32-level recursion runs, rows 32..63 at the
// end; the caller waits for the stores before publishing W.
template <int VAR, bool TIMED>
__device__ __forceinline__ int chol_inv_tile_mfma_t(double* S, double* Wl, double* rinv, double* tmp, int* fail_sh, int tid,
                                                    long long* ts, int* early_flag = nullptr, double* Wg = nullptr) {
  const int r = tid & 63, q = tid >> 6;
  if (TIMED && tid == 0) ts[0] = __builtin_amdgcn_s_memrealtime();
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    if (p == 0 && q != 0) {
      // waves 1..3 are idle during panel 0: clear W here (its blocks above the
      // diagonal stay zero; the diagonal and lower blocks are written below)
      for (int e = 2 * (tid - 64); e < 64 * 64; e += 2 * (NT - 64))
        *reinterpret_cast<d2v*>(Wl + (e >> 6) * LDS_LD + (e & 63)) = d2v{0.0, 0.0};
    }
    if (q == p) {
      double s[16];
#pragma unroll
      for (int m = 0; m < 16; ++m) s[m] = S[r * LDS_LD + 16 * p + m];
      double dn = s[0];
#pragma unroll
      for (int m = 0; m < 16; ++m) {
        const int k = 16 * p + m;
        const double d = rd_lane(VAR == 1 ? dn : s[m], k);
        // (pivots are checked once after the panels, from rinv)
        const double ri = rsqrt_refined(d);
        if (r == 0) rinv[k] = ri;
        // rows below the pivot get L(r,k) = s * ri, the pivot row sqrt(d) = d * ri
        // (its s is d); rows above hold upper-triangle values that no later step
        // reads (the trailing updates and broadcasts only use rows > k) and that
        // are written back as zeros
        const double lv = s[m] * ri;
        s[m] = lv;
        if (VAR == 1 && m + 1 < 16) dn = __builtin_fma(-lv, lv, s[m + 1]);
        // column m+1 (the next pivot) by a cross-lane read; the other columns
        // through a double-buffered LDS copy of the column (results in VGPRs,
        // off the next pivot's critical path)
        if (m + 1 < 16) s[m + 1] -= lv * rd_lane(lv, k + 1);
        if (m + 2 < 16) {
          double* cb = tmp + (m & 1) * 64;
          cb[r] = lv;
#pragma unroll
          for (int mm = m + 2; mm < 16; ++mm) s[mm] -= lv * cb[16 * p + mm];
        }
      }
      // the rows above the diagonal keep stale values: nothing reads them, and
      // the stores of L write zeros there
#pragma unroll
      for (int m = 0; m < 16; ++m) S[r * LDS_LD + 16 * p + m] = s[m];
    }
    if (p == 0 && early_flag) __builtin_amdgcn_s_waitcnt(0);  // every wave's earlier stores complete
    __syncthreads();
    if (p == 0 && early_flag && tid == 192)
      __hip_atomic_store(early_flag, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    if (TIMED && tid == 0) ts[1 + 2 * p] = __builtin_amdgcn_s_memrealtime();
    if (p < 3) {
      // rank-16 update of the trailing lower blocks (I, J), p < J <= I
      const int nb = (3 - p) * (4 - p) / 2;
      for (int e = q; e < nb; e += 4) {
        int J = p + 1, rem = e;
        while (rem >= 4 - J) { rem -= 4 - J; ++J; }
        const int I = J + rem;
        d4 c;
        blk_load(c, S + 16 * I * LDS_LD + 16 * J, LDS_LD, r);
        mma16x16(c, S + 16 * I * LDS_LD + 16 * p, LDS_LD, S + 16 * J * LDS_LD + 16 * p, LDS_LD, false, -1.0, r);
        blk_store(c, S + 16 * I * LDS_LD + 16 * J, LDS_LD, r);
      }
      __syncthreads();
      if (TIMED && tid == 0) ts[2 + 2 * p] = __builtin_amdgcn_s_memrealtime();
    }
  }
  // ---- W: diagonal 16 x 16 blocks, wave q inverts block q, lane j < 16 computes column j
  {
    if (TIMED && tid == 0) ts[11] = __builtin_amdgcn_s_memrealtime();
    const int Q = q, j = r;
    double w[16], acc[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) acc[i] = 0.0;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      w[i] = ((i == j ? 1.0 : 0.0) - acc[i]) * rinv[16 * Q + i];
#pragma unroll
      for (int i2 = i + 1; i2 < 16; ++i2) acc[i2] += S[(16 * Q + i2) * LDS_LD + 16 * Q + i] * w[i];
    }
    if (TIMED && tid == 0) ts[12] = __builtin_amdgcn_s_memrealtime();
    if (j < 16) {
#pragma unroll
      for (int i = 0; i < 16; ++i) Wl[(16 * Q + i) * LDS_LD + 16 * Q + j] = (i >= j) ? w[i] : 0.0;
    }
    if (TIMED && tid == 0) ts[13] = __builtin_amdgcn_s_memrealtime();
  }
  __syncthreads();
  if (TIMED && tid == 0) ts[8] = __builtin_amdgcn_s_memrealtime();
  // first pivot that is not a positive finite number (checked by wave 2, idle
  // at level 16): its reciprocal square root is then NaN (d <= 0, NaN or +inf;
  // zero gives 0 * inf) instead of a positive finite number
  if (q == 2) {
    const double ri = rinv[r];
    const unsigned long long bad = __builtin_amdgcn_ballot_w64(!(ri > 0.0 && ri < 1.7976931348623157e308));
    if (r == 0) *fail_sh = bad ? __builtin_ctzll(bad) + 1 : 0x7fffffff;
  }
  // ---- level 16: W(1,0) = -W(1,1) L(1,0) W(0,0) (wave 0), W(3,2) = -W(3,3) L(3,2) W(2,2) (wave 1)
  if (q < 2) {
    const int I = 2 * q + 1, J = 2 * q;
    double* T = tmp + q * 16 * 17;
    d4 t = {0.0, 0.0, 0.0, 0.0};
    mma16x16(t, S + 16 * I * LDS_LD + 16 * J, LDS_LD, Wl + 16 * J * LDS_LD + 16 * J, LDS_LD, true, 1.0, r);
    blk_store(t, T, 17, r);
    __builtin_amdgcn_s_waitcnt(0);
    __builtin_amdgcn_wave_barrier();
    d4 o = {0.0, 0.0, 0.0, 0.0};
    mma16x16(o, Wl + 16 * I * LDS_LD + 16 * I, LDS_LD, T, 17, true, -1.0, r);
    blk_store(o, Wl + 16 * I * LDS_LD + 16 * J, LDS_LD, r);
  }
  __syncthreads();
  if (TIMED && tid == 0) ts[9] = __builtin_amdgcn_s_memrealtime();
  // rows 0..31 of W are final: their global stores overlap the 32-level recursion
  if (Wg) tile_store_rows_dev(Wl, Wg, 64, 0, 32, tid);
  // ---- level 32: U = L21 W11 (one 16 x 16 block per wave), then W21 = -W22 U
  {
    const int I = 2 + (q >> 1), J = q & 1;
    double* U = tmp + q * 16 * 17;
    d4 u = {0.0, 0.0, 0.0, 0.0};
    for (int K = J; K < 2; ++K)
      mma16x16(u, S + 16 * I * LDS_LD + 16 * K, LDS_LD, Wl + 16 * K * LDS_LD + 16 * J, LDS_LD, true, 1.0, r);
    blk_store(u, U, 17, r);
  }
  __syncthreads();
  {
    const int I = 2 + (q >> 1), J = q & 1;
    d4 o = {0.0, 0.0, 0.0, 0.0};
    for (int K = 2; K <= I; ++K)
      mma16x16(o, Wl + 16 * I * LDS_LD + 16 * K, LDS_LD, tmp + (2 * (K - 2) + J) * 16 * 17, 17, true, -1.0, r);
    blk_store(o, Wl + 16 * I * LDS_LD + 16 * J, LDS_LD, r);
  }
  __syncthreads();
  if (TIMED && tid == 0) ts[10] = __builtin_amdgcn_s_memrealtime();
  if (Wg) tile_store_rows_dev(Wl, Wg, 64, 32, 32, tid);
  const int f = *fail_sh;
  return f == 0x7fffffff ? 0 : f;
}

__device__ __forceinline__ int chol_inv_tile_mfma(double* S, double* Wl, double* rinv, double* tmp, int* fail_sh, int tid) {
  return chol_inv_tile_mfma_t<0, false>(S, Wl, rinv, tmp, fail_sh, tid, nullptr);
}

// chol_inv_tile_mfma with the early publication and the global W stores above.
__device__ __forceinline__ int chol_inv_tile_mfma_pub(double* S, double* Wl, double* rinv, double* tmp, int* fail_sh,
                                                      int tid, int* early_flag, double* Wg) {
  return chol_inv_tile_mfma_t<0, false>(S, Wl, rinv, tmp, fail_sh, tid, nullptr, early_flag, Wg);
}

// In-LDS inverse of a lower-triangular 64 x 64 tile by forward substitution on
// the identity: thread (r, q) keeps row r, columns 16q .. 16q+15 of the
// inverse; row k is finished (scaled by 1/L_kk) by lane k of every wave and
// then eliminated from the rows below with cross-lane reads only.
__device__ __forceinline__ void trinv_tile(const double* S, double* w, int tid) {
  const int r = tid & 63, q = tid >> 6;
#pragma unroll
  for (int m = 0; m < 16; ++m) w[m] = (r == 16 * q + m) ? 1.0 : 0.0;
  for (int qo = 0; qo < 4; ++qo) {
#pragma unroll
    for (int m = 0; m < 16; ++m) {
      const int k = 16 * qo + m;
      const double lr = S[r * LDS_LD + k];
      const double inv = 1.0 / S[k * LDS_LD + k];
      if (r == k) {
#pragma unroll
        for (int mm = 0; mm < 16; ++mm) w[mm] *= inv;
      }
      if (q < qo) {
#pragma unroll
        for (int mm = 0; mm < 16; ++mm) {
          const double wk = rd_lane(w[mm], k);
          if (r > k) w[mm] -= lr * wk;
        }
      } else if (q == qo) {
#pragma unroll
        for (int mm = 0; mm <= m; ++mm) {
          const double wk = rd_lane(w[mm], k);
          if (r > k) w[mm] -= lr * wk;
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Cross-workgroup completion flags (one int per tile, 0 = pending).  Producer:
// every wave's stores complete, a barrier, then one thread sets the flag with
// an agent-scope release.  Consumer: one thread polls with relaxed loads, then
// an agent-scope acquire makes the producer's writes visible to the whole
// workgroup (L1 is per CU, L2 per XCD).
__device__ __forceinline__ bool flag_set(const int* flag) {
  return __hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
}

// Spin (thread 0 only) until *flag != 0.  Gives up and raises *abort after
// about `limit` polls, or returns at once if *abort is already raised, so
// that every wave always reaches the end of the kernel.
__device__ __forceinline__ bool spin_wait(const int* flag, int* abort, long long limit) {
  long long polls = 0;
  while (!flag_set(flag)) {
    if (__hip_atomic_load(abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return false;
    __builtin_amdgcn_s_sleep(4);
    if (++polls > limit) {
      __hip_atomic_store(abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return false;
    }
  }
  return true;
}

__device__ __forceinline__ void acquire_fence() { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent"); }

}  // namespace bta
