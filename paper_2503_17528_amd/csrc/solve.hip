// Triangular solves with the BTA factor (A x = y via L z = y, L^T x = z) and
// the log-determinant 2 * sum log diag(L).  Neither is in the paper; both are
// needed for f(A) = log det A + y^T A^{-1} y and its gradient.
//
// The solve is memory bound (O(n b^2) reads of L per sweep) and sequential in
// the block index.  The diagonal blocks are inverted up front in batched MFMA
// launches (W_i = L_ii^{-1}, the same inverse-factor form as the selected
// inversion), so that every step of both sweeps is a pair of dense
// matrix-vector products spread over many workgroups:
//   forward   t = y_i - L_{i,i-1} z_{i-1},               z_i = W_i t
//   backward  t = z_i - L_{i+1,i}^T x_{i+1} - L_{n,i}^T x_n,  x_i = W_i^T t
// with L_{i+1,i}^T and W_i^T transposed once into the workspace, so that every
// product reads its matrix by rows (lanes along the row, coalesced), and the
// arrow terms, which do not depend on the chain, computed for all blocks at
// once.  Every sum runs in a fixed order (deterministic).
#include <algorithm>

#include "bta_device.hpp"
#include "bta_internal.hpp"

namespace bta {

#define BTA_TRY_E(x)                    \
  do {                                  \
    hipError_t e_ = (x);                \
    if (e_ != hipSuccess) return e_;    \
  } while (0)

// ---------------------------------------------------------------- logdet
__global__ __launch_bounds__(256) void logdet_partial_kernel(const double* LD, const double* LT, int64_t n, int64_t b,
                                                             int64_t a, double* partial) {
  __shared__ double red[256];
  const int64_t blk = blockIdx.x;
  const double* L;
  int64_t m;
  if (blk < n) { L = LD + blk * b * b; m = b; } else { L = LT; m = a; }
  double s = 0.0;
  for (int64_t k = threadIdx.x; k < m; k += 256) s += log(L[k * m + k]);
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blk] = red[0];
}

__global__ __launch_bounds__(256) void logdet_final_kernel(const double* partial, int64_t count, double* out) {
  __shared__ double red[256];
  double s = 0.0;
  for (int64_t k = threadIdx.x; k < count; k += 256) s += partial[k];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = 2.0 * red[0];
}

size_t logdet_work_bytes(int64_t n, int64_t b, int64_t a) { return 8 * (size_t)(n + 1 + 1024) + 256; }

// ---------------------------------------------------------------- quadratic term and gradient

// partial[blk] = sum over a fixed slice of the elementwise product y * x
__global__ __launch_bounds__(256) void dot_partial_kernel(const double* y, const double* x, int64_t count, int nslices,
                                                          double* partial) {
  __shared__ double red[256];
  const int64_t per = (count + nslices - 1) / nslices;
  const int64_t lo = (int64_t)blockIdx.x * per, hi = std::min<int64_t>(count, lo + per);
  double s = 0.0;
  for (int64_t k = lo + threadIdx.x; k < hi; k += 256) s += y[k] * x[k];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// out = 2 * sum(logs) + sum(dots), every partial summed in a fixed order
__global__ __launch_bounds__(256) void logdet_quad_final_kernel(const double* plog, int64_t nlog, const double* pdot,
                                                                int ndot, double* out) {
  __shared__ double red[256];
  double s = 0.0, t = 0.0;
  for (int64_t k = threadIdx.x; k < nlog; k += 256) s += plog[k];
  for (int64_t k = threadIdx.x; k < ndot; k += 256) t += pdot[k];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  const double ls = red[0];
  __syncthreads();
  red[threadIdx.x] = t;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = 2.0 * ls + red[0];
}

hipError_t logdet_quad_launch(int64_t n, int64_t b, int64_t a, const double* LD, const double* LT, const double* y,
                              const double* x, int64_t nrhs, double* out, void* work, hipStream_t stream) {
  double* plog = static_cast<double*>(work);
  double* pdot = plog + (n + 1);
  const int64_t nb = n + (a > 0 ? 1 : 0);
  hipLaunchKernelGGL(logdet_partial_kernel, dim3((unsigned)nb), dim3(256), 0, stream, LD, LT, n, b, a, plog);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t count = (n * b + a) * nrhs;
  const int nslices = (int)std::min<int64_t>(1024, (count + 4095) / 4096);
  hipLaunchKernelGGL(dot_partial_kernel, dim3((unsigned)nslices), dim3(256), 0, stream, y, x, count, nslices, pdot);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(logdet_quad_final_kernel, dim3(1), dim3(256), 0, stream, plog, nb, pdot, nslices, out);
  return hipGetLastError();
}

// G = s * f * (X - sum_j x_j x_j^T) on the pattern (f = 1 for the diagonal and
// tip blocks, 2 for the lower and arrow blocks, which also stand at their
// mirrored positions), gy = 2 s x.  Elementwise: G may alias X.
struct GradParams {
  int64_t n, b, a, nrhs;
  const double* XD; const double* XB; const double* XR; const double* XT;
  const double* x;
  const double* scale;
  double* GD; double* GB; double* GR; double* GT;
  double* gy;
};

__global__ __launch_bounds__(256) void grad_pattern_kernel(GradParams p) {
  const int64_t n = p.n, b = p.b, a = p.a, nr = p.nrhs;
  const int64_t bb = b * b, ab = a * b;
  const int64_t nD = n * bb, nB = (n - 1) * bb, nR = n * ab, nT = a * a, N = n * b + a;
  const int64_t total = nD + nB + nR + nT + (p.gy ? N * nr : 0);
  const double s = p.scale ? *p.scale : 1.0;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    int64_t k = e;
    int64_t row, col;  // global row / column indices into x
    const double* X;
    double* G;
    double f;
    if (k < nD) {
      const int64_t i = k / bb, rc = k - i * bb, r = rc / b, c = rc - r * b;
      row = i * b + r; col = i * b + c; X = p.XD; G = p.GD; f = 1.0;
    } else if ((k -= nD) < nB) {
      const int64_t i = k / bb, rc = k - i * bb, r = rc / b, c = rc - r * b;
      row = (i + 1) * b + r; col = i * b + c; X = p.XB; G = p.GB; f = 2.0;
    } else if ((k -= nB) < nR) {
      const int64_t i = k / ab, rc = k - i * ab, r = rc / b, c = rc - r * b;
      row = n * b + r; col = i * b + c; X = p.XR; G = p.GR; f = 2.0;
    } else if ((k -= nR) < nT) {
      const int64_t r = k / a, c = k - r * a;
      row = n * b + r; col = n * b + c; X = p.XT; G = p.GT; f = 1.0;
    } else {
      k -= nT;
      p.gy[k] = 2.0 * s * p.x[k];
      continue;
    }
    double o = 0.0;
    for (int64_t j = 0; j < nr; ++j) o += p.x[row * nr + j] * p.x[col * nr + j];
    G[k] = s * f * (X[k] - o);
  }
}

hipError_t grad_launch(int64_t n, int64_t b, int64_t a, const double* XD, const double* XB, const double* XR,
                       const double* XT, const double* x, int64_t nrhs, const double* scale, double* GD, double* GB,
                       double* GR, double* GT, double* gy, hipStream_t stream) {
  GradParams p{n, b, a, nrhs, XD, XB, XR, XT, x, scale, GD, GB, GR, GT, gy};
  const int64_t total = n * b * b + (n - 1) * b * b + n * a * b + a * a + (gy ? (n * b + a) * nrhs : 0);
  const unsigned grid = (unsigned)std::min<int64_t>(16384, (total + 255) / 256);
  hipLaunchKernelGGL(grad_pattern_kernel, dim3(grid), dim3(256), 0, stream, p);
  return hipGetLastError();
}

hipError_t logdet_launch(int64_t n, int64_t b, int64_t a, const double* LD, const double* LT, double* out, void* work,
                         hipStream_t stream) {
  double* partial = static_cast<double*>(work);
  const int64_t nb = n + (a > 0 ? 1 : 0);
  hipLaunchKernelGGL(logdet_partial_kernel, dim3((unsigned)nb), dim3(256), 0, stream, LD, LT, n, b, a, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(logdet_final_kernel, dim3(1), dim3(256), 0, stream, partial, nb, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------- solve

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// out[r] = base[r] + sign * sum_k M[r*ld + k] x[k] for the rows of this
// workgroup, batched over blockIdx.y (right-hand sides) and blockIdx.z
// (independent blocks).  tri = 0: k < K; tri = 1 (lower triangular M): only
// k < r0 + rows of the workgroup are read; tri = 2 (upper): only k >= r0.
// Elements of a triangular M outside its triangle must be zero.  base may be
// null (out = sign * sum) and M may be null (K = 0: out = base).
struct MvArgs {
  const double* M; int64_t ld, sMz;
  const double* x; int64_t sxy, sxz;
  const double* base; int64_t sby, sbz;
  double* out; int64_t soy, soz;
  int64_t rows, K;
  int tri;
  double sign;
};

// Wave w takes RPW consecutive rows; its lanes run along k in 64-wide chunks,
// CH chunks per trip, so RPW * CH loads per lane are in flight at once.  Rows
// past the end read the last row and columns past the end read column 0 (both
// inside the matrix) and contribute zero: no per-load branch.
template <int RPW, int CH>
__global__ __launch_bounds__(256) void matvec_rows_kernel(MvArgs p) {
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t y = blockIdx.y, z = blockIdx.z;
  const int64_t r0 = (int64_t)blockIdx.x * (4 * RPW);
  const int64_t rw = r0 + (int64_t)w * RPW;
  int64_t k0 = 0, k1 = p.K;
  if (p.tri == 1) k1 = std::min<int64_t>(p.K, r0 + 4 * RPW);
  if (p.tri == 2) k0 = r0;
  double s[RPW];
#pragma unroll
  for (int j = 0; j < RPW; ++j) s[j] = 0.0;
  if (p.M != nullptr && k1 > k0) {
    const double* M = p.M + z * p.sMz;
    const double* x = p.x + y * p.sxy + z * p.sxz;
    int64_t roff[RPW];
#pragma unroll
    for (int j = 0; j < RPW; ++j) roff[j] = std::min<int64_t>(rw + j, p.rows - 1) * p.ld;
    for (int64_t kb = k0; kb < k1; kb += 64 * CH) {
      double xv[CH];
      int64_t kk[CH];
#pragma unroll
      for (int c = 0; c < CH; ++c) {
        const int64_t k = kb + 64 * c + lane;
        const bool in = k < k1;
        kk[c] = in ? k : 0;
        xv[c] = in ? x[kk[c]] : 0.0;
      }
      double mv[RPW][CH];
#pragma unroll
      for (int j = 0; j < RPW; ++j)
#pragma unroll
        for (int c = 0; c < CH; ++c) mv[j][c] = M[roff[j] + kk[c]];
#pragma unroll
      for (int j = 0; j < RPW; ++j)
#pragma unroll
        for (int c = 0; c < CH; ++c) s[j] = __builtin_fma(mv[j][c], xv[c], s[j]);
    }
  }
#pragma unroll
  for (int j = 0; j < RPW; ++j) {
    const double t = wave_sum(s[j]);
    const int64_t r = rw + j;
    if (lane == 0 && r < p.rows) {
      const double b0 = p.base ? p.base[y * p.sby + z * p.sbz + r] : 0.0;
      p.out[y * p.soy + z * p.soz + r] = b0 + p.sign * t;
    }
  }
}

static hipError_t matvec_rows(const MvArgs& a, int nrhs, int nz, hipStream_t s) {
  if (a.rows <= 0 || nrhs <= 0 || nz <= 0) return hipSuccess;
  // short rows: one row per wave and many workgroups; long rows: two per wave
  if (a.K <= 1024) {
    const unsigned gx = (unsigned)((a.rows + 3) / 4);
    hipLaunchKernelGGL((matvec_rows_kernel<1, 8>), dim3(gx, (unsigned)nrhs, (unsigned)nz), dim3(256), 0, s, a);
  } else {
    const unsigned gx = (unsigned)((a.rows + 7) / 8);
    hipLaunchKernelGGL((matvec_rows_kernel<2, 8>), dim3(gx, (unsigned)nrhs, (unsigned)nz), dim3(256), 0, s, a);
  }
  return hipGetLastError();
}

// dst[z](c, r) = src[z](r, c) for rows x cols matrices (64 x 64 tiles through
// LDS; grid (tiles, 1, nz)).
__global__ __launch_bounds__(256) void transpose_kernel(const double* src, int64_t lds, int64_t ss, double* dst,
                                                        int64_t ldd, int64_t sd, int64_t rows, int64_t cols) {
  __shared__ double tile[64][65];
  const int64_t tc = (cols + 63) / 64;
  const int64_t tr = blockIdx.x / tc, tcol = blockIdx.x - tr * tc;
  const double* S = src + (int64_t)blockIdx.z * ss;
  double* Dm = dst + (int64_t)blockIdx.z * sd;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int rr = w; rr < 64; rr += 4) {
    const int64_t r = tr * 64 + rr, c = tcol * 64 + lane;
    if (r < rows && c < cols) tile[rr][lane] = S[r * lds + c];
  }
  __syncthreads();
  for (int cc = w; cc < 64; cc += 4) {
    const int64_t c = tcol * 64 + cc, r = tr * 64 + lane;
    if (r < rows && c < cols) Dm[c * ldd + r] = tile[lane][cc];
  }
}

static hipError_t transpose_launch(const double* src, int64_t lds, int64_t ss, double* dst, int64_t ldd, int64_t sd,
                                   int64_t rows, int64_t cols, int nz, hipStream_t s) {
  if (rows <= 0 || cols <= 0 || nz <= 0) return hipSuccess;
  const unsigned g = (unsigned)(((rows + 63) / 64) * ((cols + 63) / 64));
  hipLaunchKernelGGL(transpose_kernel, dim3(g, 1, (unsigned)nz), dim3(256), 0, s, src, lds, ss, dst, ldd, sd, rows,
                     cols);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void solve_gather_kernel(const double* rhs, int64_t nrhs, int64_t N, double* vec) {
  const int64_t j = blockIdx.y;
  for (int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x; r < N; r += (int64_t)gridDim.x * 256) vec[j * N + r] = rhs[r * nrhs + j];
}
__global__ __launch_bounds__(256) void solve_scatter_kernel(double* rhs, int64_t nrhs, int64_t N, const double* vec) {
  const int64_t j = blockIdx.y;
  for (int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x; r < N; r += (int64_t)gridDim.x * 256) rhs[r * nrhs + j] = vec[j * N + r];
}

// t[j][r] = vec[j][n*b + r] - sum_i ptip[j][i][r], the blocks summed in order.
__global__ __launch_bounds__(256) void solve_tip_rhs_kernel(const double* vec, int64_t N, int64_t nb, const double* ptip,
                                                            int64_t n, int64_t a, double* t) {
  const int64_t j = blockIdx.y;
  for (int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x; r < a; r += (int64_t)gridDim.x * 256) {
    double acc = 0.0;
    for (int64_t i = 0; i < n; ++i) acc += ptip[(j * n + i) * a + r];
    t[j * a + r] = vec[j * N + nb + r] - acc;
  }
}

// vec[j][i*b + c] -= sum_{r<a} L_{n,i}[r][c] x_n[r] for every block i < n
// (the arrow terms of the backward sweep: x_n is final before it starts).
__global__ __launch_bounds__(256) void solve_arrow_terms_kernel(const double* LR, int64_t n, int64_t b, int64_t a,
                                                                const double* xn, int64_t N, double* vec) {
  const int64_t j = blockIdx.y;
  const int64_t total = n * b;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
    const int64_t i = e / b, c = e - i * b;
    const double* M = LR + i * a * b + c;
    const double* x = xn + j * N;
    double acc = 0.0;
    for (int64_t r = 0; r < a; ++r) acc = __builtin_fma(M[r * b], x[r], acc);
    vec[j * N + e] -= acc;
  }
}

// Workspace layout of one solve.  C blocks per chunk of inverses: the whole
// matrix when the inverses, their transposes and the transposed coupling
// blocks fit in the budget (then each inverse is formed once for both
// sweeps), else chunks that are formed again for the backward sweep.
struct SolvePlan {
  int64_t C, nchunks;
  size_t off_W, off_T1, off_LBt, off_WT, off_WTt, off_vec, off_t, off_t2, off_ptip, bytes;
};

static SolvePlan solve_plan(int64_t n, int64_t b, int64_t a, int64_t nrhs) {
  SolvePlan sp{};
  const size_t per_block = 3 * 8 * (size_t)b * (size_t)b;
  const size_t budget = size_t(2) << 30;
  sp.C = std::max<int64_t>(1, std::min<int64_t>(n, (int64_t)(budget / per_block)));
  sp.nchunks = (n + sp.C - 1) / sp.C;
  const int64_t N = n * b + a;
  size_t off = 0;
  auto take = [&](size_t x) { size_t o = off; off += (std::max<size_t>(x, 8) + 255) & ~size_t(255); return o; };
  const size_t cbb = 8 * (size_t)sp.C * (size_t)b * (size_t)b;
  sp.off_W = take(cbb);
  sp.off_T1 = take(cbb);
  sp.off_LBt = take(cbb);
  sp.off_WT = take(8 * (size_t)(a * a));
  sp.off_WTt = take(8 * (size_t)(a * a));
  sp.off_vec = take(8 * (size_t)(N * nrhs));
  sp.off_t = take(8 * (size_t)(std::max(b, a) * nrhs));
  sp.off_t2 = take(8 * (size_t)(a * nrhs));
  sp.off_ptip = take(8 * (size_t)(n * a * nrhs));
  sp.bytes = off;
  return sp;
}

size_t solve_work_bytes(int64_t n, int64_t b, int64_t a, int64_t nrhs) { return solve_plan(n, b, a, nrhs).bytes; }

hipError_t solve_launch(int64_t n, int64_t b, int64_t a, const double* LD, const double* LB, const double* LR,
                        const double* LT, double* rhs, int64_t nrhs, void* work, hipStream_t stream) {
  const SolvePlan sp = solve_plan(n, b, a, nrhs);
  char* w = static_cast<char*>(work);
  double* W = reinterpret_cast<double*>(w + sp.off_W);
  double* T1 = reinterpret_cast<double*>(w + sp.off_T1);   // TRTRI scratch, then W_i^T
  double* LBt = reinterpret_cast<double*>(w + sp.off_LBt);
  double* WT = reinterpret_cast<double*>(w + sp.off_WT);
  double* WTt = reinterpret_cast<double*>(w + sp.off_WTt);
  double* vec = reinterpret_cast<double*>(w + sp.off_vec);
  double* tb = reinterpret_cast<double*>(w + sp.off_t);
  double* t2 = reinterpret_cast<double*>(w + sp.off_t2);
  double* ptip = reinterpret_cast<double*>(w + sp.off_ptip);
  const int64_t N = n * b + a, bb = b * b, ab = a * b;
  const int nr = (int)nrhs;
  const int64_t tstride = std::max(b, a);
  auto ok = [&]() { return hipGetLastError(); };

  const unsigned gN = (unsigned)std::min<int64_t>(1024, (N + 255) / 256);
  hipLaunchKernelGGL(solve_gather_kernel, dim3(gN, (unsigned)nrhs), dim3(256), 0, stream, rhs, nrhs, N, vec);
  if (hipError_t e = ok()) return e;

  auto invert_chunk = [&](int64_t i0, int64_t cnt) -> hipError_t {
    BTA_TRY_E(fill_zero_launch(W, (size_t)(cnt * bb), stream));
    return trtri_batched(LD + i0 * bb, b, bb, W, T1, b, bb, (int)b, (int)cnt, stream, 0, 0);
  };

  // ---- forward: z_i = W_i (y_i - L_{i,i-1} z_{i-1})
  for (int64_t c = 0; c < sp.nchunks; ++c) {
    const int64_t i0 = c * sp.C, cnt = std::min<int64_t>(sp.C, n - i0);
    BTA_TRY_E(invert_chunk(i0, cnt));
    for (int64_t i = i0; i < i0 + cnt; ++i) {
      MvArgs cp{};
      cp.M = i > 0 ? LB + (i - 1) * bb : nullptr; cp.ld = b;
      cp.x = vec + (i - 1) * b; cp.sxy = N;
      cp.base = vec + i * b; cp.sby = N;
      cp.out = tb; cp.soy = tstride;
      cp.rows = b; cp.K = i > 0 ? b : 0; cp.tri = 0; cp.sign = -1.0;
      BTA_TRY_E(matvec_rows(cp, nr, 1, stream));
      MvArgs ap{};
      ap.M = W + (i - i0) * bb; ap.ld = b;
      ap.x = tb; ap.sxy = tstride;
      ap.out = vec + i * b; ap.soy = N;
      ap.rows = b; ap.K = b; ap.tri = 1; ap.sign = 1.0;
      BTA_TRY_E(matvec_rows(ap, nr, 1, stream));
    }
  }

  // ---- the tip: z_n = W_T (y_n - sum_i L_{n,i} z_i), x_n = W_T^T z_n, then
  // the arrow terms of every block's backward right-hand side
  if (a > 0) {
    MvArgs pp{};
    pp.M = LR; pp.ld = b; pp.sMz = ab;
    pp.x = vec; pp.sxy = N; pp.sxz = b;
    pp.out = ptip; pp.soy = n * a; pp.soz = a;
    pp.rows = a; pp.K = b; pp.tri = 0; pp.sign = 1.0;
    BTA_TRY_E(matvec_rows(pp, nr, (int)n, stream));
    hipLaunchKernelGGL(solve_tip_rhs_kernel, dim3((unsigned)((a + 255) / 256), (unsigned)nrhs), dim3(256), 0, stream, vec,
                       N, n * b, ptip, n, a, t2);
    if (hipError_t e = ok()) return e;
    BTA_TRY_E(fill_zero_launch(WT, (size_t)(a * a), stream));
    BTA_TRY_E(trtri_batched(LT, a, 0, WT, WTt, a, 0, (int)a, 1, stream, 0, 0));
    BTA_TRY_E(transpose_launch(WT, a, 0, WTt, a, 0, a, a, 1, stream));
    MvArgs fz{};
    fz.M = WT; fz.ld = a;
    fz.x = t2; fz.sxy = a;
    fz.out = tb; fz.soy = tstride;
    fz.rows = a; fz.K = a; fz.tri = 1; fz.sign = 1.0;
    BTA_TRY_E(matvec_rows(fz, nr, 1, stream));
    MvArgs bx{};
    bx.M = WTt; bx.ld = a;
    bx.x = tb; bx.sxy = tstride;
    bx.out = vec + n * b; bx.soy = N;
    bx.rows = a; bx.K = a; bx.tri = 2; bx.sign = 1.0;
    BTA_TRY_E(matvec_rows(bx, nr, 1, stream));
    const unsigned g = (unsigned)std::min<int64_t>(4096, (n * b + 255) / 256);
    hipLaunchKernelGGL(solve_arrow_terms_kernel, dim3(g, (unsigned)nrhs), dim3(256), 0, stream, LR, n, b, a, vec + n * b, N,
                       vec);
    if (hipError_t e = ok()) return e;
  }

  // ---- backward: x_i = W_i^T (z_i - L_{n,i}^T x_n - L_{i+1,i}^T x_{i+1})
  for (int64_t c = sp.nchunks - 1; c >= 0; --c) {
    const int64_t i0 = c * sp.C, cnt = std::min<int64_t>(sp.C, n - i0);
    if (sp.nchunks > 1) BTA_TRY_E(invert_chunk(i0, cnt));
    BTA_TRY_E(transpose_launch(W, b, bb, T1, b, bb, b, b, (int)cnt, stream));
    const int64_t nsub = std::min<int64_t>(cnt, (n - 1) - i0);
    if (nsub > 0) BTA_TRY_E(transpose_launch(LB + i0 * bb, b, bb, LBt, b, bb, b, b, (int)nsub, stream));
    for (int64_t i = i0 + cnt - 1; i >= i0; --i) {
      MvArgs cp{};
      cp.M = i < n - 1 ? LBt + (i - i0) * bb : nullptr; cp.ld = b;
      cp.x = vec + (i + 1) * b; cp.sxy = N;
      cp.base = vec + i * b; cp.sby = N;
      cp.out = tb; cp.soy = tstride;
      cp.rows = b; cp.K = i < n - 1 ? b : 0; cp.tri = 0; cp.sign = -1.0;
      BTA_TRY_E(matvec_rows(cp, nr, 1, stream));
      MvArgs ap{};
      ap.M = T1 + (i - i0) * bb; ap.ld = b;
      ap.x = tb; ap.sxy = tstride;
      ap.out = vec + i * b; ap.soy = N;
      ap.rows = b; ap.K = b; ap.tri = 2; ap.sign = 1.0;
      BTA_TRY_E(matvec_rows(ap, nr, 1, stream));
    }
  }
  hipLaunchKernelGGL(solve_scatter_kernel, dim3(gN, (unsigned)nrhs), dim3(256), 0, stream, rhs, nrhs, N, vec);
  return ok();
}

}  // namespace bta
