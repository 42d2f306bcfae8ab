// Triangular solves with the BTA factor (A x = y via L z = y, L^T x = z) and
// the log-determinant 2 * sum log diag(L).  Neither is in the paper; both are
// needed for f(A) = log det A + y^T A^{-1} y and its gradient.
//
// The solve is memory bound (O(n b^2) reads of L per sweep).  Per block row
// and right-hand side, the coupling to the block solved before it (L_{i,i-1}
// z_{i-1} forward; L_{i+1,i}^T x_{i+1} and L_{n,i}^T x_n backward) is a
// matrix-vector product spread over many workgroups (split along the
// reduction, partial sums summed in a fixed order), and the substitution with
// the diagonal block goes tile by tile in one workgroup per right-hand side,
// with the 64 x 64 diagonal tiles applied through their precomputed inverses.
#include <algorithm>

#include "bta_device.hpp"
#include "bta_internal.hpp"

namespace bta {

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

// Compact 64 x 64 inverses of the diagonal tiles of nblk m x m lower-triangular
// blocks: tile t of block blk goes to Wc + (blk*T + t) * 4096 (ld 64).
__global__ __launch_bounds__(NT) void tile_inverses_kernel(const double* L, int64_t m, int64_t sL, int T, double* Wc) {
  __shared__ double S[TS * LDS_LD];
  const int tid = threadIdx.x;
  const int64_t blk = blockIdx.x / T;
  const int t = (int)(blockIdx.x - blk * T);
  const int ext = (int)std::min<int64_t>(64, m - (int64_t)t * 64);
  const double* Lt = L + blk * sL + (int64_t)t * 64 * m + (int64_t)t * 64;
  for (int e = tid; e < 64 * 64; e += NT) {
    const int rr = e >> 6, cc = e & 63;
    double v;
    if (rr < ext && cc < ext) v = (cc <= rr) ? Lt[(int64_t)rr * m + cc] : 0.0;
    else v = (rr == cc) ? 1.0 : 0.0;
    S[rr * LDS_LD + cc] = v;
  }
  __syncthreads();
  double w[16];
  trinv_tile(S, w, tid);
  const int r = tid & 63, q = tid >> 6;
  double* Wt = Wc + (blk * T + t) * 4096;
#pragma unroll
  for (int mm = 0; mm < 16; ++mm) {
    const int c = 16 * q + mm;
    Wt[r * 64 + c] = (c <= r) ? w[mm] : 0.0;
  }
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// out[r] (r < R <= 64) += sign * sum_{k<K} M[r*ld + k] x[k]   (row access, lanes over k).
// Wave w takes rows w, w+4, ..., w+60 together, so the loads of all its rows
// are in flight at once; the per-lane partial sums are then reduced through
// LDS (part: 64 x 65 doubles), four threads per row, instead of one chain of
// cross-lane shuffles per row.  Ends with a barrier.
__device__ void rowdot_acc(const double* M, int64_t ld, int R, int64_t K, const double* x, double* out, double sign,
                           double* part, int tid) {
  const int w = tid >> 6, lane = tid & 63;
  double s[16];
#pragma unroll
  for (int j = 0; j < 16; ++j) s[j] = 0.0;
  // branchless: rows past R read row R-1 and columns past K column 0, and
  // contribute zero (a per-row branch would make the compiler wait for each
  // load before the next); two 64-wide k chunks per trip, so that 32 loads per
  // lane are in flight
  for (int64_t k0 = 0; k0 < K; k0 += 128) {
    const int64_t k1 = k0 + lane, k2 = k0 + 64 + lane;
    const bool in1 = k1 < K, in2 = k2 < K;
    const int64_t ka = in1 ? k1 : 0, kb = in2 ? k2 : 0;
    const double xa = in1 ? x[ka] : 0.0, xb = in2 ? x[kb] : 0.0;
    double ma[16], mb[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const int64_t row = (int64_t)((w + 4 * j) < R ? (w + 4 * j) : R - 1) * ld;
      ma[j] = M[row + ka];
      mb[j] = M[row + kb];
    }
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const double t = ma[j] * xa + mb[j] * xb;
      s[j] += (w + 4 * j < R) ? t : 0.0;
    }
  }
#pragma unroll
  for (int j = 0; j < 16; ++j) part[(w + 4 * j) * 65 + lane] = s[j];
  __syncthreads();
  const int r = tid >> 2, q = tid & 3;
  double t = 0.0;
#pragma unroll
  for (int l = 0; l < 16; ++l) t += part[r * 65 + 16 * q + l];
  t += __shfl_xor(t, 1, 64);
  t += __shfl_xor(t, 2, 64);
  if (q == 0 && r < R) out[r] += sign * t;
  __syncthreads();
}

// out[k] (k < Kc <= 64) += sign * sum_{r<R} M[r*ld + k] x[r]   (column access).
// Sixteen independent partial sums per thread keep sixteen rows' loads in flight.
__device__ void coldot_acc(const double* M, int64_t ld, int64_t R, int Kc, const double* x, double* out, double* red,
                           double sign, int tid) {
  const int k = tid & 63, ph = tid >> 6;
  double s[16];
#pragma unroll
  for (int u = 0; u < 16; ++u) s[u] = 0.0;
  if (k < Kc) {
    int64_t r = ph;
    for (; r + 60 < R; r += 64) {
#pragma unroll
      for (int u = 0; u < 16; ++u) s[u] += M[(r + 4 * u) * ld + k] * x[r + 4 * u];
    }
    for (; r < R; r += 4) s[0] += M[r * ld + k] * x[r];
  }
#pragma unroll
  for (int u = 0; u < 8; ++u) s[u] += s[u + 8];
  red[ph * 64 + k] = ((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7]));
  __syncthreads();
  if (tid < 64 && tid < Kc) out[tid] += sign * (red[tid] + red[64 + tid] + red[128 + tid] + red[192 + tid]);
  __syncthreads();
}

// rowdot_acc over one 64 x 64 tile M (row stride 64) whose elements were
// loaded before: m[j] = M[(w + 4j) * 64 + lane] (wave w, rows w + 4j).
// Rows >= R and columns >= K contribute zero.  Ends with a barrier.
__device__ void rowdot_tile_regs(const double (&m)[16], int R, int K, const double* x, double* out, double sign,
                                 double* part, int tid) {
  const int w = tid >> 6, lane = tid & 63;
  const double xk = lane < K ? x[lane] : 0.0;
#pragma unroll
  for (int j = 0; j < 16; ++j) part[(w + 4 * j) * 65 + lane] = (w + 4 * j < R) ? m[j] * xk : 0.0;
  __syncthreads();
  const int r = tid >> 2, q = tid & 3;
  double t = 0.0;
#pragma unroll
  for (int l = 0; l < 16; ++l) t += part[r * 65 + 16 * q + l];
  t += __shfl_xor(t, 1, 64);
  t += __shfl_xor(t, 2, 64);
  if (q == 0 && r < R) out[r] += sign * t;
  __syncthreads();
}

struct SolveParams {
  int64_t n, b, a, nrhs, N;
  int T, TA;
  const double* LD; const double* LB; const double* LR; const double* LT;
  const double* Wd;  // [n*T] tile inverses
  const double* Wt;  // [TA] tip tile inverses
  double* vec;       // [nrhs][N] contiguous working copies
  double* part;      // [nrhs][SP][b] partial sums of the coupling products
  double* ptip;      // [nrhs][n][a] partial sums of the arrow coupling
  int SF, SB, SR;    // splits: forward (along b), backward L_{i+1,i} and L_{n,i} (64 rows each)
  int64_t SP;        // split capacity per right-hand side
};

__global__ __launch_bounds__(256) void solve_gather_kernel(const double* rhs, int64_t nrhs, int64_t N, double* vec) {
  const int64_t j = blockIdx.y;
  for (int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x; r < N; r += (int64_t)gridDim.x * 256) vec[j * N + r] = rhs[r * nrhs + j];
}
__global__ __launch_bounds__(256) void solve_scatter_kernel(double* rhs, int64_t nrhs, int64_t N, const double* vec) {
  const int64_t j = blockIdx.y;
  for (int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x; r < N; r += (int64_t)gridDim.x * 256) rhs[r * nrhs + j] = vec[j * N + r];
}

// part[j][s][r] = sum over k in split s of L_{i,i-1}[r][k] z_{i-1}[k]; a
// workgroup covers 16 rows (4 per wave, lanes along k), grid (b/16, SF, nrhs).
__global__ __launch_bounds__(256) void solve_fwd_couple_kernel(SolveParams p, int64_t i) {
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t j = blockIdx.z, s = blockIdx.y, b = p.b;
  const int64_t kc = (b + p.SF - 1) / p.SF, k0 = s * kc, k1 = std::min<int64_t>(b, k0 + kc);
  const double* M = p.LB + (i - 1) * b * b;
  const double* x = p.vec + j * p.N + (i - 1) * b;
  const int64_t rbase = (int64_t)blockIdx.x * 16 + 4 * w;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int64_t k = k0 + lane; k < k1; k += 64) {
    const double xk = x[k];
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (rbase + u < b) acc[u] += M[(rbase + u) * b + k] * xk;
  }
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const double t = wave_sum(acc[u]);
    if (lane == 0 && rbase + u < b) p.part[(j * p.SP + s) * b + rbase + u] = t;
  }
}

// ptip[j][i][r] = L_{n,i}[r] . z_i for every block i (grid (n, 1, nrhs)).
__global__ __launch_bounds__(256) void solve_tip_couple_kernel(SolveParams p) {
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t j = blockIdx.z, i = blockIdx.x, b = p.b, a = p.a;
  const double* M = p.LR + i * a * b;
  const double* x = p.vec + j * p.N + i * b;
  for (int64_t r = w; r < a; r += 4) {
    double acc = 0.0;
    for (int64_t k = lane; k < b; k += 64) acc += M[r * b + k] * x[k];
    acc = wave_sum(acc);
    if (lane == 0) p.ptip[(j * p.n + i) * a + r] = acc;
  }
}

// part[j][s][k] = sum over the 64 rows r of split s of M[r][k] x[r], with
// M = L_{i+1,i} and x = x_{i+1} for s < nb, M = L_{n,i} and x = x_n after;
// lanes along k, the four waves over the rows; grid (b/64, splits, nrhs).
__global__ __launch_bounds__(256) void solve_bwd_couple_kernel(SolveParams p, int64_t i, int nb) {
  __shared__ double red[256];
  const int ph = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t j = blockIdx.z, s = blockIdx.y, b = p.b, a = p.a;
  const int64_t k = (int64_t)blockIdx.x * 64 + lane;
  const bool sub = s < nb;
  const double* M = sub ? p.LB + i * b * b : p.LR + i * a * b;
  const double* x = sub ? p.vec + j * p.N + (i + 1) * b : p.vec + j * p.N + p.n * b;
  const int64_t R = sub ? b : a;
  const int64_t r0 = (sub ? s : s - nb) * 64, r1 = std::min<int64_t>(R, r0 + 64);
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  if (k < b) {
    int64_t r = r0 + ph;
    for (; r + 12 < r1; r += 16) {
#pragma unroll
      for (int u = 0; u < 4; ++u) acc[u] += M[(r + 4 * u) * b + k] * x[r + 4 * u];
    }
    for (; r < r1; r += 4) acc[0] += M[r * b + k] * x[r];
  }
  red[threadIdx.x] = (acc[0] + acc[1]) + (acc[2] + acc[3]);
  __syncthreads();
  if (ph == 0 && k < b) p.part[(j * p.SP + s) * b + k] = (red[lane] + red[64 + lane]) + (red[128 + lane] + red[192 + lane]);
}

// Block i forward: z_i = L_ii^{-1} (z_i - sum_s part[s]) (nsplit partials), tile by tile.
// The block's vector is kept in LDS (dynamic, b doubles, b <= 4096), so the
// tile chain does not round-trip through global memory.
__global__ __launch_bounds__(NT, 1) void solve_fwd_diag_kernel(SolveParams p, int64_t i, int nsplit, int in_lds) {
  extern __shared__ double zsh[];
  __shared__ double v[64];
  __shared__ double red[256];
  __shared__ double rpart[64 * 65];
  const int tid = threadIdx.x;
  const int64_t j = blockIdx.x, b = p.b, bb = b * b;
  double* zg = p.vec + j * p.N + i * b;
  double* z = in_lds ? zsh : zg;
  const double* pt = p.part + j * p.SP * b;
  for (int64_t r = tid; r < b; r += NT) {
    double t = 0.0;
    for (int s2 = 0; s2 < nsplit; ++s2) t += pt[s2 * b + r];
    z[r] = zg[r] - t;
  }
  __syncthreads();
  const double* Ld = p.LD + i * bb;
  for (int c = 0; c < p.T; ++c) {
    const int ext = (int)std::min<int64_t>(64, b - (int64_t)c * 64);
    const int64_t r0 = (int64_t)c * 64;
    // the tile's inverse does not depend on z: its loads go out first
    double wr[16];
    const double* Wc = p.Wd + (i * p.T + c) * 4096;
#pragma unroll
    for (int j = 0; j < 16; ++j) wr[j] = Wc[((tid >> 6) + 4 * j) * 64 + (tid & 63)];
    if (tid < 64) v[tid] = tid < ext ? z[r0 + tid] : 0.0;
    __syncthreads();
    if (c > 0) rowdot_acc(Ld + r0 * b, b, ext, r0, z, v, -1.0, rpart, tid);
    if (tid < 64) red[tid] = 0.0;
    __syncthreads();
    rowdot_tile_regs(wr, ext, ext, v, red, 1.0, rpart, tid);
    if (tid < ext) z[r0 + tid] = red[tid];
    __syncthreads();
  }
  if (in_lds)
    for (int64_t r = tid; r < b; r += NT) zg[r] = z[r];
}

// Tip forward: z_n = L_nn^{-1} (z_n - sum_i ptip[i]) (blocks summed in order), then
// the tip backward x_n = L_nn^{-T} z_n.
__global__ __launch_bounds__(NT, 1) void solve_tip_kernel(SolveParams p) {
  __shared__ double v[64];
  __shared__ double red[256];
  __shared__ double red2[256];
  __shared__ double rpart[64 * 65];
  const int tid = threadIdx.x;
  const int64_t j = blockIdx.x, a = p.a, n = p.n;
  double* z = p.vec + j * p.N + n * p.b;
  for (int64_t r = tid; r < a; r += NT) {
    double t = 0.0;
    for (int64_t i = 0; i < n; ++i) t += p.ptip[(j * n + i) * a + r];
    z[r] -= t;
  }
  __syncthreads();
  for (int c = 0; c < p.TA; ++c) {
    const int ext = (int)std::min<int64_t>(64, a - (int64_t)c * 64);
    const int64_t r0 = (int64_t)c * 64;
    if (tid < 64) v[tid] = tid < ext ? z[r0 + tid] : 0.0;
    __syncthreads();
    if (c > 0) rowdot_acc(p.LT + r0 * a, a, ext, r0, z, v, -1.0, rpart, tid);
    __syncthreads();
    if (tid < 64) red[tid] = 0.0;
    __syncthreads();
    rowdot_acc(p.Wt + (int64_t)c * 4096, 64, ext, ext, v, red, 1.0, rpart, tid);
    __syncthreads();
    if (tid < ext) z[r0 + tid] = red[tid];
    __syncthreads();
  }
  for (int c = p.TA - 1; c >= 0; --c) {
    const int ext = (int)std::min<int64_t>(64, a - (int64_t)c * 64);
    const int64_t r0 = (int64_t)c * 64;
    if (tid < 64) v[tid] = tid < ext ? z[r0 + tid] : 0.0;
    __syncthreads();
    const int64_t below = a - (r0 + ext);
    if (below > 0) coldot_acc(p.LT + (r0 + ext) * a + r0, a, below, ext, z + r0 + ext, v, red, -1.0, tid);
    if (tid < 64) red2[tid] = 0.0;
    __syncthreads();
    coldot_acc(p.Wt + (int64_t)c * 4096, 64, ext, ext, v, red2, red, 1.0, tid);
    if (tid < ext) z[r0 + tid] = red2[tid];
    __syncthreads();
  }
}

// Block i backward: x_i = L_ii^{-T} (z_i - sum_s part[s]), tile by tile from the
// last, the block's vector in LDS when it fits (as in the forward).
__global__ __launch_bounds__(NT) void solve_bwd_diag_kernel(SolveParams p, int64_t i, int nsplit, int in_lds) {
  extern __shared__ double zsh[];
  __shared__ double v[64];
  __shared__ double red[256];
  __shared__ double red2[256];
  const int tid = threadIdx.x;
  const int64_t j = blockIdx.x, b = p.b, bb = b * b;
  double* zg = p.vec + j * p.N + i * b;
  double* z = in_lds ? zsh : zg;
  const double* pt = p.part + j * p.SP * b;
  for (int64_t r = tid; r < b; r += NT) {
    double t = 0.0;
    for (int s2 = 0; s2 < nsplit; ++s2) t += pt[s2 * b + r];
    z[r] = zg[r] - t;
  }
  __syncthreads();
  const double* Ld = p.LD + i * bb;
  for (int c = p.T - 1; c >= 0; --c) {
    const int ext = (int)std::min<int64_t>(64, b - (int64_t)c * 64);
    const int64_t r0 = (int64_t)c * 64;
    if (tid < 64) v[tid] = tid < ext ? z[r0 + tid] : 0.0;
    __syncthreads();
    const int64_t below = b - (r0 + ext);
    if (below > 0) coldot_acc(Ld + (r0 + ext) * b + r0, b, below, ext, z + r0 + ext, v, red, -1.0, tid);
    if (tid < 64) red2[tid] = 0.0;
    __syncthreads();
    coldot_acc(p.Wd + (i * p.T + c) * 4096, 64, ext, ext, v, red2, red, 1.0, tid);
    if (tid < ext) z[r0 + tid] = red2[tid];
    __syncthreads();
  }
  if (in_lds)
    for (int64_t r = tid; r < b; r += NT) zg[r] = z[r];
}

static void solve_splits(int64_t b, int64_t a, int& SF, int& SB, int& SR, int64_t& SP) {
  SF = (int)std::max<int64_t>(1, (b + 255) / 256);
  SB = (int)((b + 63) / 64);
  SR = (int)((a + 63) / 64);
  SP = std::max<int64_t>(SF, (int64_t)SB + SR);
}

size_t solve_work_bytes(int64_t n, int64_t b, int64_t a, int64_t nrhs) {
  const int64_t T = (b + 63) / 64, TA = (a + 63) / 64;
  const int64_t N = n * b + a;
  int SF, SB, SR;
  int64_t SP;
  solve_splits(b, a, SF, SB, SR, SP);
  size_t bytes = 0;
  auto take = [&](size_t x) { bytes += (x + 255) & ~size_t(255); };
  take(8 * 4096 * (size_t)(n * T));
  take(8 * 4096 * (size_t)std::max<int64_t>(TA, 1));
  take(8 * (size_t)(N * nrhs));
  take(8 * (size_t)(SP * b * nrhs));
  take(8 * (size_t)std::max<int64_t>(1, n * a * nrhs));
  return bytes;
}

hipError_t solve_launch(int64_t n, int64_t b, int64_t a, const double* LD, const double* LB, const double* LR,
                        const double* LT, double* rhs, int64_t nrhs, void* work, hipStream_t stream) {
  const int64_t T = (b + 63) / 64, TA = (a + 63) / 64;
  char* w = static_cast<char*>(work);
  size_t off = 0;
  auto take = [&](size_t x) { size_t o = off; off += (x + 255) & ~size_t(255); return o; };
  SolveParams p;
  p.n = n; p.b = b; p.a = a; p.nrhs = nrhs; p.N = n * b + a;
  p.T = (int)T; p.TA = (int)TA;
  p.LD = LD; p.LB = LB; p.LR = LR; p.LT = LT;
  solve_splits(b, a, p.SF, p.SB, p.SR, p.SP);
  double* Wd = reinterpret_cast<double*>(w + take(8 * 4096 * (size_t)(n * T)));
  double* Wt = reinterpret_cast<double*>(w + take(8 * 4096 * (size_t)std::max<int64_t>(TA, 1)));
  p.vec = reinterpret_cast<double*>(w + take(8 * (size_t)(p.N * nrhs)));
  p.part = reinterpret_cast<double*>(w + take(8 * (size_t)(p.SP * b * nrhs)));
  p.ptip = reinterpret_cast<double*>(w + take(8 * (size_t)std::max<int64_t>(1, n * a * nrhs)));
  p.Wd = Wd; p.Wt = Wt;
  auto ok = [&]() { return hipGetLastError(); };
  hipLaunchKernelGGL(tile_inverses_kernel, dim3((unsigned)(n * T)), dim3(NT), 0, stream, LD, b, b * b, (int)T, Wd);
  if (hipError_t e = ok()) return e;
  if (a > 0) {
    hipLaunchKernelGGL(tile_inverses_kernel, dim3((unsigned)TA), dim3(NT), 0, stream, LT, a, (int64_t)0, (int)TA, Wt);
    if (hipError_t e = ok()) return e;
  }
  const unsigned gN = (unsigned)std::min<int64_t>(1024, (p.N + 255) / 256);
  // the diagonal-block kernels keep the block's vector in LDS up to b = 4096
  // (32 KB of dynamic LDS, within the default limit)
  const int in_lds = b <= 4096 ? 1 : 0;
  const size_t zbytes = in_lds ? 8 * (size_t)b : 0;
  hipLaunchKernelGGL(solve_gather_kernel, dim3(gN, (unsigned)nrhs), dim3(256), 0, stream, rhs, nrhs, p.N, p.vec);
  if (hipError_t e = ok()) return e;
  // forward over the blocks
  for (int64_t i = 0; i < n; ++i) {
    if (i > 0) {
      hipLaunchKernelGGL(solve_fwd_couple_kernel, dim3((unsigned)((b + 15) / 16), (unsigned)p.SF, (unsigned)nrhs), dim3(256),
                         0, stream, p, i);
      if (hipError_t e = ok()) return e;
    }
    hipLaunchKernelGGL(solve_fwd_diag_kernel, dim3((unsigned)nrhs), dim3(NT), zbytes, stream, p, i, i > 0 ? p.SF : 0, in_lds);
    if (hipError_t e = ok()) return e;
  }
  // the tip, forward then backward
  if (a > 0) {
    hipLaunchKernelGGL(solve_tip_couple_kernel, dim3((unsigned)n, 1, (unsigned)nrhs), dim3(256), 0, stream, p);
    if (hipError_t e = ok()) return e;
    hipLaunchKernelGGL(solve_tip_kernel, dim3((unsigned)nrhs), dim3(NT), 0, stream, p);
    if (hipError_t e = ok()) return e;
  }
  // backward over the blocks
  for (int64_t i = n - 1; i >= 0; --i) {
    const int nb = i < n - 1 ? p.SB : 0;
    const int ns = nb + (a > 0 ? p.SR : 0);
    if (ns > 0) {
      hipLaunchKernelGGL(solve_bwd_couple_kernel, dim3((unsigned)((b + 63) / 64), (unsigned)ns, (unsigned)nrhs), dim3(256), 0,
                         stream, p, i, nb);
      if (hipError_t e = ok()) return e;
    }
    hipLaunchKernelGGL(solve_bwd_diag_kernel, dim3((unsigned)nrhs), dim3(NT), zbytes, stream, p, i, ns, in_lds);
    if (hipError_t e = ok()) return e;
  }
  hipLaunchKernelGGL(solve_scatter_kernel, dim3(gN, (unsigned)nrhs), dim3(256), 0, stream, rhs, nrhs, p.N, p.vec);
  return ok();
}

}  // namespace bta
