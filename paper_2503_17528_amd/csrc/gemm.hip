// Grouped, batched FP64 MFMA GEMM over 64 x 64 output tiles:
//   Cout = beta * Cin + alpha * sum_seg sum_k A(m,k) B(c,k)
// with either operand stored k-contiguous or m-contiguous, k ranges clipped
// to the nonzero part of a triangular operand, and lower-triangle or
// lower-plus-mirror stores for symmetric results.  Used by the selected
// inversion for its products with the inverses of the diagonal factor blocks
// (TRMM/LAUUM/TRTRI steps) and the two GEMMs of each backward step.
#include <algorithm>

#include "bta_device.hpp"
#include "bta_internal.hpp"

namespace bta {

__device__ __forceinline__ void seg_krange(const GSeg& s, int tm, int tn, int& k0, int& k1) {
  k0 = 0;
  k1 = s.K;
  switch (s.tri) {
    case TRI_K_GE_COL: k0 = tn * 64; break;
    case TRI_K_GE_ROW: k0 = tm * 64; break;
    case TRI_K_LE_ROW: k1 = min(s.K, (tm + 1) * 64); break;
    case TRI_K_LE_COL: k1 = min(s.K, (tn + 1) * 64); break;
    default: break;
  }
  if (k0 > k1) k0 = k1;
}

__device__ __forceinline__ OpTile op_tile(const double* base, int64_t ld, int trans, int m0, int mext, int k, int kext) {
  if (!trans) return OpTile{base + (int64_t)m0 * ld + k, ld, mext, kext, false};
  return OpTile{base + (int64_t)k * ld + m0, ld, mext, kext, true};
}

__global__ __launch_bounds__(NT, 2) void gemm_kernel(GemmArgs args) {
  __shared__ double As[TS * LDS_LD];
  __shared__ double Bs[TS * LDS_LD];
  const int tid = threadIdx.x;
  const long long t = blockIdx.x;
  int j = 0;
  while (j + 1 < args.nprob && t >= args.p[j + 1].tile_begin) ++j;
  const GProb& P = args.p[j];
  const long long local = t - P.tile_begin;
  const int batch = (int)(local / P.tiles_per_batch);
  int tile = (int)(local - (long long)batch * P.tiles_per_batch);
  const int b0 = batch / P.nb1, b1 = batch - b0 * P.nb1;
  int tm, tn;
  if (P.lower_tiles) {
    // tile -> (tm, tn), tm >= tn, row by row
    tm = (int)((sqrt(8.0 * tile + 1.0) - 1.0) * 0.5);
    while ((tm + 1) * (tm + 2) / 2 <= tile) ++tm;
    while (tm * (tm + 1) / 2 > tile) --tm;
    tn = tile - tm * (tm + 1) / 2;
  } else {
    tm = tile / P.ntn;
    tn = tile - tm * P.ntn;
  }
  const int mext = min(64, P.M - tm * 64), next = min(64, P.N - tn * 64);

  // flattened k tiles over the segments
  int kbeg[2], kend[2], nk[2];
  const double* Ab[2];
  const double* Bb[2];
  for (int s = 0; s < 2; ++s) {
    nk[s] = 0;
    if (s < P.nseg) {
      seg_krange(P.seg[s], tm, tn, kbeg[s], kend[s]);
      nk[s] = (kend[s] - kbeg[s] + 63) / 64;
      Ab[s] = P.seg[s].A + b0 * P.seg[s].sA0 + b1 * P.seg[s].sA1;
      Bb[s] = P.seg[s].B + b0 * P.seg[s].sB0 + b1 * P.seg[s].sB1;
    }
  }
  const int total = nk[0] + nk[1];

  Acc acc;
  acc_zero(acc);
  Stage ra, rb;
  auto load = [&](int kk) {
    const int s = kk < nk[0] ? 0 : 1;
    const int q = s == 0 ? kk : kk - nk[0];
    const int k = kbeg[s] + q * 64;
    const int kext = min(64, kend[s] - k);
    const GSeg& g = P.seg[s];
    stage_load(ra, op_tile(Ab[s], g.lda, g.at, tm * 64, mext, k, kext), tid);
    stage_load(rb, op_tile(Bb[s], g.ldb, g.bt, tn * 64, next, k, kext), tid);
  };
  if (total > 0) load(0);
  for (int kk = 0; kk < total; ++kk) {
    const int s = kk < nk[0] ? 0 : 1;
    __syncthreads();
    stage_store(ra, As, P.seg[s].at != 0, tid);
    stage_store(rb, Bs, P.seg[s].bt != 0, tid);
    __syncthreads();
    if (kk + 1 < total) load(kk + 1);
    mma_tile(acc, As, Bs, tid);
  }

  // epilogue: final values first (Cin may alias Cout), then the stores
  double* C = P.Cout + b0 * P.sC0 + b1 * P.sC1 + (int64_t)tm * 64 * P.ldc + tn * 64;
  const double* Ci = P.Cin ? P.Cin + b0 * P.sC0 + b1 * P.sC1 + (int64_t)tm * 64 * P.ldc + tn * 64 : nullptr;
  const bool diag_tile = (tm == tn);
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int r = tile_row(tid, bi, e), c = tile_col(tid, bj);
        double v = P.alpha * acc.v[bi][bj][e];
        const bool live = r < mext && c < next && !(P.store != ST_FULL && diag_tile && c > r);
        if (live && P.beta != 0.0) v += P.beta * Ci[(int64_t)r * P.ldc + c];
        acc.v[bi][bj][e] = v;
      }
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int r = tile_row(tid, bi, e), c = tile_col(tid, bj);
        if (r >= mext || c >= next) continue;
        if (P.store != ST_FULL && diag_tile && c > r) continue;
        C[(int64_t)r * P.ldc + c] = acc.v[bi][bj][e];
      }
  if (P.store == ST_LOWER_MIRROR) {
    // mirror into the transposed position (c, r) of the global matrix
    double* Ct = P.Cout + b0 * P.sC0 + b1 * P.sC1 + (int64_t)tn * 64 * P.ldc + tm * 64;
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
      for (int bj = 0; bj < 2; ++bj)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int r = tile_row(tid, bi, e), c = tile_col(tid, bj);
          if (r >= mext || c >= next) continue;
          if (diag_tile && c >= r) continue;
          Ct[(int64_t)c * P.ldc + r] = acc.v[bi][bj][e];
        }
  }
}

thread_local DryRecorder* g_dry = nullptr;

// ---------------------------------------------------------------- kernel timer
namespace {
struct KernelTimer {
  bool on = false;
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  std::vector<std::pair<int, std::pair<size_t, size_t>>> spans;  // (kind, (start event, stop event))
  size_t open_start[KT_COUNT] = {0, 0, 0, 0};
};
KernelTimer g_timer;
}  // namespace

bool timing_on() { return g_timer.on; }

void timing_mark(int kind, bool start, hipStream_t stream) {
  if (!g_timer.on || g_timer.used >= g_timer.pool.size()) return;
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
        g_dry->windows.push_back(g.at ? Window{A, g.K, p.M, g.lda, false} : Window{A, p.M, g.K, g.lda, false});
        g_dry->windows.push_back(g.bt ? Window{B, g.K, p.N, g.ldb, false} : Window{B, p.N, g.K, g.ldb, false});
      }
      const int64_t off = b0 * p.sC0 + b1 * p.sC1;
      if (p.beta != 0.0) g_dry->windows.push_back(Window{p.Cin + off, p.M, p.N, p.ldc, false});
      g_dry->windows.push_back(Window{p.Cout + off, p.M, p.N, p.ldc, true});
      if (p.store == ST_LOWER_MIRROR) g_dry->windows.push_back(Window{p.Cout + off, p.N, p.M, p.ldc, true});
    }
}

hipError_t gemm_launch(GProb* probs, int nprob, hipStream_t stream) {
  if (g_dry) {
    for (int i = 0; i < nprob; ++i)
      if (probs[i].M > 0 && probs[i].N > 0) record_gemm(probs[i]);
    return hipSuccess;
  }
  GemmArgs args{};
  args.nprob = 0;
  long long total = 0;
  for (int i = 0; i < nprob; ++i) {
    GProb p = probs[i];
    if (p.M <= 0 || p.N <= 0 || p.nb0 <= 0 || p.nb1 <= 0) continue;
    p.ntm = (p.M + 63) / 64;
    p.ntn = (p.N + 63) / 64;
    p.tiles_per_batch = p.lower_tiles ? p.ntm * (p.ntm + 1) / 2 : p.ntm * p.ntn;
    p.tile_begin = total;
    total += (long long)p.tiles_per_batch * p.nb0 * p.nb1;
    args.p[args.nprob++] = p;
    if (args.nprob == GEMM_MAX_PROBS) break;
  }
  args.ntiles = total;
  if (total == 0) return hipSuccess;
  timing_mark(KT_GEMM, true, stream);
  hipLaunchKernelGGL(gemm_kernel, dim3((unsigned)total), dim3(NT), 0, stream, args);
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
  if (g_dry) {
    for (int blk = 0; blk < nblk; ++blk) {
      g_dry->windows.push_back(Window{L + blk * sL, m, m, ldL, false});
      g_dry->windows.push_back(Window{W + blk * sW, m, m, ldW, true});
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
  if (g_dry) {
    g_dry->windows.push_back(Window{p, 1, (int64_t)count, (int64_t)count, true});
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
  const long long total = (long long)rows * cols;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (long long)gridDim.x * blockDim.x) {
    const int r = (int)(e / cols), c = (int)(e - (long long)r * cols);
    d[(int64_t)r * ldd + c] = s[(int64_t)r * lds + c];
  }
}

hipError_t copy2d_launch(const double* src, int64_t lds, int64_t ss, double* dst, int64_t ldd, int64_t sd,
                         int rows, int cols, int nb, hipStream_t stream) {
  if (rows <= 0 || cols <= 0 || nb <= 0) return hipSuccess;
  if (g_dry) {
    for (int b = 0; b < nb; ++b) {
      g_dry->windows.push_back(Window{src + b * ss, rows, cols, lds, false});
      g_dry->windows.push_back(Window{dst + b * sd, rows, cols, ldd, true});
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

// Internal timing controls (not part of the public header): enable with a
// pool of event pairs, read back per-kind total milliseconds and launch counts.
extern "C" __attribute__((visibility("default"))) int bta_internal_timing(int on, int max_launches) {
  using namespace bta;
  for (hipEvent_t e : g_timer.pool) (void)hipEventDestroy(e);
  g_timer.pool.clear();
  g_timer.spans.clear();
  g_timer.used = 0;
  g_timer.on = false;
  if (!on) return 0;
  g_timer.pool.resize((size_t)2 * max_launches);
  for (auto& e : g_timer.pool)
    if (hipEventCreate(&e) != hipSuccess) return 1;
  g_timer.on = true;
  return 0;
}

extern "C" __attribute__((visibility("default"))) int bta_internal_timing_read(double* ms, long long* launches) {
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
