// C ABI entry points (include/bta.h): argument validation, workspace sizing,
// dispatch to the launchers.  Validation happens before any HIP call, so the
// argument checks work on a host without a GPU.
#include <algorithm>
#include <map>
#include <mutex>
#include <utility>
#include <vector>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>

#include "../../include/bta.h"
#include "bta_internal.hpp"

namespace {

thread_local std::string g_last_error;

bta_status fail(bta_status code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
bta_status fail(bta_status code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

bta_status hip_fail(hipError_t e, const char* where) {
  return fail(BTA_EHIP, "%s: %s", where, hipGetErrorString(e));
}

bool dims_ok(int64_t n, int64_t b, int64_t a) {
  if (n < 1 || b < 1 || a < 0) return false;
  // 32-bit tile bookkeeping inside the kernels
  if (b > (1 << 20) || a > (1 << 20) || n > (1LL << 30)) return false;
  return true;
}

struct Arr {
  const void* p;
  size_t bytes;
  const char* name;
};

// Every array present must be non-null and 8-byte aligned; arrays may
// coincide exactly only within an (input, output) pair; any other overlap is
// an error.
bta_status check_arrays(const Arr* arr, int count, const int* pair_of) {
  for (int i = 0; i < count; ++i) {
    if (arr[i].bytes == 0) continue;
    if (!arr[i].p) return fail(BTA_EINVAL, "%s is NULL", arr[i].name);
    if (reinterpret_cast<uintptr_t>(arr[i].p) & 7) return fail(BTA_EINVAL, "%s is not 8-byte aligned", arr[i].name);
  }
  for (int i = 0; i < count; ++i) {
    for (int j = i + 1; j < count; ++j) {
      if (arr[i].bytes == 0 || arr[j].bytes == 0) continue;
      const uintptr_t a0 = reinterpret_cast<uintptr_t>(arr[i].p), a1 = a0 + arr[i].bytes;
      const uintptr_t b0 = reinterpret_cast<uintptr_t>(arr[j].p), b1 = b0 + arr[j].bytes;
      const bool overlap = a0 < b1 && b0 < a1;
      if (!overlap) continue;
      const bool exact_pair = (pair_of[i] == j || pair_of[j] == i) && a0 == b0 && arr[i].bytes == arr[j].bytes;
      if (!exact_pair) return fail(BTA_EINVAL, "%s overlaps %s", arr[i].name, arr[j].name);
    }
  }
  return BTA_OK;
}

bta_status device_ok() {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  hipDeviceProp_t prop;
  e = hipGetDeviceProperties(&prop, dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(BTA_ENOTSUP, "device %d is %s; this library is built for gfx950", dev, prop.gcnArchName);
  return BTA_OK;
}

size_t blk_bytes(int64_t count, int64_t r, int64_t c) { return (size_t)std::max<int64_t>(count, 0) * r * c * 8; }

bta_status check_work(void* work, size_t work_bytes, size_t need) {
  if (need == 0) return BTA_OK;
  if (!work) return fail(BTA_EINVAL, "workspace is NULL (%zu bytes needed)", need);
  if (reinterpret_cast<uintptr_t>(work) & 255) return fail(BTA_EINVAL, "workspace must be 256-byte aligned");
  if (work_bytes < need) return fail(BTA_EINVAL, "workspace too small: %zu < %zu bytes", work_bytes, need);
  return BTA_OK;
}

}  // namespace

// Fixed device scratch of bta_factor_noalloc: one copy per device, created
// when the library's code object is loaded on that device and kept until the
// process ends.  Host code never passes `scratch` itself to a kernel (its
// host-side name is not a device address): it takes the device address from
// hipGetSymbolAddress, once per device, and passes that.
static __device__ __align__(256) unsigned char scratch[BTA_NOALLOC_SCRATCH_BYTES];

namespace {

std::mutex g_scratch_mu;
std::map<int, void*> g_scratch_addr;  // device ordinal -> address of that device's `scratch`

// The current device's address of `scratch` (looked up on first use, with
// that device current).
bta_status scratch_address(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_addr.find(dev);
  if (it != g_scratch_addr.end()) {
    *out = it->second;
    return BTA_OK;
  }
  void* ptr = nullptr;
  e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
  if (!ptr || (reinterpret_cast<uintptr_t>(ptr) & 255)) return fail(BTA_EHIP, "scratch address %p is not 256-byte aligned", ptr);
  g_scratch_addr[dev] = ptr;
  *out = ptr;
  return BTA_OK;
}

// Argument checks shared by bta_factor and bta_factor_noalloc.
bta_status factor_args(int64_t n, int64_t b, int64_t a, const double* D, const double* B, const double* R, const double* T,
                       double* LD, double* LB, double* LR, double* LT, int64_t* d_info) {
  if (!dims_ok(n, b, a)) return fail(BTA_EINVAL, "invalid sizes n=%lld b=%lld a=%lld", (long long)n, (long long)b, (long long)a);
  const Arr arr[9] = {
      {D, blk_bytes(n, b, b), "D"},        {B, blk_bytes(n - 1, b, b), "B"}, {R, blk_bytes(n, a, b), "R"},
      {T, blk_bytes(1, a, a), "T"},        {LD, blk_bytes(n, b, b), "LD"},   {LB, blk_bytes(n - 1, b, b), "LB"},
      {LR, blk_bytes(n, a, b), "LR"},      {LT, blk_bytes(1, a, a), "LT"},   {d_info, 8, "d_info"}};
  const int pair[9] = {4, 5, 6, 7, 0, 1, 2, 3, -1};
  return check_arrays(arr, 9, pair);
}

}  // namespace

extern "C" {

size_t bta_workspace_bytes(int op, int64_t n, int64_t b, int64_t a, int64_t nrhs) {
  if (!dims_ok(n, b, a)) return 0;
  switch (op) {
    case BTA_OP_FACTOR: return bta::factor_plan(n, b, a).bytes;
    case BTA_OP_SELINV: return bta::selinv_plan(n, b, a).bytes;
    case BTA_OP_SOLVE: return nrhs >= 1 ? bta::solve_work_bytes(n, b, a, nrhs) : 0;
    case BTA_OP_LOGDET: return bta::logdet_work_bytes(n, b, a);
    default: return 0;
  }
}

bta_status bta_factor(int64_t n, int64_t b, int64_t a, const double* D, const double* B, const double* R, const double* T,
               double* LD, double* LB, double* LR, double* LT, void* work, size_t work_bytes, int64_t* d_info,
               bta_stream_t stream) {
  bta_status st = factor_args(n, b, a, D, B, R, T, LD, LB, LR, LT, d_info);
  if (st) return st;
  const bta::FactorPlan fp = bta::factor_plan(n, b, a);
  st = check_work(work, work_bytes, fp.bytes);
  if (st) return st;
  st = device_ok();
  if (st) return st;
  hipError_t e = bta::factor_launch(fp, n, b, a, D, B, R, T, LD, LB, LR, LT, work, d_info,
                                    reinterpret_cast<hipStream_t>(stream), bta::device_cu_count());
  return e == hipSuccess ? BTA_OK : hip_fail(e, "bta_factor launch");
}

bta_status bta_factor_noalloc(int64_t n, int64_t b, int64_t a, const double* D, const double* B, const double* R,
                              const double* T, double* LD, double* LB, double* LR, double* LT, int64_t* d_info,
                              bta_stream_t stream) {
  bta_status st = factor_args(n, b, a, D, B, R, T, LD, LB, LR, LT, d_info);
  if (st) return st;
  const bta::FactorPlan fp = bta::factor_plan(n, b, a);
  if (fp.bytes > (size_t)BTA_NOALLOC_SCRATCH_BYTES)
    return fail(BTA_EINVAL, "bta_factor_noalloc: n=%lld b=%lld a=%lld needs %zu bytes of scratch, above the fixed %zu "
                "(use bta_factor with a workspace)", (long long)n, (long long)b, (long long)a, fp.bytes,
                (size_t)BTA_NOALLOC_SCRATCH_BYTES);
  st = device_ok();
  if (st) return st;
  void* ptr = nullptr;
  st = scratch_address(&ptr);
  if (st) return st;
  hipError_t e = bta::factor_launch(fp, n, b, a, D, B, R, T, LD, LB, LR, LT, ptr, d_info,
                                    reinterpret_cast<hipStream_t>(stream), bta::device_cu_count());
  return e == hipSuccess ? BTA_OK : hip_fail(e, "bta_factor_noalloc launch");
}

bta_status bta_selinv(int64_t n, int64_t b, int64_t a, const double* LD, const double* LB, const double* LR, const double* LT,
               double* XD, double* XB, double* XR, double* XT, void* work, size_t work_bytes, bta_stream_t stream) {
  if (!dims_ok(n, b, a)) return fail(BTA_EINVAL, "invalid sizes n=%lld b=%lld a=%lld", (long long)n, (long long)b, (long long)a);
  const Arr arr[8] = {
      {LD, blk_bytes(n, b, b), "LD"}, {LB, blk_bytes(n - 1, b, b), "LB"}, {LR, blk_bytes(n, a, b), "LR"},
      {LT, blk_bytes(1, a, a), "LT"}, {XD, blk_bytes(n, b, b), "XD"},     {XB, blk_bytes(n - 1, b, b), "XB"},
      {XR, blk_bytes(n, a, b), "XR"}, {XT, blk_bytes(1, a, a), "XT"}};
  const int pair[8] = {4, 5, 6, 7, 0, 1, 2, 3};
  bta_status st = check_arrays(arr, 8, pair);
  if (st) return st;
  const bta::SelinvPlan sp = bta::selinv_plan(n, b, a);
  st = check_work(work, work_bytes, sp.bytes);
  if (st) return st;
  st = device_ok();
  if (st) return st;
  hipError_t e = bta::selinv_launch(sp, n, b, a, LD, LB, LR, LT, XD, XB, XR, XT, work, reinterpret_cast<hipStream_t>(stream));
  return e == hipSuccess ? BTA_OK : hip_fail(e, "bta_selinv launch");
}

bta_status bta_solve(int64_t n, int64_t b, int64_t a, const double* LD, const double* LB, const double* LR, const double* LT,
              double* rhs, int64_t nrhs, void* work, size_t work_bytes, bta_stream_t stream) {
  if (!dims_ok(n, b, a)) return fail(BTA_EINVAL, "invalid sizes n=%lld b=%lld a=%lld", (long long)n, (long long)b, (long long)a);
  if (nrhs < 1 || nrhs > (1 << 20)) return fail(BTA_EINVAL, "invalid nrhs=%lld", (long long)nrhs);
  const int64_t N = n * b + a;
  const Arr arr[5] = {{LD, blk_bytes(n, b, b), "LD"}, {LB, blk_bytes(n - 1, b, b), "LB"}, {LR, blk_bytes(n, a, b), "LR"},
                      {LT, blk_bytes(1, a, a), "LT"}, {rhs, blk_bytes(1, N, nrhs), "rhs"}};
  const int pair[5] = {-1, -1, -1, -1, -1};
  bta_status st = check_arrays(arr, 5, pair);
  if (st) return st;
  st = check_work(work, work_bytes, bta::solve_work_bytes(n, b, a, nrhs));
  if (st) return st;
  st = device_ok();
  if (st) return st;
  hipError_t e = bta::solve_launch(n, b, a, LD, LB, LR, LT, rhs, nrhs, work, reinterpret_cast<hipStream_t>(stream));
  return e == hipSuccess ? BTA_OK : hip_fail(e, "bta_solve launch");
}

bta_status bta_logdet(int64_t n, int64_t b, int64_t a, const double* LD, const double* LT, double* d_out, void* work,
               size_t work_bytes, bta_stream_t stream) {
  if (!dims_ok(n, b, a)) return fail(BTA_EINVAL, "invalid sizes n=%lld b=%lld a=%lld", (long long)n, (long long)b, (long long)a);
  const Arr arr[3] = {{LD, blk_bytes(n, b, b), "LD"}, {LT, blk_bytes(1, a, a), "LT"}, {d_out, 8, "d_out"}};
  const int pair[3] = {-1, -1, -1};
  bta_status st = check_arrays(arr, 3, pair);
  if (st) return st;
  st = check_work(work, work_bytes, bta::logdet_work_bytes(n, b, a));
  if (st) return st;
  st = device_ok();
  if (st) return st;
  hipError_t e = bta::logdet_launch(n, b, a, LD, LT, d_out, work, reinterpret_cast<hipStream_t>(stream));
  return e == hipSuccess ? BTA_OK : hip_fail(e, "bta_logdet launch");
}

bta_status bta_logdet_quad(int64_t n, int64_t b, int64_t a, const double* LD, const double* LT, const double* y, const double* x,
                    int64_t nrhs, double* d_out, void* work, size_t work_bytes, bta_stream_t stream) {
  if (!dims_ok(n, b, a)) return fail(BTA_EINVAL, "invalid sizes n=%lld b=%lld a=%lld", (long long)n, (long long)b, (long long)a);
  if (nrhs < 1 || nrhs > (1 << 20)) return fail(BTA_EINVAL, "invalid nrhs=%lld", (long long)nrhs);
  const int64_t N = n * b + a;
  const Arr arr[5] = {{LD, blk_bytes(n, b, b), "LD"}, {LT, blk_bytes(1, a, a), "LT"}, {y, blk_bytes(1, N, nrhs), "y"},
                      {x, blk_bytes(1, N, nrhs), "x"}, {d_out, 8, "d_out"}};
  const int pair[5] = {-1, -1, 3, 2, -1};  // y and x may coincide (f = logdet + y^T y)
  bta_status st = check_arrays(arr, 5, pair);
  if (st) return st;
  st = check_work(work, work_bytes, bta::logdet_work_bytes(n, b, a));
  if (st) return st;
  st = device_ok();
  if (st) return st;
  hipError_t e = bta::logdet_quad_launch(n, b, a, LD, LT, y, x, nrhs, d_out, work, reinterpret_cast<hipStream_t>(stream));
  return e == hipSuccess ? BTA_OK : hip_fail(e, "bta_logdet_quad launch");
}

bta_status bta_grad_logdet_quad(int64_t n, int64_t b, int64_t a, const double* XD, const double* XB, const double* XR,
                         const double* XT, const double* x, int64_t nrhs, const double* d_scale, double* GD, double* GB,
                         double* GR, double* GT, double* gy, bta_stream_t stream) {
  if (!dims_ok(n, b, a)) return fail(BTA_EINVAL, "invalid sizes n=%lld b=%lld a=%lld", (long long)n, (long long)b, (long long)a);
  if (nrhs < 1 || nrhs > (1 << 20)) return fail(BTA_EINVAL, "invalid nrhs=%lld", (long long)nrhs);
  const int64_t N = n * b + a;
  const Arr arr[11] = {{XD, blk_bytes(n, b, b), "XD"}, {XB, blk_bytes(n - 1, b, b), "XB"}, {XR, blk_bytes(n, a, b), "XR"},
                       {XT, blk_bytes(1, a, a), "XT"}, {GD, blk_bytes(n, b, b), "GD"}, {GB, blk_bytes(n - 1, b, b), "GB"},
                       {GR, blk_bytes(n, a, b), "GR"}, {GT, blk_bytes(1, a, a), "GT"}, {x, blk_bytes(1, N, nrhs), "x"},
                       {d_scale, d_scale ? 8u : 0u, "d_scale"}, {gy, gy ? blk_bytes(1, N, nrhs) : 0u, "gy"}};
  const int pair[11] = {4, 5, 6, 7, 0, 1, 2, 3, -1, -1, -1};
  bta_status st = check_arrays(arr, 11, pair);
  if (st) return st;
  st = device_ok();
  if (st) return st;
  hipError_t e = bta::grad_launch(n, b, a, XD, XB, XR, XT, x, nrhs, d_scale, GD, GB, GR, GT, gy,
                                  reinterpret_cast<hipStream_t>(stream));
  return e == hipSuccess ? BTA_OK : hip_fail(e, "bta_grad_logdet_quad launch");
}

namespace {

bta_status validate_batch(int count, const bta_desc* d, bool factor) {
  if (count < 1 || count > (1 << 20)) return fail(BTA_EINVAL, "invalid batch count %d", count);
  if (!d) return fail(BTA_EINVAL, "descriptor array is NULL");
  std::vector<std::pair<uintptr_t, uintptr_t>> spans;
  for (int m = 0; m < count; ++m) {
    const int64_t n = d[m].n, b = d[m].b, a = d[m].a;
    if (!dims_ok(n, b, a)) return fail(BTA_EINVAL, "matrix %d: invalid sizes n=%lld b=%lld a=%lld", m, (long long)n, (long long)b, (long long)a);
    bta_status st;
    if (factor) {
      const Arr arr[9] = {{d[m].D, blk_bytes(n, b, b), "D"},   {d[m].B, blk_bytes(n - 1, b, b), "B"}, {d[m].R, blk_bytes(n, a, b), "R"},
                          {d[m].T, blk_bytes(1, a, a), "T"},   {d[m].LD, blk_bytes(n, b, b), "LD"}, {d[m].LB, blk_bytes(n - 1, b, b), "LB"},
                          {d[m].LR, blk_bytes(n, a, b), "LR"}, {d[m].LT, blk_bytes(1, a, a), "LT"}, {d[m].d_info, 8, "d_info"}};
      const int pair[9] = {4, 5, 6, 7, 0, 1, 2, 3, -1};
      st = check_arrays(arr, 9, pair);
      if (st) return fail(st, "matrix %d: %s", m, g_last_error.c_str());
      for (const Arr& x : arr)
        if (x.bytes) spans.push_back({reinterpret_cast<uintptr_t>(x.p), reinterpret_cast<uintptr_t>(x.p) + x.bytes});
    } else {
      const Arr arr[8] = {{d[m].LD, blk_bytes(n, b, b), "LD"}, {d[m].LB, blk_bytes(n - 1, b, b), "LB"}, {d[m].LR, blk_bytes(n, a, b), "LR"},
                          {d[m].LT, blk_bytes(1, a, a), "LT"}, {d[m].XD, blk_bytes(n, b, b), "XD"}, {d[m].XB, blk_bytes(n - 1, b, b), "XB"},
                          {d[m].XR, blk_bytes(n, a, b), "XR"}, {d[m].XT, blk_bytes(1, a, a), "XT"}};
      const int pair[8] = {4, 5, 6, 7, 0, 1, 2, 3};
      st = check_arrays(arr, 8, pair);
      if (st) return fail(st, "matrix %d: %s", m, g_last_error.c_str());
      for (const Arr& x : arr)
        if (x.bytes) spans.push_back({reinterpret_cast<uintptr_t>(x.p), reinterpret_cast<uintptr_t>(x.p) + x.bytes});
    }
  }
  // arrays of different matrices must not overlap (exact in-place pairs repeat the same span)
  std::sort(spans.begin(), spans.end());
  spans.erase(std::unique(spans.begin(), spans.end()), spans.end());
  for (size_t i = 1; i < spans.size(); ++i)
    if (spans[i].first < spans[i - 1].second) return fail(BTA_EINVAL, "arrays of the batch overlap");
  return BTA_OK;
}

void batch_sizes(int count, const bta_desc* d, std::vector<int64_t>& n, std::vector<int64_t>& b, std::vector<int64_t>& a) {
  n.resize(count); b.resize(count); a.resize(count);
  for (int m = 0; m < count; ++m) { n[m] = d[m].n; b[m] = d[m].b; a[m] = d[m].a; }
}

std::vector<bta::BatchMatrix> batch_mats(int count, const bta_desc* d) {
  std::vector<bta::BatchMatrix> v(count);
  for (int m = 0; m < count; ++m)
    v[m] = bta::BatchMatrix{d[m].n, d[m].b, d[m].a, d[m].D, d[m].B, d[m].R, d[m].T, d[m].LD, d[m].LB, d[m].LR, d[m].LT,
                            d[m].XD, d[m].XB, d[m].XR, d[m].XT, d[m].d_info};
  return v;
}

}  // namespace

size_t bta_batched_workspace_bytes(int op, int count, const bta_desc* descs) {
  if (count < 1 || !descs) return 0;
  for (int m = 0; m < count; ++m)
    if (!dims_ok(descs[m].n, descs[m].b, descs[m].a)) return 0;
  std::vector<int64_t> n, b, a;
  batch_sizes(count, descs, n, b, a);
  if (op == BTA_OP_FACTOR) return bta::factor_batch_plan(count, n.data(), b.data(), a.data(), 0).bytes;
  if (op == BTA_OP_SELINV) return bta::selinv_batch_bytes(count, n.data(), b.data(), a.data());
  return 0;
}

bta_status bta_factor_batched(int count, const bta_desc* descs, void* work, size_t work_bytes, bta_stream_t stream) {
  bta_status st = validate_batch(count, descs, true);
  if (st) return st;
  std::vector<int64_t> n, b, a;
  batch_sizes(count, descs, n, b, a);
  st = device_ok();
  if (st) return st;
  const bta::FactorBatchPlan bp = bta::factor_batch_plan(count, n.data(), b.data(), a.data(), bta::device_cu_count());
  st = check_work(work, work_bytes, bp.bytes);
  if (st) return st;
  const std::vector<bta::BatchMatrix> mats = batch_mats(count, descs);
  hipError_t e = bta::factor_batch_launch(bp, mats.data(), work, reinterpret_cast<hipStream_t>(stream), bta::device_cu_count());
  return e == hipSuccess ? BTA_OK : hip_fail(e, "bta_factor_batched launch");
}

bta_status bta_selinv_batched(int count, const bta_desc* descs, void* work, size_t work_bytes, bta_stream_t stream) {
  bta_status st = validate_batch(count, descs, false);
  if (st) return st;
  std::vector<int64_t> n, b, a;
  batch_sizes(count, descs, n, b, a);
  st = check_work(work, work_bytes, bta::selinv_batch_bytes(count, n.data(), b.data(), a.data()));
  if (st) return st;
  st = device_ok();
  if (st) return st;
  const std::vector<bta::BatchMatrix> mats = batch_mats(count, descs);
  hipError_t e = bta::selinv_batch_launch(count, mats.data(), work, reinterpret_cast<hipStream_t>(stream));
  return e == hipSuccess ? BTA_OK : hip_fail(e, "bta_selinv_batched launch");
}

const char* bta_status_string(int status) {
  switch (status) {
    case BTA_OK: return "BTA_OK";
    case BTA_EINVAL: return "BTA_EINVAL: invalid argument";
    case BTA_EHIP: return "BTA_EHIP: HIP runtime error";
    case BTA_ENOTSUP: return "BTA_ENOTSUP: unsupported device";
    default: return "unknown bta status";
  }
}

const char* bta_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
