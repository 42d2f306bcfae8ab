// Batched selected inversion: the launch sequences of all matrices are
// recorded as stage-keyed operations (the stage key names the position of an
// operation in the per-matrix sequence: tip, preprocessing chunk/level, backward
// step), operations with the same key are independent across matrices and are
// merged into one list-driven launch, and the merged sequence is captured once
// per descriptor set in a HIP graph and replayed.  For every merged GEMM launch
// an autotuner picks the tile shape (64 x 64 or 128 x 128) by timing both on
// first use of its shape class (only for stages whose outputs do not feed their
// own inputs, so the second run reproduces the first); the choice is cached
// per process.
#include <algorithm>
#include <cstring>
#include <list>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "bta_device.hpp"
#include "bta_internal.hpp"
#include "bta_testing.h"

#define BTA_TRY_E(x)                    \
  do {                                  \
    hipError_t e_ = (x);                \
    if (e_ != hipSuccess) return e_;    \
  } while (0)

namespace bta {

// ---------------------------------------------------------------- list kernels

__global__ void fill_list_kernel(const FillOp* ops) {
  const FillOp f = ops[blockIdx.y];
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < f.count; e += (long long)gridDim.x * blockDim.x)
    f.p[e] = 0.0;
}

__global__ void copy_list_kernel(const CopyOp* ops) {
  const CopyOp c = ops[blockIdx.y];
  const long long per = (long long)c.rows * c.cols, total = per * c.nb;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (long long)gridDim.x * blockDim.x) {
    const long long bi = e / per, rc = e - bi * per;
    const int r = (int)(rc / c.cols), q = (int)(rc - (long long)r * c.cols);
    c.dst[bi * c.sd + (int64_t)r * c.ldd + q] = c.src[bi * c.ss + (int64_t)r * c.lds + q];
  }
}

// one workgroup per 64 x 64 diagonal tile of one block of one entry
__global__ __launch_bounds__(NT) void trinv_list_kernel(const TrinvOp* ops, const long long* wg_begin, int nops) {
  __shared__ double S[TS * LDS_LD];
  const int tid = threadIdx.x;
  int lo = 0, hi = nops - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (wg_begin[mid] <= (long long)blockIdx.x) lo = mid; else hi = mid - 1;
  }
  const TrinvOp op = ops[lo];
  const long long local = blockIdx.x - wg_begin[lo];
  const int T = (op.m + 63) / 64;
  const int blk = (int)(local / T), t = (int)(local - (long long)blk * T);
  const int ext = min(64, op.m - t * 64);
  const double* Lt = op.L + blk * op.sL + (int64_t)t * 64 * op.ldL + t * 64;
  for (int e = tid; e < 64 * 64; e += NT) {
    const int rr = e >> 6, cc = e & 63;
    double v;
    if (rr < ext && cc < ext) v = (cc <= rr) ? Lt[(int64_t)rr * op.ldL + cc] : 0.0;
    else v = (rr == cc) ? 1.0 : 0.0;
    S[rr * LDS_LD + cc] = v;
  }
  __syncthreads();
  double w[16];
  trinv_tile(S, w, tid);
  const int r = tid & 63, q = tid >> 6;
  double* Wt = op.W + blk * op.sW + (int64_t)t * 64 * op.ldW + t * 64;
  if (r < ext) {
#pragma unroll
    for (int mm = 0; mm < 16; ++mm) {
      const int c = 16 * q + mm;
      if (c < ext) Wt[(int64_t)r * op.ldW + c] = (c <= r) ? w[mm] : 0.0;
    }
  }
}

// ---------------------------------------------------------------- merged plan

namespace {

struct StageExec {
  StageKey key;       // (phase, major, minor) of the merged stage
  int kind;           // 0 gemm, 1 fill, 2 copy, 3 trinv
  size_t off;         // op array offset in the table region (gemm: problems with 64-tile metadata)
  size_t off_pre;     // prefix array offset (gemm: 64-tile prefix; trinv: workgroup prefix)
  size_t off_p128;    // gemm: problems with 128-tile metadata
  size_t off_pre128;  // gemm: 128-tile prefix
  int count;          // number of ops / problems
  long long work;   // trinv: workgroups; gemm: 64-tile count
  long long work2;  // gemm: 128-tile count
  bool pure;        // gemm: outputs do not feed the stage's inputs (safe to run twice)
  bool skinny;      // gemm: every problem takes the skinny kernel (at most 16 rows: the arrow rows)
  std::string shape;
};

struct MergedPlan {
  std::vector<StageExec> stages;
  std::vector<char> table;  // host image of the device table region
};

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

template <class T>
size_t append(std::vector<char>& tab, const std::vector<T>& v) {
  const size_t off = align256(tab.size());
  tab.resize(off + sizeof(T) * v.size());
  if (!v.empty()) std::memcpy(tab.data() + off, v.data(), sizeof(T) * v.size());
  return off;
}

bool windows_overlap(const double* a0, const double* a1, const double* b0, const double* b1) { return a0 < b1 && b0 < a1; }

// coarse [first, last] address span of a problem operand / output
void span_of(const double* base, int64_t rows, int64_t cols, int64_t ld, int64_t s0, int64_t s1, int nb0, int nb1,
             const double*& lo, const double*& hi) {
  lo = base;
  hi = base + (rows - 1) * ld + cols + (int64_t)(nb0 - 1) * s0 + (int64_t)(nb1 - 1) * s1;
}

bool stage_pure(const std::vector<GProb>& ps) {
  for (const GProb& p : ps)
    if (p.beta != 0.0) return false;
  for (const GProb& o : ps) {
    const double *c0, *c1;
    span_of(o.Cout, o.store == ST_LOWER_MIRROR ? std::max(o.M, o.N) : o.M, o.store == ST_LOWER_MIRROR ? std::max(o.M, o.N) : o.N,
            o.ldc, o.sC0, o.sC1, o.nb0, o.nb1, c0, c1);
    for (const GProb& p : ps)
      for (int s = 0; s < p.nseg; ++s) {
        const GSeg& g = p.seg[s];
        const double *a0, *a1, *b0, *b1;
        span_of(g.A, g.at ? g.K : p.M, g.at ? p.M : g.K, g.lda, g.sA0, g.sA1, p.nb0, p.nb1, a0, a1);
        span_of(g.B, g.bt ? g.K : p.N, g.bt ? p.N : g.K, g.ldb, g.sB0, g.sB1, p.nb0, p.nb1, b0, b1);
        if (windows_overlap(c0, c1, a0, a1) || windows_overlap(c0, c1, b0, b1)) return false;
      }
  }
  return true;
}

std::string shape_key(const std::vector<GProb>& ps) {
  std::map<std::string, long long> hist;
  for (const GProb& p : ps) {
    int K = 0;
    for (int s = 0; s < p.nseg; ++s) K += p.seg[s].K;
    const std::string k = std::to_string(p.M) + "x" + std::to_string(p.N) + "x" + std::to_string(K) + "/" +
                          std::to_string(p.lower_tiles) + std::to_string(p.store) + std::to_string(p.nseg);
    hist[k] += (long long)p.nb0 * p.nb1;
  }
  std::string key;
  for (auto& kv : hist) key += kv.first + "*" + std::to_string(kv.second) + ";";
  return key;
}

MergedPlan build_plan(const StageRecorder& rec) {
  MergedPlan mp;
  for (const auto& kv : rec.stages) {
    const StageRecorder::Stage& st = kv.second;
    StageExec ex{};
    ex.key = kv.first;
    ex.kind = st.kind;
    if (st.kind == 0) {
      std::vector<GProb> p64 = st.gemms, p128 = st.gemms;
      std::vector<long long> pre64, pre128;
      long long t64 = 0, t128 = 0;
      for (size_t i = 0; i < p64.size(); ++i) {
        pre64.push_back(t64);
        t64 += gemm_prob_tiles(p64[i], 64);
        pre128.push_back(t128);
        t128 += gemm_prob_tiles(p128[i], 128);
      }
      // the same problems with both tilings: store the 64-tile and 128-tile copies
      ex.off = append(mp.table, p64);
      ex.off_pre = append(mp.table, pre64);
      ex.off_p128 = append(mp.table, p128);
      ex.off_pre128 = append(mp.table, pre128);
      ex.count = (int)p64.size();
      ex.work = t64;
      ex.work2 = t128;
      ex.pure = stage_pure(st.gemms);
      long long v = 0;
      ex.skinny = !(env_int("BTA_BATCH_SKINNY", 0, 1, &v) && v == 0);  // measurement override
      for (const GProb& q : st.gemms) ex.skinny = ex.skinny && gemm_skinny_ok(q);
      ex.shape = shape_key(st.gemms);
      mp.stages.push_back(ex);
    } else if (st.kind == 1) {
      ex.off = append(mp.table, st.fills);
      ex.count = (int)st.fills.size();
      mp.stages.push_back(ex);
    } else if (st.kind == 2) {
      ex.off = append(mp.table, st.copies);
      ex.count = (int)st.copies.size();
      mp.stages.push_back(ex);
    } else if (st.kind == 3) {
      std::vector<long long> pre;
      long long wgs = 0;
      for (const TrinvOp& t : st.trinvs) {
        pre.push_back(wgs);
        wgs += (long long)((t.m + 63) / 64) * t.nblk;
      }
      ex.off = append(mp.table, st.trinvs);
      ex.off_pre = append(mp.table, pre);
      ex.count = (int)st.trinvs.size();
      ex.work = wgs;
      mp.stages.push_back(ex);
    }
  }
  mp.table.resize(align256(mp.table.size()));
  return mp;
}

// ---------------------------------------------------------------- autotuner / graph cache

// The replay of one descriptor set: its merged stages with their tilings,
// the sweep's waits, a pinned copy of the table image (uploaded on the
// caller's stream before every replay, so the upload never blocks the host)
// and the captured graph.  Recent descriptor sets are kept most recently used
// first; at most kGraphCache of them, the oldest released on insertion (after
// its last upload has completed).
constexpr size_t kGraphCache = 8;
struct Replay {
  std::string sig;
  std::vector<StageExec> stages;
  std::vector<int> choice;
  std::map<int, int> need;    // sweep step -> preprocessing stage index it waits for
  std::map<int, int> ev_of;   // preprocessing stage index -> event number (2, 3, ...)
  int nev = 2;                // events used: 0 fork, 1 end of the preprocessing branch
  void* htab = nullptr;       // pinned table image
  size_t tab_bytes = 0;
  hipEvent_t uploaded = nullptr;  // recorded after each upload of htab
  hipGraphExec_t exec = nullptr;
  ~Replay() {
    if (uploaded) { (void)hipEventSynchronize(uploaded); (void)hipEventDestroy(uploaded); }
    if (htab) (void)hipHostFree(htab);
    if (exec) (void)hipGraphExecDestroy(exec);
  }
};
std::mutex g_mu;
std::list<std::shared_ptr<Replay>> g_replays;

int heuristic_big(const StageExec& ex) { return ex.work2 >= 200 ? 1 : 0; }

hipError_t launch_stage(const StageExec& ex, char* dtab, int big, hipStream_t s) {
  switch (ex.kind) {
    case 0: {
      if (ex.skinny)
        return gemm_skinny_list_launch(reinterpret_cast<const GProb*>(dtab + ex.off),
                                       reinterpret_cast<const long long*>(dtab + ex.off_pre), ex.count, ex.work, s);
      if (big)
        return gemm_list_launch(reinterpret_cast<const GProb*>(dtab + ex.off_p128),
                                reinterpret_cast<const long long*>(dtab + ex.off_pre128), ex.count, ex.work2, 1, s);
      return gemm_list_launch(reinterpret_cast<const GProb*>(dtab + ex.off), reinterpret_cast<const long long*>(dtab + ex.off_pre),
                              ex.count, ex.work, 0, s);
    }
    case 1:
      hipLaunchKernelGGL(fill_list_kernel, dim3(64, (unsigned)ex.count), dim3(256), 0, s, reinterpret_cast<const FillOp*>(dtab + ex.off));
      return hipGetLastError();
    case 2:
      hipLaunchKernelGGL(copy_list_kernel, dim3(64, (unsigned)ex.count), dim3(256), 0, s, reinterpret_cast<const CopyOp*>(dtab + ex.off));
      return hipGetLastError();
    case 3:
      if (ex.work == 0) return hipSuccess;
      hipLaunchKernelGGL(trinv_list_kernel, dim3((unsigned)ex.work), dim3(NT), 0, s, reinterpret_cast<const TrinvOp*>(dtab + ex.off),
                         reinterpret_cast<const long long*>(dtab + ex.off_pre), ex.count);
      return hipGetLastError();
  }
  return hipSuccess;
}

// The tuning-table key of a merged GEMM stage's shape class (every matrix's
// b and a are in the shape string, so the op's b and a fields stay 0).
std::string stage_key(const StageExec& ex) { return tune_key(("selinv_batched[" + ex.shape + "]").c_str(), 0, 0, "tile128"); }

}  // namespace

// Workspace: per-matrix selected-inversion slices, then the table region.
struct BatchLayout {
  std::vector<size_t> slice;
  size_t table_off = 0, bytes = 0;
};

static BatchLayout batch_layout(int count, const int64_t* n, const int64_t* b, const int64_t* a, size_t table_bytes) {
  BatchLayout L;
  size_t off = 0;
  for (int m = 0; m < count; ++m) {
    L.slice.push_back(off);
    off += align256(selinv_plan(n[m], b[m], a[m], false).bytes);
  }
  L.table_off = off;
  L.bytes = off + table_bytes;
  return L;
}

static hipError_t record_batch(int count, const BatchMatrix* mats, char* work, const BatchLayout& L, StageRecorder& rec) {
  g_rec = &rec;
  hipError_t e = hipSuccess;
  rec.span = 0;
  long long v = 0;
  if (!(env_int("BTA_BATCH_SPREAD", 0, 1, &v) && v == 0))  // measurement override: 0 aligns the sweeps' first steps
    for (int m = 0; m < count; ++m) rec.span = std::max<int64_t>(rec.span, mats[m].n);
  for (int m = 0; m < count && e == hipSuccess; ++m) {
    const BatchMatrix& x = mats[m];
    rec.cur = m;
    rec.cur_n = x.n;
    e = selinv_launch(selinv_plan(x.n, x.b, x.a, false), x.n, x.b, x.a, x.LD, x.LB, x.LR, x.LT, x.XD, x.XB, x.XR, x.XT,
                      work + L.slice[m], nullptr);
  }
  g_rec = nullptr;
  return e;
}

// For each merged backward-sweep step, the index of the preprocessing-branch
// stage (phase < 2) after which every block worked on at that step is ready
// (the block of each matrix that has a step there); a step with a block never
// marked ready waits for the whole branch (absent from the map).
static std::map<int, int> sweep_waits(const MergedPlan& mp, const StageRecorder& rec) {
  std::map<StageKey, int> index;
  for (size_t k = 0; k < mp.stages.size(); ++k) index.emplace(mp.stages[k].key, (int)k);
  std::map<int, int> need;
  std::map<int, bool> whole;
  for (size_t m = 0; m < rec.sweep_block.size(); ++m)
    for (const auto& kv : rec.sweep_block[m]) {
      const int S = kv.first;
      const int64_t i = kv.second;
      if (whole.count(S)) continue;
      int idx = -1;
      if (m < rec.ready.size() && i >= 0 && i < (int64_t)rec.ready[m].size()) {
        const auto it = index.find(rec.ready[m][i]);
        if (it != index.end() && mp.stages[it->second].key.phase < 2) idx = it->second;
      }
      if (idx < 0) {
        whole[S] = true;
        need.erase(S);
        continue;
      }
      const auto it = need.find(S);
      need[S] = it == need.end() ? idx : std::max(it->second, idx);
    }
  return need;
}

size_t selinv_batch_bytes(int count, const int64_t* n, const int64_t* b, const int64_t* a) {
  // record with placeholder pointers to size the table region
  std::vector<BatchMatrix> mats(count);
  const uintptr_t G = uintptr_t(1) << 40;
  for (int m = 0; m < count; ++m) {
    double* base = reinterpret_cast<double*>((uintptr_t)(m + 1) * G);
    mats[m] = BatchMatrix{n[m], b[m], a[m], nullptr, nullptr, nullptr, nullptr, base, base, base, base, base, base, base, base, nullptr};
  }
  BatchLayout L0 = batch_layout(count, n, b, a, 0);
  StageRecorder rec;
  if (record_batch(count, mats.data(), reinterpret_cast<char*>(uintptr_t(1) << 50), L0, rec) != hipSuccess) return 0;
  const MergedPlan mp = build_plan(rec);
  return batch_layout(count, n, b, a, mp.table.size()).bytes;
}

// Issue a replay's stages: the preprocessing and arrow-row stages (phases 0
// and 1) on `side`, forked from `main`, the backward sweep (phase 2) on
// `main`, each sweep step waiting only for the preprocessing stage after
// which every block it works on is ready; `side` joins `main` at the end.  The preprocessing branch is issued first, so every wait follows
// the record of its event.  (Issuing each sweep step right after the stage it
// waits for measured slower in the captured graph: 45.9 ms against 42.5 ms
// per step of the 64-matrix workload; launching the same sequence directly on
// two streams instead of replaying a graph, 43.8 ms.)
static hipError_t issue_replay(const Replay& r, char* dtab, hipStream_t main, hipStream_t side, SyncCtx* cx) {
  BTA_TRY_E(hipEventRecord(cx->event(0), main));
  BTA_TRY_E(hipStreamWaitEvent(side, cx->event(0), 0));
  for (size_t k = 0; k < r.stages.size(); ++k) {
    if (r.stages[k].key.phase >= 2) continue;
    BTA_TRY_E(launch_stage(r.stages[k], dtab, r.choice[k], side));
    const auto it = r.ev_of.find((int)k);
    if (it != r.ev_of.end()) BTA_TRY_E(hipEventRecord(cx->event(it->second), side));
  }
  BTA_TRY_E(hipEventRecord(cx->event(1), side));
  int step = INT32_MIN;
  for (size_t k = 0; k < r.stages.size(); ++k) {
    const StageExec& ex = r.stages[k];
    if (ex.key.phase < 2) continue;
    if (ex.key.major != step) {  // a new sweep step: wait for the stage that completes its blocks
      step = ex.key.major;
      const auto it = r.need.find(step);
      BTA_TRY_E(hipStreamWaitEvent(main, cx->event(it != r.need.end() ? r.ev_of.at(it->second) : 1), 0));
    }
    BTA_TRY_E(launch_stage(ex, dtab, r.choice[k], main));
  }
  return hipStreamWaitEvent(main, cx->event(1), 0);  // join the preprocessing branch
}

hipError_t selinv_batch_launch(int count, const BatchMatrix* mats, void* work, hipStream_t stream) {
  std::vector<int64_t> n(count), b(count), a(count);
  for (int m = 0; m < count; ++m) { n[m] = mats[m].n; b[m] = mats[m].b; a[m] = mats[m].a; }
  char* w = static_cast<char*>(work);
  const BatchLayout L0 = batch_layout(count, n.data(), b.data(), a.data(), 0);
  StageRecorder rec;
  BTA_TRY_E(record_batch(count, mats, w, L0, rec));
  const MergedPlan mp = build_plan(rec);
  char* dtab = w + L0.table_off;
  int dev = 0;
  BTA_TRY_E(hipGetDevice(&dev));

  // descriptor-set signature: the table image holds every pointer and size
  std::string sig(mp.table.begin(), mp.table.end());
  sig += "|" + std::to_string(reinterpret_cast<uintptr_t>(work)) + "|" + std::to_string(dev);
  std::shared_ptr<Replay> hit;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    for (auto it = g_replays.begin(); it != g_replays.end(); ++it)
      if ((*it)->sig == sig) {
        g_replays.splice(g_replays.begin(), g_replays, it);  // most recently used
        hit = g_replays.front();
        break;
      }
  }
  if (hit) {
    BTA_TRY_E(hipMemcpyAsync(dtab, hit->htab, hit->tab_bytes, hipMemcpyHostToDevice, stream));
    BTA_TRY_E(hipEventRecord(hit->uploaded, stream));
    return hipGraphLaunch(hit->exec, stream);
  }
  BTA_TRY_E(hipMemcpyAsync(dtab, mp.table.data(), mp.table.size(), hipMemcpyHostToDevice, stream));

  // first use: run eagerly; a pure GEMM stage whose shape class is not in the
  // tuning table is timed with both tilings (median of three runs each; the
  // stage's outputs do not feed its inputs, so repeating it is harmless) and
  // the faster one recorded.  This first call waits for those timings on the
  // host (hipEventSynchronize on the caller's stream); later calls only enqueue.
  std::vector<int> choice(mp.stages.size(), 0);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  for (size_t k = 0; k < mp.stages.size(); ++k) {
    const StageExec& ex = mp.stages[k];
    if (ex.kind != 0) {
      BTA_TRY_E(launch_stage(ex, dtab, 0, stream));
      continue;
    }
    long long tuned = -1;
    if (!tune_get(stage_key(ex), &tuned) || (tuned != 0 && tuned != 1)) tuned = -1;
    if (ex.skinny) {  // one kernel: nothing to tune
      BTA_TRY_E(launch_stage(ex, dtab, 0, stream));
      continue;
    }
    if (tuned < 0 && ex.pure && ex.work2 > 0) {
      if (!e0) {
        BTA_TRY_E(hipEventCreate(&e0));
        BTA_TRY_E(hipEventCreate(&e1));
      }
      float med[2] = {0.f, 0.f};
      for (int big = 0; big < 2; ++big) {
        float t[3];
        for (int rep = 0; rep < 3; ++rep) {
          BTA_TRY_E(hipEventRecord(e0, stream));
          BTA_TRY_E(launch_stage(ex, dtab, big, stream));
          BTA_TRY_E(hipEventRecord(e1, stream));
          BTA_TRY_E(hipEventSynchronize(e1));
          BTA_TRY_E(hipEventElapsedTime(&t[rep], e0, e1));
        }
        std::sort(t, t + 3);
        med[big] = t[1];
      }
      tuned = med[1] < med[0] ? 1 : 0;
      tune_set(stage_key(ex), tuned, true);
      // the last timed run used the 128 tiling: leave the chosen tiling's
      // result, so that this call's bits are those of the replays
      if (tuned == 0) BTA_TRY_E(launch_stage(ex, dtab, 0, stream));
    } else {
      if (tuned < 0) tuned = heuristic_big(ex);
      BTA_TRY_E(launch_stage(ex, dtab, (int)tuned, stream));
    }
    choice[k] = (int)tuned;
  }
  if (e0) { (void)hipEventDestroy(e0); (void)hipEventDestroy(e1); }

  // the replay of the next calls with this descriptor set
  auto r = std::make_shared<Replay>();
  r->sig = sig;
  r->stages = mp.stages;
  r->choice = choice;
  r->need = sweep_waits(mp, rec);
  for (const auto& kv : r->need) r->ev_of.emplace(kv.second, 0);
  for (auto& kv : r->ev_of) kv.second = r->nev++;
  BTA_TRY_E(hipHostMalloc(&r->htab, mp.table.size(), 0));
  std::memcpy(r->htab, mp.table.data(), mp.table.size());
  r->tab_bytes = mp.table.size();
  BTA_TRY_E(hipEventCreateWithFlags(&r->uploaded, hipEventDisableTiming));
  {
    SyncLease lease;
    SyncCtx* cx = lease.get();
    if (!cx) return hipErrorInvalidResourceHandle;
    for (int k = 0; k < r->nev; ++k)
      if (!cx->event(k)) return hipErrorInvalidResourceHandle;  // created before the capture
    BTA_TRY_E(hipStreamBeginCapture(cx->capture, hipStreamCaptureModeThreadLocal));
    const hipError_t ce = issue_replay(*r, dtab, cx->capture, cx->side, cx);
    hipGraph_t graph = nullptr;
    const hipError_t ee = hipStreamEndCapture(cx->capture, &graph);
    if (ce != hipSuccess) { if (graph) (void)hipGraphDestroy(graph); return ce; }
    if (ee != hipSuccess) return ee;
    const hipError_t ie = hipGraphInstantiate(&r->exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ie != hipSuccess) return ie;
  }
  std::lock_guard<std::mutex> lk(g_mu);
  g_replays.push_front(r);
  while (g_replays.size() > kGraphCache) g_replays.pop_back();
  return hipSuccess;
}

// Host check of the merged batch plan with placeholder arrays: (1) every
// stage holds operations of one kind; (2) the operations merged into one
// launch touch disjoint memory except for shared reads (no write of one
// operation overlaps a read or a write of another one in the same stage);
// (3) every matrix contributes its operations in its own stage order;
// (4) in the replayed graph, no sweep stage shares a written element with a
// preprocessing stage it is not ordered after.  Out of place and in place.
// Returns 0 when the plan is valid.
static int selinv_batch_check_one(int count, const int64_t* n, const int64_t* b, const int64_t* a, bool inplace) {
  std::vector<BatchMatrix> mats(count);
  const uintptr_t G = uintptr_t(1) << 36;
  for (int m = 0; m < count; ++m) {
    double* L = reinterpret_cast<double*>((uintptr_t)(2 * m + 1) * G);
    double* X = inplace ? L : reinterpret_cast<double*>((uintptr_t)(2 * m + 2) * G);
    const int64_t bb = b[m] * b[m], ab = a[m] * b[m];
    mats[m] = BatchMatrix{n[m], b[m], a[m], nullptr, nullptr, nullptr, nullptr,
                          L, L + n[m] * bb, L + n[m] * bb + (n[m] - 1) * bb, L + n[m] * bb + (n[m] - 1) * bb + n[m] * ab,
                          X, X + n[m] * bb, X + n[m] * bb + (n[m] - 1) * bb, X + n[m] * bb + (n[m] - 1) * bb + n[m] * ab,
                          nullptr};
  }
  const BatchLayout L0 = batch_layout(count, n, b, a, 0);
  StageRecorder rec;
  if (record_batch(count, mats.data(), reinterpret_cast<char*>(uintptr_t(1) << 52), L0, rec) != hipSuccess) return 1;
  // byte spans of every element window a stage reads or writes, by operation
  struct Span { const char* lo; const char* hi; bool w; int op; };
  auto spans_of = [](const StageRecorder::Stage& st) {
    std::vector<Span> spans;
    auto add = [&](const void* base, int64_t rows, int64_t cols, int64_t ld, bool w, int op) {
      if (rows <= 0 || cols <= 0) return;
      const char* lo = static_cast<const char*>(base);
      spans.push_back({lo, lo + 8 * ((rows - 1) * ld + cols), w, op});
    };
    int op = 0;
    for (const GProb& p : st.gemms) {
      for (int b0 = 0; b0 < p.nb0; ++b0)
        for (int b1 = 0; b1 < p.nb1; ++b1) {
          const int64_t off = b0 * p.sC0 + b1 * p.sC1;
          add(p.Cout + off, p.M, p.N, p.ldc, true, op);
          if (p.store == ST_LOWER_MIRROR) add(p.Cout + off, p.N, p.M, p.ldc, true, op);
          for (int q = 0; q < p.nseg; ++q) {
            const GSeg& g = p.seg[q];
            add(g.A + b0 * g.sA0 + b1 * g.sA1, g.at ? g.K : p.M, g.at ? p.M : g.K, g.lda, false, op);
            add(g.B + b0 * g.sB0 + b1 * g.sB1, g.bt ? g.K : p.N, g.bt ? p.N : g.K, g.ldb, false, op);
          }
        }
      ++op;
    }
    for (const FillOp& f : st.fills) { add(f.p, 1, f.count, f.count, true, op); ++op; }
    for (const CopyOp& c : st.copies) {
      for (int q = 0; q < c.nb; ++q) {
        add(c.src + q * c.ss, c.rows, c.cols, c.lds, false, op);
        add(c.dst + q * c.sd, c.rows, c.cols, c.ldd, true, op);
      }
      ++op;
    }
    for (const TrinvOp& t : st.trinvs) {
      for (int q = 0; q < t.nblk; ++q) {
        add(t.L + q * t.sL, t.m, t.m, t.ldL, false, op);
        add(t.W + q * t.sW, t.m, t.m, t.ldW, true, op);
      }
      ++op;
    }
    std::sort(spans.begin(), spans.end(), [](const Span& x, const Span& y) { return x.lo < y.lo; });
    return spans;
  };
  // operations merged into one stage run concurrently: no element written by
  // one may be touched by another
  std::map<StageKey, std::vector<Span>> by_key;
  for (const auto& kv : rec.stages) {
    const StageRecorder::Stage& st = kv.second;
    const int kinds = (!st.gemms.empty()) + (!st.fills.empty()) + (!st.copies.empty()) + (!st.trinvs.empty());
    if (kinds != 1) return 2;
    const std::vector<Span> spans = spans_of(st);
    for (size_t i = 0; i < spans.size(); ++i)
      for (size_t j = i + 1; j < spans.size() && spans[j].lo < spans[i].hi; ++j)
        if (spans[i].op != spans[j].op && (spans[i].w || spans[j].w)) return 3;
    by_key.emplace(kv.first, spans);
  }
  // the replayed graph runs the sweep (phase 2) beside the preprocessing
  // branch: a sweep step is ordered only after the preprocessing stage it
  // waits for, so it must share no written element with any later one
  const MergedPlan mp = build_plan(rec);
  const std::map<int, int> need = sweep_waits(mp, rec);
  for (const StageExec& sx : mp.stages) {
    if (sx.key.phase < 2) continue;
    const auto it = need.find(sx.key.major);
    if (it == need.end()) continue;  // waits for the whole branch
    const std::vector<Span>& ss = by_key.at(sx.key);
    for (size_t k = (size_t)it->second + 1; k < mp.stages.size(); ++k) {
      if (mp.stages[k].key.phase >= 2) continue;
      for (const Span& x : by_key.at(mp.stages[k].key))
        for (const Span& y : ss)
          if (x.lo < y.hi && y.lo < x.hi && (x.w || y.w)) return 4;
    }
  }
  return 0;
}

BTA_TESTING_API int bta_internal_selinv_batch_check(int count, const int64_t* n, const int64_t* b, const int64_t* a) {
  const int r = selinv_batch_check_one(count, n, b, a, false);
  return r != 0 ? r : selinv_batch_check_one(count, n, b, a, true);
}

}  // namespace bta
