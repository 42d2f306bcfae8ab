// POBTASI (Algorithm 2) on gfx950, in the inverse-factor form.
//
// With W_i = L_ii^{-1}, P_i = [L_{i+1,i}; L_{n,i}] W_i and the already final
// window S_{i+1} = [[X_{i+1,i+1}, X_{n,i+1}^T], [X_{n,i+1}, X_{n,n}]], the
// backward step of Algorithm 2 reads
//
//   [X_{i+1,i}; X_{n,i}] = -S_{i+1} P_i
//   X_{i,i}              = W_i^T W_i - [X_{i+1,i}; X_{n,i}]^T P_i
//
// which is the listing's U blocks followed by its right-side solves with
// L_ii, with each solve replaced by the product with W_i (the paper's own
// substitution of repeated TRSMs by one inversion plus GEMMs).  W_i, P_i and
// V_i = W_i^T W_i depend on the factor only, so they are computed for all
// blocks up front in large batched launches (chunks of blocks); the
// sequential backward sweep is then two MFMA GEMM launches per step.
//   X_{n,n} = L_nn^{-T} L_nn^{-1} comes from the same inverse + product.
//
// The arrow rows form a recursion of their own, X_{n,i} = -(X_{n,i+1} P_B +
// X_nn P_R), which does not involve the diagonal blocks; it runs on the
// preprocessing stream right after each chunk's products, so that the sweep
// proper is one b x b product and one lower-triangular b x b product per step.
#include <algorithm>
#include <map>
#include <mutex>
#include <vector>

#include "bta_device.hpp"
#include "bta_internal.hpp"
#include "bta_testing.h"

namespace bta {

static GProb prob_init() {
  GProb p{};
  p.nseg = 0;
  p.nb0 = 1;
  p.nb1 = 1;
  p.alpha = 1.0;
  p.beta = 0.0;
  p.store = ST_FULL;
  p.lower_tiles = 0;
  return p;
}

static GSeg seg(const double* A, int64_t lda, int at, const double* B, int64_t ldb, int bt, int K, int tri,
                int64_t sA0 = 0, int64_t sB0 = 0, int64_t sA1 = 0, int64_t sB1 = 0) {
  GSeg s{};
  s.A = A; s.B = B; s.lda = lda; s.ldb = ldb; s.at = at; s.bt = bt; s.K = K; s.tri = tri;
  s.sA0 = sA0; s.sB0 = sB0; s.sA1 = sA1; s.sB1 = sB1;
  return s;
}

#define BTA_TRY(x)                      \
  do {                                  \
    hipError_t e_ = (x);                \
    if (e_ != hipSuccess) return e_;    \
  } while (0)

// Inverse of nblk lower-triangular m x m matrices L (ld ldL, stride sL) into W
// (ld ldW, stride sW; must be zero on entry), using T1 (same layout as W) as
// scratch.  64-tile inverses first, then doubling: for neighbouring groups of
// g tiles, W21 = -W22 (L21 W11).
hipError_t trtri_batched(const double* L, int64_t ldL, int64_t sL, double* W, double* T1, int64_t ldW, int64_t sW,
                                int m, int nblk, hipStream_t s, int phase, int major) {
  set_stage(phase, major, 1);
  BTA_TRY(trinv_diag_tiles_launch(L, ldL, sL, W, ldW, sW, m, nblk, s));
  const int T = (m + 63) / 64;
  int lg = 0;
  for (int g = 1; g < T; g *= 2, ++lg) {
    // groups start at tiles 0, 2g, 4g, ... and exist while start + g < T; all
    // but possibly the last have g + g full 64-row tiles
    const int ngroups = (T - g + 2 * g - 1) / (2 * g);
    const int s_last = 2 * g * (ngroups - 1);
    const bool last_full = (s_last + 2 * g < T) || (s_last + 2 * g == T && m % 64 == 0);
    const int nfull = last_full ? ngroups : ngroups - 1;
    const int s_part = s_last;
    const bool part = !last_full;
    const int m1 = 64 * g;
    const int64_t gstepL = (int64_t)2 * g * 64 * (ldL + 1);
    const int64_t gstepW = (int64_t)2 * g * 64 * (ldW + 1);
    GProb pr[2];
    int np = 0;
    set_stage(phase, major, 2 + 2 * lg);
    // T1 = L21 * W11
    for (int which = 0; which < 2; ++which) {
      const int s0 = which == 0 ? 0 : s_part;
      const int cnt = which == 0 ? nfull : (part ? 1 : 0);
      if (cnt == 0) continue;
      const int m2 = which == 0 ? 64 * g : (m - 64 * (s0 + g));
      GProb p = prob_init();
      const double* L21 = L + (int64_t)(s0 + g) * 64 * ldL + (int64_t)s0 * 64;
      const double* W11 = W + (int64_t)s0 * 64 * ldW + (int64_t)s0 * 64;
      p.seg[0] = seg(L21, ldL, 0, W11, ldW, 1, m1, TRI_K_GE_COL, sL, sW, gstepL, gstepW);
      p.nseg = 1;
      p.Cout = T1 + (int64_t)(s0 + g) * 64 * ldW + (int64_t)s0 * 64;
      p.ldc = ldW; p.sC0 = sW; p.sC1 = gstepW;
      p.M = m2; p.N = m1; p.nb0 = nblk; p.nb1 = cnt;
      pr[np++] = p;
    }
    BTA_TRY(gemm_launch(pr, np, s));
    np = 0;
    set_stage(phase, major, 3 + 2 * lg);
    // W21 = -W22 * T1
    for (int which = 0; which < 2; ++which) {
      const int s0 = which == 0 ? 0 : s_part;
      const int cnt = which == 0 ? nfull : (part ? 1 : 0);
      if (cnt == 0) continue;
      const int m2 = which == 0 ? 64 * g : (m - 64 * (s0 + g));
      GProb p = prob_init();
      const double* W22 = W + (int64_t)(s0 + g) * 64 * (ldW + 1);
      const double* T1b = T1 + (int64_t)(s0 + g) * 64 * ldW + (int64_t)s0 * 64;
      p.seg[0] = seg(W22, ldW, 0, T1b, ldW, 1, m2, TRI_K_LE_ROW, sW, sW, gstepW, gstepW);
      p.nseg = 1;
      p.Cout = W + (int64_t)(s0 + g) * 64 * ldW + (int64_t)s0 * 64;
      p.ldc = ldW; p.sC0 = sW; p.sC1 = gstepW;
      p.M = m2; p.N = m1; p.nb0 = nblk; p.nb1 = cnt;
      p.alpha = -1.0;
      pr[np++] = p;
    }
    BTA_TRY(gemm_launch(pr, np, s));
  }
  return hipSuccess;
}

// ---------------------------------------------------------------- per-call stream contexts
namespace {
std::mutex g_sync_mu;
std::map<int, std::vector<SyncCtx*>> g_sync_free;  // idle contexts per device
}  // namespace

hipEvent_t SyncCtx::event(int k) {
  while ((int)ev.size() <= k) {
    hipEvent_t e;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
    ev.push_back(e);
  }
  return ev[k];
}

SyncLease::SyncLease() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return;
  {
    std::lock_guard<std::mutex> lk(g_sync_mu);
    std::vector<SyncCtx*>& fr = g_sync_free[dev];
    if (!fr.empty()) {
      ctx_ = fr.back();
      fr.pop_back();
      return;
    }
  }
  SyncCtx* c = new SyncCtx;
  c->dev = dev;
  if (hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking) != hipSuccess ||
      hipStreamCreateWithFlags(&c->copy, hipStreamNonBlocking) != hipSuccess ||
      hipStreamCreateWithFlags(&c->capture, hipStreamNonBlocking) != hipSuccess) {
    for (hipStream_t st : {c->side, c->copy, c->capture})
      if (st) (void)hipStreamDestroy(st);
    delete c;
    return;
  }
  ctx_ = c;
}

SyncLease::~SyncLease() {
  if (!ctx_) return;
  std::lock_guard<std::mutex> lk(g_sync_mu);
  g_sync_free[ctx_->dev].push_back(ctx_);
}

// Largest split count of a sweep product: BTA_SELINV_SPLIT (1..GEMM_MAX_PROBS),
// else the tuning table's "split" entry for (b, a), else GEMM_MAX_PROBS.
static int selinv_split_max(int64_t b, int64_t a) {
  long long v = 0;
  if (env_int("BTA_SELINV_SPLIT", 1, GEMM_MAX_PROBS, &v)) return (int)v;
  if (tune_get(tune_key("selinv", b, a, "split"), &v) && v >= 1 && v <= GEMM_MAX_PROBS) return (int)v;
  return GEMM_MAX_PROBS;
}

SelinvPlan selinv_plan(int64_t n, int64_t b, int64_t a, bool split) {
  SelinvPlan sp{};
  const int64_t T = (b + 63) / 64;
  // enough blocks per chunk to give the 64-tile inverses ~512 workgroups,
  // within ~4 GB of workspace (W and T1 per block of the chunk)
  int64_t chunk = (512 + T - 1) / T;
  const int64_t per_block = 8 * (2 * b * b);
  chunk = std::min<int64_t>(chunk, std::max<int64_t>(1, (int64_t(4) << 30) / per_block));
  chunk = std::max<int64_t>(1, std::min<int64_t>(chunk, 64));
  chunk = std::min<int64_t>(chunk, n);
  sp.chunk = chunk;
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off += (bytes + 255) & ~size_t(255); return o; };
  const size_t bb = (size_t)b * b;
  sp.off_W = take(8 * bb * chunk);
  sp.off_T1 = take(8 * bb * chunk);
  sp.off_PR = take(8 * (size_t)std::max<int64_t>(1, a * b * n));
  sp.off_Xp = take(8 * 2 * bb);  // X_{i+1,i} of two consecutive steps
  sp.off_WT = take(8 * (size_t)std::max<int64_t>(1, 2 * a * a));
  // split-k partial products of the sweep at small b (few output tiles)
  sp.split_doubles = (split && b <= 1024) ? (size_t)GEMM_MAX_PROBS * bb : 0;
  sp.split_max = selinv_split_max(b, a);
  sp.off_split = take(8 * std::max<size_t>(1, sp.split_doubles));
  sp.bytes = off;
  return sp;
}

// Preprocessing chunks [i0, i1), from the last block down: the first ones
// small, so that the sweep starts early, then doubling up to sp.chunk.
static std::vector<std::pair<int64_t, int64_t>> selinv_chunks(const SelinvPlan& sp, int64_t n) {
  std::vector<std::pair<int64_t, int64_t>> c;
  int64_t size = std::min<int64_t>(sp.chunk, 2), i1 = n;
  while (i1 > 0) {
    const int64_t i0 = std::max<int64_t>(0, i1 - size);
    c.emplace_back(i0, i1);
    i1 = i0;
    size = std::min<int64_t>(sp.chunk, 2 * size);
  }
  return c;
}

hipError_t selinv_launch(const SelinvPlan& sp, int64_t n, int64_t b, int64_t a,
                         const double* LD, const double* LB, const double* LR, const double* LT,
                         double* XD, double* XB, double* XR, double* XT,
                         void* work, hipStream_t s) {
  char* w = static_cast<char*>(work);
  double* Ws = reinterpret_cast<double*>(w + sp.off_W);
  double* T1 = reinterpret_cast<double*>(w + sp.off_T1);
  double* Xp = reinterpret_cast<double*>(w + sp.off_Xp);
  double* PR = reinterpret_cast<double*>(w + sp.off_PR);  // P_R of every block (a x b each)
  double* WT = reinterpret_cast<double*>(w + sp.off_WT);
  double* SK = sp.split_doubles ? reinterpret_cast<double*>(w + sp.off_split) : nullptr;
  const int64_t bb = b * b, ab = a * b;
  const int ib = (int)b, ia = (int)a;
  // outputs may alias the inputs exactly: P_B = L_{i+1,i} W_i then goes to
  // staging (T1, free once the inverses are done) and is copied afterwards
  const bool inplace = n > 1 && XB == LB;

  // ---- tip: X_nn = W_T^T W_T
  if (a > 0) {
    double* WTt = WT + a * a;
    set_stage(0, 0, 0);
    BTA_TRY(fill_zero_launch(WT, (size_t)(2 * a * a), s));
    BTA_TRY(trtri_batched(LT, a, 0, WT, WTt, a, 0, ia, 1, s, 0, 0));
    set_stage(0, 0, 100);
    GProb p = prob_init();
    p.seg[0] = seg(WT, a, 1, WT, a, 1, ia, TRI_K_GE_ROW);
    p.nseg = 1;
    p.Cout = XT; p.ldc = a;
    p.M = ia; p.N = ia;
    p.lower_tiles = 1;
    p.store = ST_LOWER_MIRROR;
    BTA_TRY(gemm_launch(&p, 1, s));
  }

  // ---- per-block preprocessing and the arrow-row recursion on a side
  // stream, chunk by chunk from the last block down, so that the backward
  // sweep (on `s`) can start on the first finished blocks while later chunks
  // fill the CUs the sweep leaves idle; each step of the sweep waits for its
  // own block only (an event per block, after its arrow row).
  const bool dry = recording();
  SyncLease lease;  // this call's side stream, copy stream and events
  SyncCtx* cx = lease.get();
  if (!dry && !cx) return hipErrorInvalidResourceHandle;
  auto event_at = [cx](int k) { return cx->event(k); };
  hipStream_t sa = dry ? s : cx->side;
  if (!dry) {
    BTA_TRY(hipEventRecord(event_at(0), s));
    BTA_TRY(hipStreamWaitEvent(sa, event_at(0), 0));
  }
  const auto chunks = selinv_chunks(sp, n);
  for (size_t k = 0; k < chunks.size(); ++k) {
    const int64_t i0 = chunks[k].first, i1 = chunks[k].second;
    const int nblk = (int)(i1 - i0);
    const int nsub = (int)std::min<int64_t>(nblk, (n - 1) - i0);  // blocks of the chunk with an L_{i+1,i}
    set_stage(1, (int)k, 0);
    BTA_TRY(fill_zero_launch(Ws, (size_t)bb * nblk, sa));
    BTA_TRY(trtri_batched(LD + i0 * bb, b, bb, Ws, T1, b, bb, ib, nblk, sa, 1, (int)k));
    set_stage(1, (int)k, 100);
    GProb pr[3];
    int np = 0;
    if (nsub > 0) {  // P_B = L_{i+1,i} W_i into the X_{i+1,i} slot
      GProb p = prob_init();
      p.seg[0] = seg(LB + i0 * bb, b, 0, Ws, b, 1, ib, TRI_K_GE_COL, bb, bb);
      p.nseg = 1;
      p.Cout = inplace ? T1 : XB + i0 * bb; p.ldc = b; p.sC0 = bb;
      p.M = ib; p.N = ib; p.nb0 = nsub;
      pr[np++] = p;
    }
    if (a > 0) {  // P_R = L_{n,i} W_i
      GProb p = prob_init();
      p.seg[0] = seg(LR + i0 * ab, b, 0, Ws, b, 1, ib, TRI_K_GE_COL, ab, bb);
      p.nseg = 1;
      p.Cout = PR + i0 * ab; p.ldc = b; p.sC0 = ab;
      p.M = ia; p.N = ib; p.nb0 = nblk;
      pr[np++] = p;
    }
    {  // V_i = W_i^T W_i (lower) into X_ii
      GProb p = prob_init();
      p.seg[0] = seg(Ws, b, 1, Ws, b, 1, ib, TRI_K_GE_ROW, bb, bb);
      p.nseg = 1;
      p.Cout = XD + i0 * bb; p.ldc = b; p.sC0 = bb;
      p.M = ib; p.N = ib; p.nb0 = nblk;
      p.lower_tiles = 1;
      p.store = ST_LOWER;
      pr[np++] = p;
    }
    BTA_TRY(gemm_launch(pr, np, sa));
    if (inplace) {  // every L_{i+1,i} of the chunk has been read
      set_stage(1, (int)k, 101);
      BTA_TRY(copy2d_launch(T1, b, bb, XB + i0 * bb, b, bb, ib, ib, nsub, sa));
    }
    // arrow rows of the chunk: X_{n,i} = -(X_{n,i+1} P_B + X_nn P_R); block i
    // is ready for the sweep once its row is (event 1 + i)
    if (a == 0 && !dry)
      for (int64_t i = i1 - 1; i >= i0; --i) BTA_TRY(hipEventRecord(event_at(1 + (int)i), sa));
    if (a == 0 && g_rec)
      for (int64_t i = i1 - 1; i >= i0; --i) g_rec->mark_ready(i);
    for (int64_t i = i1 - 1; a > 0 && i >= i0; --i) {
      set_stage(1, (int)k, 200 + (int)(i1 - 1 - i));
      GProb p = prob_init();
      if (i < n - 1) {
        p.seg[0] = seg(XR + (i + 1) * ab, b, 0, XB + i * bb, b, 1, ib, TRI_NONE);
        p.seg[1] = seg(XT, a, 0, PR + i * ab, b, 1, ia, TRI_NONE);
        p.nseg = 2;
      } else {
        p.seg[0] = seg(XT, a, 0, PR + i * ab, b, 1, ia, TRI_NONE);
        p.nseg = 1;
      }
      p.Cout = XR + i * ab; p.ldc = b;
      p.M = ia; p.N = ib;
      p.alpha = -1.0;
      BTA_TRY(gemm_launch(&p, 1, sa));
      if (!dry) BTA_TRY(hipEventRecord(event_at(1 + (int)i), sa));
      if (g_rec) g_rec->mark_ready(i);
    }
  }

  // ---- backward sweep.  X_{i+1,i} goes to one of two buffers; its copy over
  // P_B (the X_{i+1,i} slot) runs on a copy stream after the step's second
  // product, off the sweep's critical path, and the buffer is reused two steps
  // later.
  hipStream_t sc = dry ? s : cx->copy;
  const int E0 = 1 + (int)n;
  for (int64_t i = n - 1; i >= 0; --i) {
    // block i's preprocessing and arrow row
    if (!dry) BTA_TRY(hipStreamWaitEvent(s, event_at(1 + (int)i), 0));
    const bool has_sub = i < n - 1;
    const int step = (int)(n - 1 - i);
    set_stage(2, step, 0);
    const double* PB = XB + i * bb;
    const double* PRi = PR + i * ab;
    double* Xb = Xp + (step & 1) * bb;
    if (has_sub) {  // X_{i+1,i} = -(X_{i+1,i+1} P_B + X_{n,i+1}^T P_R)
      if (!dry && step >= 2) BTA_TRY(hipStreamWaitEvent(s, event_at(E0 + 2 * (step - 2) + 1), 0));  // buffer copied out
      GProb p = prob_init();
      p.seg[0] = seg(XD + (i + 1) * bb, b, 0, PB, b, 1, ib, TRI_NONE);
      p.nseg = 1;
      if (a > 0) { p.seg[1] = seg(XR + (i + 1) * ab, b, 1, PRi, b, 1, ia, TRI_NONE); p.nseg = 2; }
      p.Cout = Xb; p.ldc = b;
      p.M = ib; p.N = ib;
      p.alpha = -1.0;
      BTA_TRY(gemm_launch_split(&p, 1, s, SK, sp.split_doubles, sp.split_max));
    }
    set_stage(2, step, 1);
    {  // X_ii = V_i - X_{i+1,i}^T P_B - X_{n,i}^T P_R  (lower, mirrored; no
       // segments when n == 1 and a == 0: the mirror of V_0)
      GProb p = prob_init();
      p.nseg = 0;
      if (has_sub) p.seg[p.nseg++] = seg(Xb, b, 1, PB, b, 1, ib, TRI_NONE);
      if (a > 0) p.seg[p.nseg++] = seg(XR + i * ab, b, 1, PRi, b, 1, ia, TRI_NONE);
      p.Cin = XD + i * bb; p.Cout = XD + i * bb; p.ldc = b;
      p.M = ib; p.N = ib;
      p.alpha = -1.0; p.beta = 1.0;
      p.lower_tiles = 1;
      p.store = ST_LOWER_MIRROR;
      BTA_TRY(gemm_launch_split(&p, 1, s, SK, sp.split_doubles, sp.split_max));
    }
    set_stage(2, step, 3);
    if (has_sub) {
      if (!dry) {
        BTA_TRY(hipEventRecord(event_at(E0 + 2 * step), s));
        BTA_TRY(hipStreamWaitEvent(sc, event_at(E0 + 2 * step), 0));
      }
      BTA_TRY(copy2d_launch(Xb, b, 0, XB + i * bb, b, 0, ib, ib, 1, sc));
      if (!dry) BTA_TRY(hipEventRecord(event_at(E0 + 2 * step + 1), sc));
    }
  }
  // the last copy (step n-1) before the call's work on `s` is complete
  if (!dry && n > 1) BTA_TRY(hipStreamWaitEvent(s, event_at(E0 + 2 * (int)(n - 1) + 1), 0));
  return hipSuccess;
}

// Whether two windows of one launch share an element (exact rectangle test
// when both have the same leading dimension, byte spans otherwise).
static bool windows_meet(const Window& x, const Window& y) {
  const intptr_t bx = reinterpret_cast<intptr_t>(x.base), by = reinterpret_cast<intptr_t>(y.base);
  const intptr_t ex = bx + 8 * ((x.rows - 1) * x.ld + x.cols), ey = by + 8 * ((y.rows - 1) * y.ld + y.cols);
  if (ex <= by || ey <= bx) return false;
  if (x.ld != y.ld || (bx - by) % 8 != 0) return true;
  const int64_t ox = (bx - std::min(bx, by)) / 8, oy = (by - std::min(bx, by)) / 8;
  const int64_t rx = ox / x.ld, cx = ox % x.ld, ry = oy / y.ld, cy = oy % y.ld;
  if (cx + x.cols > x.ld || cy + y.cols > y.ld) return true;
  return rx < ry + y.rows && ry < rx + x.rows && cx < cy + y.cols && cy < cx + x.cols;
}

// Host dry run of selinv_launch with fake, widely separated array bases:
// every window any launch would touch must lie inside one array (inputs are
// never written out of place), and no launch may write an element that it
// also reads through another window (identical windows are the epilogue's
// read-then-write of its own C tile).  In place (outputs = inputs) the same
// checks run with the bounds of the shared arrays.  Returns 0 when all hold.
static int selinv_dry_run(int64_t n, int64_t b, int64_t a, bool inplace) {
  const SelinvPlan sp = selinv_plan(n, b, a);
  const uintptr_t G = uintptr_t(1) << 40;
  const size_t sz[9] = {(size_t)(n * b * b) * 8, (size_t)((n - 1) * b * b) * 8, (size_t)(n * a * b) * 8, (size_t)(a * a) * 8,
                        (size_t)(n * b * b) * 8, (size_t)((n - 1) * b * b) * 8, (size_t)(n * a * b) * 8, (size_t)(a * a) * 8,
                        sp.bytes};
  auto base = [&](int k) { return reinterpret_cast<double*>((uintptr_t)(k + 1) * G); };
  const int xo = inplace ? 0 : 4;
  DryRecorder rec;
  g_dry = &rec;
  hipError_t e = selinv_launch(sp, n, b, a, base(0), base(1), base(2), base(3), base(xo), base(xo + 1), base(xo + 2),
                               base(xo + 3), reinterpret_cast<void*>(base(8)), nullptr);
  g_dry = nullptr;
  if (e != hipSuccess) return 1;
  for (const Window& w : rec.windows) {
    if (w.rows <= 0 || w.cols <= 0) continue;
    const uintptr_t addr = reinterpret_cast<uintptr_t>(w.base);
    const int arr = (int)(addr / G) - 1;
    if (arr < 0 || arr > 8) return 2;
    if (w.cols > w.ld) return 3;
    const size_t first = addr - (uintptr_t)(arr + 1) * G;
    const size_t last = first + 8 * ((size_t)(w.rows - 1) * w.ld + (w.cols - 1));
    if (last + 8 > sz[arr]) return 4;
    if (!inplace && w.write && arr < 4) return 5;
  }
  for (size_t i = 0; i < rec.windows.size(); ++i) {
    const Window& x = rec.windows[i];
    if (!x.write || x.rows <= 0 || x.cols <= 0) continue;
    for (size_t j = 0; j < rec.windows.size(); ++j) {
      const Window& y = rec.windows[j];
      if (j == i || y.op != x.op || y.rows <= 0 || y.cols <= 0) continue;
      const bool same = y.base == x.base && y.rows == x.rows && y.cols == x.cols && y.ld == x.ld;
      if (!same && windows_meet(x, y)) return 6;
    }
  }
  return 0;
}

int selinv_dry_check(int64_t n, int64_t b, int64_t a) {
  const int r = selinv_dry_run(n, b, a, false);
  if (r) return r;
  const int q = selinv_dry_run(n, b, a, true);
  return q ? 10 + q : 0;
}

}  // namespace bta

BTA_TESTING_API int bta_internal_selinv_dry_check(int64_t n, int64_t b, int64_t a) {
  return bta::selinv_dry_check(n, b, a);
}
