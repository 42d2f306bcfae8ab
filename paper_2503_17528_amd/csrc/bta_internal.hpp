// Host-side interfaces between the C ABI and the kernel launchers.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <array>
#include <map>
#include <string>
#include <vector>

namespace bta {

// ---------------------------------------------------------------- factor
// Columns by which a diagonal task is dispatched ahead of its column (at most
// this many tasks wait on tasks with larger tickets; the factor kernel keeps
// more resident workgroups than that).
constexpr int FACTOR_LOOKAHEAD = 8;

struct FactorPlan {
  int T, TA, look;
  int sub_delay;  // SUB tasks of column c are dispatched with column c + sub_delay of their step
  long long nflags, step_full, step_last, ntasks;
  size_t off_ctl, off_flags, off_Wd, off_Wt, off_P, bytes;
};
FactorPlan factor_plan(int64_t n, int64_t b, int64_t a);
hipError_t factor_launch(const FactorPlan& fp, int64_t n, int64_t b, int64_t a,
                         const double* D, const double* B, const double* R, const double* T,
                         double* LD, double* LB, double* LR, double* LT,
                         void* work, int64_t* info, hipStream_t stream, int num_cus,
                         unsigned long long* trace = nullptr);

// One matrix of a batch (sizes and the pointers of include/bta.h's bta_desc).
struct BatchMatrix {
  int64_t n, b, a;
  const double *D, *B, *R, *T;
  double *LD, *LB, *LR, *LT;
  double *XD, *XB, *XR, *XT;
  int64_t* info;
};

struct FactorBatchPlan {
  int count = 0;
  std::vector<FactorPlan> plans;
  std::vector<long long> flag_off;
  std::vector<std::array<size_t, 2>> ws_off;
  long long nflags = 0, ntasks = 0, nseg = 0;
  size_t off_ctl = 0, off_mats = 0, off_segs = 0, off_flags = 0, bytes = 0;
  int order = 1;  // segment order: 0 by chain position, 1 by the fraction of the chain
};
FactorBatchPlan factor_batch_plan(int count, const int64_t* n, const int64_t* b, const int64_t* a, int num_cus);
hipError_t factor_batch_launch(const FactorBatchPlan& bp, const BatchMatrix* mats, void* work, hipStream_t stream,
                               int num_cus);

// ---------------------------------------------------------------- grouped GEMM
// One product term: sum_k A(m,k) B(c,k) over a k range.  A(m,k) is
// A[m*lda + k] (at == 0) or A[k*lda + m] (at == 1); B likewise with bt.
// Batched operands advance by s*0 per first batch index and s*1 per second.
enum : int { TRI_NONE = 0, TRI_K_GE_COL = 1, TRI_K_GE_ROW = 2, TRI_K_LE_ROW = 3, TRI_K_LE_COL = 4 };
enum : int { ST_FULL = 0, ST_LOWER = 1, ST_LOWER_MIRROR = 3 };

struct GSeg {
  const double* A;
  const double* B;
  int64_t lda, ldb;
  int64_t sA0, sA1, sB0, sB1;
  int K;
  int at, bt, tri;
};

struct GProb {
  GSeg seg[2];
  int nseg;
  const double* Cin;  // may be null when beta == 0
  double* Cout;
  int64_t ldc, sC0, sC1;
  int M, N;
  int nb0, nb1;        // batch = nb0 x nb1
  double alpha, beta;  // Cout = beta*Cin + alpha*sum
  int store;           // ST_*
  int lower_tiles;     // only tiles with tile_row >= tile_col
  // filled by gemm_launch
  int ntm, ntn, tiles_per_batch;
  long long tile_begin;
};

constexpr int GEMM_MAX_PROBS = 4;
struct GemmArgs {
  GProb p[GEMM_MAX_PROBS];
  int nprob;
  long long ntiles;
};

// Launch the problems (at most GEMM_MAX_PROBS) as one grid; empty problems are skipped.
hipError_t gemm_launch(GProb* probs, int nprob, hipStream_t stream);
// One problem whose 64 x 64 tiles fill less than half of the CUs, with plain
// (not triangular) operands: its k range is split into S <= GEMM_MAX_PROBS
// parts computed as one launch into ws (S*M*N doubles), then summed in split
// order by a second launch with the problem's alpha, beta and store mode.
// Anything else (or ws == nullptr) goes to gemm_launch.
hipError_t gemm_launch_split(GProb* probs, int nprob, hipStream_t stream, double* ws, size_t ws_doubles,
                             int smax = GEMM_MAX_PROBS);
// The split count gemm_launch_split would use for p (1 = no split; at most smax).
int splitk_factor(const GProb& p, size_t ws_doubles, int smax = GEMM_MAX_PROBS);

// ---------------------------------------------------------------- selinv
struct SelinvPlan {
  int64_t chunk;  // blocks per preprocessing chunk
  size_t split_doubles;  // split-k partials of the sweep products (0: no split)
  int split_max;         // largest split count of a sweep product (tuning knob "split")
  size_t off_W, off_T1, off_PR, off_Xp, off_WT, off_split, bytes;
};
// split: reserve the split-k partials of the sweep products (single-matrix
// calls; the batched selected inversion has parallelism across matrices).
SelinvPlan selinv_plan(int64_t n, int64_t b, int64_t a, bool split = true);
hipError_t selinv_launch(const SelinvPlan& sp, int64_t n, int64_t b, int64_t a,
                         const double* LD, const double* LB, const double* LR, const double* LT,
                         double* XD, double* XB, double* XR, double* XT,
                         void* work, hipStream_t stream);

// batched selected inversion
size_t selinv_batch_bytes(int count, const int64_t* n, const int64_t* b, const int64_t* a);
hipError_t selinv_batch_launch(int count, const BatchMatrix* mats, void* work, hipStream_t stream);

// ---------------------------------------------------------------- solve / logdet
size_t solve_work_bytes(int64_t n, int64_t b, int64_t a, int64_t nrhs);
hipError_t solve_launch(int64_t n, int64_t b, int64_t a, const double* LD, const double* LB,
                        const double* LR, const double* LT, double* rhs, int64_t nrhs,
                        void* work, hipStream_t stream);
size_t logdet_work_bytes(int64_t n, int64_t b, int64_t a);
hipError_t logdet_launch(int64_t n, int64_t b, int64_t a, const double* LD, const double* LT,
                         double* out, void* work, hipStream_t stream);
hipError_t logdet_quad_launch(int64_t n, int64_t b, int64_t a, const double* LD, const double* LT, const double* y,
                              const double* x, int64_t nrhs, double* out, void* work, hipStream_t stream);
hipError_t grad_launch(int64_t n, int64_t b, int64_t a, const double* XD, const double* XB, const double* XR,
                       const double* XT, const double* x, int64_t nrhs, const double* scale, double* GD, double* GB,
                       double* GR, double* GT, double* gy, hipStream_t stream);

// ---------------------------------------------------------------- shared small kernels
// Triangular inverse of 64 x 64 diagonal tiles: for batch index (blk, t),
// W tile t of block blk = inverse of lower-triangular L tile t (ragged last
// tile padded with the identity); writes the full 64 x 64 tile of W with
// zeros above the diagonal into W (row-major, ld = m, block stride sW).
hipError_t trinv_diag_tiles_launch(const double* L, int64_t ldL, int64_t sL, double* W, int64_t ldW, int64_t sW,
                                   int m, int nblk, hipStream_t stream);
// Inverses W = L^{-1} of nblk lower-triangular m x m matrices (L: ld ldL,
// block stride sL; W and the scratch T1: ld ldW, block stride sW).  W must be
// zero on entry and receives zeros above the diagonal.  phase/major label the
// launches for the batched recorder.
hipError_t trtri_batched(const double* L, int64_t ldL, int64_t sL, double* W, double* T1, int64_t ldW, int64_t sW,
                         int m, int nblk, hipStream_t s, int phase, int major);
// Fill `count` doubles with zero.
hipError_t fill_zero_launch(double* p, size_t count, hipStream_t stream);
// Copy a rows x cols row-major matrix (batched by nb with strides).
hipError_t copy2d_launch(const double* src, int64_t lds, int64_t ss, double* dst, int64_t ldd, int64_t sd,
                         int rows, int cols, int nb, hipStream_t stream);

int device_cu_count();
// ---------------------------------------------------------------- tuning table (tune.hip)
// Key of a tuned decision: "<arch>|<op>|b=<b>|a=<a>|<knob>".
std::string tune_key(const char* op, int64_t b, int64_t a, const char* knob);
bool tune_get(const std::string& key, long long* out);
// persist: rewrite the BTA_TUNE_CACHE file (when set) with the whole table.
void tune_set(const std::string& key, long long val, bool persist);
// Integer environment override in [lo, hi] (false when unset or invalid).
bool env_int(const char* name, long long lo, long long hi, long long* out);

// Library-owned streams and events for one call.  Every call that needs more
// than the caller's stream leases a context for its whole enqueue sequence
// (SyncLease) and returns it afterwards, so that calls enqueued concurrently by
// different host threads never record each other's events: a stream wait
// refers to the record made before it, and a context's next user only records
// after the previous one has finished enqueueing.  Contexts are created on
// first need (per device, default-priority non-blocking streams) and kept
// until the process ends; they hold no device memory.
struct SyncCtx {
  int dev = -1;
  hipStream_t side = nullptr;     // preprocessing and arrow rows of the selected inversion
  hipStream_t copy = nullptr;     // copy-outs of the backward sweep
  hipStream_t capture = nullptr;  // graph capture of the batched selected inversion
  std::vector<hipEvent_t> ev;
  hipEvent_t event(int k);  // event k of this context (created on demand; nullptr on failure)
};
class SyncLease {
 public:
  SyncLease();  // takes a free context of the current device (or makes one)
  ~SyncLease();
  SyncLease(const SyncLease&) = delete;
  SyncLease& operator=(const SyncLease&) = delete;
  SyncCtx* get() const { return ctx_; }  // nullptr if no context could be made
 private:
  SyncCtx* ctx_ = nullptr;
};

// Host dry run: when a recorder is installed on this thread, the launchers
// above only record what they would touch (no HIP calls).  Used to check
// every operand window against its array bounds on the CPU.
struct Window {
  const void* base;
  int64_t rows, cols, ld;  // row-major window: element (r, c) at base + r*ld + c (doubles)
  bool write;
  int op;  // launch that touches it
};
struct DryRecorder {
  std::vector<Window> windows;
  int op = 0;
  void add(const void* base, int64_t rows, int64_t cols, int64_t ld, bool write) {
    windows.push_back(Window{base, rows, cols, ld, write, op});
  }
};
extern thread_local DryRecorder* g_dry;

// Stage recorder (batched selected inversion): while installed, the launchers
// record their work under the current stage key instead of launching.
struct FillOp { double* p; long long count; };
struct CopyOp { const double* src; int64_t lds, ss; double* dst; int64_t ldd, sd; int rows, cols, nb; };
struct TrinvOp { const double* L; int64_t ldL, sL; double* W; int64_t ldW, sW; int m, nblk; };
struct StageKey {
  int phase, major, minor;
  bool operator<(const StageKey& o) const {
    if (phase != o.phase) return phase < o.phase;
    if (major != o.major) return major < o.major;
    return minor < o.minor;
  }
};
struct StageRecorder {
  StageKey key{0, 0, 0};
  struct Stage {
    int kind = -1;  // 0 gemm, 1 fill, 2 copy, 3 trinv
    std::vector<GProb> gemms;
    std::vector<FillOp> fills;
    std::vector<CopyOp> copies;
    std::vector<TrinvOp> trinvs;
  };
  std::map<StageKey, Stage> stages;
  // cur: the matrix being recorded, cur_n its block count.  ready[m][i]: the
  // stage after which block i of matrix m is ready for the backward sweep
  // (its preprocessing and arrow row done; {-1,-1,-1} if never marked).
  // span > 1: the sweep of every matrix is spread over `span` merged steps
  // (its step s of cur_n becomes s (span-1) / (cur_n-1), strictly increasing),
  // so that short sweeps do not crowd the first steps of the longest one;
  // sweep_block[m][S] = the block matrix m works on at merged step S.
  int cur = -1;
  int64_t cur_n = 0, span = 0;
  std::vector<std::vector<StageKey>> ready;
  std::vector<std::map<int, int64_t>> sweep_block;
  void mark_ready(int64_t i) {
    if (cur < 0) return;
    if ((int)ready.size() <= cur) ready.resize(cur + 1);
    if ((int64_t)ready[cur].size() <= i) ready[cur].resize(i + 1, StageKey{-1, -1, -1});
    ready[cur][i] = key;
  }
  int sweep_step(int s) const { return (span > 1 && cur_n > 1) ? (int)((int64_t)s * (span - 1) / (cur_n - 1)) : s; }
  void note_sweep(int S, int64_t block) {
    if (cur < 0) return;
    if ((int)sweep_block.size() <= cur) sweep_block.resize(cur + 1);
    sweep_block[cur][S] = block;
  }
  void gemm(const GProb& p) { Stage& s = stages[key]; s.kind = 0; s.gemms.push_back(p); }
  void fill(const FillOp& f) { Stage& s = stages[key]; s.kind = 1; s.fills.push_back(f); }
  void copy(const CopyOp& c) { Stage& s = stages[key]; s.kind = 2; s.copies.push_back(c); }
  void trinv(const TrinvOp& t) { Stage& s = stages[key]; s.kind = 3; s.trinvs.push_back(t); }
};
extern thread_local StageRecorder* g_rec;
inline void set_stage(int phase, int major, int minor) {
  if (!g_rec) return;
  if (phase == 2) {  // backward-sweep step `major`: block cur_n - 1 - major
    const int S = g_rec->sweep_step(major);
    if (minor == 0) g_rec->note_sweep(S, g_rec->cur_n - 1 - major);
    major = S;
  }
  g_rec->key = StageKey{phase, major, minor};
}
inline bool recording() { return g_dry != nullptr || g_rec != nullptr; }

// problem-list GEMM launch (device-resident problem array and tile prefix)
hipError_t gemm_list_launch(const GProb* d_probs, const long long* d_tile_begin, int nprob, long long ntiles, int big,
                            hipStream_t stream);
long long gemm_prob_tiles(GProb& p, int tile);
// Products of at most 16 rows with plain k ranges, A by rows, B by k rows, one
// batch entry and a full store; launched one workgroup per 64 columns
// (tile_begin[] as for 64 x 64 tiles).
bool gemm_skinny_ok(const GProb& p);
hipError_t gemm_skinny_list_launch(const GProb* d_probs, const long long* d_tile_begin, int nprob, long long ntiles,
                                   hipStream_t stream);

// Optional per-kernel timing with HIP events recorded on the launch stream
// around each launch of the main kernels (off unless enabled).
enum : int { KT_FACTOR = 0, KT_GEMM = 1, KT_TRINV = 2, KT_OTHER = 3, KT_COUNT = 4 };
bool timing_on();
void timing_mark(int kind, bool start, hipStream_t stream);

}  // namespace bta
