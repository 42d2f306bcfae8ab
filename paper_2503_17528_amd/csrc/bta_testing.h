/*
 * bta_testing.h -- internal hooks of libbta.so for the test suite and the
 * benchmark.  They are not part of the C ABI (include/bta.h): they expose host
 * replays of the kernels' schedules, measurement switches and single kernels,
 * and may change without notice.  They are exported (default visibility) only
 * so that the tests can reach them through ctypes; every other symbol of the
 * library is hidden.  None of them allocates device memory.
 */
#ifndef BTA_TESTING_H
#define BTA_TESTING_H

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#define BTA_TESTING_API extern "C" __attribute__((visibility("default")))

/* ---- factorization (factor.hip) */
/* Override of the DIAG lookahead in band columns for later factorizations
 * (1..64; 0 removes the override); returns the previous override (0 = none;
 * any other argument only queries). */
BTA_TESTING_API int bta_internal_factor_lookahead(int look);
/* The DIAG lookahead (after the T-1 clamp) and the k-loop load path (1 = L2)
 * a factorization of (n, b, a) would use now. */
BTA_TESTING_API int bta_internal_factor_plan_knobs(int64_t n, int64_t b, int64_t a, int* look, int* cached);
/* Cap on the single-matrix factor kernel's workgroups (0 = one per CU);
 * returns the previous value (a negative argument only queries). */
BTA_TESTING_API int bta_internal_factor_max_grid(int g);
/* bta_factor with a trace buffer of 8 words per ticket (device memory); the
 * number of records is returned through *ntasks.  Returns 0 on success. */
BTA_TESTING_API int bta_internal_factor_traced(int64_t n, int64_t b, int64_t a, const double* D, const double* B,
                                               const double* R, const double* T, double* LD, double* LB, double* LR,
                                               double* LT, void* work, int64_t* info, unsigned long long* trace,
                                               long long* ntasks, hipStream_t stream);
/* Override: 1 the factor kernels read their k-loop operand tiles through the
 * L2 where the tiles are cache-line aligned, 0 device-coherent loads, -1 no
 * override.  Returns the previous override (any other argument only queries). */
BTA_TESTING_API int bta_internal_factor_cached_loads(int on);
/* The pivot reciprocal square root of the diagonal-tile Cholesky
 * (hardware estimate + one third-order refinement) applied to count device
 * doubles: d_out[k] = rsqrt_refined(d_in[k]).  Returns 0 on launch success. */
BTA_TESTING_API int bta_internal_rsqrt(const double* d_in, double* d_out, int64_t count, hipStream_t s);
/* Latency probe of the diagonal-tile Cholesky + inverse: one workgroup
 * factors the 64 x 64 SPD tile d_A (row-major) `iters` times with panel
 * variant `var`; d_ticks[0] gets the summed 100 MHz ticks, d_ticks[1] the
 * failure column (0 = none), d_ticks[2..11] the summed phase ticks,
 * d_ticks[12..15] those of the steps inside the diagonal-block inverses (16
 * entries in all), d_L and d_W (64 x 64 each) the factor and its inverse. */
BTA_TESTING_API int bta_internal_diag_link_probe(const double* d_A, double* d_L, double* d_W, long long* d_ticks,
                                                 int iters, int var, hipStream_t s);
/* Round-trip latency of the cross-workgroup flag hand-off between the first
 * and last workgroup of a grid of `grid` (d_flags: 128 zeroed ints); mode 0
 * release/acquire, mode 1 relaxed after a store wait.  d_ticks[0] = summed
 * 100 MHz ticks of `iters` round trips.  Every poll is bounded. */
BTA_TESTING_API int bta_internal_flag_pingpong(int* d_flags, long long* d_ticks, int iters, int mode, int grid,
                                               hipStream_t s);
/* Throughput probe of the factor's k loop: `grid` workgroups each run
 * `steps` double-buffered k steps on 64 x 64 tiles at pseudo-random positions
 * of the first span_rows rows of the row-major matrix d_M (leading dimension
 * ld, a multiple of 64); mode 0 device-coherent loads, 1 no loads, 2 loads
 * through the L2.  d_ticks[g]: workgroup g's 100 MHz ticks; d_out: grid*256. */
BTA_TESTING_API int bta_internal_kloop_probe(const double* d_M, int64_t ld, int64_t span_rows, int steps, int mode,
                                             int grid, long long* d_ticks, double* d_out, hipStream_t s);
/* Host replay of the single-matrix task schedule (0 = valid); counts[7]
 * receives the number of tiles of each task type. */
BTA_TESTING_API int bta_internal_factor_schedule_check(int64_t n, int64_t b, int64_t a, long long* counts);
/* Host replay of the batched task interleaving for `num_cus` workgroups
 * (0 = valid); *ahead receives the largest number of waiting tasks. */
BTA_TESTING_API int bta_internal_factor_batch_check(int count, const int64_t* n, const int64_t* b, const int64_t* a,
                                                    int num_cus, long long* ahead);

/* ---- selected inversion (selinv.hip, batched.hip) */
/* Host dry run of every launch of bta_selinv, out of place and in place: each
 * operand window inside its array, no launch writing what it reads (0 = valid). */
BTA_TESTING_API int bta_internal_selinv_dry_check(int64_t n, int64_t b, int64_t a);
/* Host check of the merged batched plan: the operations merged into one stage
 * touch no element that another of them writes, and in the replayed graph no
 * backward-sweep stage shares a written element with a preprocessing stage it
 * is not ordered after.  0 = valid; 2 = a stage mixes operation kinds, 3 = an
 * overlap inside a stage, 4 = an overlap between the graph's two branches. */
BTA_TESTING_API int bta_internal_selinv_batch_check(int count, const int64_t* n, const int64_t* b, const int64_t* a);
/* The tuning table (tune.hip) as "key=value" lines (up to cap bytes); returns
 * the number of entries.  Keys: "<arch>|<op>|b=<b>|a=<a>|<knob>", e.g. the
 * factor's "look" (DIAG lookahead) and "cached" (L2 loads), the batched
 * selected inversion's per-stage-class "tile128". */
BTA_TESTING_API int bta_internal_autotune_dump(char* out, int cap);
/* Tuning table access: set (in memory), get (0 = found), the key of
 * (op, b, a, knob) for this device, save / load the JSON file at path, clear.
 * The file named by BTA_TUNE_CACHE is loaded on first use and rewritten when
 * a first-use measurement adds an entry. */
BTA_TESTING_API int bta_internal_tune_set(const char* key, long long value);
BTA_TESTING_API int bta_internal_tune_get(const char* key, long long* value);
BTA_TESTING_API int bta_internal_tune_key(const char* op, int64_t b, int64_t a, const char* knob, char* out, int cap);
BTA_TESTING_API int bta_internal_tune_save(const char* path);
BTA_TESTING_API int bta_internal_tune_load(const char* path);
BTA_TESTING_API int bta_internal_tune_clear(void);

/* ---- GEMM engine and measurement (gemm.hip) */
/* GEMM kernel family of the selected inversion (0 automatic, 1 register-staged,
 * 2 direct-to-LDS where allowed, 3..7 one direct-to-LDS body); returns the
 * previous mode (-1 only queries). */
BTA_TESTING_API int bta_internal_gemm_mode(int mode);
/* One product through the grouped GEMM: C = beta*Cin + alpha*sum_k A(m,k) B(c,k). */
BTA_TESTING_API int bta_internal_gemm(int M, int N, int K, const double* A, int64_t lda, int at, const double* B,
                                      int64_t ldb, int bt, int tri, const double* Cin, double* C, int64_t ldc,
                                      double alpha, double beta, int store, int lower_tiles, hipStream_t s);
/* nprob copies of one product (problem q offset by q*stride in A, B and C)
 * through the batched list kernel: 64 x 64 tiles with four LDS stages, or
 * 128 x 128 tiles with big; dlist is device memory of at least
 * 512 * (nprob + 1) bytes; synchronizes `s`.  -1 on a bad nprob (1..64). */
BTA_TESTING_API int bta_internal_gemm_list(int M, int N, int K, const double* A, int64_t lda, int at, const double* B,
                                           int64_t ldb, int bt, int tri, const double* Cin, double* C, int64_t ldc,
                                           double alpha, double beta, int store, int lower_tiles, int nprob,
                                           int64_t strideA, int64_t strideB, int64_t strideC, int big, void* dlist,
                                           hipStream_t s);
/* A product of at most 16 rows through the skinny list kernel, as two k
 * segments [0, K1) and [K1, K) (A by rows, B by k rows, full store); dlist is
 * device memory of at least 512 bytes; synchronizes `s`.  -1 when the product
 * does not qualify. */
BTA_TESTING_API int bta_internal_gemm_skinny(int M, int N, int K, int K1, const double* A, int64_t lda, const double* B,
                                             int64_t ldb, const double* Cin, double* C, int64_t ldc, double alpha,
                                             double beta, void* dlist, hipStream_t s);
/* The same product through the split-k path of the selected inversion's sweep
 * (ws: device partials of ws_doubles; *splits receives the split count used). */
BTA_TESTING_API int bta_internal_gemm_split(int M, int N, int K, const double* A, int64_t lda, int at, const double* B,
                                            int64_t ldb, int bt, const double* Cin, double* C, int64_t ldc,
                                            double alpha, double beta, int store, int lower_tiles, double* ws,
                                            size_t ws_doubles, int* splits, hipStream_t s);
/* Per-kernel HIP-event timing of the main kernels: `kinds` is a bit mask of
 * the kinds recorded (bit 0 factor, 1 GEMM, 2 TRTRI leaves, 3 other; 0 turns
 * timing off) with a pool of 2*max_launches events; not thread safe. */
BTA_TESTING_API int bta_internal_timing(int kinds, int max_launches);
/* Per-kind milliseconds and launch counts of the timed spans (0 = complete). */
BTA_TESTING_API int bta_internal_timing_read(double* ms, long long* launches);
/* Register-only FP64 MFMA rate probe: grid workgroups of 256 threads, each
 * wave running `chains` (8 or 16) independent MFMA chains; d_out holds
 * grid*256 doubles; flops = grid * 4 * iters * chains * 2048. */
BTA_TESTING_API int bta_internal_mfma_probe(double* d_out, int grid, int iters, int chains, hipStream_t s);

#endif /* BTA_TESTING_H */
