/* fastmm -- single-precision C = A*B by Winograd's variant of Strassen's
 * recursion with MFMA leaf products, for AMD Instinct MI355X (gfx950).
 *
 * The operation: the paper computes C = AB for operands of any shape
 * (Section 3.1) by a recursion over the quadrant split of equation (1)
 * (quadrant 0 is ceil(m/2) x ceil(n/2), quadrant 3 floor(m/2) x floor(n/2))
 * that hands a small enough problem to a leaf product (Table 2) computing
 * c_ij = sum_k a_ik b_kj (equation (6)).  Its leaf call moves the operands to
 * the device, runs the kernel and moves the result back, and returns only
 * when done, like a function call (Section 3.3).  The fast 7-product
 * recursion in place of the classic 8-product one (Table 1) is the paper's
 * stated next step (Section 4.3, closing remarks); this library performs it:
 * per level S1..S4 / T1..T4 pre-additions, seven sub-products, U post-
 * additions (Winograd's schedule), down to a leaf cutoff.
 *
 * Conventions for every entry point
 *   - Matrices are row-major FP32: element (i, j) of X is X[i * ldx + j].
 *   - Return value: FASTMM_SUCCESS (0) or a negative fastmm_status; the text
 *     of the last error of the calling thread is fastmm_get_last_error().
 *   - Arguments are validated before anything is written: on
 *     FASTMM_ERROR_INVALID_VALUE or FASTMM_ERROR_NOT_SUPPORTED the outputs are
 *     untouched.
 *   - Every call is synchronous: it is enqueued on the library stream
 *     (fastmm_set_stream) and returns after that stream has drained.  With
 *     host operands the top recursion level runs piece by piece, alternating
 *     between the library stream and a second compute stream of the
 *     library's (FASTMM_PIPE_STREAMS=1: the library stream alone), while two
 *     copy streams move operand blocks in and result blocks out (set
 *     FASTMM_PIPELINE=0 to copy everything first instead).  One or two
 *     compute streams give bit for bit the same result; the pipelined
 *     Winograd product splits its inner recursion by bands and so differs
 *     from the copy-first (and device-resident) one in the last bits, while
 *     a plain product is bit for bit the same on every path.  The other
 *     streams start after the work queued on the library stream before the
 *     call, and the call returns once all of them have drained.
 *   - The caller owns A, B and C; the library never keeps them.  The library
 *     owns its workspace (device memory for the recursion's temporaries and
 *     for staging host operands), which grows on demand and is released by
 *     fastmm_finalize().
 *   - No C++ exception crosses this interface.  Calls are serialised by one
 *     process-wide lock.
 */
#ifndef FASTMM_H
#define FASTMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  FASTMM_SUCCESS = 0,
  FASTMM_ERROR_INVALID_VALUE = -1, /* bad size, ld, pointer, depth or overlap */
  FASTMM_ERROR_OUT_OF_MEMORY = -2, /* workspace over device memory or the limit */
  FASTMM_ERROR_DEVICE = -3,        /* a HIP call failed; message has the reason */
  FASTMM_ERROR_NOT_SUPPORTED = -4  /* e.g. A, B, C not all device or all host */
} fastmm_status;

enum { FASTMM_AUTO = -1 }; /* depth < 0 (or tile < 0): let the planner choose */

/* Planner modes (fastmm_plan). */
enum {
  FASTMM_PLAN_DEFAULT = 0,   /* fixed rule: deepest split with leaf >= 1280; 64x64
                                tiles when 128x128 ones would number under 512 */
  FASTMM_PLAN_MODEL = 1,     /* learned cost model chooses depth and tile among all
                                candidates (mean predicted time of its networks),
                                keeping DEFAULT's choice unless another is predicted
                                1% faster; untrained: EXHAUSTIVE */
  FASTMM_PLAN_EXHAUSTIVE = 2 /* time every candidate on the device, cache it */
};

/* Leaf tile shapes (BM x BN of C per workgroup). */
enum {
  FASTMM_TILE_128x128 = 0,
  FASTMM_TILE_256x128 = 1,
  FASTMM_TILE_128x64 = 2,
  FASTMM_TILE_64x64 = 3,
  FASTMM_TILE_128x128_K32 = 4, /* 128x128, K-slabs of 32 */
  FASTMM_TILE_256x128_W8 = 5,  /* 256x128 on 8 wavefronts */
  FASTMM_TILE_256x256_W8 = 6,  /* 256x256 on 8 wavefronts */
  FASTMM_TILE_128x256 = 7,
  /* Precision forms of the leaf, never chosen by the planner.  Each FP32
   * operand element becomes hi + lo in 16 bits and every product is taken as
   * hi*hi + hi*lo + lo*hi, accumulated in FP32 on the 16-bit matrix cores;
   * the quadrant additions stay FP32.  fastmm_gemm_ex (device or host
   * operands) first packs both operands of every leaf as hi/lo tiles
   * (workspace about the size of the FP32 leaf operands) and runs 256x256
   * tiles on them; fastmm_rmul runs BF16X3 on 128x128 tiles that
   * split in registers and rejects FP16X3 (FASTMM_ERROR_NOT_SUPPORTED).
   * BF16X3: split BF16, about 2^-16 relative accuracy per product instead of
   * FP32's 2^-24.
   * FP16X3: scaled split FP16.  Each row of a leaf's left operand and each
   * column of its right operand is scaled by the power of two that brings
   * its largest magnitude into [2^14, 2^15) (a pass over the operands before
   * the leaf, exponents kept in the workspace), split into hi + lo FP16, and
   * the scales are undone on the result: about 2^-21 relative accuracy per
   * product. */
  FASTMM_TILE_BF16X3 = 8,
  FASTMM_TILE_FP16X3 = 9
};

typedef struct {
  int depth;              /* Winograd levels to take (0 = plain MFMA SGEMM) */
  int64_t leaf;           /* leaf cutoff passed to fastmm_gemm */
  int tile;               /* FASTMM_TILE_* of the leaf kernel */
  size_t workspace_bytes; /* device workspace of the plan's temporaries (S, T, P
                             blocks, packed split-precision operands); staging
                             copies of host or misaligned operands come on top */
  double predicted_ms;    /* model prediction or measured time; <0 unknown */
  int source;             /* FASTMM_PLAN_* mode that produced it */
} fastmm_plan_t;

typedef struct {
  int depth;               /* levels actually taken by the last call */
  int tile;                /* leaf tile used */
  int64_t leaves;          /* number of leaf products (7^depth per problem) */
  int64_t leaf_m, leaf_k, leaf_n; /* leaf extents (single-problem calls) */
  double leaf_flops;       /* sum of 2*m*n*k over leaves */
  double add_bytes;        /* algorithmic bytes of the pre/post additions */
  double transfer_bytes;   /* host<->device bytes moved */
  int launches;            /* kernel launches issued */
  size_t workspace_bytes;  /* device workspace in use */
  /* Phase times of the last call from HIP events on the library's streams,
   * in milliseconds; -1 when profiling is off (fastmm_set_profiling) or the
   * phase is not timed on that path.  leaf_ms is the time during which at
   * least one leaf launch of the call ran: the union of the launches'
   * intervals (host operands: the pieces' launches on the two compute
   * streams overlap). */
  double h2d_ms, preadd_ms, leaf_ms, postadd_ms, d2h_ms, total_ms;
  int leaf_launches;       /* grouped leaf launches of the call */
  int graph_replayed;      /* batched: 1 if a cached HIP graph was replayed */
} fastmm_stats_t;

/* C = A*B.  M, N, K >= 0.  lda >= max(1,K), ldb >= max(1,N), ldc >= max(1,N).
 * A, B, C must all be device memory or all host memory (pinned or pageable;
 * host operands are staged through the workspace and the transfer is part
 * of the call, as in the paper's three-step leaf call, Section 3.3).
 * M == 0 or N == 0: nothing is done.  K == 0: C is set to zero.
 * depth >= 0: at most that many Winograd levels (0 = classic product on the
 * MFMA leaf kernel); depth < 0: the planner chooses depth, leaf and tile,
 * except that with host operands a product whose smallest extent is under
 * 6656 takes depth 0 (there the transfers bound the call, and the plain
 * product's pipeline finishes sooner).
 * leaf: a node (m, k, n) splits iff levels remain and
 * floor(min(m, k, n) / 2) >= max(leaf, 1) (leaf = 3008 reproduces the
 * paper's recursion point 6016, Section 3.1).  depth > 16 is invalid.
 * C must not overlap A or B.  M above 2^31 - 1, K or N above 2^31 - 4, lda
 * above 2^21 or ldb above 2^24 give FASTMM_ERROR_NOT_SUPPORTED (the leaf
 * kernels address a tile's slab with 32-bit offsets, and operands are
 * padded to multiples of 4 columns).  Every argument is checked before the
 * device is touched.  Device operands whose rows are not 16-byte aligned, or
 * whose K or N is not a multiple of 4, are first copied into zero-padded
 * workspace buffers (host operands always are): A and B are only read. */
int fastmm_gemm(int64_t M, int64_t N, int64_t K, const float* A, int64_t lda, const float* B,
                int64_t ldb, float* C, int64_t ldc, int depth, int64_t leaf);

/* As fastmm_gemm with an explicit leaf tile (FASTMM_TILE_*, or < 0 for the
 * planner's or the default choice). */
int fastmm_gemm_ex(int64_t M, int64_t N, int64_t K, const float* A, int64_t lda,
                   const float* B, int64_t ldb, float* C, int64_t ldc, int depth, int64_t leaf,
                   int tile);

/* For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  The same
 * product as fastmm_gemm (same schedule, same kernels, bit for bit the same
 * result), run in a fixed workspace of FASTMM_NOALLOC_WORKSPACE_BYTES that
 * the library holds in a statically allocated device array: reserved on
 * every GPU the library is loaded on, held until the process ends, shared by
 * every call on that GPU (calls of one process are serialised and return
 * when done; nothing else may use it concurrently).  No device or pinned
 * allocation happens in the call (the schedule itself is built in host heap
 * memory).
 *   - A, B, C must be device memory with 16-byte aligned rows of A and B,
 *     lda and ldb multiples of 4 and K, N multiples of 4 (what fastmm_gemm
 *     would otherwise copy into staging buffers); else
 *     FASTMM_ERROR_NOT_SUPPORTED.  The current device must be the one the
 *     library was initialised on.
 *   - depth < 0 takes the planner's fixed rule (FASTMM_PLAN_DEFAULT), which
 *     needs no device; depth >= 0 and leaf as in fastmm_gemm.
 *   - A product whose temporaries and descriptors need more than the fixed
 *     workspace gives FASTMM_ERROR_OUT_OF_MEMORY (the message states both
 *     sizes) before anything is written; a smaller depth needs less.
 *   - Other arguments and errors as fastmm_gemm. */
enum { FASTMM_NOALLOC_WORKSPACE_BYTES = 256 << 20 };
int fastmm_gemm_noalloc(int64_t M, int64_t N, int64_t K, const float* A, int64_t lda,
                        const float* B, int64_t ldb, float* C, int64_t ldc, int depth,
                        int64_t leaf);

/* C = A*B by the paper's classic recursion (Table 1): eight sub-products per
 * level over the quadrant split of equation (1), the second product of each
 * result quadrant accumulated (C += AB), down to the same stop rule as
 * fastmm_gemm (depth >= 0 levels, leaf cutoff; leaf = 3008 is the paper's
 * recursion point 6016, Section 3.1).  A comparator: it performs all 2MNK
 * flops.  Leaves run on the MFMA kernel `tile`, one grouped launch per
 * reduction chunk (2^depth launches).  Arguments, residency and errors as
 * fastmm_gemm. */
int fastmm_rmul(int64_t M, int64_t N, int64_t K, const float* A, int64_t lda, const float* B,
                int64_t ldb, float* C, int64_t ldc, int depth, int64_t leaf, int tile);

/* count independent products C[i] = A[i]*B[i], each with its own extents and
 * leading dimensions (same rules as fastmm_gemm, per problem).  The paper
 * runs two independent products at once, one per GPU, to fill its devices
 * (Section 4.2, the two-GPU measurement); here many uneven products share
 * each launch of one device.  depth == NULL: each problem's depth from
 * the planner (mode set by fastmm_set_plan_mode), always with 128x128 tiles
 * (the batch's shared leaf launch fills the device): DEFAULT's fixed rule,
 * or, in the MODEL and EXHAUSTIVE modes, the fastest predicted or timed
 * depth among those whose leaf launch would fill the device on its own, when
 * it is at least 5% faster than the fixed rule's; depth != NULL: 128x128
 * tiles and leaf[i] (NULL: the default cutoff 1280).  Every level of
 * every problem is one grouped launch (or one per group of up to three levels,
 * the additions of levels that halve exactly); the launch sequence is captured once
 * per set of shapes and plans into a HIP graph and replayed.  A call that
 * repeats one of the last eight device-operand calls exactly (problems,
 * pointers, leading dimensions, depth and leaf arrays, planner mode and
 * state, stream) replays its graph without validating, planning or
 * building again (unless FASTMM_WORKSPACE_LIMIT or FASTMM_POISON=1 is set:
 * those act on every call); its descriptors are uploaded again, so the operands'
 * contents may change between calls, not their addresses or extents.  All
 * problems are validated first: on error nothing is written. */
int fastmm_gemm_batched(int count, const int64_t* M, const int64_t* N, const int64_t* K,
                        const float* const* A, const int64_t* lda, const float* const* B,
                        const int64_t* ldb, float* const* C, const int64_t* ldc, const int* depth,
                        const int64_t* leaf);

/* Choose (depth, leaf, tile) for an M x K by K x N product.  The paper picks
 * its leaf engine by problem size against fixed thresholds (Table 2 and the
 * K0 = 400, K1 ~ 3000 operating points of Section 3.2); here the choice is
 * made per shape by a rule, by exhaustive timing, or by a learned cost model.
 * out must be non-NULL. */
int fastmm_plan(int64_t M, int64_t N, int64_t K, int mode, fastmm_plan_t* out);

/* Planner mode used when depth < 0 is passed (default FASTMM_PLAN_DEFAULT). */
int fastmm_set_plan_mode(int mode);

/* Load / save the planner's state: the timing database (JSON) and the cost
 * model weights (raw little-endian FP32, FASTMM_MODEL_NETS x
 * FASTMM_MLP_PARAMS values: the networks one after another).  NULL path:
 * skip. */
int fastmm_planner_load(const char* timing_db_path, const char* model_path);
int fastmm_planner_save(const char* timing_db_path, const char* model_path);

/* Train the cost model on the timing database with the GPU forward/backward
 * and Adam kernels: each of its FASTMM_MODEL_NETS networks takes `epochs`
 * passes of minibatches of `batch` at learning rate lr, network j drawing its
 * initial weights and minibatch order from seed + j.  The paper sets its leaf
 * thresholds by hand from measurements (Section 3.2, Table 2); the model
 * learns them from this library's own timings.  Mean final training loss of
 * the networks in *loss (may be NULL). */
int fastmm_planner_train(int epochs, int batch, float lr, uint64_t seed, float* loss);

/* Number of timing records in the planner's database. */
int64_t fastmm_planner_records(void);

/* The paper keeps, per device, an "MM queue": the device's memory context,
 * its buffers, its compiled kernels and the command queue every product is
 * issued on, created once and reused by every call (Section 3.3).  Here the
 * library's state plays that role: one workspace, pinned staging, cached
 * graphs and a command stream.
 *
 * Run all kernels on this HIP stream (a hipStream_t; NULL: the library's own
 * stream, created at default priority).  The call first drains the stream in
 * use; later calls are ordered after any work the caller queued on the new
 * stream before them, and still return only when their own work on it is
 * done.  The caller keeps ownership of the stream and must not destroy it
 * while it is set. */
int fastmm_set_stream(void* hip_stream);

/* Record HIP events per phase in every later call (fastmm_get_stats). */
int fastmm_set_profiling(int on);

/* Structure counts and phase times of the last successful product call. */
int fastmm_get_stats(fastmm_stats_t* out);

/* Message of the calling thread's last error ("" if none): what failed in
 * the MM queue's last command (Section 3.3), e.g. the HIP error string of a
 * failed copy or launch.  Valid until the thread's next fastmm call. */
const char* fastmm_get_last_error(void);

/* Tear the MM queue down (Section 3.3 builds it once before any product):
 * drain the stream, release the workspace, the pinned staging, the cached
 * graphs, the events and the library's own streams, and forget a stream set
 * by fastmm_set_stream.  The next call builds everything again; calling it
 * twice, or before any other call, does nothing. */
void fastmm_finalize(void);

/* ---- Kernel-level entry points (device pointers only), for verification of
 * the individual steps against a CPU evaluation. ---- */

/* One level of pre-additions on one operand.  X is the parent operand
 * (rows x cols valid, ldx); the quadrants are ceil(rows/2) x ceil(cols/2)
 * per equation (1), zero-padded.  side 0 (A operand) writes S1..S4, side 1
 * (B operand) writes T1..T4, as four consecutive dense h_r x h_c blocks at
 * out (h_r = ceil(rows/2), h_c = ceil(cols/2)). */
int fastmm_preadd(int side, int64_t rows, int64_t cols, const float* X, int64_t ldx,
                  float* out);

/* One level of post-additions: P holds P1..P7 as seven consecutive dense
 * h_r x h_c blocks; writes C11, C12, C21, C22 into C (rows x cols, ldc),
 * clipped to rows <= 2 h_r, cols <= 2 h_c. */
int fastmm_postadd(int64_t h_r, int64_t h_c, const float* P, float* C, int64_t ldc,
                   int64_t rows, int64_t cols);

/* ---- Cost-model network kernels (device pointers only).  Network 5 -> 64
 * -> 64 -> 1 with ReLU; flat parameters [W1 (5x64), b1, W2 (64x64), b2,
 * W3 (64x1), b3], W stored (fan_in, fan_out) row-major; X is (batch x 5).
 * Loss: mean squared error.  These are the planner's training kernels. ---- */
enum { FASTMM_MLP_PARAMS = 4609, FASTMM_MODEL_NETS = 3 };

/* y[batch] = network(X).  */
int fastmm_mlp_forward(int batch, const float* params, const float* X, float* y);

/* grad[4609] = d loss / d params for targets t; *loss_out (device, 1 float)
 * receives the loss (may be NULL). */
int fastmm_mlp_backward(int batch, const float* params, const float* X, const float* t,
                        float* grad, float* loss_out);

/* One Adam step (step counts from 1) on params with moments m, v. */
int fastmm_mlp_adam(const float* grad, float* params, float* m, float* v, int step, float lr,
                    float beta1, float beta2, float eps);

#ifdef __cplusplus
}
#endif

#endif /* FASTMM_H */
