/*
 * desc.h -- C ABI of the MI355X (gfx950) data-parallel kernel library.
 *
 * The operations are the four computations the Descend paper evaluates
 * (Sec. 5: block-wide parallel reduction, matrix transposition, scan and
 * matrix multiplication) and their segmented / batched forms.  The argument
 * conventions follow the paper's statement of a GPU function (Sec. 1,
 * Listing 2; Sec. 3.3-3.4):
 *
 *   - inputs are shared, read-only references and outputs are unique
 *     references: an output must not overlap any input (DESC_ERR_ALIAS);
 *   - every array lives in GPU memory: a pointer the GPU would reach through
 *     host memory is rejected (DESC_ERR_HOST_POINTER), the error the paper's
 *     separation of cpu.mem and gpu.global rules out statically;
 *   - sizes are element counts, never bytes, and the library derives the
 *     launch shape itself, so a caller cannot launch more threads than there
 *     are elements (the bytes-versus-elements mistake of Sec. 2);
 *   - memory is owned by the caller; the library frees nothing it did not
 *     allocate and allocates nothing in these calls.
 *
 * Every call is asynchronous and ordered on `stream` (a hipStream_t; NULL is
 * the default stream); none reads device memory from the host, allocates or
 * synchronises, so a call may be captured into a HIP graph.  Arguments are
 * checked in the order null -> size -> host pointer -> alias -> workspace,
 * and a failed check returns before anything is launched.
 *
 * Workspace contract.  Calls that take `ws` keep a little state in it
 * between calls (a generation number and counters) so that each runs as a
 * single launch without a clearing pass.  A workspace must be filled with
 * zero bytes once before its first use; after that the library leaves it
 * ready for the next call.  Calls that share one workspace must be ordered
 * (one stream, or synchronised): overlapping calls on one workspace race.
 * The required size comes from the matching *_workspace() query.
 */
#ifndef DESC_H
#define DESC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  DESC_OK = 0,
  DESC_ERR_NULL = -1,          /* a required pointer is NULL */
  DESC_ERR_SIZE = -2,          /* negative size, or bytes overflow int64 */
  DESC_ERR_HOST_POINTER = -3,  /* pointer is host memory or unknown to HIP */
  DESC_ERR_ALIAS = -4,         /* an output overlaps an input */
  DESC_ERR_WORKSPACE = -5,     /* workspace smaller than the query returned */
  DESC_ERR_UNSUPPORTED = -6,   /* mode or shape the library does not provide */
  DESC_ERR_HIP = -7,           /* a HIP call failed; see desc_last_hip_error() */
  DESC_ERR_ALIGNMENT = -8,     /* pointer not aligned to its element size */
  DESC_ERR_LIMIT = -9          /* size above an allocation-free call's fixed scratch */
} desc_status;

/* Human-readable name of a status code (static storage). */
const char* desc_status_string(desc_status s);

/* Raw hipError_t behind the last DESC_ERR_HIP returned to this thread. */
int desc_last_hip_error(void);

/* Library version, as MAJOR * 10000 + MINOR * 100 + PATCH. */
int desc_version(void);

/*
 * Pointer classifier hook, for embedding and for exercising the argument
 * checks on a machine without a GPU.  `fn(p)` returns 0 if `p` is GPU
 * memory, 1 if it is host memory and -1 if it is unknown.  NULL restores the
 * default classifier (hipPointerGetAttributes).  Process-wide.
 */
typedef int (*desc_pointer_classifier)(const void* p);
void desc_set_pointer_classifier(desc_pointer_classifier fn);

/* ------------------------------------------------------------------------
 * Device status of a workspace.  A few failures can only be seen on the GPU,
 * after the call has returned DESC_OK; the kernels record them in the
 * 32-bit status word at byte 4 of the workspace:
 *   DESC_DEV_WAIT_LIMIT  a block's bounded wait for another block ran out.
 *                        The output of that call is wrong.  Causes: a
 *                        workspace that was not zeroed before its first use,
 *                        two calls overlapping on one workspace, or a wait
 *                        limit set below (debugging).  Sticky: it stays set
 *                        until read.  Reported by the workspaces of
 *                        desc_reduce_i32, desc_reduce_op (min/max, float
 *                        sum), desc_scan_i32 / desc_scan_exclusive_i32,
 *                        desc_scan_f32, the segmented reduce and scan and
 *                        the batched scan.
 *   DESC_DEV_PLANES      desc_gemm_grouped or desc_gemm_strided_batched in
 *                        DESC_GEMM_BF16X3 mode found that the bf16 planes do
 *                        not fit the workspace (or a dimension above 2^40)
 *                        and computed nothing.  Written by every such call
 *                        (0 when it computed), so it describes the last call.
 *
 * desc_workspace_status: a kernel on `stream` copies the word into
 * status[0] (int32, GPU memory) and resets it to 0; stream-ordered after the
 * calls before it, no host read, capture-safe.  `ws` is the workspace of one
 * of the calls above (8-byte aligned, ws_bytes >= 64).  On another
 * workspace of the library the value has no meaning, and resetting it does
 * not disturb later calls (those workspaces are scratch, rewritten by every
 * call, or leave the word alone).
 *
 * desc_workspace_set_wait_limit (debugging): every bounded wait of a call on
 * this workspace gives up after at most max_polls polls (0: at once, without
 * polling); max_polls < 0 restores the built-in limit (2^20 polls).  Kept in
 * the workspace header until changed (zeroing the workspace restores the
 * default).  For the workspaces that report DESC_DEV_WAIT_LIMIT.  A wait
 * that gives up leaves its block to finish with a partial value, so every
 * kernel still ends normally; the affected outputs are unspecified.
 * max_polls above 2^32 - 2 is DESC_ERR_SIZE.
 * ---------------------------------------------------------------------- */
enum {
  DESC_DEV_OK = 0,
  DESC_DEV_WAIT_LIMIT = 1,
  DESC_DEV_PLANES = 2
};
desc_status desc_workspace_status(void* ws, size_t ws_bytes, int32_t* status, void* stream);
desc_status desc_workspace_set_wait_limit(void* ws, size_t ws_bytes, int64_t max_polls,
                                          void* stream);

/* ------------------------------------------------------------------------
 * Reduction (Sec. 5, "block-wide parallel reduction", read as the full sum).
 * out[0] = sum of in[0..n), exact: int32 values are summed in int64.  n = 0
 * writes 0.  `in` int32[n] (may be NULL when n = 0), `out` int64[1].
 * ---------------------------------------------------------------------- */
size_t desc_reduce_i32_workspace(int64_t n);
desc_status desc_reduce_i32(const int32_t* in, int64_t n, int64_t* out, void* ws,
                            size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * Two more reductions over the block-wide structure of the sum (Sec. 5,
 * "block-wide parallel reduction", with other operators and element types).
 *
 * desc_reduce_minmax_i32: out[0] = min, out[1] = max of in[0..n); n = 0
 * writes the identities {INT32_MAX, INT32_MIN}.  `out` int32[2].
 *
 * desc_reduce_sum_f32: out[0] = the sum of the float32 values in[0..n),
 * accumulated in FP64 in an order fixed by the element indices and n alone
 * (not by the input address, the run or the hardware's scheduling), so
 * equal inputs give bit-equal results.  The order: elements are taken in
 * chunks of 4096; lane j (0..255) of block b adds, from 0.0, elements
 * 1024u + 4j + e (u, e = 0..3) of chunks b, b + G, b + 2G, ... in that order;
 * the 256 lane values of a block meet in a tree (inside each 64-lane wave
 * lane i adds lane i^32, then i^16, 8, 4, 2, 1; then the four waves as
 * (w0 + w1) + (w2 + w3)); lane t of the last block adds the values of blocks
 * t, t + 256, ... from 0.0 and the same tree combines those.  G = min(max(
 * ceil(n / 4096), 1), 2048).  The error against the exact sum is at most
 * d * 2^-53 * sum|in[i]|, d = 16 ceil(ceil(n / 4096) / G) + ceil(G / 256)
 * + 16.  Non-finite inputs follow IEEE addition (NaN, or +inf with -inf,
 * gives NaN).  n = 0 writes +0.0.  `out` double[1], 8-byte aligned.
 *
 * Both: `in` 4-byte aligned (may be NULL when n = 0); one workspace of
 * desc_reduce_op_workspace(n) bytes, zeroed before first use, may serve both
 * calls but no other entry point.
 * ---------------------------------------------------------------------- */
size_t desc_reduce_op_workspace(int64_t n);
desc_status desc_reduce_minmax_i32(const int32_t* in, int64_t n, int32_t* out, void* ws,
                                   size_t ws_bytes, void* stream);
desc_status desc_reduce_sum_f32(const float* in, int64_t n, double* out, void* ws,
                                size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * Inclusive scan (Sec. 5, "scan"): out[i] = in[0] + ... + in[i] modulo 2^32
 * (two's-complement wrap), int32 in and out, out-of-place.  n = 0 launches
 * nothing.
 * ---------------------------------------------------------------------- */
size_t desc_scan_i32_workspace(int64_t n);
desc_status desc_scan_i32(const int32_t* in, int32_t* out, int64_t n, void* ws,
                          size_t ws_bytes, void* stream);

/* Exclusive form of the same scan: out[0] = 0, out[i] = in[0] + ... +
 * in[i-1] modulo 2^32.  Same single pass, same workspace
 * (desc_scan_i32_workspace(n) bytes), same checks. */
desc_status desc_scan_exclusive_i32(const int32_t* in, int32_t* out, int64_t n, void* ws,
                                    size_t ws_bytes, void* stream);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, hosts that forbid hipMalloc): desc_scan_i32 without a
 * workspace.  Its state lives in a fixed device array of the library
 * (2 MiB + 64 bytes per GPU, held until the process ends, set up and
 * cleared by the first call on each GPU); n up to DESC_SCAN_NOALLOC_MAX_N
 * elements, larger n returns DESC_ERR_LIMIT before anything is launched.
 * Every call on one GPU shares that array: calls that overlap in time race
 * (order them on one stream or synchronise), and a device-side failure of
 * a call is not reported (it can only come from such an overlap).  Same
 * result, checks and stream semantics as desc_scan_i32; nothing is
 * allocated, freed or synchronised. */
#define DESC_SCAN_NOALLOC_MAX_N ((int64_t)1 << 31)
desc_status desc_scan_i32_noalloc(const int32_t* in, int32_t* out, int64_t n, void* stream);

/* ------------------------------------------------------------------------
 * Inclusive scan of float32 values (the scan of Sec. 5 over floats):
 * out[i] = the prefix in[0] + ... + in[i], accumulated in FP64 in an order
 * fixed by the element indices and n alone, and rounded once to float32, so
 * equal inputs give bit-equal outputs on every run and at every address.
 * The order: tiles of 65536 elements, each [16 waves][16 rounds][64 lanes]
 * [4]; within a tile, lane sums of four, a wave scan in DPP order and
 * sequential carries over rounds and waves; across tiles, the aggregates of
 * each group of 64 tiles meet in a butterfly and the groups' sums are
 * chained in order (the full statement is in the kernel's source).  Error
 * against the exact prefix S_i: at most 2^-24 |S_i| + 2^-149 +
 * d 2^-53 sum_{k<=i} |in[k]|, d = ceil(ceil(n / 65536) / 64) + 160.
 * Non-finite inputs follow IEEE addition; zero prefixes come out as +0.
 * Out-of-place; `in`, `out` 4-byte aligned; n = 0 launches nothing.  The
 * workspace (desc_scan_f32_workspace(n) bytes, zeroed before first use)
 * serves no other entry point.
 * ---------------------------------------------------------------------- */
size_t desc_scan_f32_workspace(int64_t n);
desc_status desc_scan_f32(const float* in, float* out, int64_t n, void* ws, size_t ws_bytes,
                          void* stream);

/* ------------------------------------------------------------------------
 * The paper's own forms of the two operations above (Sec. 5), for
 * comparison with the single-pass forms.
 *
 * Block-wide reduction: out[b] = exact int64 sum of in[b*E .. min(n,(b+1)*E))
 * for b < ceil(n / E), one GPU block per chunk, each block combining its
 * threads' sums in a split/synchronise tree (Sec. 2-3).  E (elements per
 * block) must be a multiple of 1024 (DESC_ERR_SIZE otherwise); `out` holds
 * ceil(n / E) int64.  n = 0 launches nothing.  No workspace.
 *
 * Two-kernel scan: the inclusive scan of desc_scan_i32 computed as kernel 1,
 * the sum of every 65536-element tile into the workspace, then kernel 2, each
 * tile's carry (the sum of the tile sums before it) and its scan.  It reads
 * the input twice (3n words of traffic against 2n).  The workspace holds one
 * word per tile, scratch between the two kernels (no initialisation).
 * ---------------------------------------------------------------------- */
desc_status desc_reduce_blocks_i32(const int32_t* in, int64_t n, int64_t E, int64_t* out,
                                   void* stream);
size_t desc_scan_two_pass_i32_workspace(int64_t n);
desc_status desc_scan_two_pass_i32(const int32_t* in, int32_t* out, int64_t n, void* ws,
                                   size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * Transposition (Sec. 1, Listings 1-2; Sec. 5, "matrix transposition"):
 * `in` is a row-major rows x cols matrix of 32-bit words, `out` receives
 * the row-major cols x rows matrix with out[c][r] = in[r][c].  The words are
 * moved as bit patterns.  The batched form transposes `batch` matrices
 * stored one after another in both arrays.  Any size is accepted (ragged
 * edges included); rows = 0 or cols = 0 launches nothing.
 * ---------------------------------------------------------------------- */
desc_status desc_transpose_f32(const float* in, float* out, int64_t rows, int64_t cols,
                               void* stream);
desc_status desc_transpose_batched_f32(const float* in, float* out, int64_t batch,
                                       int64_t rows, int64_t cols, void* stream);

/* The same transposition for elements of elem_bytes = 1, 2, 4 or 8 bytes
 * (8: the doubles of the paper's own example), moved as bit patterns;
 * pointers aligned to the element size.  Other sizes return
 * DESC_ERR_UNSUPPORTED; elem_bytes = 4 is desc_transpose_batched_f32. */
desc_status desc_transpose_batched(const void* in, void* out, int64_t elem_bytes, int64_t batch,
                                   int64_t rows, int64_t cols, void* stream);

/* ------------------------------------------------------------------------
 * Matrix multiplication (Sec. 5, "matrix multiplication"; the paper fixes
 * neither precision nor layout): C = A * B with A M x K, B K x N and C
 * M x N, all row-major FP32 with row strides lda >= K, ldb >= N, ldc >= N
 * (in elements).  C is overwritten (K = 0 writes zeros).  C must not overlap
 * A, B or the workspace.  Modes:
 *   DESC_GEMM_F32         FP32 products, FP32 accumulation (matrix cores);
 *                         no workspace (ws may be NULL).
 *   DESC_GEMM_BF16X3      a = hi + lo with hi = bf16(a), lo = bf16(a - hi)
 *                         (round to nearest even), likewise b;
 *                         C = Ah*Bh + Ah*Bl + Al*Bh on the bf16 matrix cores
 *                         with FP32 accumulation.
 *   DESC_GEMM_FP8_ROWCOL  row i of A scaled by 448 / max_k |a_ik| and column
 *                         j of B by 448 / max_k |b_kj|, encoded as OCP e4m3
 *                         (round to nearest even, saturating), multiplied on
 *                         the fp8 matrix cores with FP32 accumulation and
 *                         rescaled: C_ij = (alpha_i/448)(beta_j/448) sum q q.
 * The two low-precision modes prepare padded operands in the workspace
 * (desc_gemm_workspace bytes, 256-byte aligned); its contents need no
 * initialisation and are overwritten by every call.
 * ---------------------------------------------------------------------- */
typedef enum {
  DESC_GEMM_F32 = 0,
  DESC_GEMM_BF16X3 = 1,
  DESC_GEMM_FP8_ROWCOL = 2
} desc_gemm_mode;

size_t desc_gemm_workspace(desc_gemm_mode mode, int64_t M, int64_t N, int64_t K);
desc_status desc_gemm(desc_gemm_mode mode, int64_t M, int64_t N, int64_t K, const float* A,
                      int64_t lda, const float* B, int64_t ldb, float* C, int64_t ldc, void* ws,
                      size_t ws_bytes, void* stream);

/* Operand preparation steps of the precision modes, with the conversions the
 * GEMM modes use (bit patterns as uint16 bfloat16 and uint8 e4m3 codes):
 *   split_bf16_rows : hi, lo (M x K, stride ldh) of the rows of A (stride lda);
 *   split_bf16_cols : hi^T, lo^T (N x K, stride ldh) of the columns of B;
 *   quant_e4m3_rows : codes (M x K, stride ldq) and scale[i] = alpha_i / 448;
 *   quant_e4m3_cols : codes of the columns of B transposed (N x K, stride ldq)
 *                     and scale[j] = beta_j / 448; needs a workspace of
 *                     desc_quant_e4m3_cols_workspace(K, N) bytes (scratch,
 *                     no initialisation). */
desc_status desc_split_bf16_rows(const float* A, int64_t M, int64_t K, int64_t lda,
                                 uint16_t* hi, uint16_t* lo, int64_t ldh, void* stream);
desc_status desc_split_bf16_cols(const float* B, int64_t K, int64_t N, int64_t ldb,
                                 uint16_t* hi_t, uint16_t* lo_t, int64_t ldh, void* stream);
desc_status desc_quant_e4m3_rows(const float* A, int64_t M, int64_t K, int64_t lda, uint8_t* q,
                                 int64_t ldq, float* scale, void* stream);
size_t desc_quant_e4m3_cols_workspace(int64_t K, int64_t N);
desc_status desc_quant_e4m3_cols(const float* B, int64_t K, int64_t N, int64_t ldb,
                                 uint8_t* q_t, int64_t ldq, float* scale, void* ws,
                                 size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * Grouped GEMM (batched Sec. 5 matrix multiplication): G independent
 * problems C_g = A_g * B_g, each with its own shape, row strides and
 * pointers, described by a device array of desc_gemm_problem (row-major
 * FP32, lda >= K, ldb >= N, ldc >= N as for desc_gemm; an M, N <= 0 problem
 * is skipped, K = 0 writes zeros).  The descriptors and the memory they
 * point to are read on the GPU only; the library cannot check them on the
 * host, so they are a precondition (valid GPU pointers, C_g not overlapping
 * any operand).  The workspace needs no initialisation.  Modes:
 *   DESC_GEMM_F32     one planning kernel and one persistent kernel;
 *                     desc_gemm_grouped_workspace(G) bytes, 64-byte aligned.
 *   DESC_GEMM_BF16X3  desc_gemm's BF16X3 arithmetic per problem.  A planning
 *                     kernel, then, in the built-in configuration, one
 *                     persistent kernel over 128 x 128 output tiles that
 *                     splits the FP32 operands into hi and lo while staging
 *                     them (no operand copies).  Problems with lda or ldb
 *                     above 2^24, and every problem in the "tile64" and
 *                     "tile128" configurations, go through bf16 planes: a
 *                     persistent kernel splits their operands into planes
 *                     padded to multiples of 128 (M, N) and 64 (K, at least
 *                     64) inside the workspace, and a persistent kernel
 *                     computes their tiles from the planes.  The workspace
 *                     (256-byte aligned) must hold
 *                     desc_gemm_grouped_workspace_for(DESC_GEMM_BF16X3, G,
 *                     problems_host) bytes, computed from a host copy of the
 *                     descriptors (M, N, K, lda, ldb are read) for the
 *                     configuration in effect when the call is made.  The
 *                     host can only check the planning part; the planning
 *                     kernel checks the rest on the GPU, and if the planes do
 *                     not fit, or a problem has M, N or K above 2^40, it
 *                     computes nothing and sets the device status word (byte
 *                     4 of the workspace) to DESC_DEV_PLANES, 0 after a call
 *                     that computed (see desc_workspace_status).
 * desc_gemm_grouped_workspace_for returns 0 for an unsupported mode, G < 0,
 * problems_host = NULL with G > 0, or a refused shape.
 * ---------------------------------------------------------------------- */
typedef struct {
  int64_t M, N, K;
  int64_t lda, ldb, ldc;
  const float* A;
  const float* B;
  float* C;
} desc_gemm_problem;

size_t desc_gemm_grouped_workspace(int64_t G);
size_t desc_gemm_grouped_workspace_for(desc_gemm_mode mode, int64_t G,
                                       const desc_gemm_problem* problems_host);
desc_status desc_gemm_grouped(desc_gemm_mode mode, int64_t G, const desc_gemm_problem* problems,
                              void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * Strided batched GEMM: C_g = A_g B_g for g < G, one shape M x N x K, with
 * A_g = A + g * stride_a, B_g = B + g * stride_b, C_g = C + g * stride_c
 * (strides in elements, >= 0; row-major, lda >= K, ldb >= N, ldc >= N as
 * for desc_gemm).  Modes DESC_GEMM_F32 and DESC_GEMM_BF16X3, with the
 * arithmetic of desc_gemm_grouped: a kernel writes the G problem
 * descriptors into the back of the workspace and the grouped kernels run
 * on them.  The workspace (256-byte aligned, no initialisation) must hold
 * desc_gemm_strided_batched_workspace(mode, G, M, N, K, lda, ldb) bytes (0
 * for an unsupported mode or a refused shape).  Checks as for desc_gemm on
 * the spans of all batches; outputs of two batches that would overlap
 * (stride_c < (M - 1) ldc + N with G > 1) are DESC_ERR_ALIAS.  G = 0, M = 0
 * or N = 0 launches nothing; K = 0 writes zeros.
 * ---------------------------------------------------------------------- */
size_t desc_gemm_strided_batched_workspace(desc_gemm_mode mode, int64_t G, int64_t M, int64_t N,
                                           int64_t K, int64_t lda, int64_t ldb);
desc_status desc_gemm_strided_batched(desc_gemm_mode mode, int64_t G, int64_t M, int64_t N,
                                      int64_t K, const float* A, int64_t lda, int64_t stride_a,
                                      const float* B, int64_t ldb, int64_t stride_b, float* C,
                                      int64_t ldc, int64_t stride_c, void* ws, size_t ws_bytes,
                                      void* stream);

/* ------------------------------------------------------------------------
 * Uniform batched reduce and scan: `in` is a row-major batch x len int32
 * matrix, each row one segment of the segmented forms below (offsets
 * s * len, written by a kernel into the back of the workspace).
 *   reduce : out[b] = exact int64 sum of row b (0 when len = 0).
 *   scan   : out[b][i] = in[b][0] + ... + in[b][i] modulo 2^32.
 * Workspaces (8-byte aligned, zeroed once before first use as for the
 * segmented forms, whose workspace is their front part): the matching
 * *_batched_i32_workspace(batch, len) bytes.  batch = 0 (and, for the scan,
 * len = 0) launches nothing.
 * ---------------------------------------------------------------------- */
size_t desc_reduce_batched_i32_workspace(int64_t batch, int64_t len);
desc_status desc_reduce_batched_i32(const int32_t* in, int64_t batch, int64_t len, int64_t* out,
                                    void* ws, size_t ws_bytes, void* stream);
size_t desc_scan_batched_i32_workspace(int64_t batch, int64_t len);
desc_status desc_scan_batched_i32(const int32_t* in, int32_t* out, int64_t batch, int64_t len,
                                  void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * Segmented forms (batched Sec. 5 reduction and scan): `in` holds n int32
 * values; segment s covers positions [offsets[s], offsets[s+1]) for
 * s < num_segments, with offsets int64[num_segments + 1] in GPU memory,
 * non-decreasing and within [0, n] (a precondition the library does not
 * check, since that would read device memory on the host; offsets that
 * break it give unspecified results but no access outside the arrays).
 *   reduce : out[s] = exact int64 sum of segment s (0 for an empty segment).
 *   scan   : out[i] = in[offsets[s]] + ... + in[i] modulo 2^32 for i in
 *            segment s; positions outside every segment are not written.
 * The reduce of up to 8192 segments runs as one persistent launch (every
 * block plans the units of all segments in its LDS and then takes every
 * G-th unit, G the blocks that fit the device at once; no block waits for
 * another before the end of the call); the scan, a larger reduce and the
 * batched forms run as a one-block planning kernel and one main kernel.
 * All state lives in the workspace, so every form may be captured in a HIP
 * graph and replayed.  The workspace is zeroed once before its first use
 * (its header holds the device status word, the wait limit and the
 * generation that tags the state words); one workspace may serve both
 * operations if it has the larger size.
 * ---------------------------------------------------------------------- */
size_t desc_reduce_segmented_i32_workspace(int64_t n, int64_t num_segments);
desc_status desc_reduce_segmented_i32(const int32_t* in, int64_t n, const int64_t* offsets,
                                      int64_t num_segments, int64_t* out, void* ws,
                                      size_t ws_bytes, void* stream);
size_t desc_scan_segmented_i32_workspace(int64_t n, int64_t num_segments);
desc_status desc_scan_segmented_i32(const int32_t* in, int32_t* out, int64_t n,
                                    const int64_t* offsets, int64_t num_segments, void* ws,
                                    size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * Copy of n 32-bit words: the plain bandwidth ceiling the HBM-bound
 * operations are measured against.  `in` and `out` must not overlap.
 * ---------------------------------------------------------------------- */
desc_status desc_copy_32(const void* in, void* out, int64_t n, void* stream);

/* Reversal of n 32-bit words, out[i] = in[n - 1 - i] (bit patterns moved):
 * the copy read through the `reverse` view (Sec. 3.2).  `in` and `out` must
 * not overlap; 4-byte aligned; n = 0 launches nothing. */
desc_status desc_reverse_u32(const void* in, void* out, int64_t n, void* stream);

/* ------------------------------------------------------------------------
 * Configurations.  Tile shapes are compile-time parameters of the kernels
 * (the paper keeps sizes as nats in the types); each operation is compiled
 * for a few shapes and a table picks one per problem-size class.  The
 * built-in table can be overridden per class, or from a text file written
 * by the offline tuner with lines "<op name> <size class> <config name>"
 * ('#' starts a comment).  Process-wide; changing it while calls are in
 * flight only affects later calls.
 * ---------------------------------------------------------------------- */
typedef enum {
  DESC_OP_REDUCE_I32 = 0,
  DESC_OP_SCAN_I32 = 1,
  DESC_OP_TRANSPOSE_32 = 2,
  DESC_OP_COPY_32 = 3,
  DESC_OP_GEMM_F32 = 4,
  DESC_OP_GEMM_BF16X3 = 5,
  DESC_OP_GEMM_FP8 = 6,
  DESC_OP_SEG_REDUCE_I32 = 7,
  DESC_OP_SEG_SCAN_I32 = 8,
  DESC_OP_GEMM_GROUPED = 9,
  DESC_OP_GEMM_GROUPED_BF16X3 = 10
} desc_op;

int desc_config_count(desc_op op);                     /* 0 for an op not built */
const char* desc_config_name(desc_op op, int cfg);     /* NULL if out of range */
const char* desc_op_name(desc_op op);                  /* NULL if not built */
/* Size class (0..3) of a problem: element count, M*N*K for GEMM, and the
 * problem count G for the grouped GEMM (on the GEMM scale: G < 2^24 is
 * class 0). */
int desc_size_class(desc_op op, int64_t size);
/* cfg < 0 restores the built-in choice; DESC_ERR_UNSUPPORTED if out of range. */
desc_status desc_config_set(desc_op op, int size_class, int cfg);
int desc_config_get(desc_op op, int size_class);       /* -1 if out of range */
desc_status desc_config_load(const char* path);

#ifdef __cplusplus
}
#endif

#endif /* DESC_H */
