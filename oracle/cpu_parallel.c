/*
 * cpu_parallel.c -- the oracle's reduce, scan and transpose loops spread over
 * the host's cores with OpenMP.  MEASUREMENT BASELINE ONLY: the benchmark's
 * CPU leg times these beside the single-thread oracle, so that the GPU
 * figures can be read against a whole host as well as one core.  Nothing in
 * the GPU library includes, links or calls this file, and the tests check it
 * against the single-thread oracle.
 *
 *   - reduce    : each thread sums a contiguous chunk in int64, the chunk
 *                 sums are added (integer addition: the exact sum);
 *   - scan      : two passes over contiguous chunks (chunk sums, then each
 *                 chunk scanned from its carry), wrapping modulo 2^32, which
 *                 equals the sequential definition bit for bit;
 *   - transpose : out[c][r] = in[r][c] as 32-bit patterns, 64 x 64 blocks
 *                 shared out over the threads.
 *
 * Build: gcc -O2 -std=c11 -fopenmp -shared -fPIC.
 */
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>

int omp_threads(void) { return omp_get_max_threads(); }

int64_t omp_reduce_i32(const int32_t* x, int64_t n) {
  int64_t s = 0;
#pragma omp parallel for reduction(+ : s) schedule(static)
  for (int64_t i = 0; i < n; ++i) s += x[i];
  return s;
}

void omp_scan_i32(const int32_t* x, int32_t* y, int64_t n) {
  const int T = omp_get_max_threads();
  uint32_t* carry = (uint32_t*)calloc((size_t)T + 1, sizeof(uint32_t));
#pragma omp parallel num_threads(T)
  {
    const int t = omp_get_thread_num(), nt = omp_get_num_threads();
    const int64_t lo = n * t / nt, hi = n * (t + 1) / nt;
    uint32_t s = 0;
    for (int64_t i = lo; i < hi; ++i) s += (uint32_t)x[i];
    carry[t + 1] = s;
#pragma omp barrier
#pragma omp single
    for (int k = 1; k <= nt; ++k) carry[k] += carry[k - 1];
    uint32_t acc = carry[t];
    for (int64_t i = lo; i < hi; ++i) {
      acc += (uint32_t)x[i];
      y[i] = (int32_t)acc;
    }
  }
  free(carry);
}

void omp_transpose_u32(const uint32_t* in, uint32_t* out, int64_t rows, int64_t cols) {
  const int64_t B = 64;
  const int64_t br = (rows + B - 1) / B, bc = (cols + B - 1) / B;
#pragma omp parallel for schedule(static)
  for (int64_t blk = 0; blk < br * bc; ++blk) {
    const int64_t r0 = blk / bc * B, c0 = blk % bc * B;
    const int64_t r1 = r0 + B < rows ? r0 + B : rows, c1 = c0 + B < cols ? c0 + B : cols;
    for (int64_t r = r0; r < r1; ++r)
      for (int64_t c = c0; c < c1; ++c) out[c * rows + r] = in[r * cols + c];
  }
}
