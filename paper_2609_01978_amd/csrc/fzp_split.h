// Device helpers shared by the split-BF16 row-pass kernels: the binary-stripe
// GEMM (fzp_gemm.hip) and the complex-stripe GEMM (fzp_cplx.hip).
#pragma once

#include <cstdint>

#include "fzp_device.h"
#include "fzp_internal.h"

namespace fzp {

namespace {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;
typedef __attribute__((__vector_size__(4 * sizeof(uint32_t)))) uint32_t u32x4;

__device__ __forceinline__ uint16_t bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__device__ __forceinline__ u32x4 lds_ld16(const char *p) { return *(const u32x4 *)p; }

// Disc chord of the tile rows [r0, r1] (union = chord of the row nearest the axis),
// in aperture columns [lo, hi).
__device__ __forceinline__ void tile_chord(const InstDev &d, int64_t r0, int64_t r1, int64_t &lo, int64_t &hi) {
  const int64_t N = d.N;
  int64_t rc = (N - 1) / 2;
  if (rc < r0) rc = r0;
  if (rc > r1) rc = r1;
  double cc = fabs((double)(2 * rc - N + 1));
  if (rc + 1 <= r1) cc = fmin(cc, fabs((double)(2 * (rc + 1) - N + 1)));
  const double rem = d.kmax - cc * cc;
  lo = hi = 0;
  if (rem < 0.0) return;
  int64_t m = (int64_t)sqrt(rem);
  while ((double)(m + 1) * (double)(m + 1) <= rem) ++m;
  while (m > 0 && (double)m * (double)m > rem) --m;
  const int64_t lo2 = N - 1 - m, hi2 = N - 1 + m;
  lo = lo2 >= 0 ? (lo2 + 1) / 2 : 0;
  hi = (hi2 / 2 < N - 1 ? hi2 / 2 : N - 1) + 1;
}

// Epilogue of both row-pass GEMMs.  The partial sums are stored column-major,
// Ts[c][r - row_begin] with column stride rs (the chunk's row count), so the
// column pass reads each real column of T contiguously.  Register v of lane l
// holds row 8(v/4) + 4(l/32) + (v%4) of its 32 x 32 block and column l%32: the
// four registers 4a .. 4a+3 are four consecutive rows, one 16-byte store.
__device__ __forceinline__ void store_partials(const f32x16 (&acc)[4][2], float *__restrict__ Ts, int64_t rs, int cbase,
                                               int M2, int64_t rbase, int64_t row_begin, int64_t row_end) {
#pragma unroll
  for (int cb = 0; cb < 2; ++cb) {
    const int c = cbase + cb * 32;
    if (c >= M2) continue;
    float *col = Ts + (int64_t)c * rs - row_begin;
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        const int64_t r = rbase + rb * 32 + 8 * a;
        if (r + 3 < row_end) {
          *(float4 *)(col + r) = make_float4(acc[rb][cb][4 * a], acc[rb][cb][4 * a + 1], acc[rb][cb][4 * a + 2],
                                             acc[rb][cb][4 * a + 3]);
        } else {
#pragma unroll
          for (int e = 0; e < 4; ++e)
            if (r + e < row_end) col[r + e] = acc[rb][cb][4 * a + e];
        }
      }
  }
}

}  // namespace

}  // namespace fzp
