// Split-BF16 row pass on the CDNA4 matrix cores.
//
// The row pass of the separable CZT (Sec. 2.6) is a product of the stripe
// (S aperture rows x N columns) with the N x M kernel matrix
//   A[i][q] = exp(2 pi i (beta c_i^2/2 - alpha c_i d_q))
// (the x chirp of Eq. 2 times the Eq. 10 Fourier kernel), i.e. a complex GEMM
// whose left operand is the binary zone mask, generated on the fly from the
// exact integer radius (Sec. 2.2, Eq. 4).  A is stored once per plan as two
// BF16 planes, hi = bf16(A) and lo = bf16(A - hi), for the real and imaginary
// parts; the mask is exact in BF16, so T = mask.A_hi + mask.A_lo (two MFMA
// products, float32 accumulation) carries A to about 2^-16 relative.
//
// Table layout: At[plane][c][i], plane 0 = hi, 1 = lo, c = 2q + {0: re, 1: im},
// i = 0 .. Npad-1 (zero beyond N), so an MFMA B operand (8 consecutive k of one
// column) is one 16-byte load and the accumulator columns interleave re/im as
// the float2 T buffer does.

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
__device__ __forceinline__ double bf16_to_double(uint16_t h) { return (double)__uint_as_float((uint32_t)h << 16); }

__global__ __launch_bounds__(256) void k_build_split_table(InstDev d, uint16_t *At) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int q = blockIdx.y;
  if (i >= d.Npad) return;
  const int M = d.M;
  const int64_t plane = (int64_t)2 * M * d.Npad;
  uint16_t hr = 0, hi_ = 0, lr = 0, li = 0;
  if (i < d.N) {
    const double c = (double)i - 0.5 * (double)(d.N - 1);
    const double dq = (double)q - 0.5 * (double)M + d.sx;
    const double ph = (0.5 * d.beta * (c * c));
    const double lin = d.alpha * c * dq;
    const double t = (ph - rint(ph)) - (lin - rint(lin));
    const double2 a = cexp_turns(t);
    hr = bf16_rne((float)a.x);
    hi_ = bf16_rne((float)a.y);
    lr = bf16_rne((float)(a.x - bf16_to_double(hr)));
    li = bf16_rne((float)(a.y - bf16_to_double(hi_)));
  }
  At[(int64_t)(2 * q) * d.Npad + i] = hr;
  At[(int64_t)(2 * q + 1) * d.Npad + i] = hi_;
  At[plane + (int64_t)(2 * q) * d.Npad + i] = lr;
  At[plane + (int64_t)(2 * q + 1) * d.Npad + i] = li;
}

constexpr int kWaves = 4;
constexpr int kRowsPerWave = 32;
constexpr int kTileRows = kWaves * kRowsPerWave;  // 128
constexpr int kColBlocks = 2;                     // 32 real columns each
constexpr int kTileCols = 32 * kColBlocks;        // real columns per work-group

// One work-group: kTileRows aperture rows x kTileCols real columns of T.
// MFMA 32x32x16 BF16 operand layout: lane l supplies row (A) / column (B)
// l % 32 and k = 8 (l / 32) .. 8 (l / 32) + 7.
__global__ __launch_bounds__(256) void k_row_pass_split(InstDev d, int64_t row_begin, int64_t row_end,
                                                        float *__restrict__ T) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t N = d.N;
  const int M = d.M;
  const int64_t tile_r0 = row_begin + (int64_t)blockIdx.x * kTileRows;
  const int c0 = blockIdx.y * kTileCols;  // first real column
  // K range: chord of the tile row closest to the optical axis
  const double halfN = 0.5 * (double)(N - 1);
  int64_t rlast = tile_r0 + kTileRows - 1;
  if (rlast > row_end - 1) rlast = row_end - 1;
  int64_t rc = (int64_t)halfN;
  if (rc < tile_r0) rc = tile_r0;
  if (rc > rlast) rc = rlast;
  double cc = (double)(2 * rc - N + 1);
  // the row with the smallest |c| in [tile_r0, rlast]
  {
    const int64_t alt = rc + 1 <= rlast ? rc + 1 : rc;
    const double ca = (double)(2 * alt - N + 1);
    if (fabs(ca) < fabs(cc)) cc = ca;
  }
  const double rem = d.kmax - cc * cc;
  int64_t k_lo = 0, k_hi = 0;
  if (rem >= 0.0) {
    int64_t m = (int64_t)sqrt(rem);
    while ((double)(m + 1) * (double)(m + 1) <= rem) ++m;
    while (m > 0 && (double)m * (double)m > rem) --m;
    const int64_t lo2 = N - 1 - m, hi2 = N - 1 + m;
    k_lo = lo2 >= 0 ? (lo2 + 1) / 2 : 0;
    k_hi = (hi2 / 2 < N - 1 ? hi2 / 2 : N - 1) + 1;
    k_lo = k_lo / 16 * 16;
    k_hi = (k_hi + 15) / 16 * 16;
    if (k_hi > d.Npad) k_hi = d.Npad;
  }
  // this lane's aperture row and its K offset within a 16-wide step
  const int64_t row = tile_r0 + wave * kRowsPerWave + (lane & 31);
  const bool row_ok = row < row_end;
  const double cj = (double)(2 * row - N + 1);
  const double bj = cj * cj;
  const int koff = 8 * (lane >> 5);
  const int col = lane & 31;
  const int64_t plane = (int64_t)2 * M * d.Npad;
  const uint16_t *Bh[kColBlocks];
#pragma unroll
  for (int cb = 0; cb < kColBlocks; ++cb) Bh[cb] = d.A + (int64_t)(c0 + cb * 32 + col) * d.Npad + koff;

  f32x16 acc[kColBlocks];
#pragma unroll
  for (int cb = 0; cb < kColBlocks; ++cb)
#pragma unroll
    for (int e = 0; e < 16; ++e) acc[cb][e] = 0.0f;

  for (int64_t k = k_lo; k < k_hi; k += 16) {
    // mask operand: 8 consecutive columns i = k + koff .. +7 of this lane's row
    uint32_t pk[4];
#pragma unroll
    for (int e2 = 0; e2 < 4; ++e2) {
      uint32_t w = 0;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int64_t i = k + koff + 2 * e2 + h;
        const double ci = (double)(2 * i - N + 1);
        const double K = ci * ci + bj;
        const int zone = (int)(K * d.kappa);
        const bool open = row_ok && i < N && K <= d.kmax && (((zone & 1) ^ d.centre_open) != 0);
        w |= (open ? 0x3f80u : 0u) << (16 * h);
      }
      pk[e2] = w;
    }
    u32x4 av = {pk[0], pk[1], pk[2], pk[3]};
    const bf16x8 a = __builtin_bit_cast(bf16x8, av);
#pragma unroll
    for (int cb = 0; cb < kColBlocks; ++cb) {
      const u32x4 bh = *(const u32x4 *)(Bh[cb] + k);
      const u32x4 bl = *(const u32x4 *)(Bh[cb] + plane + k);
      acc[cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, __builtin_bit_cast(bf16x8, bh), acc[cb], 0, 0, 0);
      acc[cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, __builtin_bit_cast(bf16x8, bl), acc[cb], 0, 0, 0);
    }
  }
  // accumulator layout (32x32 MFMA): register v of lane l holds
  // row 8 (v / 4) + 4 (l / 32) + (v % 4), column l % 32.
#pragma unroll
  for (int cb = 0; cb < kColBlocks; ++cb) {
    const int c = c0 + cb * 32 + col;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int rloc = 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
      const int64_t r = tile_r0 + wave * kRowsPerWave + rloc;
      if (r < row_end && c < 2 * M) T[(r - row_begin) * (int64_t)(2 * M) + c] = acc[cb][v];
    }
  }
}

}  // namespace

hipError_t launch_build_split_table(const Plan &p, const InstHost &ih, char *ws, hipStream_t st) {
  (void)p;
  InstDev d = ih.dev;
  const dim3 grid((unsigned)((d.Npad + 255) / 256), (unsigned)d.M);
  hipLaunchKernelGGL(k_build_split_table, grid, dim3(256), 0, st, d, (uint16_t *)(ws + ih.off_A));
  return hipGetLastError();
}

hipError_t launch_row_pass_split(const InstDev &d, int32_t S, int64_t row_begin, int64_t row_end, float2 *T,
                                 hipStream_t st) {
  (void)S;
  const int64_t rows = row_end - row_begin;
  if (rows <= 0) return hipSuccess;
  if ((2 * d.M) % kTileCols != 0) return hipErrorInvalidValue;
  const dim3 grid((unsigned)((rows + kTileRows - 1) / kTileRows), (unsigned)(2 * d.M / kTileCols));
  hipLaunchKernelGGL(k_row_pass_split, grid, dim3(256), 0, st, d, row_begin, row_end, (float *)T);
  return hipGetLastError();
}

}  // namespace fzp
