// Row pass on the int8 matrix cores for binary stripes (FZP_FLAG_SPLIT_INT8).
//
// Same product as the split-BF16 row pass (Sec. 2.6: the binary zone mask of
// Eq. 4, generated on the fly, times the N x M kernel matrix
//   A[i][q] = exp(2 pi i (beta c_i^2/2 - alpha c_i d_q))),
// with A held in fixed point instead of a BF16 hi/lo pair: v = rint(A s),
// s = kI8Scale = 16256, split into two balanced int8 digits v = 128 v0 + v1.
// The mask is 0 / 1 in int8, so both digit products sum exactly in int32 and
// the only error is the quantisation of A (at most 0.5 / 16256 = 3.1e-5 per
// component).  Per 32 columns of K the int8 MFMA does the work of two BF16
// MFMA K-steps, so the two digits cost what one BF16 plane does.
//
// Table layout, blocked by 64 aperture columns (one 64-byte row per column and
// block, as the BF16 table's 32-column blocks):
//   A8[digit][i / 64][c][i % 64],  digit 0 = v0, 1 = v1,  c = 2q + {0: re, 1: im},
// zero for i >= N.  It occupies the first half of the split table's space.

#include <atomic>
#include <cmath>

#include "fzp_split.h"

namespace fzp {

namespace {

__global__ __launch_bounds__(256) void k_build_i8_table(InstDev d, int8_t *__restrict__ A8) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int q = blockIdx.y;
  if (i >= d.Npad) return;
  const int M = d.M;
  const int64_t plane = (int64_t)2 * M * d.Npad;  // bytes per digit plane
  const int64_t b8 = (i >> 6) * (int64_t)(2 * M) * 64 + (i & 63);
  int8_t r0 = 0, r1 = 0, i0 = 0, i1 = 0;
  if (i < d.N) {
    const double c = (double)i - 0.5 * (double)(d.N - 1);
    const double dq = (double)q - 0.5 * (double)M + d.sx;
    const double ph = (0.5 * d.beta * (c * c));
    const double lin = d.alpha * c * dq;
    const double2 a = cexp_turns((ph - rint(ph)) - (lin - rint(lin)));
    // v1 = v mod 128 in [-64, 63], v0 = (v - v1) / 128 in [-127, 127]
    const int vr = (int)rint(a.x * kI8Scale), vi = (int)rint(a.y * kI8Scale);
    const int lr = ((vr + 64) & 127) - 64, li = ((vi + 64) & 127) - 64;
    r0 = (int8_t)((vr - lr) >> 7);
    i0 = (int8_t)((vi - li) >> 7);
    r1 = (int8_t)lr;
    i1 = (int8_t)li;
  }
  A8[b8 + (int64_t)(2 * q) * 64] = r0;
  A8[b8 + (int64_t)(2 * q + 1) * 64] = i0;
  A8[plane + b8 + (int64_t)(2 * q) * 64] = r1;
  A8[plane + b8 + (int64_t)(2 * q + 1) * 64] = i1;
}

constexpr int kTC = 128;  // real columns per tile (64 complex ROI columns), as the BF16 row pass

// LDS slab rows are 64 bytes; chunk j of row r sits at chunk j ^ swz8(r), which
// keeps the MFMA operand reads (32 consecutive rows, one chunk) conflict-free.
__device__ __forceinline__ int swz8(int r) { return ((r >> 1) ^ (r >> 3)) & 3; }

// ---------------------------------------------------------------------------
// The row-pass kernel: T = (128 (mask . v0) + mask . v1), in int32 (the
// column pass scales it by 1 / 16256); |T| <= 65536 (127 * 128 + 64) < 2^31
// for K segments up to 65536 columns.  One v_mfma_i32_32x32x32_i8 covers 32
// columns of K.
//
// Same work-group tile (512 rows x 128 real columns), wave layout (4 x 2 waves
// of 4 x 2 MFMA blocks), XCD-aware order, K trimming to the disc chord and
// direct global -> LDS ring as the BF16 binary row pass; a stage is 64
// columns of K (two MFMA K-steps: a 64-byte table row per ROI column, two mask
// words per row).  The two digit planes are swept one after the other over the
// K segment (the accumulators of both would not fit beside the operands):
// digit 0, the accumulators times 128, then digit 1.  Partial sums are stored
// as int32 bits in the float32 partial planes; the column pass converts them
// (k_col_operand).
// ---------------------------------------------------------------------------
constexpr int kKT8 = 64;                         // K columns per stage
constexpr int kRing8 = 8, kAhead8 = 7;
constexpr int kSlab8 = kTC * 64;                 // 8 KiB: 128 columns x 64 bytes
constexpr int kWords8 = 512 * 2 * 4;             // two mask words per tile row
constexpr int kStage8 = kSlab8 + kWords8;
constexpr int kLds8 = kRing8 * kStage8;          // 98304
// each wave copies one slab piece and two word pieces per stage; at a stage's
// end the copies of the kRing8 - 2 stages after the next may stay in flight
constexpr int kWait8 = (kRing8 - 2) * 3;

typedef int32_t i32x4 __attribute__((ext_vector_type(4)));
typedef int32_t i32x16 __attribute__((ext_vector_type(16)));

// 16 mask bits (column order) -> 16 int8 values 0 / 1: each nibble times
// 0x00204081 puts its bits at 0, 8, 16, 24 (no overlaps, no carries).
__device__ __forceinline__ i32x4 expand16_i8(uint32_t x) {
  i32x4 v;
#pragma unroll
  for (int j = 0; j < 4; ++j) v[j] = (int32_t)((((x >> (4 * j)) & 0xfu) * 0x00204081u) & 0x01010101u);
  return v;
}

template <int N> __device__ __forceinline__ void wait_barrier8() {
  static_assert(N == 18, "add the count");
  asm volatile("s_waitcnt vmcnt(18) lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

__global__ __launch_bounds__(512, 1) void k_row_pass_i8(InstDev d, int64_t row_begin, int64_t row_end, int n_rt,
                                                        int n_ct, int seg_lo, int n_seg,
                                                        const uint32_t *__restrict__ bits, int W, int64_t bits_rows,
                                                        float *__restrict__ T, int64_t seg_stride_f) {
  extern __shared__ __attribute__((aligned(16))) char lds[];
  constexpr int kTR = 512;
  char *const sbuf = lds;                          // kRing8 x kSlab8
  char *const wbuf = lds + kRing8 * kSlab8;        // kRing8 x kWords8
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int G = n_rt * n_ct * n_seg;
  const int slot = blockIdx.x >> 3;
  const int g = (slot / 32) * 256 + (blockIdx.x & 7) * 32 + (slot % 32);
  if (g >= G) return;
  const int rt = g % n_rt;
  const int ct = (g / n_rt) % n_ct;
  const int seg = seg_lo + g / (n_rt * n_ct);

  const int M2 = 2 * d.M;
  const int64_t r0 = row_begin + (int64_t)rt * kTR;
  int64_t rl = r0 + kTR - 1;
  if (rl > row_end - 1) rl = row_end - 1;
  const int c0 = ct * kTC;
  const int64_t s_lo = (int64_t)seg * d.seg_len;
  const int64_t s_hi = s_lo + d.seg_len < d.Npad ? s_lo + d.seg_len : d.Npad;
  int64_t k_lo, k_hi;
  tile_chord(d, r0, rl, k_lo, k_hi);
  k_lo = k_lo / kKT8 * kKT8;
  k_hi = (k_hi + kKT8 - 1) / kKT8 * kKT8;
  if (k_lo < s_lo) k_lo = s_lo;
  if (k_hi > s_hi) k_hi = s_hi;

  // ---- copy roles: thread tid copies the two mask words of tile row tid;
  // wave w copies slab rows (ROI columns) 16 w .. 16 w + 15, lane L chunk L & 3
  // of row 16 w + L / 4 from global chunk (L & 3) ^ swz8(row).  Columns past 2M
  // read column 0: they feed only accumulators that are never stored.
  const uint32_t *wsrc = bits + (r0 + tid - row_begin);
  const int R = wave * 16 + (lane >> 2);
  const int gc = c0 + R < M2 ? c0 + R : 0;
  const int64_t plane = (int64_t)M2 * d.Npad;     // bytes per digit plane
  const int8_t *bsrc0 = (const int8_t *)d.A + (int64_t)gc * 64 + 16 * ((lane & 3) ^ swz8(R));

  // ---- compute role: wave (wr, wc) covers rows wr*128.., columns wc*64..
  const int wr = wave >> 1, wc = wave & 1;
  const int l32 = lane & 31, lhi = lane >> 5;
  const int lsw = swz8(l32);
  const int cks0 = ((0 + lhi) ^ lsw) << 4, cks1 = ((2 + lhi) ^ lsw) << 4;
  const int brow = (wc * 64 + l32) * 64;

  i32x16 acc[4][2];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[a][b][e] = 0;

  if (k_lo < k_hi) {
    const int kb = (int)k_lo;
    const int nst = (int)((k_hi - k_lo) / kKT8);
    const int klast = (int)d.Npad - kKT8;
#pragma unroll 1
    for (int dg = 0; dg < 2; ++dg) {
      const int8_t *bsrc = bsrc0 + dg * plane;
      auto copy_stage = [&](int s) {
        const int k = min(kb + s * kKT8, klast);
        __builtin_amdgcn_global_load_lds((const void *)(bsrc + (int64_t)(k >> 6) * M2 * 64),
                                         (__attribute__((address_space(3))) void *)(sbuf + (s % kRing8) * kSlab8 +
                                                                                    wave * 1024),
                                         16, 0, 0);
        const int wi = k >> 5;  // k <= Npad - 64: words wi and wi + 1 exist
        char *wd = wbuf + (s % kRing8) * kWords8 + wave * 256;
        __builtin_amdgcn_global_load_lds((const void *)(wsrc + (int64_t)wi * bits_rows),
                                         (__attribute__((address_space(3))) void *)wd, 4, 0, 0);
        __builtin_amdgcn_global_load_lds((const void *)(wsrc + (int64_t)(wi + 1) * bits_rows),
                                         (__attribute__((address_space(3))) void *)(wd + kTR * 4), 4, 0, 0);
      };
      for (int s = 0; s < kAhead8; ++s) copy_stage(s);
      wait_barrier8<kWait8>();
      for (int s = 0; s < nst; ++s) {
        copy_stage(s + kAhead8);
        const uint32_t *sw = (const uint32_t *)(wbuf + (s % kRing8) * kWords8) + wr * 128 + l32;
        const char *sb = sbuf + (s % kRing8) * kSlab8 + brow;
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) {
          i32x4 bq[2], aq[4];
#pragma unroll
          for (int cb = 0; cb < 2; ++cb)
            bq[cb] = __builtin_bit_cast(i32x4, lds_ld16(sb + cb * 32 * 64 + (ks ? cks1 : cks0)));
#pragma unroll
          for (int rb = 0; rb < 4; ++rb) aq[rb] = expand16_i8((sw[rb * 32 + ks * kTR] >> (16 * lhi)) & 0xffffu);
#pragma unroll
          for (int rb = 0; rb < 4; ++rb)
#pragma unroll
            for (int cb = 0; cb < 2; ++cb)
              acc[rb][cb] = __builtin_amdgcn_mfma_i32_32x32x32_i8(aq[rb], bq[cb], acc[rb][cb], 0, 0, 0);
        }
        wait_barrier8<kWait8>();
      }
      // drain the copies past the end, and let every wave finish reading the
      // ring before the next digit's prologue overwrites it
      asm volatile("s_waitcnt vmcnt(0)\n\ts_barrier" ::: "memory");
      if (dg == 0) {
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int e = 0; e < 16; ++e) acc[a][b][e] *= 128;
      }
    }
  }
  // epilogue: the int32 sums as raw bits in the float32 partial planes
  f32x16 out[4][2];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int e = 0; e < 16; ++e) out[a][b][e] = __int_as_float(acc[a][b][e]);
  store_partials(out, T + (int64_t)(seg - seg_lo) * seg_stride_f, seg_stride_f / M2, c0 + wc * 64 + l32, M2,
                 r0 + wr * 128 + 4 * lhi, row_begin, row_end);
}

}  // namespace

hipError_t init_i8_attributes() {
  static std::atomic<bool> done{false};
  if (done.load(std::memory_order_acquire)) return hipSuccess;
  const hipError_t e =
      hipFuncSetAttribute((const void *)k_row_pass_i8, hipFuncAttributeMaxDynamicSharedMemorySize, kLds8);
  if (e == hipSuccess) done.store(true, std::memory_order_release);
  return e;
}

hipError_t launch_build_i8_table(const InstHost &ih, char *ws, hipStream_t st) {
  const InstDev &d = ih.dev;
  const dim3 grid((unsigned)((d.Npad + 255) / 256), (unsigned)d.M);
  hipLaunchKernelGGL(k_build_i8_table, grid, dim3(256), 0, st, d, (int8_t *)(ws + ih.off_A));
  return hipGetLastError();
}

hipError_t launch_row_pass_i8(const InstDev &d, int64_t row_begin, int64_t row_end, float2 *T, int64_t seg_stride,
                              const uint32_t *bits, hipStream_t st) {
  if (row_end <= row_begin) return hipSuccess;
  int seg_lo, seg_hi;
  split_seg_range(d, row_begin, row_end, seg_lo, seg_hi);
  if (seg_hi <= seg_lo) return hipSuccess;
  hipError_t e = init_i8_attributes();
  if (e != hipSuccess) return e;
  const int n_seg = seg_hi - seg_lo;
  const int64_t rows = row_end - row_begin;
  const int W = (int)(d.Npad / 32);
  const int n_rt = (int)((rows + 511) / 512);
  const int n_ct = (2 * d.M + kTC - 1) / kTC;
  const int64_t G = (int64_t)n_rt * n_ct * n_seg;
  const int64_t grid = (G + 255) / 256 * 256;  // whole rounds of 32 work-groups on each of 8 XCDs
  hipLaunchKernelGGL(k_row_pass_i8, dim3((unsigned)grid), dim3(512), kLds8, st, d, row_begin, row_end, n_rt, n_ct,
                     seg_lo, n_seg, bits, W, bits_rows_pad(rows), (float *)T, 2 * seg_stride);
  return hipGetLastError();
}

}  // namespace fzp
