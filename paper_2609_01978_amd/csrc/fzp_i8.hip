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
// ---------------------------------------------------------------------------
// Zone-mask bits for the int8 row pass.  The same bits as k_mask_bits (Sec.
// 2.2, Eq. 4: zone = floor(K kappa) from the exact integer K, the disc chord,
// the centre-open flip), in another order:
//   - the four words of a 128-column block of one row are adjacent,
//     bits[k / 128][r - row_begin][w % 4], so one 16-byte direct copy per row
//     fills a pipeline stage;
//   - inside a word, column 16 h + 4 j + b (h: MFMA lane half, j: byte group,
//     b: byte) sits at bit 8 b + 4 h + j, so that lane half h forms its
//     operand dword j as (word >> (4 h + j)) & 0x01010101.
// With N = 32 W the words of the right half are the mirrored left ones.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t perm_i8(uint32_t v) {
  uint32_t r = 0;
#pragma unroll
  for (int e = 0; e < 32; ++e) r |= ((v >> e) & 1u) << (8 * (e & 3) + 4 * (e >> 4) + ((e >> 2) & 3));
  return r;
}

template <bool FOUR>
__global__ __launch_bounds__(256) void k_mask_bits_i8(InstDev d, int64_t row_begin, int64_t row_end, int64_t rows_pad,
                                                      int W, uint32_t *__restrict__ bits,
                                                      uint32_t *__restrict__ bits2) {
  const int64_t N = d.N;
  const int64_t Nm1 = N - 1;
  const uint32_t flip = d.centre_open ? 0xffffffffu : 0u;
  const int64_t rows = row_end - row_begin;
  const int64_t rl = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;  // thread = one row
  if (rl >= rows_pad) return;
  // rows past the chunk (up to the padded row count) get empty chords: zero words
  const int64_t row = row_begin + rl;
  const double cj = (double)(2 * row - N + 1);
  const double bj = cj * cj;
  int64_t rlo = 0, rhi = 0;
  const double rem = d.kmax - bj;
  if (rl < rows && rem >= 0.0) {
    int64_t m = (int64_t)sqrt(rem);
    while ((double)(m + 1) * (double)(m + 1) <= rem) ++m;
    while (m > 0 && (double)m * (double)m > rem) --m;
    rlo = (Nm1 - m + 1) >> 1;
    rhi = ((Nm1 + m) >> 1) + 1;
  }
  // groups of four words (one 128-column block), one 16-byte store each; with
  // N = 32 W the group G - 1 - g holds the mirrored words of group g in
  // reverse order (G = W / 4), so only the first (G + 1) / 2 groups are
  // evaluated (a middle group is its own mirror)
  const int G = W / 4;
  const bool mirror = (int64_t)32 * W == N;
  const int gend = mirror ? (G + 1) / 2 : G;
  const int g0 = blockIdx.y * 16, g1 = min(g0 + 16, gend);
  for (int g = g0; g < g1; ++g) {
    uint32_t v[4], v2[4], vm[4], vm2[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      // each bit goes straight to its permuted place, and for the mirrored
      // word to the place of its bit-reversed position; the chord mask is
      // permuted the same way (perm_i8 distributes over and / xor, and the
      // centre-open flip is all ones or zero)
      const int64_t i0 = 32 * (int64_t)(4 * g + q);
      v[q] = v2[q] = vm[q] = vm2[q] = 0;
      if (i0 < rhi && i0 + 32 > rlo) {
        double ci = (double)(2 * i0 - Nm1);
        uint32_t a = 0, a2 = 0, am = 0, am2 = 0;
#pragma unroll
        for (int e = 0; e < 32; ++e) {
          const int pe = 8 * (e & 3) + 4 * (e >> 4) + ((e >> 2) & 3);
          const int f = 31 - e, pf = 8 * (f & 3) + 4 * (f >> 4) + ((f >> 2) & 3);
          const double K = fma(ci, ci, bj);
          if constexpr (FOUR) {
            const int z = (int)(K * d.kappa_l);
            const uint32_t b1 = (uint32_t)(z >> 1) & 1u, b2 = (uint32_t)(z ^ (z >> 1)) & 1u;
            a |= b1 << pe;
            a2 |= b2 << pe;
            am |= b1 << pf;
            am2 |= b2 << pf;
          } else {
            const uint32_t b1 = (uint32_t)(int)(K * d.kappa) & 1u;
            a |= b1 << pe;
            am |= b1 << pf;
          }
          ci += 2.0;
        }
        const int lo = (int)min(max(rlo - i0, (int64_t)0), (int64_t)32);
        const int hi = (int)min(max(rhi - i0, (int64_t)0), (int64_t)32);
        const uint32_t valid = (hi >= 32 ? 0xffffffffu : ((1u << hi) - 1u)) & ~((1u << lo) - 1u);
        uint32_t pv = 0xffffffffu, pvm = 0xffffffffu;
        if (valid != 0xffffffffu) {
          pv = perm_i8(valid);
          pvm = perm_i8(__builtin_bitreverse32(valid));
        }
        v[q] = (a ^ flip) & pv;
        vm[q] = (am ^ flip) & pvm;
        v2[q] = a2 & pv;
        vm2[q] = am2 & pvm;
      }
    }
    uint4 *o = (uint4 *)bits + (int64_t)g * rows_pad + rl;
    *o = make_uint4(v[0], v[1], v[2], v[3]);
    if (mirror) *((uint4 *)bits + (int64_t)(G - 1 - g) * rows_pad + rl) = make_uint4(vm[3], vm[2], vm[1], vm[0]);
    if constexpr (FOUR) {
      *((uint4 *)bits2 + (int64_t)g * rows_pad + rl) = make_uint4(v2[0], v2[1], v2[2], v2[3]);
      if (mirror)
        *((uint4 *)bits2 + (int64_t)(G - 1 - g) * rows_pad + rl) = make_uint4(vm2[3], vm2[2], vm2[1], vm2[0]);
    }
  }
}

// ---------------------------------------------------------------------------
// The row-pass kernel: T = 128 (mask . v0) + mask . v1 in int32 (the column
// pass scales it by 1 / 16256); |T| <= 65536 (127 * 128 + 64) < 2^31 for K
// segments up to 65536 columns.  One v_mfma_i32_32x32x32_i8 covers 32
// columns of K.
//
// Work-group tile 512 rows x 128 real columns, 8 waves of 64 x 128 (2 x 4
// MFMA blocks of 32 x 32; each expanded mask operand feeds 4 MFMAs), in the
// XCD-aware order of the BF16 binary row pass, K trimmed to the tile's disc
// chord.  A pipeline stage is 128 columns of K (four MFMA K-steps): per ROI
// column a 128-byte slab row (two 64-byte table rows), per tile row 16 bytes
// of mask words; both arrive by direct global -> LDS copies into a 6-deep
// ring, issued 5 stages ahead, one barrier per stage.  The two digit planes
// are swept one after the other over the K segment (the accumulators of both
// would not fit beside the operands): digit 0, the accumulators times 128,
// then digit 1.  Partial sums are stored as int32 bits in the float32 partial
// planes; the column pass converts them (k_col_operand).
// ---------------------------------------------------------------------------
constexpr int kKT8 = 128;                        // K columns per stage
constexpr int kRB8 = 2, kCB8 = 4;                // MFMA blocks per wave (rows, columns)
constexpr int kRowB8 = kKT8;                     // slab bytes per ROI column
constexpr int kSlab8 = kTC * kRowB8;             // 16 KiB
constexpr int kWords8 = 512 * 16;                // 4 mask words per tile row
constexpr int kRing8 = 6, kAhead8 = 5;
constexpr int kLds8 = kRing8 * (kSlab8 + kWords8);  // 147456
// per wave and stage: two 1 KiB slab copies and one 1 KiB word copy; at a
// stage's end the copies of the kRing8 - 2 stages after the next may be in flight
constexpr int kWait8 = (kRing8 - 2) * 3;
static_assert(kWait8 == 12, "the s_waitcnt counts below");

typedef int32_t i32x4 __attribute__((ext_vector_type(4)));
typedef int32_t i32x16 __attribute__((ext_vector_type(16)));

// LDS slab rows hold their eight 16-byte chunks in the order chunk ^ swz(row),
// which keeps the MFMA operand reads (32 consecutive rows, one chunk)
// conflict-free; row bits 0 .. 4 only, so every 32-row block has the same order.
__device__ __forceinline__ int swz_i8(int r) { return (r & 7) ^ ((r >> 3) & 3); }

// Lane half h's operand (16 int8 values 0 / 1) from a permuted mask word.
__device__ __forceinline__ i32x4 expand_i8(uint32_t w, int h) {
  const uint32_t x = w >> (4 * h);
  i32x4 v;
#pragma unroll
  for (int j = 0; j < 4; ++j) v[j] = (int32_t)((x >> j) & 0x01010101u);
  return v;
}

__global__ __launch_bounds__(512, 1) void k_row_pass_i8(InstDev d, int64_t row_begin, int64_t row_end, int n_rt,
                                                        int n_ct, int seg_lo, int n_seg,
                                                        const uint32_t *__restrict__ bits, int64_t bits_rows,
                                                        float *__restrict__ T, int64_t seg_stride_f) {
  extern __shared__ __attribute__((aligned(16))) char lds[];
  constexpr int kTR = 512;
  char *const sbuf = lds;                         // kRing8 x kSlab8
  char *const wbuf = lds + kRing8 * kSlab8;       // kRing8 x kWords8
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

  // ---- copy roles: thread tid copies the 16 mask-word bytes of tile row tid;
  // slab copy x of wave w fills slab rows (ROI columns) 8 (2 w + x) .. + 7, lane
  // L chunk L % 8 of row L / 8, read from global chunk (L % 8) ^ swz(row): table
  // block k / 64 + gch / 4, bytes 16 (gch % 4).  Columns past 2M read column 0:
  // they feed only accumulators that are never stored.
  const uint32_t *wsrc = bits + (r0 + tid - row_begin) * 4;
  const int64_t plane = (int64_t)M2 * d.Npad;    // bytes per digit plane
  const int8_t *bsrc0[2];
#pragma unroll
  for (int x = 0; x < 2; ++x) {
    const int R = (wave * 2 + x) * 8 + (lane >> 3);
    const int gc = c0 + R < M2 ? c0 + R : 0;
    const int gch = (lane & 7) ^ swz_i8(R);
    bsrc0[x] = (const int8_t *)d.A + (int64_t)(gch >> 2) * M2 * 64 + (int64_t)gc * 64 + 16 * (gch & 3);
  }

  // ---- compute role: wave w covers rows 64 w .., all 128 columns
  const int l32 = lane & 31, lhi = lane >> 5;
  const int lsw = swz_i8(l32);
  const int brow = l32 * kRowB8;
  const int wrow = (wave * 64 + l32) * 16;

  i32x16 acc[kRB8][kCB8];
#pragma unroll
  for (int a = 0; a < kRB8; ++a)
#pragma unroll
    for (int b = 0; b < kCB8; ++b)
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[a][b][e] = 0;

  if (k_lo < k_hi) {
    const int64_t kb = k_lo;
    const int nst = (int)((k_hi - k_lo) / kKT8);
    const int64_t klast = d.Npad - kKT8;
#pragma unroll 1
    for (int dg = 0; dg < 2; ++dg) {
      auto copy_stage = [&](int s) {
        const int64_t k = min(kb + (int64_t)s * kKT8, klast);
        char *sd = sbuf + (s % kRing8) * kSlab8 + wave * 2048;
#pragma unroll
        for (int x = 0; x < 2; ++x)
          __builtin_amdgcn_global_load_lds((const void *)(bsrc0[x] + dg * plane + (k >> 6) * M2 * 64),
                                           (__attribute__((address_space(3))) void *)(sd + x * 1024), 16, 0, 0);
        __builtin_amdgcn_global_load_lds((const void *)(wsrc + (k >> 7) * bits_rows * 4),
                                         (__attribute__((address_space(3))) void *)(wbuf + (s % kRing8) * kWords8 +
                                                                                    wave * 1024),
                                         16, 0, 0);
      };
      for (int s = 0; s < kAhead8; ++s) copy_stage(s);
      asm volatile("s_waitcnt vmcnt(12) lgkmcnt(0)\n\ts_barrier" ::: "memory");
      for (int s = 0; s < nst; ++s) {
        copy_stage(s + kAhead8);
        const char *sb = sbuf + (s % kRing8) * kSlab8 + brow;
        const char *swp = wbuf + (s % kRing8) * kWords8 + wrow;
        u32x4 wq[kRB8];
#pragma unroll
        for (int rb = 0; rb < kRB8; ++rb) wq[rb] = lds_ld16(swp + rb * 32 * 16);
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
          i32x4 bq[kCB8], aq[kRB8];
          const int cko = ((2 * ks + lhi) ^ lsw) << 4;
#pragma unroll
          for (int cb = 0; cb < kCB8; ++cb)
            bq[cb] = __builtin_bit_cast(i32x4, lds_ld16(sb + cb * 32 * kRowB8 + cko));
#pragma unroll
          for (int rb = 0; rb < kRB8; ++rb) aq[rb] = expand_i8(wq[rb][ks], lhi);
#pragma unroll
          for (int rb = 0; rb < kRB8; ++rb)
#pragma unroll
            for (int cb = 0; cb < kCB8; ++cb)
              acc[rb][cb] = __builtin_amdgcn_mfma_i32_32x32x32_i8(aq[rb], bq[cb], acc[rb][cb], 0, 0, 0);
        }
        asm volatile("s_waitcnt vmcnt(12) lgkmcnt(0)\n\ts_barrier" ::: "memory");
      }
      // drain the copies past the end, and let every wave finish reading the
      // ring before the next digit's prologue overwrites it
      asm volatile("s_waitcnt vmcnt(0)\n\ts_barrier" ::: "memory");
      if (dg == 0) {
#pragma unroll
        for (int a = 0; a < kRB8; ++a)
#pragma unroll
          for (int b = 0; b < kCB8; ++b)
#pragma unroll
            for (int e = 0; e < 16; ++e) acc[a][b][e] *= 128;
      }
    }
  }
  // epilogue: the int32 sums as raw bits in the float32 partial planes,
  // column-major Ts[c][r - row_begin]; register v of lane l holds row
  // 8(v/4) + 4(l/32) + v%4 of its block and column l%32, four consecutive
  // rows per 16-byte store
  float *Ts = T + (int64_t)(seg - seg_lo) * seg_stride_f;
  const int64_t rs = seg_stride_f / M2;
  const int64_t rbase = r0 + wave * 64 + 4 * lhi;
#pragma unroll
  for (int cb = 0; cb < kCB8; ++cb) {
    const int c = c0 + cb * 32 + l32;
    if (c >= M2) continue;
    float *col = Ts + (int64_t)c * rs - row_begin;
#pragma unroll
    for (int rb = 0; rb < kRB8; ++rb)
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        const int64_t r = rbase + rb * 32 + 8 * a;
        const i32x16 &v = acc[rb][cb];
        if (r + 3 < row_end) {
          *(float4 *)(col + r) = make_float4(__int_as_float(v[4 * a]), __int_as_float(v[4 * a + 1]),
                                             __int_as_float(v[4 * a + 2]), __int_as_float(v[4 * a + 3]));
        } else {
#pragma unroll
          for (int e = 0; e < 4; ++e)
            if (r + e < row_end) col[r + e] = __int_as_float(v[4 * a + e]);
        }
      }
  }
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

hipError_t launch_mask_bits_i8(const InstDev &d, int64_t row_begin, int64_t row_end, uint32_t *bits, hipStream_t st,
                               uint32_t *bits2) {
  const int64_t rows = row_end - row_begin;
  if (rows <= 0) return hipSuccess;
  const int W = (int)(d.Npad / 32);
  const int64_t rows_pad = bits_rows_pad(rows);
  const int G = W / 4, gend = (int64_t)32 * W == d.N ? (G + 1) / 2 : G;  // mirrored halves
  const dim3 grid((unsigned)((rows_pad + 255) / 256), (unsigned)((gend + 15) / 16));
  if (bits2)
    hipLaunchKernelGGL(k_mask_bits_i8<true>, grid, dim3(256), 0, st, d, row_begin, row_end, rows_pad, W, bits, bits2);
  else
    hipLaunchKernelGGL(k_mask_bits_i8<false>, grid, dim3(256), 0, st, d, row_begin, row_end, rows_pad, W, bits,
                       bits2);
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
  const int n_rt = (int)((rows + 511) / 512);
  const int n_ct = (2 * d.M + kTC - 1) / kTC;
  const int64_t G = (int64_t)n_rt * n_ct * n_seg;
  const int64_t grid = (G + 255) / 256 * 256;  // whole rounds of 32 work-groups on each of 8 XCDs
  hipLaunchKernelGGL(k_row_pass_i8, dim3((unsigned)grid), dim3(512), kLds8, st, d, row_begin, row_end, n_rt, n_ct,
                     seg_lo, n_seg, bits, bits_rows_pad(rows), (float *)T, 2 * seg_stride);
  return hipGetLastError();
}

}  // namespace fzp
