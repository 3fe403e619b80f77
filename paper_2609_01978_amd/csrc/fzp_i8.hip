// Row pass on the int8 matrix cores (FZP_FLAG_SPLIT_INT8).
//
// Same product as the split-BF16 row pass (Sec. 2.6: the stripe of Eq. 4
// zones, generated on the fly, times the N x M kernel matrix
//   A[i][q] = exp(2 pi i (beta c_i^2/2 - alpha c_i d_q))),
// with A held in fixed point instead of a BF16 hi/lo pair: v = rint(A s),
// s = kI8Scale = 16256, split into two balanced int8 digits v = 128 v0 + v1.
// Binary stripes: the mask is 0 / 1 in int8, so both digit products sum
// exactly in int32 and the only error is the quantisation of A (at most
// 0.5 / 16256 = 3.1e-5 per component); per 32 columns of K the int8 MFMA does
// the work of two BF16 MFMA K-steps, so the two digits cost what one BF16
// plane does.  Complex stripes (creases, L-level plates) hold the stripe in
// digits too (k_row_pass_i8_cplx below).
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
  int8_t r0 = 0, r1 = 0, i0 = 0, i1 = 0;  // digits of A_re, A_im
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
      // each bit is gathered into its permuted place; the chord mask is
      // permuted the same way (perm_i8 distributes over and / xor, and the
      // centre-open flip is all ones or zero).  The mirrored word is the
      // bit-reversed natural word, and bit reversal commutes with the
      // permutation (reversing a 5-bit index complements each of its fields,
      // which maps position p to 31 - p), so it is the permuted word reversed.
      const int64_t i0 = 32 * (int64_t)(4 * g + q);
      v[q] = v2[q] = vm[q] = vm2[q] = 0;
      if (i0 < rhi && i0 + 32 > rlo) {
        double ci = (double)(2 * i0 - Nm1);
        // Column e goes to bit 8 (e & 3) + (e >> 2) of the permuted word: inside
        // byte lane e & 3 the bit position rises with e, so each lane collects
        // its 8 bits by a funnel shift from the top (one instruction per
        // sample) and ends with them in bits 24..31.
        uint32_t acc[4] = {0u, 0u, 0u, 0u}, acc2[4] = {0u, 0u, 0u, 0u};
#pragma unroll
        for (int e = 0; e < 32; ++e) {
          const double K = fma(ci, ci, bj);
          if constexpr (FOUR) {
            const int z = (int)(K * d.kappa_l);
            acc[e & 3] = __builtin_amdgcn_alignbit((uint32_t)(z >> 1), acc[e & 3], 1);
            acc2[e & 3] = __builtin_amdgcn_alignbit((uint32_t)(z ^ (z >> 1)), acc2[e & 3], 1);
          } else {
            acc[e & 3] = __builtin_amdgcn_alignbit((uint32_t)(int)(K * d.kappa), acc[e & 3], 1);
          }
          ci += 2.0;
        }
        const uint32_t a = (acc[0] >> 24) | ((acc[1] >> 16) & 0xff00u) | ((acc[2] >> 8) & 0xff0000u) |
                           (acc[3] & 0xff000000u);
        const uint32_t a2 = (acc2[0] >> 24) | ((acc2[1] >> 16) & 0xff00u) | ((acc2[2] >> 8) & 0xff0000u) |
                            (acc2[3] & 0xff000000u);
        const int lo = (int)min(max(rlo - i0, (int64_t)0), (int64_t)32);
        const int hi = (int)min(max(rhi - i0, (int64_t)0), (int64_t)32);
        const uint32_t valid = (hi >= 32 ? 0xffffffffu : ((1u << hi) - 1u)) & ~((1u << lo) - 1u);
        const uint32_t pv = valid != 0xffffffffu ? perm_i8(valid) : 0xffffffffu;
        v[q] = (a ^ flip) & pv;
        v2[q] = a2 & pv;
        vm[q] = __builtin_bitreverse32(v[q]);
        vm2[q] = __builtin_bitreverse32(v2[q]);
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

// ---------------------------------------------------------------------------
// Row pass on the int8 matrix cores for complex stripes (creases, L-level
// phase plates): T = S A with S = mask e^{i phi} per sample (Sec. 2.2, the
// deformation map as a phase screen; Eq. 4 zones), both operands in two int8
// digits, S = (128 s0 + s1) / s and A = (128 a0 + a1) / s, s = kI8Scale:
//   S A s^2 = 128^2 s0 a0 + 128 (s0 a1 + s1 a0) + s1 a1,
// the last term (at most 64^2 / s^2 = 1.5e-5) left out.  As a real GEMM,
// [S_re | S_im] against [[A_re, A_im], [-A_im, A_re]]: the lower block A' is
// not stored but made in registers from the upper one, column n's operand
// from column n ^ 1 (the neighbouring lane) negated on even columns (negated
// digits stay digits: |v0| <= 127, |v1| <= 64).  Per 32 columns of K and
// 32 x 32 block:
//   hi += s0_re a0 + s0_im a0',   x += s0_re a1 + s1_re a0 + s0_im a1' + s1_im a0',
// six v_mfma_i32_32x32x32_i8 against twelve BF16 MFMAs of the three-product
// split.  Both sums are exact in int32 per K segment (|hi| <= 2 * 127^2 * 65536,
// |x| <= 4 * 127 * 64 * 65536, both < 2^31); the epilogue forms 128^2 hi + 128 x
// exactly in int64 and stores it rounded once to float32 (relative 6e-8) in
// the partial planes T, which the column pass adds in float64 and scales by
// 1 / s^2.
//
// Work-group tile 256 rows x 128 real columns, 8 waves of 64 x 64 (2 x 2 MFMA
// blocks, two sets of 64 int32 accumulators), XCD-aware order and K trimming
// as the BF16 complex row pass; a stage is 32 columns of K: four stripe planes
// (s0_re, s1_re, s0_im, s1_im) x 256 rows x 32 bytes and two table planes
// (a0, a1) x 128 columns x 32 bytes, by direct copies into a 3-deep ring, 2
// stages ahead.  LDS rows are 32 bytes; the 16-byte halves of rows
// 8 .. 15 of every 16 are swapped so that 16 rows read at one half hit 64
// distinct banks.
// ---------------------------------------------------------------------------
constexpr int kCTR8 = 256, kCTC8 = 128, kCKT8 = 32, kCRowB8 = 32;
constexpr int kCG8 = 4 * kCTR8 * kCRowB8;     // 32768: four stripe planes
constexpr int kCT8b = 2 * kCTC8 * kCRowB8;    // 8192: two table planes
constexpr int kCStage8 = kCG8 + kCT8b;
constexpr int kCRing8 = 3, kCAhead8 = 2;
constexpr int kCLds8 = kCRing8 * kCStage8;    // 122880
// per wave and stage: four stripe pieces and one table piece of 1 KiB; with
// two stages ahead the newest stage's five may stay in flight at a stage's end
constexpr int kCWait8 = 5;

__device__ __forceinline__ int chalf8(int row, int half) { return half ^ ((row >> 3) & 1); }

// Column n's B operand from lane l ^ 1 (column n ^ 1, the same K half), each
// byte negated on even columns.  For a byte b other than -128 (digits lie in
// [-127, 127]), -b = ((b ^ 0x7f) + 1) ^ 0x80 with no carry out of the byte
// (b ^ 0x7f keeps the sign bit and takes the low seven bits to 0x7f - l, and
// adding one carries into bit 7 only for l = 0, where b = 0 gives 0x80 and
// the final flip 0).  The lane's constants are zero on odd columns, where
// the expression is the identity: k7 = 0x7f7f7f7f, k1 = 0x01010101,
// k8 = 0x80808080 on even lanes.
__device__ __forceinline__ i32x4 swap_neg_i8(i32x4 b, uint32_t k7, uint32_t k1, uint32_t k8) {
  i32x4 r;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const uint32_t u = (uint32_t)__builtin_amdgcn_mov_dpp(b[j], 0xb1, 0xf, 0xf, true);  // quad_perm [1,0,3,2]
    r[j] = (int32_t)(((u ^ k7) + k1) ^ k8);
  }
  return r;
}

__global__ __launch_bounds__(512, 1) void k_row_pass_i8_cplx(InstDev d, int64_t row_begin, int64_t row_end, int n_rt,
                                                             int n_ct, int seg_lo, int n_seg,
                                                             const int8_t *__restrict__ G, int64_t rows_pad,
                                                             int64_t kb0, int64_t nkb, float *__restrict__ T,
                                                             int64_t seg_stride_f) {
  static_assert(kCWait8 == 5, "the s_waitcnt counts below");
  extern __shared__ __attribute__((aligned(16))) char lds[];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int Gn = n_rt * n_ct * n_seg;
  const int slot = blockIdx.x >> 3;
  const int g = (slot / 32) * 256 + (blockIdx.x & 7) * 32 + (slot % 32);
  if (g >= Gn) return;
  const int rt = g % n_rt;
  const int ct = (g / n_rt) % n_ct;
  const int seg = seg_lo + g / (n_rt * n_ct);

  const int M2 = 2 * d.M;
  const int64_t r0 = row_begin + (int64_t)rt * kCTR8;
  int64_t rl = r0 + kCTR8 - 1;
  if (rl > row_end - 1) rl = row_end - 1;
  const int c0 = ct * kCTC8;
  const int64_t s_lo = (int64_t)seg * d.seg_len;
  const int64_t s_hi = s_lo + d.seg_len < d.Npad ? s_lo + d.seg_len : d.Npad;
  int64_t k_lo, k_hi;
  tile_chord(d, r0, rl, k_lo, k_hi);
  k_lo = k_lo / kCKT8 * kCKT8;
  k_hi = (k_hi + kCKT8 - 1) / kCKT8 * kCKT8;
  if (k_lo < s_lo) k_lo = s_lo;
  if (k_hi > s_hi) k_hi = s_hi;
  if (k_lo < 16 * kb0) k_lo = 16 * kb0;
  if (k_hi > 16 * (kb0 + nkb)) k_hi = 16 * (kb0 + nkb);

  // ---- copy roles.  Stripe: wave w copies pieces x = 4w .. 4w+3 (plane x / 8,
  // rows 32 (x % 8) ..); table: piece w (plane w / 4, columns 32 (w % 4) ..).
  // Lane L fills LDS row L / 2, half L & 1, which holds the global half
  // chalf8(row, L & 1): stripe block k / 16 + half, table bytes k % 64 +
  // 16 half.  Table columns past 2M read column 0: they feed only accumulator
  // columns that are never stored.
  const int64_t gplane = nkb * rows_pad * 16;     // bytes per stripe plane
  const int64_t tplane = (int64_t)M2 * d.Npad;    // bytes per table plane
  const int8_t *gsrc[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int x = 4 * wave + j;
    const int row = (x & 7) * 32 + (lane >> 1);
    gsrc[j] = G + (x >> 3) * gplane + (int64_t)chalf8(row, lane & 1) * rows_pad * 16 +
              ((int64_t)rt * kCTR8 + row) * 16;
  }
  const int8_t *bsrc;
  {
    const int col = (wave & 3) * 32 + (lane >> 1);
    const int gc = c0 + col < M2 ? c0 + col : 0;
    bsrc = (const int8_t *)d.A + (wave >> 2) * tplane + (int64_t)gc * 64 + 16 * chalf8(col, lane & 1);
  }

  // ---- compute role: wave (wr, wc) covers rows wr*64 .., columns wc*64 ..
  const int wr = wave >> 1, wc = wave & 1;
  const int l32 = lane & 31, lhi = lane >> 5;
  const int hofs = chalf8(l32, lhi) * 16;
  const int aoff = (wr * 64 + l32) * kCRowB8 + hofs;
  const int boff = kCG8 + (wc * 64 + l32) * kCRowB8 + hofs;
  const bool even = (lane & 1) == 0;
  const uint32_t k7 = even ? 0x7f7f7f7fu : 0u, k1 = even ? 0x01010101u : 0u, k8 = even ? 0x80808080u : 0u;

  i32x16 ah[2][2], ax[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int e = 0; e < 16; ++e) ah[a][b][e] = ax[a][b][e] = 0;

  if (k_lo < k_hi) {
    const int64_t kb = k_lo;
    const int nst = (int)((k_hi - k_lo) / kCKT8);
    const int64_t klast = k_hi - kCKT8;  // copies past the end repeat the last stage
    auto copy_stage = [&](int s) {
      const int64_t k = kb + (int64_t)s * kCKT8 < klast ? kb + (int64_t)s * kCKT8 : klast;
      char *dst = lds + (s % kCRing8) * kCStage8;
      const int64_t gofs = (k / 16 - kb0) * rows_pad * 16;
#pragma unroll
      for (int j = 0; j < 4; ++j)
        __builtin_amdgcn_global_load_lds((const void *)(gsrc[j] + gofs),
                                         (__attribute__((address_space(3))) void *)(dst + (4 * wave + j) * 1024), 16,
                                         0, 0);
      const int64_t tofs = (k >> 6) * M2 * 64 + (k & 63);
      __builtin_amdgcn_global_load_lds((const void *)(bsrc + tofs),
                                       (__attribute__((address_space(3))) void *)(dst + kCG8 + wave * 1024), 16, 0,
                                       0);
    };
    for (int s = 0; s < kCAhead8; ++s) copy_stage(s);
    asm volatile("s_waitcnt vmcnt(5) lgkmcnt(0)\n\ts_barrier" ::: "memory");
    for (int s = 0; s < nst; ++s) {
      copy_stage(s + kCAhead8);
      const char *sb = lds + (s % kCRing8) * kCStage8;
      i32x4 b[2][4];  // [cb][a0, a1, a0', a1']
#pragma unroll
      for (int cb = 0; cb < 2; ++cb) {
#pragma unroll
        for (int t = 0; t < 2; ++t)
          b[cb][t] = __builtin_bit_cast(i32x4, lds_ld16(sb + boff + t * kCTC8 * kCRowB8 + cb * 32 * kCRowB8));
        b[cb][2] = swap_neg_i8(b[cb][0], k7, k1, k8);
        b[cb][3] = swap_neg_i8(b[cb][1], k7, k1, k8);
      }
#pragma unroll
      for (int rb = 0; rb < 2; ++rb) {
        const char *pa = sb + aoff + rb * 32 * kCRowB8;
        const i32x4 s0r = __builtin_bit_cast(i32x4, lds_ld16(pa));
        const i32x4 s1r = __builtin_bit_cast(i32x4, lds_ld16(pa + 1 * kCTR8 * kCRowB8));
        const i32x4 s0i = __builtin_bit_cast(i32x4, lds_ld16(pa + 2 * kCTR8 * kCRowB8));
        const i32x4 s1i = __builtin_bit_cast(i32x4, lds_ld16(pa + 3 * kCTR8 * kCRowB8));
#pragma unroll
        for (int cb = 0; cb < 2; ++cb) {
          ah[rb][cb] = __builtin_amdgcn_mfma_i32_32x32x32_i8(s0r, b[cb][0], ah[rb][cb], 0, 0, 0);
          ax[rb][cb] = __builtin_amdgcn_mfma_i32_32x32x32_i8(s0r, b[cb][1], ax[rb][cb], 0, 0, 0);
          ah[rb][cb] = __builtin_amdgcn_mfma_i32_32x32x32_i8(s0i, b[cb][2], ah[rb][cb], 0, 0, 0);
          ax[rb][cb] = __builtin_amdgcn_mfma_i32_32x32x32_i8(s0i, b[cb][3], ax[rb][cb], 0, 0, 0);
          ax[rb][cb] = __builtin_amdgcn_mfma_i32_32x32x32_i8(s1r, b[cb][0], ax[rb][cb], 0, 0, 0);
          ax[rb][cb] = __builtin_amdgcn_mfma_i32_32x32x32_i8(s1i, b[cb][2], ax[rb][cb], 0, 0, 0);
        }
      }
      asm volatile("s_waitcnt vmcnt(5) lgkmcnt(0)\n\ts_barrier" ::: "memory");
    }
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  }
  // epilogue: 128^2 hi + 128 x per element, column-major per real column;
  // register v of lane l holds row 8(v/4) + 4(l/32) + v%4 of its block and
  // column l%32
  const int64_t rs = seg_stride_f / M2;
  const int64_t rbase = r0 + wr * 64 + 4 * lhi;
  float *Ts = T + (int64_t)(seg - seg_lo) * seg_stride_f;
  auto val = [&](int rb, int cb, int e) {
    return (float)(16384 * (int64_t)ah[rb][cb][e] + 128 * (int64_t)ax[rb][cb][e]);
  };
#pragma unroll
  for (int cb = 0; cb < 2; ++cb) {
    const int c = c0 + wc * 64 + cb * 32 + l32;
    if (c >= M2) continue;
    float *col = Ts + (int64_t)c * rs - row_begin;
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        const int64_t r = rbase + rb * 32 + 8 * a;
        if (r + 3 < row_end) {
          *(float4 *)(col + r) = make_float4(val(rb, cb, 4 * a), val(rb, cb, 4 * a + 1), val(rb, cb, 4 * a + 2),
                                             val(rb, cb, 4 * a + 3));
        } else {
#pragma unroll
          for (int e = 0; e < 4; ++e)
            if (r + e < row_end) col[r + e] = val(rb, cb, 4 * a + e);
        }
      }
  }
}

}  // namespace

hipError_t init_i8_attributes() {
  static std::atomic<bool> done{false};
  if (done.load(std::memory_order_acquire)) return hipSuccess;
  hipError_t e = hipFuncSetAttribute((const void *)k_row_pass_i8, hipFuncAttributeMaxDynamicSharedMemorySize, kLds8);
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void *)k_row_pass_i8_cplx, hipFuncAttributeMaxDynamicSharedMemorySize, kCLds8);
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

hipError_t launch_row_pass_i8_cplx(const InstDev &d, int64_t row_begin, int64_t row_end, float2 *T,
                                   int64_t seg_stride, const void *G, hipStream_t st) {
  const int64_t rows = row_end - row_begin;
  if (rows <= 0) return hipSuccess;
  int64_t rows_pad, kb0, nkb;
  split_stripe_extent(d, row_begin, row_end, rows_pad, kb0, nkb);
  int seg_lo, seg_hi;
  split_seg_range(d, row_begin, row_end, seg_lo, seg_hi);
  if (seg_hi <= seg_lo || nkb <= 0) return hipSuccess;
  hipError_t e = init_i8_attributes();
  if (e != hipSuccess) return e;
  const int n_rt = (int)((rows + kCTR8 - 1) / kCTR8);
  const int n_ct = (2 * d.M + kCTC8 - 1) / kCTC8;
  const int n_seg = seg_hi - seg_lo;
  const int64_t Gn = (int64_t)n_rt * n_ct * n_seg;
  const int64_t grid = (Gn + 255) / 256 * 256;  // whole rounds of 32 work-groups on each of 8 XCDs
  hipLaunchKernelGGL(k_row_pass_i8_cplx, dim3((unsigned)grid), dim3(512), kCLds8, st, d, row_begin, row_end, n_rt,
                     n_ct, seg_lo, n_seg, (const int8_t *)G, rows_pad, kb0, nkb, (float *)T, 2 * seg_stride);
  return hipGetLastError();
}

}  // namespace fzp
