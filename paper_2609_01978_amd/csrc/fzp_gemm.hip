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
// Table layout, blocked by 32 aperture columns:
//   At[plane][i / 32][c][i % 32],  plane 0 = hi, 1 = lo,  c = 2q + {0: re, 1: im},
// i = 0 .. Npad-1 (zero beyond N).  One pipeline stage of a column tile (32 k
// of 128 columns) is then one contiguous 8 KiB slab per plane, an MFMA B
// operand (8 consecutive k of one column) is one 16-byte chunk, and the
// accumulator columns interleave re/im as the float2 T buffer does.

#include <atomic>
#include <cmath>

#include "fzp_split.h"

namespace fzp {

namespace {


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
  const int64_t blk = (i >> 5) * (int64_t)(2 * M) * 32 + (i & 31);
  At[blk + (int64_t)(2 * q) * 32] = hr;
  At[blk + (int64_t)(2 * q + 1) * 32] = hi_;
  At[plane + blk + (int64_t)(2 * q) * 32] = lr;
  At[plane + blk + (int64_t)(2 * q + 1) * 32] = li;
}

// ---------------------------------------------------------------------------
// Zone-mask bits of a chunk of aperture rows, word-major: bits[w][r - row_begin]
// (row stride `rows`), bit e of word w is the mask at column 32 w + e (zero
// outside the row's disc chord); one pipeline stage of a row tile is then one
// contiguous run of words.
// K = c_i^2 + c_j^2 is exact in float64 and zone = floor(K kappa) is the same
// single float64 product the reference rule uses (Sec. 2.2, Eq. 4).  Each
// element is evaluated once here instead of once per GEMM column tile.
// ---------------------------------------------------------------------------
// FOUR: the two masks of a 4-level plate in one pass: with z = floor(K kappa_L),
// kappa_L = 2 kappa (exactly, so z >> 1 = floor(K kappa)), the level is z mod 4;
// `bits` gets the odd zones (z >> 1) & 1 = levels 2 and 3, `bits2` the levels 1
// and 2, (z xor (z >> 1)) & 1 (a sample's (-i)^l is then
// 1 - (1 - i) odd - (1 + i) half, see k_col_operand).
template <bool FOUR>
__global__ __launch_bounds__(256) void k_mask_bits(InstDev d, int64_t row_begin, int64_t row_end, int64_t rows_pad,
                                                   int W, uint32_t *__restrict__ bits, uint32_t *__restrict__ bits2) {
  const int64_t N = d.N;
  const int Nm1 = (int)(N - 1);
  const double kappa = d.kappa;
  const uint32_t flip = d.centre_open ? 0xffffffffu : 0u;
  const int64_t rows = row_end - row_begin;
  const int64_t rl = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;  // thread = one row
  if (rl >= rows_pad) return;
  // rows past the chunk (up to the padded row count) get empty chords: zero words
  const int64_t row = row_begin + rl;
  const double cj = (double)(2 * row - N + 1);
  const double bj = cj * cj;
  int rlo = 0, rhi = 0;
  const double rem = d.kmax - bj;
  if (rl < rows && rem >= 0.0) {
    int m = (int)sqrt(rem);
    while ((double)(m + 1) * (double)(m + 1) <= rem) ++m;
    while (m > 0 && (double)m * (double)m > rem) --m;
    rlo = (Nm1 - m + 1) >> 1;
    rhi = ((Nm1 + m) >> 1) + 1;
  }
  // With N = 32 W, columns i and N-1-i (offsets c and -c) have the same K and
  // the chord is symmetric, so word W-1-w is word w bit-reversed: only the
  // left half of the words is evaluated.
  const bool mirror = (int64_t)32 * W == N;
  const int wend = mirror ? W / 2 : W;
  const int w0 = blockIdx.y * 64, w1 = min(w0 + 64, wend);
  for (int w = w0; w < w1; ++w) {
    const int i0 = 32 * w;
    uint32_t v = 0, v2 = 0;
    if (i0 < rhi && i0 + 32 > rlo) {
      double ci = (double)(2 * i0 - Nm1);
#pragma unroll
      for (int e = 0; e < 32; ++e) {
        const double K = fma(ci, ci, bj);
        if constexpr (FOUR) {
          const int z = (int)(K * d.kappa_l);
          v |= ((uint32_t)(z >> 1) & 1u) << e;
          v2 |= ((uint32_t)(z ^ (z >> 1)) & 1u) << e;
        } else {
          const int zone = (int)(K * kappa);
          v |= ((uint32_t)zone & 1u) << e;
        }
        ci += 2.0;
      }
      const int lo = min(max(rlo - i0, 0), 32), hi = min(max(rhi - i0, 0), 32);
      const uint32_t valid = (hi >= 32 ? 0xffffffffu : ((1u << hi) - 1u)) & ~((1u << lo) - 1u);
      v = (v ^ flip) & valid;
      v2 &= valid;
    }
    bits[(int64_t)w * rows_pad + rl] = v;
    if (mirror) bits[(int64_t)(W - 1 - w) * rows_pad + rl] = __builtin_bitreverse32(v);
    if constexpr (FOUR) {
      bits2[(int64_t)w * rows_pad + rl] = v2;
      if (mirror) bits2[(int64_t)(W - 1 - w) * rows_pad + rl] = __builtin_bitreverse32(v2);
    }
  }
}

// ---------------------------------------------------------------------------
// Row-pass GEMM.  Work-group tile: kTR aperture rows x kTC real columns of T
// over one K segment (d.seg_len aperture columns, trimmed to the disc chord
// of the tile's rows).  8 waves in a 4 (rows) x 2 (columns) grid, each wave
// 128 rows x 64 columns = 4 x 2 MFMA 32x32 blocks, 128 float32 accumulators
// per lane.  The tall tile (512 rows) gives 512 flops per byte of operand
// slab, above the BF16-MFMA / HBM ridge even without cache reuse.
//
// K advances in stages of kKT = 32 columns (two MFMA K-steps).  All global
// traffic is direct (register-free) global -> LDS copies into 4-deep rings,
// issued kAhead = 3 stages before use, so no wave waits on a load it has
// just issued; one barrier per stage:
//   - copy the hi/lo operand slab and the mask-bit words of stage s+3,
//   - each lane expands the mask bits of its own 4 rows for stage s straight
//     into MFMA A operands (no LDS round trip for the mask),
//   - 32 MFMAs of stage s on the LDS slab,
//   - wait for the copies issued two stages ago, barrier.
// Each K segment's partial sum is written in float32 and the column pass adds
// the segments in float64, which bounds the float32 accumulation length.
//
// LDS slab rows are 64 bytes (32 BF16); the four 16-byte chunks of row r sit
// in the order chunk ^ swz(r), which keeps the MFMA operand reads (32
// consecutive rows, one chunk) free of bank conflicts without padding.
// ---------------------------------------------------------------------------

constexpr int kTC = 128;     // real columns per tile (64 complex ROI columns)
constexpr int kKT = 32;      // K columns per pipeline stage
constexpr int kRowB = 64;    // LDS bytes per slab row of a stage
constexpr int kBBytes = 2 * kTC * kRowB;           // 16384 (hi and lo planes)
constexpr int kRing = 4, kAhead = 3;

// Binary-stripe GEMM variants, by WR = waves along the rows: the tile has
// 128 WR rows and 2 WR waves (WR = 4: 512 rows, 8 waves, one work-group per
// CU; WR = 2: 256 rows, 4 waves, two work-groups per CU, so that one
// work-group's barrier and pipeline start-up are covered by the other's
// MFMAs).  Each wave copies 8 / WR slab pieces and one mask-word piece per
// stage.
template <int WR, int RING = kRing, bool PF = false, bool IL = false> struct BinTile {
  static constexpr int rows = 128 * WR;
  static constexpr int threads = 128 * WR;
  static constexpr int waves = 2 * WR;
  static constexpr int per_cu = 4 / WR;
  static constexpr int slab_copies = 8 / WR;               // 1 KiB pieces per wave
  static constexpr int copies = slab_copies + 1;          // + one mask-word piece
  static constexpr int bits_bytes = rows * 4;             // one mask word per tile row
  static constexpr int ring = RING;                       // LDS stages
  static constexpr int ahead = RING - 1;                  // stages copied ahead of use
  static constexpr int lds = RING * (kBBytes + bits_bytes);
  static constexpr int round = 32 * per_cu;               // concurrent work-groups per XCD
  // copies a wave may leave outstanding at the end of a stage: those of the
  // RING - 2 stages after the next one; with PF (fragments of the next stage
  // read one stage early) the stage after the next must be complete as well
  static constexpr int wait = (RING - (PF ? 3 : 2)) * copies;
};

// s_waitcnt vmcnt(N) + s_barrier for the outstanding-copy counts used above.
template <int N> __device__ __forceinline__ void wait_barrier() {
  static_assert(N == 6 || N == 10 || N == 12 || N == 15 || N == 18 || N == 20, "add the count");
  if constexpr (N == 6) asm volatile("s_waitcnt vmcnt(6) lgkmcnt(0)\n\ts_barrier" ::: "memory");
  if constexpr (N == 10) asm volatile("s_waitcnt vmcnt(10) lgkmcnt(0)\n\ts_barrier" ::: "memory");
  if constexpr (N == 12) asm volatile("s_waitcnt vmcnt(12) lgkmcnt(0)\n\ts_barrier" ::: "memory");
  if constexpr (N == 15) asm volatile("s_waitcnt vmcnt(15) lgkmcnt(0)\n\ts_barrier" ::: "memory");
  if constexpr (N == 18) asm volatile("s_waitcnt vmcnt(18) lgkmcnt(0)\n\ts_barrier" ::: "memory");
  if constexpr (N == 20) asm volatile("s_waitcnt vmcnt(20) lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

__device__ __forceinline__ int swz(int r) { return ((r >> 1) ^ (r >> 3)) & 3; }


// 8 mask bits (one byte, column order) -> 8 packed BF16 values (1.0 / 0).
// y = x | x << 15 puts bit 2p at bit 2p and bit 2p+1 at bit 2p+16; masking
// those two bits and multiplying by 0x3f80 / 4^p (an integer for p <= 3)
// moves them to bits 0 and 16 as BF16 1.0 = 0x3f80: two operations per pair.
__device__ __forceinline__ bf16x8 expand8(uint32_t x) {
  const uint32_t y = x | (x << 15);
  u32x4 v;
  v[0] = (y & 0x00010001u) * 0x3f80u;
  v[1] = (y & 0x00040004u) * 0x0fe0u;
  v[2] = (y & 0x00100010u) * 0x03f8u;
  v[3] = (y & 0x00400040u) * 0x00feu;
  return __builtin_bit_cast(bf16x8, v);
}



template <int WR, int RING, bool PF, bool IL>
__global__ __launch_bounds__(BinTile<WR>::threads, BinTile<WR>::per_cu) void k_row_pass_split(InstDev d, int64_t row_begin, int64_t row_end,
                                                                int n_rt, int n_ct, int seg_lo, int n_seg,
                                                                const uint32_t *__restrict__ bits, int W,
                                                                int64_t bits_rows, float *__restrict__ T,
                                                                int64_t seg_stride_f) {
  extern __shared__ __attribute__((aligned(16))) char lds[];
  using BT = BinTile<WR, RING, PF, IL>;
  constexpr int kTR = BT::rows;
  constexpr int kBitsBytes = BT::bits_bytes;
  constexpr int kRing = BT::ring, kAhead = BT::ahead;
  char *const bbuf = lds;                            // kRing x kBBytes
  char *const wbuf = lds + kRing * kBBytes;          // kRing x kBitsBytes
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  // XCD-aware tile order.  Work-groups are dealt to the 8 XCDs round robin;
  // the XCD's own sequence is cut into rounds of 32 (one per CU).  In round
  // q, XCD x takes the 32 consecutive logical tiles 256 q + 32 x .. (row tile
  // fastest), so the tiles resident on one XCD share the operand slab in its
  // L2 while every XCD draws from all K segments (whose work differs).
  const int G = n_rt * n_ct * n_seg;
  const int slot = blockIdx.x >> 3;
  const int g = (slot / BT::round) * (8 * BT::round) + (blockIdx.x & 7) * BT::round + (slot % BT::round);
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
  k_lo = k_lo / kKT * kKT;
  k_hi = (k_hi + kKT - 1) / kKT * kKT;
  if (k_lo < s_lo) k_lo = s_lo;
  if (k_hi > s_hi) k_hi = s_hi;

  // ---- bit-word copy role: lane tid copies the word of tile row tid (the mask
  // buffer's rows are padded to a multiple of 512 with zero words)
  const uint32_t *wsrc = bits + (r0 + tid - row_begin);
  // ---- slab-copy role: wave w copies slab rows [16 c w, 16 c (w + 1)) (c direct
  // loads of 16 rows, c = 8 / WR); lane L carries chunk L&3 of row 16 x + L/4 of
  // its block, read from global chunk (L&3) ^ swz(row) so the LDS image is the
  // swizzled layout.  Columns past 2M read column 0 instead: they only feed
  // accumulator columns that are never stored.
  constexpr int SC = BT::slab_copies;
  const uint16_t *bsrc[SC];
#pragma unroll
  for (int x = 0; x < SC; ++x) {
    const int R = (wave * SC + x) * 16 + (lane >> 2);
    const int plane = R / kTC, col = R % kTC;
    const int gc = c0 + col < M2 ? c0 + col : 0;
    const int chunk = (lane & 3) ^ swz(R);
    bsrc[x] = d.A + (int64_t)plane * M2 * d.Npad + (int64_t)gc * 32 + 8 * chunk;
  }

  // ---- compute role: wave (wr, wc) covers rows wr*128.., columns wc*64..
  const int wr = wave >> 1, wc = wave & 1;
  const int l32 = lane & 31, lhi = lane >> 5;
  const int lsw = swz(l32);
  // byte offsets of this lane's slab chunks for K-step ks (row & 31 == l32 everywhere)
  const int cks0 = ((0 + lhi) ^ lsw) << 4, cks1 = ((2 + lhi) ^ lsw) << 4;
  const int brow = (wc * 64 + l32) * kRowB;

  f32x16 acc[4][2];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[a][b][e] = 0.0f;

  if (k_lo < k_hi) {
    // The pipeline also copies up to kAhead stages past the end: their slab
    // loads are clamped to the table's last slab and their mask is zero.
    const int kb = (int)k_lo;
    const int nst = (int)((k_hi - k_lo) / kKT);
    const int klast = (int)d.Npad - kKT;
    auto copy_stage = [&](int s) {
      const int k = min(kb + s * kKT, klast);
      const int64_t kofs = (int64_t)(k >> 5) * M2 * 32;  // 32-column block of the table
      char *dst = bbuf + (s % kRing) * kBBytes + wave * SC * 1024;
#pragma unroll
      for (int x = 0; x < SC; ++x)
        __builtin_amdgcn_global_load_lds((const void *)(bsrc[x] + kofs),
                                         (__attribute__((address_space(3))) void *)(dst + x * 1024), 16, 0, 0);
      const int wi = min((kb + s * kKT) >> 5, W - 1);
      __builtin_amdgcn_global_load_lds((const void *)(wsrc + (int64_t)wi * bits_rows),
                                       (__attribute__((address_space(3))) void *)(wbuf + (s % kRing) * kBitsBytes +
                                                                                  wave * 256),
                                       4, 0, 0);
    };
    for (int s = 0; s < kAhead; ++s) copy_stage(s);
    wait_barrier<BT::wait>();
    // operand fragments: words of the stage, B chunks (hi, lo) of a K-step
    auto load_words = [&](int s, uint32_t (&word)[4]) {
      const uint32_t *sw = (const uint32_t *)(wbuf + (s % kRing) * kBitsBytes) + wr * 128 + l32;
#pragma unroll
      for (int rb = 0; rb < 4; ++rb) word[rb] = sw[rb * 32];
    };
    auto load_b = [&](int s, int ks, bf16x8 (&bh)[2], bf16x8 (&bl)[2]) {
      const char *sb = bbuf + (s % kRing) * kBBytes + brow;
      const int cofs = ks ? cks1 : cks0;
#pragma unroll
      for (int cb = 0; cb < 2; ++cb) {
        bh[cb] = __builtin_bit_cast(bf16x8, lds_ld16(sb + cb * 32 * kRowB + cofs));
        bl[cb] = __builtin_bit_cast(bf16x8, lds_ld16(sb + (kTC + cb * 32) * kRowB + cofs));
      }
    };
    // one K-step: byte (2 ks + lhi) of each row word holds this lane's 8 columns;
    // 8 independent accumulators per operand plane, so consecutive MFMAs never
    // wait on each other
    auto expand = [&](const uint32_t (&word)[4], int ks, bf16x8 (&a)[4]) {
#pragma unroll
      for (int rb = 0; rb < 4; ++rb) a[rb] = expand8((word[rb] >> (8 * (2 * ks + lhi))) & 0xffu);
    };
    auto mfmas = [&](const bf16x8 (&a)[4], const bf16x8 (&bh)[2], const bf16x8 (&bl)[2]) {
#pragma unroll
      for (int rb = 0; rb < 4; ++rb)
#pragma unroll
        for (int cb = 0; cb < 2; ++cb)
          acc[rb][cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[rb], bh[cb], acc[rb][cb], 0, 0, 0);
#pragma unroll
      for (int rb = 0; rb < 4; ++rb)
#pragma unroll
        for (int cb = 0; cb < 2; ++cb)
          acc[rb][cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[rb], bl[cb], acc[rb][cb], 0, 0, 0);
    };
    // Interleaved K-step: the mask operand of row block rb + 1 is expanded
    // while the MFMAs of row block rb run (scheduling fences keep VALU and
    // MFMA in this order; LDS reads and scalar work may still move).
    auto kstep_il = [&](const uint32_t (&word)[4], int ks, const bf16x8 (&bh)[2], const bf16x8 (&bl)[2]) {
      bf16x8 a[4];
      const int sh = 8 * (2 * ks + lhi);
      a[0] = expand8((word[0] >> sh) & 0xffu);
#pragma unroll
      for (int rb = 0; rb < 4; ++rb) {
        __builtin_amdgcn_sched_barrier(0x0104);
        acc[rb][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[rb], bh[0], acc[rb][0], 0, 0, 0);
        acc[rb][1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[rb], bh[1], acc[rb][1], 0, 0, 0);
        if (rb < 3) a[rb + 1] = expand8((word[rb + 1] >> sh) & 0xffu);
      }
      __builtin_amdgcn_sched_barrier(0x0104);
#pragma unroll
      for (int rb = 0; rb < 4; ++rb)
#pragma unroll
        for (int cb = 0; cb < 2; ++cb)
          acc[rb][cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[rb], bl[cb], acc[rb][cb], 0, 0, 0);
    };
    if constexpr (!PF) {
      for (int s = 0; s < nst; ++s) {
        copy_stage(s + kAhead);
        uint32_t word[4];
        load_words(s, word);
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) {
          bf16x8 bh[2], bl[2], a[4];
          load_b(s, ks, bh, bl);
          if constexpr (IL) {
            kstep_il(word, ks, bh, bl);
          } else {
            expand(word, ks, a);
            mfmas(a, bh, bl);
          }
        }
        wait_barrier<BT::wait>();
      }
    } else {
      // Software pipelined across the stage barrier: the first K-step's
      // operands of stage s + 1 (mask words expanded, table fragments) are
      // prepared during stage s, which is possible because stage s + 1 is
      // complete and visible since the barrier that ended stage s - 1.  After
      // each barrier the MFMAs start at once.
      uint32_t word[4], nword[4];
      bf16x8 a0[4], a1[4], bh0[2], bl0[2], bh1[2], bl1[2];
      load_words(0, word);
      load_b(0, 0, bh0, bl0);
      expand(word, 0, a0);
      for (int s = 0; s < nst; ++s) {
        copy_stage(s + kAhead);
        load_b(s, 1, bh1, bl1);
        mfmas(a0, bh0, bl0);
        expand(word, 1, a1);
        load_words(s + 1, nword);
        load_b(s + 1, 0, bh0, bl0);
        mfmas(a1, bh1, bl1);
        expand(nword, 0, a0);
#pragma unroll
        for (int rb = 0; rb < 4; ++rb) word[rb] = nword[rb];
        wait_barrier<BT::wait>();
      }
    }
    // drain the copies still in flight before the work-group retires its LDS
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  }
  // epilogue: register v of lane l holds row 8(v/4) + 4(l/32) + (v%4), column l%32
  store_partials(acc, T + (int64_t)(seg - seg_lo) * seg_stride_f, seg_stride_f / M2, c0 + wc * 64 + l32, M2,
                 r0 + wr * 128 + 4 * lhi, row_begin, row_end);
}

}  // namespace

hipError_t init_split_attributes() {
  // set once per process (the attributes belong to the functions); threads
  // racing through the first call all set the same values
  static std::atomic<bool> done{false};
  if (done.load(std::memory_order_acquire)) return hipSuccess;
  hipError_t e = hipFuncSetAttribute((const void *)k_row_pass_split<4, 4, false, false>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, BinTile<4, 4>::lds);
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void *)k_row_pass_split<4, 8, false, false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            BinTile<4, 8>::lds);
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void *)k_row_pass_split<4, 8, true, false>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, BinTile<4, 8, true>::lds);
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void *)k_row_pass_split<4, 8, false, true>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, BinTile<4, 8>::lds);
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void *)k_row_pass_split<2, 4, false, false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            BinTile<2, 4>::lds);
  if (e == hipSuccess) e = init_cplx_attributes();
  if (e == hipSuccess) done.store(true, std::memory_order_release);
  return e;
}

hipError_t launch_build_split_table(const Plan &p, const InstHost &ih, char *ws, hipStream_t st) {
  (void)p;
  InstDev d = ih.dev;
  const dim3 grid((unsigned)((d.Npad + 255) / 256), (unsigned)d.M);
  hipLaunchKernelGGL(k_build_split_table, grid, dim3(256), 0, st, d, (uint16_t *)(ws + ih.off_A));
  return hipGetLastError();
}

int split_segments(const InstDev &d) { return (int)((d.Npad + d.seg_len - 1) / d.seg_len); }

// Mask-bit rows are padded to a multiple of the largest binary tile (512 rows).
int64_t bits_rows_pad(int64_t rows) { return (rows + 511) / 512 * 512; }

size_t split_bits_bytes(const InstDev &d, int64_t chunk_rows) {
  return (size_t)bits_rows_pad(chunk_rows) * (size_t)(d.Npad / 32) * 4;
}

// Union of the disc chords of rows [row_begin, row_end): the chord of the row
// nearest the axis, aperture columns [lo, hi); lo = hi = 0 when no row meets
// the disc.
void split_chunk_chord(const InstDev &d, int64_t row_begin, int64_t row_end, int64_t &lo, int64_t &hi) {
  const int64_t N = d.N;
  lo = hi = 0;
  if (row_end <= row_begin) return;
  int64_t rc = (N - 1) / 2;
  if (rc < row_begin) rc = row_begin;
  if (rc > row_end - 1) rc = row_end - 1;
  int64_t best = -1;
  for (int64_t r = rc; r <= rc + 1 && r < row_end; ++r) {
    const int64_t c = 2 * r - N + 1;
    const int64_t rem = (int64_t)d.kmax - c * c;
    if (rem < 0) continue;
    int64_t m = (int64_t)std::sqrt((double)rem);
    while (m > 0 && m * m > rem) --m;
    while ((m + 1) * (m + 1) <= rem) ++m;
    if (m > best) best = m;
  }
  if (best < 0) return;
  lo = (N - 1 - best + 1) / 2 > 0 ? (N - 1 - best + 1) / 2 : 0;
  hi = ((N - 1 + best) / 2 < N - 1 ? (N - 1 + best) / 2 : N - 1) + 1;
}

// K segments that intersect the disc chords of rows [row_begin, row_end).
void split_seg_range(const InstDev &d, int64_t row_begin, int64_t row_end, int &seg_lo, int &seg_hi) {
  int64_t lo, hi;
  split_chunk_chord(d, row_begin, row_end, lo, hi);
  if (hi <= lo) {
    seg_lo = seg_hi = 0;
    return;
  }
  seg_lo = (int)(lo / d.seg_len);
  seg_hi = (int)((hi - 1) / d.seg_len) + 1;
}

hipError_t launch_mask_bits(const InstDev &d, int64_t row_begin, int64_t row_end, uint32_t *bits, hipStream_t st,
                            uint32_t *bits2) {
  const int64_t rows = row_end - row_begin;
  if (rows <= 0) return hipSuccess;
  const int W = (int)(d.Npad / 32);
  const int64_t rows_pad = bits_rows_pad(rows);
  const int wend = (int64_t)32 * W == d.N ? W / 2 : W;  // mirrored halves (see k_mask_bits)
  const dim3 grid((unsigned)((rows_pad + 255) / 256), (unsigned)((wend + 63) / 64));
  if (bits2)
    hipLaunchKernelGGL(k_mask_bits<true>, grid, dim3(256), 0, st, d, row_begin, row_end, rows_pad, W, bits, bits2);
  else
    hipLaunchKernelGGL(k_mask_bits<false>, grid, dim3(256), 0, st, d, row_begin, row_end, rows_pad, W, bits,
                       (uint32_t *)nullptr);
  return hipGetLastError();
}

namespace {
template <int WR, int RING, bool PF, bool IL>
hipError_t launch_bin(const InstDev &d, int64_t row_begin, int64_t row_end, float2 *T, int64_t seg_stride,
                      const uint32_t *bits, int seg_lo, int n_seg, hipStream_t st) {
  using BT = BinTile<WR, RING, PF, IL>;
  const int64_t rows = row_end - row_begin;
  const int W = (int)(d.Npad / 32);
  const int n_rt = (int)((rows + BT::rows - 1) / BT::rows);
  const int n_ct = (2 * d.M + kTC - 1) / kTC;
  const int64_t G = (int64_t)n_rt * n_ct * n_seg;
  const int64_t grid = (G + 8 * BT::round - 1) / (8 * BT::round) * (8 * BT::round);  // whole rounds over 8 XCDs
  hipLaunchKernelGGL((k_row_pass_split<WR, RING, PF, IL>), dim3((unsigned)grid), dim3(BT::threads), BT::lds, st, d, row_begin,
                     row_end, n_rt, n_ct, seg_lo, n_seg, bits, W, bits_rows_pad(rows), (float *)T, 2 * seg_stride);
  return hipGetLastError();
}
}  // namespace

hipError_t launch_row_pass_split(const InstDev &d, int32_t S, int64_t row_begin, int64_t row_end, float2 *T,
                                 int64_t seg_stride, const uint32_t *bits, hipStream_t st) {
  (void)S;
  if (row_end <= row_begin) return hipSuccess;
  int seg_lo, seg_hi;
  split_seg_range(d, row_begin, row_end, seg_lo, seg_hi);
  if (seg_hi <= seg_lo) return hipSuccess;
  hipError_t e = init_split_attributes();
  if (e != hipSuccess) return e;
  const int n_seg = seg_hi - seg_lo;
  if (d.bin_tile_rows == 256)
    return launch_bin<2, 4, false, false>(d, row_begin, row_end, T, seg_stride, bits, seg_lo, n_seg, st);
  if (d.bin_ring == 8 && d.bin_prefetch == 1)
    return launch_bin<4, 8, true, false>(d, row_begin, row_end, T, seg_stride, bits, seg_lo, n_seg, st);
  if (d.bin_ring == 8 && d.bin_prefetch == 2)
    return launch_bin<4, 8, false, true>(d, row_begin, row_end, T, seg_stride, bits, seg_lo, n_seg, st);
  if (d.bin_ring == 8)
    return launch_bin<4, 8, false, false>(d, row_begin, row_end, T, seg_stride, bits, seg_lo, n_seg, st);
  return launch_bin<4, 4, false, false>(d, row_begin, row_end, T, seg_stride, bits, seg_lo, n_seg, st);
}

}  // namespace fzp
