// Split-BF16 row pass for deformed (complex) stripes on the CDNA4 matrix
// cores, and the generator of their BF16 stripe planes.  The binary-stripe
// GEMM, the operand table and the shared schedule helpers are in
// fzp_gemm.hip and fzp_split.h.

#include <cmath>

#include "fzp_split.h"

namespace fzp {

namespace {

constexpr int kCThreads = 512;

// Every wave issues 6 copies per stage, 2 stages ahead; waiting until at most
// 6 are outstanding completes the copies of the next stage, then the
// work-group barrier makes them visible.  One asm statement, so that the
// compiler does not put a wait for all outstanding copies in front of the
// barrier.
// Wait until at most N of this wave's copies are in flight (the newest
// stage's), then barrier: N = 6 with all four stripe planes, 4 with the hi
// planes only.
template <int N> __device__ __forceinline__ void stage_barrier() {
  static_assert(N == 0 || N == 5 || N == 6, "add the count");
  if constexpr (N == 6) asm volatile("s_waitcnt vmcnt(6) lgkmcnt(0)\n\ts_barrier" ::: "memory");
  if constexpr (N == 5) asm volatile("s_waitcnt vmcnt(5) lgkmcnt(0)\n\ts_barrier" ::: "memory");
  if constexpr (N == 0) asm volatile("s_waitcnt vmcnt(0) lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// ---------------------------------------------------------------------------
// Deformed stripes.  With a membrane phase screen the stripe
// g = mask exp(2 pi i phi) is complex and the row pass is the full complex
// product
//   T_re = g_re.A_re - g_im.A_im,    T_im = g_re.A_im + g_im.A_re,
// with both operands split into BF16 hi + lo and the three leading products
//   g.A ~ g_hi.A_hi + g_hi.A_lo + g_lo.A_hi
// (g_lo.A_lo is below 2^-32 relative and dropped).  Against the table's
// interleaved columns [A_re | A_im] the imaginary stripe needs the columns
// [-A_im | A_re]: the MFMA B operand of column n is swapped with that of its
// neighbour n ^ 1 (a lane-pair DPP move, the two lanes hold the same k range)
// and negated on even columns, so both products read the same LDS slab.
//
// The stripe is generated once per chunk (phase screen in FP32 turns from
// FP64 ridge distances; zone mask from the exact integer rule) into
//   G[v][kb][row][16],  v = re_hi, re_lo, im_hi, im_lo,
// kb = 16-column block of the chunk's disc chord, rows padded to the 256-row
// tile, so one pipeline stage of a row tile is a contiguous 8 KiB per plane.
// ---------------------------------------------------------------------------
constexpr int kCTR = 256;     // rows per tile
constexpr int kCTC = 256;     // real columns per tile (128 complex ROI columns); 128 in the narrow variant
constexpr int kCKT = 16;      // K columns per pipeline stage (one MFMA K-step)
constexpr int kCRowB = 32;    // LDS bytes per slab row
constexpr int kCGBytes = 4 * kCTR * kCRowB;   // 32768: four stripe planes
constexpr int kCBBytes = 2 * kCTC * kCRowB;   // 16384: table hi and lo
constexpr int kCStage = kCGBytes + kCBBytes;  // 49152
constexpr int kCRing = 3;  // LDS stages (the default tile); copies run kCRing - 1 stages ahead
constexpr int kCLdsBytes = kCRing * kCStage;  // 147456
// LDS of a tile with CT real columns and a ring of RING stages
constexpr int cplx_lds_bytes(int CT, int RING = kCRing) { return RING * (kCGBytes + 2 * CT * kCRowB); }

// 16-byte half of a 32-byte slab row in LDS: swapped on rows 8..15 of every
// 16 so that 16 consecutive rows read at one half hit 64 distinct banks.
__device__ __forceinline__ int chalf(int row, int half) { return half ^ ((row >> 3) & 1); }

// sin and cos of 2 pi t (t in turns, |t| up to a few hundred) in float32:
// t is cut into a quarter-turn count q and a remainder r in [-1/2, 1/2]
// quarter turns, sin and cos of the angle r pi/2 (at most pi/4) come from
// their Taylor series through the x^9 and x^10 terms (truncation below
// 3e-9), and q mod 4 rotates the pair.  Enough for the BF16 hi/lo pair the
// stripe keeps (16 significant bits).
__device__ __forceinline__ void sincos_turns(float t, float &sn, float &cs) {
  const float u = 4.0f * t;
  const float q = rintf(u);
  const float x = (u - q) * 1.57079632679489662f;
  const float x2 = x * x;
  float ps = fmaf(x2, 1.0f / 362880.0f, -1.0f / 5040.0f);
  ps = fmaf(x2, ps, 1.0f / 120.0f);
  ps = fmaf(x2, ps, -1.0f / 6.0f);
  const float sx = fmaf(x * x2, ps, x);
  float pc = fmaf(x2, -1.0f / 3628800.0f, 1.0f / 40320.0f);
  pc = fmaf(x2, pc, -1.0f / 720.0f);
  pc = fmaf(x2, pc, 1.0f / 24.0f);
  pc = fmaf(x2, pc, -0.5f);
  const float cx = fmaf(x2, pc, 1.0f);
  const int k = (int)q & 3;  // angle = x + k pi/2
  const float a = (k & 1) ? cx : sx, b = (k & 1) ? sx : cx;
  sn = (k & 2) ? -a : a;
  cs = ((k + 1) & 2) ? -b : b;
}

// Round to nearest even into BF16 by the hardware conversion (one
// instruction; the same result as the integer rounding of the operand table).
__device__ __forceinline__ uint16_t bf16_cvt(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }

// PHASE: an L-level phase plate (levels != 0).  Crease-free 2- and 4-level
// plates never come here: they are sums of binary masks (k_col_operand).
// I8: the int8 row pass's operand instead of the BF16 pair: the same layout
// with one byte per sample, planes v = s0_re, s1_re, s0_im, s1_im, the two
// balanced digits of rint(kI8Scale g) (as the int8 table), and the written
// blocks rounded to that pass's 32-column stages.
template <bool PHASE, bool I8 = false>
__global__ __launch_bounds__(kCTR) void k_stripe_cplx(InstDev d, int64_t row_begin, int64_t row_end,
                                                     int64_t rows_pad, int64_t kb0, int64_t nkb,
                                                     uint16_t *__restrict__ G) {
  const int64_t rl = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (rl >= rows_pad) return;
  const int64_t N = d.N;
  const int64_t row = row_begin + rl;
  const bool live = row < row_end;
  const double cj = (double)(2 * row - N + 1);
  const double bj = cj * cj;
  const double y = 0.5 * cj * d.dx;
  const double hdx = 0.5 * d.dx;
  const int nc = d.n_creases;
  const CreaseDev *cr = d.cr;
  const int64_t plane = nkb * rows_pad * 16;
  // The GEMM reads a row tile's slab only inside that tile's disc chord
  // (rounded out to whole 16-column blocks): blocks outside it are not written.
  int64_t t_lo, t_hi;
  {
    const int64_t r0 = row_begin + (int64_t)blockIdx.x * kCTR;
    const int64_t r1 = r0 + kCTR - 1 < row_end - 1 ? r0 + kCTR - 1 : row_end - 1;
    tile_chord(d, r0, r1, t_lo, t_hi);
    constexpr int kAl = I8 ? 32 : 16;
    t_lo = t_lo / kAl * kAl;
    t_hi = (t_hi + kAl - 1) / kAl * kAl;
  }
  for (int64_t kb = blockIdx.y; kb < nkb; kb += gridDim.y) {
    const int64_t i0 = 16 * (kb0 + kb);
    if (i0 < t_lo || i0 >= t_hi) continue;
    const double c0 = (double)(2 * i0 - N + 1);
    // zone mask of the 16 samples (exact integer rule); for an L-level phase
    // plate every disc sample passes and carries -l/L turns of lens phase,
    // l = floor(K kappa_L) mod L
    uint32_t open = 0;
    float turns[16];
    if constexpr (PHASE) {
      const int L = d.levels;
      const float inv_l = 1.0f / (float)L;
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const double ci = c0 + 2.0 * e;
        const double K = fma(ci, ci, bj);
        const int lv = (int)(K * d.kappa_l) % L;
        const bool o = live && i0 + e < N && K <= d.kmax;
        open |= (o ? 1u : 0u) << e;
        turns[e] = -(float)lv * inv_l;
      }
    } else {
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const double ci = c0 + 2.0 * e;
        const double K = fma(ci, ci, bj);
        const int zone = (int)(K * d.kappa);
        const bool o = live && i0 + e < N && K <= d.kmax && (((zone & 1) ^ d.centre_open) != 0);
        open |= (o ? 1u : 0u) << e;
        turns[e] = 0.0f;
      }
    }
    // Crease phase in turns.  Along the row the ridge distance d grows by
    // st = dx cos(theta) per sample, so the Gaussian g = exp(-a d^2) obeys
    // g(i+1) = g(i) r(i) with r(i+1) = r(i) q, r(0) = exp(-a (2 d0 st + st^2)),
    // q = exp(-2 a st^2): three exponentials per ridge per 16 samples, started
    // from the float64 distance of the first sample.  A ridge whose term stays
    // below 2^-30 turns over all 16 samples (|h| exp(-a d^2) < 2^-30 at the
    // nearest of them) is skipped; neighbouring rows of a wave see nearly the
    // same distances, so the skip is close to wave-uniform.
    const double x0 = hdx * c0;
    for (int k = 0; k < nc; ++k) {
      const float dd = (float)fma(x0, cr[k].c, fma(y, cr[k].s, -cr[k].rho));
      const float st = (float)(d.dx * cr[k].c);
      const float a = (float)cr[k].inv2s2;
      const float h = (float)cr[k].h_over_lambda;
      const float d15 = fmaf(15.0f, st, dd);
      const float dmin = (dd > 0.0f) == (d15 > 0.0f) ? fminf(fabsf(dd), fabsf(d15)) : 0.0f;
      if (a * dmin * dmin > __logf(fabsf(h)) + 20.7944154f) continue;  // ln 2^30
      float g = __expf(-a * dd * dd);
      float r = __expf(-a * (2.0f * dd * st + st * st));
      const float q = __expf(-2.0f * a * st * st);
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        turns[e] = fmaf(h, g, turns[e]);
        g *= r;
        r *= q;
      }
    }
    if constexpr (I8) {
      uint32_t w8[4][4] = {};
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        // sin and cos of 2 pi t from the hardware's transcendental unit, whose
        // input is in turns and valid to +-256: t is first reduced to
        // [-1/2, 1/2] (exact in float32), so any ridge height is taken; within
        // 1.3e-7 of float64 over [-8, 8] turns (measured on 4 million points),
        // far below the digits' quantisation step of 1 / 16256
        const float tr = turns[e] - rintf(turns[e]);
        const float sn = __builtin_amdgcn_sinf(tr), cs = __builtin_amdgcn_cosf(tr);
        const bool o = (open >> e) & 1u;
        const int vr = o ? (int)rintf(cs * (float)kI8Scale) : 0, vi = o ? (int)rintf(sn * (float)kI8Scale) : 0;
        // balanced digits v = 128 d0 + d1, d1 in [-64, 63]
        const int r0 = (vr + 64) >> 7, i0 = (vi + 64) >> 7;
        const uint32_t dg[4] = {(uint32_t)(r0 & 0xff), (uint32_t)((vr - (r0 << 7)) & 0xff), (uint32_t)(i0 & 0xff),
                                (uint32_t)((vi - (i0 << 7)) & 0xff)};
#pragma unroll
        for (int v = 0; v < 4; ++v) w8[v][e >> 2] |= dg[v] << (8 * (e & 3));
      }
      int8_t *G8 = (int8_t *)G;
#pragma unroll
      for (int v = 0; v < 4; ++v)
        *(u32x4 *)(G8 + v * plane + (kb * rows_pad + rl) * 16) = u32x4{w8[v][0], w8[v][1], w8[v][2], w8[v][3]};
      continue;
    }
    uint32_t w[4][8];
#pragma unroll
    for (int e = 0; e < 16; e += 2) {
      uint32_t pr[4] = {0u, 0u, 0u, 0u};
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        float sn, cs;
        sincos_turns(turns[e + u], sn, cs);
        const bool o = (open >> (e + u)) & 1u;
        const float gr = o ? cs : 0.0f, gi = o ? sn : 0.0f;
        const uint16_t rh = bf16_cvt(gr), ih = bf16_cvt(gi);
        const uint16_t rlo = bf16_cvt(gr - __uint_as_float((uint32_t)rh << 16));
        const uint16_t ilo = bf16_cvt(gi - __uint_as_float((uint32_t)ih << 16));
        pr[0] |= (uint32_t)rh << (16 * u);
        pr[1] |= (uint32_t)rlo << (16 * u);
        pr[2] |= (uint32_t)ih << (16 * u);
        pr[3] |= (uint32_t)ilo << (16 * u);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) w[v][e >> 1] = pr[v];
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      u32x4 *dst = (u32x4 *)(G + v * plane + (kb * rows_pad + rl) * 16);
      dst[0] = u32x4{w[v][0], w[v][1], w[v][2], w[v][3]};
      dst[1] = u32x4{w[v][4], w[v][5], w[v][6], w[v][7]};
    }
  }
}

// Column n's B operand from lane l ^ 1 (column n ^ 1), negated on even columns.
__device__ __forceinline__ bf16x8 swap_neg(bf16x8 b, uint32_t nmask) {
  u32x4 u = __builtin_bit_cast(u32x4, b), r;
#pragma unroll
  for (int j = 0; j < 4; ++j)
    r[j] = (uint32_t)__builtin_amdgcn_mov_dpp((int)u[j], 0xb1, 0xf, 0xf, true) ^ nmask;  // quad_perm [1,0,3,2]
  return __builtin_bit_cast(bf16x8, r);
}

// Row-pass GEMM for complex stripes.  Work-group tile: kCTR aperture rows x
// kCTC real columns of T over one K segment (trimmed to the tiles' disc
// chord).  With COL the same kernel is the column pass of the split path:
// rows are ROI rows p, K is the chunk's aperture rows j (segments of
// seg_len_c rows, no chord), the A operand the column kernel matrix B_y and
// the B operand the chunk's row-pass result T (see k_col_operand).  8 waves
// in a 4 (rows) x 2 (columns) grid, each 64 x 128 = 2 x 4 MFMA 32x32 blocks
// (128 float32 accumulators per lane), 6 MFMAs per block per K-step.  Stripe
// and table slabs move HBM -> LDS by direct copies into a 3-deep ring, 2
// stages ahead, one barrier per stage.
// CT = 128 with RING = 2 (one stage ahead, 80 KiB of LDS) fits two
// work-groups per CU, so that one work-group's barrier waits are covered by
// the other's MFMAs.
template <bool COL, int CT = kCTC, int RING = kCRing>
__global__ __launch_bounds__(kCThreads, RING == 2 ? 2 : 1) void k_row_pass_split_cplx(
    InstDev d, int64_t row_begin, int64_t row_end, int n_rt, int n_ct, int seg_lo, int n_seg,
    const uint16_t *__restrict__ G, int64_t rows_pad, int64_t kb0, int64_t nkb, float *__restrict__ T,
    int64_t seg_stride_f, const uint16_t *__restrict__ Bop, int64_t kB0, int64_t KB, int64_t k_begin, int64_t k_end,
    int64_t seg_len_c) {
  extern __shared__ __attribute__((aligned(16))) char lds[];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int G_ = n_rt * n_ct * n_seg;
  const int slot = blockIdx.x >> 3;
  const int g = (slot >> 5) * 256 + (blockIdx.x & 7) * 32 + (slot & 31);
  if (g >= G_) return;
  const int rt = g % n_rt;
  const int ct = (g / n_rt) % n_ct;
  const int seg = seg_lo + g / (n_rt * n_ct);

  const int M2 = 2 * d.M;
  const int64_t r0 = row_begin + (int64_t)rt * kCTR;
  int64_t rl = r0 + kCTR - 1;
  if (rl > row_end - 1) rl = row_end - 1;
  // CT real columns per tile: waves 4 (rows) x 2 (columns), each CB column
  // blocks of 32; NB table pieces (32 columns of one plane) copied per wave
  static_assert(CT == 256 || CT == 128, "tile width");
  static_assert(RING == 3 || RING == 2, "ring depth");
  constexpr int CB = CT / 64, NB = CT / 128, PPP = CT / 32;
  constexpr int kStage = kCGBytes + 2 * CT * kCRowB;
  constexpr int kAheadR = RING - 1;
  // copies a wave may leave in flight at a stage's end: those of the newest
  // stage with two stages ahead, none with one
  constexpr int kWait = RING == 3 ? 4 + NB : 0;
  const int c0 = ct * CT;
  int64_t k_lo, k_hi;
  if constexpr (COL) {
    k_lo = k_begin + (int64_t)(seg - seg_lo) * seg_len_c;
    k_hi = k_lo + seg_len_c < k_end ? k_lo + seg_len_c : k_end;
  } else {
    const int64_t s_lo = (int64_t)seg * d.seg_len;
    const int64_t s_hi = s_lo + d.seg_len < d.Npad ? s_lo + d.seg_len : d.Npad;
    tile_chord(d, r0, rl, k_lo, k_hi);
    k_lo = k_lo / kCKT * kCKT;
    k_hi = (k_hi + kCKT - 1) / kCKT * kCKT;
    if (k_lo < s_lo) k_lo = s_lo;
    if (k_hi > s_hi) k_hi = s_hi;
    if (k_lo < 16 * kb0) k_lo = 16 * kb0;
    if (k_hi > 16 * (kb0 + nkb)) k_hi = 16 * (kb0 + nkb);
  }

  // ---- copy roles.  Stripe: wave w copies slab pieces x = 4w .. 4w+3 (plane
  // x / 8, rows 32 (x % 8) ..); table: pieces y = 2w, 2w+1 (plane y / 8,
  // columns 32 (y % 8) ..).  Lane L fills LDS row L / 2, half L & 1, which
  // holds global half chalf(row, L & 1).  Table columns past 2M read column 0:
  // they feed only accumulator columns that are never stored.
  const int64_t plane = nkb * rows_pad * 16;
  constexpr int NG = 4;
  const uint16_t *gsrc[NG];
  int gx[NG];
#pragma unroll
  for (int j = 0; j < NG; ++j) {
    const int x = 4 * wave + j;
    gx[j] = x;
    const int row = (x & 7) * 32 + (lane >> 1);
    gsrc[j] = G + (x >> 3) * plane + ((int64_t)rt * kCTR + row) * 16 + 8 * chalf(row, lane & 1);
  }
  const uint16_t *bsrc[NB];
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    const int y = NB * wave + j;
    const int col = (y % PPP) * 32 + (lane >> 1);
    const int gc = c0 + col < M2 ? c0 + col : 0;
    bsrc[j] = Bop + (int64_t)(y / PPP) * M2 * KB + (int64_t)gc * 32 + 8 * chalf(col, lane & 1);
  }

  // ---- compute role: wave (wr, wc) covers rows wr*64 .., columns wc*128 ..
  // (2 x 4 MFMA blocks: each stripe operand read from LDS feeds four column
  // blocks)
  const int wr = wave >> 1, wc = wave & 1;
  const int l32 = lane & 31, lhi = lane >> 5;
  const int hofs = chalf(l32, lhi) * 16;
  const int aoff = (wr * 64 + l32) * kCRowB + hofs;
  const int boff = kCGBytes + (wc * 32 * CB + l32) * kCRowB + hofs;
  const uint32_t nmask = (lane & 1) ? 0u : 0x80008000u;

  f32x16 acc[2][CB];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < CB; ++b)
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[a][b][e] = 0.0f;

  if (k_lo < k_hi) {
    const int64_t kb = k_lo;
    const int nst = (int)((k_hi - k_lo) / kCKT);
    const int64_t klast = k_hi - kCKT;  // copies past the end repeat the last stage
    auto copy_stage = [&](int s) {
      const int64_t k = kb + (int64_t)s * kCKT < klast ? kb + (int64_t)s * kCKT : klast;
      char *dst = lds + (s % RING) * kStage;
      const int64_t gofs = (k / 16 - kb0) * rows_pad * 16;
#pragma unroll
      for (int j = 0; j < NG; ++j)
        __builtin_amdgcn_global_load_lds((const void *)(gsrc[j] + gofs),
                                         (__attribute__((address_space(3))) void *)(dst + gx[j] * 1024), 16, 0, 0);
      const int64_t kr = k - kB0;  // K index of the B operand's blocked layout
      const int64_t bofs = (kr >> 5) * M2 * 32 + (kr & 31);
#pragma unroll
      for (int j = 0; j < NB; ++j)
        __builtin_amdgcn_global_load_lds((const void *)(bsrc[j] + bofs),
                                         (__attribute__((address_space(3))) void *)(dst + kCGBytes +
                                                                                    (NB * wave + j) * 1024),
                                         16, 0, 0);
    };
    for (int s = 0; s < kAheadR; ++s) copy_stage(s);
    stage_barrier<kWait>();
    for (int s = 0; s < nst; ++s) {
      copy_stage(s + kAheadR);
      const char *sb = lds + (s % RING) * kStage;
      bf16x8 bh[CB], bl[CB], bhs[CB], bls[CB];
#pragma unroll
      for (int cb = 0; cb < CB; ++cb) {
        bh[cb] = __builtin_bit_cast(bf16x8, lds_ld16(sb + boff + cb * 32 * kCRowB));
        bl[cb] = __builtin_bit_cast(bf16x8, lds_ld16(sb + boff + cb * 32 * kCRowB + CT * kCRowB));
        bhs[cb] = swap_neg(bh[cb], nmask);
        bls[cb] = swap_neg(bl[cb], nmask);
      }
#pragma unroll
      for (int rb = 0; rb < 2; ++rb) {
        const char *pa = sb + aoff + rb * 32 * kCRowB;
        const bf16x8 rh = __builtin_bit_cast(bf16x8, lds_ld16(pa));
        const bf16x8 ih = __builtin_bit_cast(bf16x8, lds_ld16(pa + 2 * kCTR * kCRowB));
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) {
          acc[rb][cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(rh, bh[cb], acc[rb][cb], 0, 0, 0);
          acc[rb][cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ih, bhs[cb], acc[rb][cb], 0, 0, 0);
        }
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) {
          acc[rb][cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(rh, bl[cb], acc[rb][cb], 0, 0, 0);
          acc[rb][cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ih, bls[cb], acc[rb][cb], 0, 0, 0);
        }
        const bf16x8 rlo = __builtin_bit_cast(bf16x8, lds_ld16(pa + 1 * kCTR * kCRowB));
        const bf16x8 ilo = __builtin_bit_cast(bf16x8, lds_ld16(pa + 3 * kCTR * kCRowB));
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) {
          acc[rb][cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(rlo, bh[cb], acc[rb][cb], 0, 0, 0);
          acc[rb][cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ilo, bhs[cb], acc[rb][cb], 0, 0, 0);
        }
      }
      stage_barrier<kWait>();
    }
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  }
  // epilogue: register v of lane l holds row 8(v/4) + 4(l/32) + (v%4) of its
  // block and column l%32.  Row pass: partials column-major per real column;
  // column pass: row-major (ROI row p, real column c), so that the finishing
  // kernel reads and writes along ROI rows.
  float *Ts = T + (int64_t)(seg - seg_lo) * seg_stride_f;
  if constexpr (COL) {
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) {
      const int c = c0 + wc * 32 * CB + cb * 32 + l32;
      if (c >= M2) continue;
#pragma unroll
      for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int64_t r = r0 + wr * 64 + 4 * lhi + rb * 32 + 8 * a + e;
            if (r < row_end) Ts[r * M2 + c] = acc[rb][cb][4 * a + e];
          }
    }
    return;
  }
  const int64_t rs = seg_stride_f / M2;
#pragma unroll
  for (int cb = 0; cb < CB; ++cb) {
    const int c = c0 + wc * 32 * CB + cb * 32 + l32;
    if (c >= M2) continue;
    float *col = Ts + (int64_t)c * rs - row_begin;
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        const int64_t r = r0 + wr * 64 + 4 * lhi + rb * 32 + 8 * a;
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

// ---------------------------------------------------------------------------
// Column pass of the split path (B_y . T, Eqs. 9-10 along y): per chunk of
// aperture rows j, C[p][q] = sum_j B_y[p][j] T[j][q] with
//   B_y[p][j] = exp(2 pi i (beta c_j^2 / 2 - alpha c_j d_p)),
//   c_j = j - (N-1)/2, d_p = p - M/2 + s_y,
// on the matrix cores with the same three-product BF16 split and float32
// accumulation per K segment; the segments and the chunks are added in
// float64 into the ROI together with the output factor of Eq. 2.
// ---------------------------------------------------------------------------

// B_y in the stripe-plane layout G[v][j/16][p][16] (v = re_hi, re_lo, im_hi,
// im_lo), p padded to the 256-row tile, j to Npad; zero outside p < M, j < N.
__global__ __launch_bounds__(256) void k_build_col_table(InstDev d, int64_t rows_pad, uint16_t *__restrict__ By) {
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t p = blockIdx.y;
  if (j >= d.Npad) return;
  const int M = d.M;
  uint16_t hr = 0, hi_ = 0, lr = 0, li = 0;
  if (j < d.N && p < M) {
    const double c = (double)j - 0.5 * (double)(d.N - 1);
    const double dp = (double)p - 0.5 * (double)M + d.sy;
    const double ph = 0.5 * d.beta * (c * c);
    const double lin = d.alpha * c * dp;
    const double2 a = cexp_turns((ph - rint(ph)) - (lin - rint(lin)));
    hr = bf16_rne((float)a.x);
    hi_ = bf16_rne((float)a.y);
    lr = bf16_rne((float)(a.x - (double)__uint_as_float((uint32_t)hr << 16)));
    li = bf16_rne((float)(a.y - (double)__uint_as_float((uint32_t)hi_ << 16)));
  }
  const int64_t plane = (d.Npad / 16) * rows_pad * 16;
  const int64_t at = ((j >> 4) * rows_pad + p) * 16 + (j & 15);
  By[at] = hr;
  By[plane + at] = lr;
  By[2 * plane + at] = hi_;
  By[3 * plane + at] = li;
}

// T of the chunk (float32 partial planes, one per K segment of the row pass,
// column-major per real column, summed here in float64) as the column GEMM's
// B operand: BF16 hi and lo planes in the operand-table layout
// Tb[h][kk/32][c][kk%32], kk = j - kB0 for j in [kB0, kB0 + KB); zero for rows
// outside [row_begin, row_end).  A work-group covers one 32-row block of kk and
// 8 columns, so each wave reads two 128-byte runs of T and writes one
// 128-byte run per plane (one 512-byte run per work-group).
// With S (a 2-level plate) the partial planes hold T_mask and the operand is
// T_disc - 2 T_mask, T_disc = S[hi] - S[lo] over row j's disc chord [lo, hi).
// With S and T2 (a 4-level plate) T holds the odd zones' T_u and T2 the
// second mask's T_v, and the operand is T_disc - (1 - i) T_u - (1 + i) T_v:
//   re: D_re - (U_re + U_im) - (V_re - V_im),  im: D_im - (U_im - U_re) - (V_im + V_re).
// The int8 row pass's planes hold int32 sums (raw bits), added exactly in int64.
__device__ __forceinline__ int64_t sum_segments_i32(const float *src, int nseg, int64_t seg_stride_f) {
  const int32_t *s32 = (const int32_t *)src;
  int64_t a = 0;
  for (int sgi = 0; sgi < nseg; ++sgi) a += s32[(int64_t)sgi * seg_stride_f];
  return a;
}

// MODE 0: float32 planes (split-BF16 row pass); 1: int32 sums of the int8
// binary row pass, in units of 1 / kI8Scale; 2: float32 planes of the int8
// complex row pass, in units of 1 / kI8Scale^2.
template <int MODE> __device__ __forceinline__ double sum_segments(const float *src, int nseg, int64_t seg_stride_f) {
  if constexpr (MODE == 1) return (double)sum_segments_i32(src, nseg, seg_stride_f) * (1.0 / kI8Scale);
  double v = 0.0;
  int sgi = 0;
  for (; sgi + 4 <= nseg; sgi += 4) {
    const float a0 = src[(int64_t)sgi * seg_stride_f], a1 = src[(int64_t)(sgi + 1) * seg_stride_f];
    const float a2 = src[(int64_t)(sgi + 2) * seg_stride_f], a3 = src[(int64_t)(sgi + 3) * seg_stride_f];
    v += (double)a0;
    v += (double)a1;
    v += (double)a2;
    v += (double)a3;
  }
  for (; sgi < nseg; ++sgi) v += (double)src[(int64_t)sgi * seg_stride_f];
  return v;
}

template <int MODE>
__global__ __launch_bounds__(256) void k_col_operand(int M2, int64_t row_begin, int64_t row_end,
                                                     const float *__restrict__ T, int nseg, int64_t seg_stride_f,
                                                     int64_t rs, int64_t kB0, int64_t KB, uint16_t *__restrict__ Tb,
                                                     const double2 *__restrict__ S, int64_t N, double kmax,
                                                     const float *__restrict__ T2) {
  const int64_t kk = blockIdx.x * (int64_t)32 + (threadIdx.x & 31);
  const int c = blockIdx.y * 8 + (threadIdx.x >> 5);
  if (kk >= KB || c >= M2) return;
  const int64_t j = kB0 + kk;
  uint16_t h = 0, l = 0;
  if (j >= row_begin && j < row_end) {
    double v = sum_segments<MODE == 2 ? 0 : MODE>(T + (int64_t)c * rs + (j - row_begin), nseg, seg_stride_f);
    if constexpr (MODE == 2) v *= 1.0 / (kI8Scale * kI8Scale);
    if (T2) {
      // c and its partner column c ^ 1 (re / im of the same ROI column)
      const double u_o = sum_segments<MODE>(T + (int64_t)(c ^ 1) * rs + (j - row_begin), nseg, seg_stride_f);
      const double v_s = sum_segments<MODE>(T2 + (int64_t)c * rs + (j - row_begin), nseg, seg_stride_f);
      const double v_o = sum_segments<MODE>(T2 + (int64_t)(c ^ 1) * rs + (j - row_begin), nseg, seg_stride_f);
      // re (c even): U_re + U_im + V_re - V_im; im (c odd): U_im - U_re + V_im + V_re
      v = (c & 1) ? (v - u_o) + (v_s + v_o) : (v + u_o) + (v_s - v_o);
    }
    if (S) {
      const double cj = (double)(2 * j - N + 1);
      const double rem = kmax - cj * cj;
      double disc = 0.0;
      if (rem >= 0.0) {
        int64_t m = (int64_t)sqrt(rem);
        while ((double)(m + 1) * (double)(m + 1) <= rem) ++m;
        while (m > 0 && (double)m * (double)m > rem) --m;
        int64_t lo = (N - 1 - m + 1) >> 1, hi = ((N - 1 + m) >> 1) + 1;
        if (lo < 0) lo = 0;  // a disc wider than the grid
        if (hi > N) hi = N;
        const double2 a = S[hi * (M2 / 2) + (c >> 1)], b = S[lo * (M2 / 2) + (c >> 1)];
        disc = (c & 1) ? a.y - b.y : a.x - b.x;
      }
      v = T2 ? disc - v : disc - 2.0 * v;
    }
    h = bf16_rne((float)v);
    l = bf16_rne((float)(v - (double)__uint_as_float((uint32_t)h << 16)));
  }
  const int64_t at = (kk >> 5) * (int64_t)M2 * 32 + (int64_t)c * 32 + (kk & 31);
  Tb[at] = h;
  Tb[(int64_t)M2 * KB + at] = l;
}

// ROI[p][q] += F[p][q] sum_seg C_seg[p][q] (float64), F the output factor of
// Eq. 2; C_seg row-major with re/im adjacent: C[seg][p][2q + {0, 1}].
__global__ __launch_bounds__(256) void k_col_finish(InstDev d, const float *__restrict__ C, int nseg,
                                                    int64_t segC, double2 *__restrict__ roi) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  const int p = blockIdx.y;
  const int M = d.M;
  if (q >= M) return;
  const float2 *src = (const float2 *)(C + (int64_t)p * (2 * M)) + q;
  float2 v = src[0];
  double2 acc = make_double2((double)v.x, (double)v.y);
  for (int sgi = 1; sgi < nseg; ++sgi) {
    v = src[(int64_t)sgi * (segC / 2)];
    acc = cadd(acc, make_double2((double)v.x, (double)v.y));
  }
  const double xq = d.x0 + ((double)q - 0.5 * (double)M) * d.dx_out;
  const double yp = d.y0 + ((double)p - 0.5 * (double)M) * d.dx_out;
  const double2 F = cscale(cexp_turns(d.kz_turns + (xq * xq + yp * yp) * d.inv2lz), d.scale);
  double2 *o = roi + (int64_t)p * M + q;
  *o = cadd(*o, cmul(F, acc));
}

}  // namespace

hipError_t init_cplx_attributes() {
  hipError_t e = hipFuncSetAttribute((const void *)k_row_pass_split_cplx<false>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, kCLdsBytes);
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void *)k_row_pass_split_cplx<true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            kCLdsBytes);
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void *)k_row_pass_split_cplx<false, 128>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, cplx_lds_bytes(128));
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void *)k_row_pass_split_cplx<false, 128, 2>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, cplx_lds_bytes(128, 2));
  return e;
}

size_t split_stripe_bytes(const InstDev &d, int64_t chunk_rows) {
  const int64_t rows_pad = (chunk_rows + kCTR - 1) / kCTR * kCTR;
  return (size_t)rows_pad * (size_t)d.Npad * 4 * sizeof(uint16_t);
}

void split_stripe_extent(const InstDev &d, int64_t row_begin, int64_t row_end, int64_t &rows_pad, int64_t &kb0,
                         int64_t &nkb) {
  int64_t lo, hi;
  split_chunk_chord(d, row_begin, row_end, lo, hi);
  rows_pad = (row_end - row_begin + kCTR - 1) / kCTR * kCTR;
  // 16-column blocks; an even count from an even block for the int8 row
  // pass's 32-column stages
  const int64_t al = d.i8 ? 32 : 16;
  kb0 = lo / al * al / 16;
  nkb = hi > lo ? (hi + al - 1) / al * al / 16 - kb0 : 0;
}

hipError_t launch_stripe_cplx(const InstDev &d, int64_t row_begin, int64_t row_end, uint16_t *G, hipStream_t st) {
  int64_t rows_pad, kb0, nkb;
  split_stripe_extent(d, row_begin, row_end, rows_pad, kb0, nkb);
  if (nkb <= 0 || rows_pad <= 0) return hipSuccess;
  // x: one work-group row per 256-row GEMM tile (the kernel takes that tile's
  // chord); y: about 4096 work-groups in all, each striding over the 16-column
  // blocks (measured a little faster than one work-group per block)
  const int64_t gx = (rows_pad + kCTR - 1) / kCTR;
  int64_t gy = 4096 / gx;
  if (gy < 1) gy = 1;
  if (gy > nkb) gy = nkb;
  if (gy > 65535) gy = 65535;
  const dim3 grid((unsigned)gx, (unsigned)gy);
  if (d.levels != 0 && d.i8)
    hipLaunchKernelGGL((k_stripe_cplx<true, true>), grid, dim3(kCTR), 0, st, d, row_begin, row_end, rows_pad, kb0,
                       nkb, G);
  else if (d.i8)
    hipLaunchKernelGGL((k_stripe_cplx<false, true>), grid, dim3(kCTR), 0, st, d, row_begin, row_end, rows_pad, kb0,
                       nkb, G);
  else if (d.levels != 0)
    hipLaunchKernelGGL(k_stripe_cplx<true>, grid, dim3(kCTR), 0, st, d, row_begin, row_end, rows_pad, kb0, nkb, G);
  else
    hipLaunchKernelGGL(k_stripe_cplx<false>, grid, dim3(kCTR), 0, st, d, row_begin, row_end, rows_pad, kb0, nkb, G);
  return hipGetLastError();
}

hipError_t launch_row_pass_split_cplx(const InstDev &d, int64_t row_begin, int64_t row_end, float2 *T,
                                      int64_t seg_stride, const uint16_t *G, hipStream_t st) {
  const int64_t rows = row_end - row_begin;
  if (rows <= 0) return hipSuccess;
  int64_t rows_pad, kb0, nkb;
  split_stripe_extent(d, row_begin, row_end, rows_pad, kb0, nkb);
  int seg_lo, seg_hi;
  split_seg_range(d, row_begin, row_end, seg_lo, seg_hi);
  if (seg_hi <= seg_lo || nkb <= 0) return hipSuccess;
  // tile width: 256 real columns, or 128 (cplx_tile = 1: twice the work-groups
  // for a small ROI, each operand read from LDS feeding half as many MFMAs;
  // cplx_tile = 2: the same with a 2-stage ring and two work-groups per CU)
  const int CT = d.cplx_tile >= 1 ? 128 : kCTC;
  const int n_rt = (int)((rows + kCTR - 1) / kCTR);
  const int n_ct = (2 * d.M + CT - 1) / CT;
  const int n_seg = seg_hi - seg_lo;
  const int64_t Gn = (int64_t)n_rt * n_ct * n_seg;
  const int64_t grid = (Gn + 255) / 256 * 256;
  hipError_t e = init_split_attributes();
  if (e != hipSuccess) return e;
  if (d.cplx_tile == 2)
    hipLaunchKernelGGL((k_row_pass_split_cplx<false, 128, 2>), dim3((unsigned)grid), dim3(kCThreads),
                       cplx_lds_bytes(128, 2), st, d, row_begin, row_end, n_rt, n_ct, seg_lo, n_seg, G, rows_pad,
                       kb0, nkb, (float *)T, 2 * seg_stride, d.A, (int64_t)0, d.Npad, (int64_t)0, (int64_t)0,
                       (int64_t)0);
  else if (CT == 128)
    hipLaunchKernelGGL((k_row_pass_split_cplx<false, 128>), dim3((unsigned)grid), dim3(kCThreads),
                       cplx_lds_bytes(128), st, d, row_begin, row_end, n_rt, n_ct, seg_lo, n_seg, G, rows_pad, kb0,
                       nkb, (float *)T, 2 * seg_stride, d.A, (int64_t)0, d.Npad, (int64_t)0, (int64_t)0, (int64_t)0);
  else
    hipLaunchKernelGGL(k_row_pass_split_cplx<false>, dim3((unsigned)grid), dim3(kCThreads), kCLdsBytes, st, d,
                       row_begin, row_end, n_rt, n_ct, seg_lo, n_seg, G, rows_pad, kb0, nkb, (float *)T,
                       2 * seg_stride, d.A, (int64_t)0, d.Npad, (int64_t)0, (int64_t)0, (int64_t)0);
  return hipGetLastError();
}


// Column pass of the split path: K extent and segments of one chunk.
namespace {
struct ColSchedule {
  int64_t kB0, KB, k_begin, k_end, seg_len;
  int n_rt, n_ct, n_seg;
};
ColSchedule col_schedule(int M, int64_t row_begin, int64_t row_end) {
  ColSchedule c;
  c.kB0 = row_begin / 32 * 32;
  c.k_begin = row_begin / 16 * 16;
  c.k_end = (row_end + 15) / 16 * 16;
  c.KB = (c.k_end - c.kB0 + 31) / 32 * 32;
  c.n_rt = (M + kCTR - 1) / kCTR;
  c.n_ct = (2 * M + kCTC - 1) / kCTC;
  // about 512 tiles in all, segments of at least 256 rows
  const int64_t target = (512 + c.n_rt * c.n_ct - 1) / (c.n_rt * c.n_ct);
  const int64_t rows = c.k_end - c.k_begin;
  int64_t len = (rows + target - 1) / target;
  len = (len + 15) / 16 * 16;
  if (len < 256) len = 256;
  c.seg_len = len;
  c.n_seg = rows > 0 ? (int)((rows + len - 1) / len) : 0;
  return c;
}
}  // namespace

size_t col_table_bytes(int M, int64_t Npad) {
  const int64_t rows_pad = (M + kCTR - 1) / kCTR * kCTR;
  return (size_t)4 * (size_t)Npad * (size_t)rows_pad * sizeof(uint16_t);
}

size_t col_operand_bytes(int M, int64_t chunk_rows) {
  // the K extent runs from row_begin rounded down to 32 to row_end rounded
  // up to 16: at most chunk_rows + 47 rows, rounded up to 32
  const int64_t KB = (chunk_rows + 47 + 31) / 32 * 32;
  return (size_t)2 * (size_t)KB * (size_t)(2 * M) * sizeof(uint16_t);
}

size_t col_partial_bytes(int M, int64_t chunk_rows) {
  // a chunk gets at most `target` segments (seg_len >= rows / target), and at
  // most one per 256 of its K rows (seg_len >= 256; the K extent is the
  // chunk's rows rounded out to 16 at both ends)
  const ColSchedule c = col_schedule(M, 0, 0);
  const int64_t target = (512 + c.n_rt * c.n_ct - 1) / (c.n_rt * c.n_ct);
  const int64_t by_rows = (chunk_rows + 30 + 255) / 256;
  const int64_t nseg = target < by_rows ? target : by_rows;
  return (size_t)nseg * (size_t)M * (size_t)(2 * M) * sizeof(float);
}

namespace {

// ---------------------------------------------------------------------------
// 2-level phase plates: prefix sums of the row kernel along the aperture row.
// S[i][q] = sum_{i' < i} A(i', q), A(i, q) = e^{2 pi i (beta c_i^2/2 - alpha c_i d_q)}
// in float64 (the same turns as the operand table, unsplit), by blocks of
// kPrefixBlock rows: local running sums, an exclusive scan of the block totals
// per column, then the offsets added; a fixed order, so the table is the same
// on every build.
// ---------------------------------------------------------------------------
constexpr int kPrefixBlock = 2048;

__global__ __launch_bounds__(256) void k_prefix_local(InstDev d, double2 *__restrict__ S, double2 *__restrict__ tot) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t b = blockIdx.y;
  const int M = d.M;
  if (q >= M) return;
  const double dq = (double)q - 0.5 * (double)M + d.sx;
  const int64_t i0 = b * kPrefixBlock;
  const int64_t i1 = i0 + kPrefixBlock < d.N ? i0 + kPrefixBlock : d.N;
  double2 acc = make_double2(0.0, 0.0);
  for (int64_t i = i0; i < i1; ++i) {
    const double c = (double)i - 0.5 * (double)(d.N - 1);
    const double ph = 0.5 * d.beta * (c * c);
    const double lin = d.alpha * c * dq;
    acc = cadd(acc, cexp_turns((ph - rint(ph)) - (lin - rint(lin))));
    S[(i + 1) * M + q] = acc;
  }
  tot[b * M + q] = acc;
}

__global__ __launch_bounds__(256) void k_prefix_offsets(int M, int64_t nb, double2 *__restrict__ tot,
                                                        double2 *__restrict__ S) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= M) return;
  double2 off = make_double2(0.0, 0.0);
  for (int64_t b = 0; b < nb; ++b) {
    const double2 t = tot[b * M + q];
    tot[b * M + q] = off;
    off = cadd(off, t);
  }
  S[q] = make_double2(0.0, 0.0);
}

__global__ __launch_bounds__(256) void k_prefix_add(int M, int64_t N, const double2 *__restrict__ tot,
                                                    double2 *__restrict__ S) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;  // element (i, q) of rows 1 .. N
  if (e >= N * (int64_t)M) return;
  const int64_t i = e / M;
  const int q = (int)(e - i * M);
  S[(i + 1) * M + q] = cadd(S[(i + 1) * M + q], tot[(i / kPrefixBlock) * M + q]);
}

}  // namespace

bool two_level_fast(const InstDev &d) { return d.levels == 2 && d.n_creases == 0 && d.S != nullptr; }

bool four_level_fast(const InstDev &d) { return d.levels == 4 && d.n_creases == 0 && d.S != nullptr; }

size_t prefix_table_bytes(int M, int64_t Npad) {
  const int64_t nb = (Npad + kPrefixBlock - 1) / kPrefixBlock;
  return (size_t)(Npad + 1 + nb) * (size_t)M * sizeof(double2);
}

hipError_t launch_build_prefix_table(const InstDev &d, double2 *S, hipStream_t st) {
  const int M = d.M;
  const int64_t nb = (d.N + kPrefixBlock - 1) / kPrefixBlock;
  double2 *tot = S + (d.Npad + 1) * (int64_t)M;  // block totals, then offsets
  hipLaunchKernelGGL(k_prefix_local, dim3((unsigned)((M + 255) / 256), (unsigned)nb), dim3(256), 0, st, d, S, tot);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_prefix_offsets, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, st, M, nb, tot, S);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t n = d.N * (int64_t)M;
  hipLaunchKernelGGL(k_prefix_add, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, M, d.N, tot, S);
  return hipGetLastError();
}

hipError_t launch_build_col_table(const InstDev &d, uint16_t *By, hipStream_t st) {
  const int64_t rows_pad = (d.M + kCTR - 1) / kCTR * kCTR;
  const dim3 grid((unsigned)((d.Npad + 255) / 256), (unsigned)rows_pad);
  hipLaunchKernelGGL(k_build_col_table, grid, dim3(256), 0, st, d, rows_pad, By);
  return hipGetLastError();
}

hipError_t launch_col_pass_split(const InstDev &d, int64_t row_begin, int64_t row_end, const float2 *T, int nseg,
                                 int64_t seg_stride, uint16_t *Tb, float *C, double2 *roi, hipStream_t st,
                                 const float2 *T2) {
  if (row_end <= row_begin || nseg <= 0) return hipSuccess;
  const int M = d.M, M2 = 2 * M;
  const ColSchedule c = col_schedule(M, row_begin, row_end);
  // T -> BF16 hi/lo operand (the row-pass partial planes: column stride = chunk rows)
  const int64_t rs = seg_stride / M;
  // the int8 row pass: binary stripes (mode 1) or complex ones (mode 2)
  const bool binary = d.n_creases == 0 && (d.levels == 0 || two_level_fast(d) || four_level_fast(d));
  const int mode = !d.i8 ? 0 : binary ? 1 : 2;
  hipLaunchKernelGGL(mode == 2 ? k_col_operand<2> : mode == 1 ? k_col_operand<1> : k_col_operand<0>,
                     dim3((unsigned)(c.KB / 32), (unsigned)((M2 + 7) / 8)), dim3(256), 0, st, M2, row_begin,
                     row_end, (const float *)T, nseg, 2 * seg_stride, rs, c.kB0, c.KB, Tb,
                     two_level_fast(d) || four_level_fast(d) ? d.S : nullptr, d.N, d.kmax,
                     four_level_fast(d) ? (const float *)T2 : nullptr);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = init_split_attributes();
  if (e != hipSuccess) return e;
  const int64_t rows_pad = (M + kCTR - 1) / kCTR * kCTR;
  const int64_t Gn = (int64_t)c.n_rt * c.n_ct * c.n_seg;
  const int64_t grid = (Gn + 255) / 256 * 256;
  const int64_t segC = (int64_t)M * M2;  // floats per partial plane
  hipLaunchKernelGGL(k_row_pass_split_cplx<true>, dim3((unsigned)grid), dim3(kCThreads), kCLdsBytes, st, d,
                     (int64_t)0, (int64_t)M, c.n_rt, c.n_ct, 0, c.n_seg, d.By, rows_pad, (int64_t)0, d.Npad / 16, C,
                     segC, (const uint16_t *)Tb, c.kB0, c.KB, c.k_begin, c.k_end, c.seg_len);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_col_finish, dim3((unsigned)((M + 255) / 256), (unsigned)M), dim3(256), 0, st, d,
                     (const float *)C, c.n_seg, segC, roi);
  return hipGetLastError();
}

}  // namespace fzp
