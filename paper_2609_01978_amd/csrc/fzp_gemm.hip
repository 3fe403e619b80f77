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

// ---------------------------------------------------------------------------
// Zone-mask bits of a chunk of aperture rows: bits[r - row_begin][w], bit e of
// word w is the mask at column 32 w + e (zero outside the row's disc chord).
// K = c_i^2 + c_j^2 is exact in float64 and zone = floor(K kappa) is the same
// single float64 product the reference rule uses (Sec. 2.2, Eq. 4).  Each
// element is evaluated once here instead of once per GEMM column tile.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_mask_bits(InstDev d, int64_t row_begin, int64_t row_end, int W,
                                                   uint32_t *__restrict__ bits) {
  const int64_t N = d.N;
  const int Nm1 = (int)(N - 1);
  const double kappa = d.kappa;
  const uint32_t flip = d.centre_open ? 0xffffffffu : 0u;
  for (int64_t row = row_begin + blockIdx.x; row < row_end; row += gridDim.x) {
    const double cj = (double)(2 * row - N + 1);
    const double bj = cj * cj;
    int rlo = 0, rhi = 0;
    const double rem = d.kmax - bj;
    if (rem >= 0.0) {
      int m = (int)sqrt(rem);
      while ((double)(m + 1) * (double)(m + 1) <= rem) ++m;
      while (m > 0 && (double)m * (double)m > rem) --m;
      rlo = (Nm1 - m + 1) >> 1;
      rhi = ((Nm1 + m) >> 1) + 1;
    }
    uint32_t *out = bits + (row - row_begin) * (int64_t)W;
    for (int w = threadIdx.x; w < W; w += blockDim.x) {
      const int i0 = 32 * w;
      uint32_t v = 0;
      if (i0 < rhi && i0 + 32 > rlo) {
        double ci = (double)(2 * i0 - Nm1);
#pragma unroll
        for (int e = 0; e < 32; ++e) {
          const double K = fma(ci, ci, bj);
          const int zone = (int)(K * kappa);
          v |= ((uint32_t)zone & 1u) << e;
          ci += 2.0;
        }
        const int lo = min(max(rlo - i0, 0), 32), hi = min(max(rhi - i0, 0), 32);
        const uint32_t valid = (hi >= 32 ? 0xffffffffu : ((1u << hi) - 1u)) & ~((1u << lo) - 1u);
        v = (v ^ flip) & valid;
      }
      out[w] = v;
    }
  }
}

// ---------------------------------------------------------------------------
// Row-pass GEMM.  Work-group tile: kTR aperture rows x kTC real columns of T
// over one K segment (kSplitSegLen aperture columns, trimmed to the disc chord
// of the tile's rows).  8 waves in a 4 (rows) x 2 (columns) grid, each wave
// 128 rows x 64 columns = 4 x 2 MFMA 32x32 blocks, 128 float32 accumulators
// per lane.  The tall tile (512 rows) gives 512 flops per byte of operand
// slab, above the BF16-MFMA / HBM ridge even without cache reuse.  K advances in stages of kKT = 32 columns (two MFMA K-steps).
// Pipeline, one barrier per stage s; all global traffic is direct
// (register-free) global -> LDS copies, so no wave ever waits on a load it
// has just issued:
//   - the hi/lo operand slab of stage s+2 and the mask-bit words of stage s+3
//     are copied into LDS ring slots freed by the previous barrier,
//   - the MFMAs of stage s run on the LDS copies of stage s,
//   - the bits of stage s+1 (copied two stages earlier) are expanded to BF16
//     into the other mask buffer,
//   - the barrier waits only for the copies issued one stage earlier.
// Each K segment's partial sum is written in float32 and the column pass adds
// the segments in float64, which bounds the float32 accumulation length.
//
// LDS rows are 64 bytes (32 BF16); the four 16-byte chunks of row r sit in
// the order chunk ^ swz(r), which spreads both the MFMA operand reads (32
// consecutive rows, one chunk) and the row writes over all banks without
// padding: 2 mask buffers + 3 slab buffers + 3 bit-word slots = 118 KiB.
// ---------------------------------------------------------------------------
constexpr int kThreads = 512;
constexpr int kTR = 512;     // rows per tile
constexpr int kTC = 128;     // real columns per tile (64 complex ROI columns)
constexpr int kKT = 32;      // K columns per pipeline stage
constexpr int kRowB = 64;    // LDS bytes per row of a stage
constexpr int kMaskBytes = kTR * kRowB;            // 32768
constexpr int kBBytes = 2 * kTC * kRowB;           // 16384 (hi and lo planes)
constexpr int kBitsBytes = 8 * 64 * 4;           // one dword copy per lane of each wave
constexpr int kMaskBufs = 2, kBBufs = 3, kBitsBufs = 3;
constexpr int kLdsBytes = kMaskBufs * kMaskBytes + kBBufs * kBBytes + kBitsBufs * kBitsBytes;  // 120832

__device__ __forceinline__ int swz(int r) { return ((r >> 1) ^ (r >> 3)) & 3; }
__device__ __forceinline__ u32x4 lds_ld16(const char *p) { return *(const u32x4 *)p; }
__device__ __forceinline__ void lds_st16(char *p, u32x4 v) { *(u32x4 *)p = v; }

// Wait until at most 3 vector-memory operations are outstanding - every wave
// issues exactly 3 copies per stage, so this completes all copies issued
// before the current stage - and this wave's LDS writes are done, then the
// work-group barrier.  One asm statement, so that the compiler does not put
// a blanket wait for all outstanding copies in front of the barrier.
__device__ __forceinline__ void stage_barrier() {
  asm volatile("s_waitcnt vmcnt(3) lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

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

__global__ __launch_bounds__(kThreads, 1) void k_row_pass_split(InstDev d, int64_t row_begin, int64_t row_end,
                                                                int n_rt, int n_ct, int n_seg,
                                                                const uint32_t *__restrict__ bits, int W,
                                                                float *__restrict__ T, int64_t seg_stride_f) {
  extern __shared__ __attribute__((aligned(16))) char lds[];
  char *const mbuf = lds;                               // 2 x kMaskBytes
  char *const bbuf = lds + kMaskBufs * kMaskBytes;      // 3 x kBBytes
  char *const wbuf = bbuf + kBBufs * kBBytes;           // 3 x kBitsBytes
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  // XCD-aware tile order: work-groups are dealt to the 8 XCDs round robin, so
  // give each XCD a contiguous run of logical tiles (row tile fastest): the
  // tiles resident on one XCD share the operand slab in its L2.
  const int G = n_rt * n_ct * n_seg;
  const int per_xcd = (G + 7) / 8;
  const int g = (blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
  if (g >= G) return;
  const int rt = g % n_rt;
  const int ct = (g / n_rt) % n_ct;
  const int seg = g / (n_rt * n_ct);

  const int M2 = 2 * d.M;
  const int64_t r0 = row_begin + (int64_t)rt * kTR;
  int64_t rl = r0 + kTR - 1;
  if (rl > row_end - 1) rl = row_end - 1;
  const int c0 = ct * kTC;
  const int64_t s_lo = (int64_t)seg * kSplitSegLen;
  const int64_t s_hi = s_lo + kSplitSegLen < d.Npad ? s_lo + kSplitSegLen : d.Npad;
  int64_t k_lo, k_hi;
  tile_chord(d, r0, rl, k_lo, k_hi);
  k_lo = k_lo / kKT * kKT;
  k_hi = (k_hi + kKT - 1) / kKT * kKT;
  if (k_lo < s_lo) k_lo = s_lo;
  if (k_hi > s_hi) k_hi = s_hi;

  // ---- mask role: thread tid expands row tid (all 32 columns of each stage)
  const int gr = tid;
  const bool grow_ok = r0 + gr < row_end;
  // bit-word copy role: wave w copies the words of tile rows [64 w, 64 w + 64),
  // lane l's word landing at dword tid of the slot; rows past the chunk read
  // its last row and are zeroed on expansion
  const int64_t wrow = min(r0 + tid, row_end - 1) - row_begin;
  const uint32_t *wsrc = bits + wrow * (int64_t)W;
  const int wslot = tid * 4;
  const int gsw = swz(gr);
  // ---- slab-copy role: wave w copies slab rows [32 w, 32 w + 32) (2 direct loads
  // of 16 rows); lane L carries chunk L&3 of row 16 x + L/4 of its block, read
  // from global chunk (L&3) ^ swz(row) so the LDS image is the swizzled layout.
  // Columns past 2M read column 0 instead: they only feed accumulator columns
  // that are never stored.
  const uint16_t *bsrc[2];
#pragma unroll
  for (int x = 0; x < 2; ++x) {
    const int R = (wave * 2 + x) * 16 + (lane >> 2);
    const int plane = R / kTC, col = R % kTC;
    const int gc = c0 + col < M2 ? c0 + col : 0;
    const int chunk = (lane & 3) ^ swz(R);
    bsrc[x] = d.A + (int64_t)plane * M2 * d.Npad + (int64_t)gc * d.Npad + 8 * chunk;
  }

  // ---- compute role: wave (wr, wc) covers rows wr*128.., columns wc*64..
  const int wr = wave >> 1, wc = wave & 1;
  const int l32 = lane & 31, lhi = lane >> 5;
  const int lsw = swz(l32);
  // byte offsets of this lane's operand chunks for K-step ks (row & 31 == l32 everywhere)
  const int cks0 = ((0 + lhi) ^ lsw) << 4, cks1 = ((2 + lhi) ^ lsw) << 4;
  const int arow = (wr * 128 + l32) * kRowB;
  const int brow = (wc * 64 + l32) * kRowB;

  f32x16 acc[4][2];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[a][b][e] = 0.0f;

  if (k_lo < k_hi) {
    // The pipeline also copies up to three stages past the end: their slab
    // loads are clamped to the table's last slab and their mask is zero.
    const int kb = (int)k_lo;
    const int nst = (int)((k_hi - k_lo) / kKT);
    const int klast = (int)d.Npad - kKT;
    auto copy_slab = [&](int s) {
      const int k = min(kb + s * kKT, klast);
      char *dst = bbuf + (s % kBBufs) * kBBytes + wave * 2 * 1024;
#pragma unroll
      for (int x = 0; x < 2; ++x)
        __builtin_amdgcn_global_load_lds((const void *)(bsrc[x] + k),
                                         (__attribute__((address_space(3))) void *)(dst + x * 1024), 16, 0, 0);
    };
    auto copy_bits = [&](int s) {
      const int wi = min((kb + s * kKT) >> 5, W - 1);
      __builtin_amdgcn_global_load_lds((const void *)(wsrc + wi),
                                       (__attribute__((address_space(3))) void *)(wbuf + (s % kBitsBufs) * kBitsBytes +
                                                                                  wave * 256),
                                       4, 0, 0);
    };
    // expand the 32 bits of row gr of stage s to packed BF16 (four 16-byte chunks)
    auto store_mask = [&](int s) {
      const uint32_t word = *(const uint32_t *)(wbuf + (s % kBitsBufs) * kBitsBytes + wslot);
      const uint32_t b32 = (grow_ok && s < nst) ? word : 0u;
      char *st = mbuf + (s & 1) * kMaskBytes + gr * kRowB;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        uint32_t w[4];
#pragma unroll
        for (int p2 = 0; p2 < 4; ++p2) {
          const uint32_t t2 = b32 >> (8 * c + 2 * p2);
          w[p2] = (t2 & 1u) * 0x3f80u + (t2 & 2u) * 0x1fc00000u;
        }
        lds_st16(st + ((c ^ gsw) << 4), u32x4{w[0], w[1], w[2], w[3]});
      }
    };
    struct Frag {
      bf16x8 a[4], h[2], l[2];
    };
    auto read_frag = [&](int s, int cofs, Frag &f) {
      const char *ma = mbuf + (s & 1) * kMaskBytes + arow + cofs;
      const char *mb = bbuf + (s % kBBufs) * kBBytes + brow + cofs;
#pragma unroll
      for (int rb = 0; rb < 4; ++rb) f.a[rb] = __builtin_bit_cast(bf16x8, lds_ld16(ma + rb * 32 * kRowB));
#pragma unroll
      for (int cb = 0; cb < 2; ++cb) {
        f.h[cb] = __builtin_bit_cast(bf16x8, lds_ld16(mb + cb * 32 * kRowB));
        f.l[cb] = __builtin_bit_cast(bf16x8, lds_ld16(mb + (kTC + cb * 32) * kRowB));
      }
    };
    // 16 MFMAs of one K-step: 8 independent accumulators per operand plane
    auto mma = [&](const Frag &f) {
#pragma unroll
      for (int rb = 0; rb < 4; ++rb)
#pragma unroll
        for (int cb = 0; cb < 2; ++cb)
          acc[rb][cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(f.a[rb], f.h[cb], acc[rb][cb], 0, 0, 0);
#pragma unroll
      for (int rb = 0; rb < 4; ++rb)
#pragma unroll
        for (int cb = 0; cb < 2; ++cb)
          acc[rb][cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(f.a[rb], f.l[cb], acc[rb][cb], 0, 0, 0);
    };
    // prologue: slabs 0, 1 and bit words 0..2 copied; stage 0's mask expanded
    copy_slab(0);
    copy_slab(1);
    copy_bits(0);
    copy_bits(1);
    copy_bits(2);
    asm volatile("s_waitcnt vmcnt(0)\n\ts_barrier" ::: "memory");
    store_mask(0);
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
    for (int s = 0; s < nst; ++s) {
      copy_slab(s + 2);
      copy_bits(s + 3);
      Frag f0, f1;
      read_frag(s, cks0, f0);
      read_frag(s, cks1, f1);
      mma(f0);
      mma(f1);
      store_mask(s + 1);
      stage_barrier();
    }
    // drain the copies still in flight before the work-group retires its LDS
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  }
  // epilogue: register v of lane l holds row 8(v/4) + 4(l/32) + (v%4), column l%32
  float *Ts = T + (int64_t)seg * seg_stride_f;
#pragma unroll
  for (int rb = 0; rb < 4; ++rb)
#pragma unroll
    for (int cb = 0; cb < 2; ++cb) {
      const int c = c0 + wc * 64 + cb * 32 + l32;
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int64_t r = r0 + wr * 128 + rb * 32 + 8 * (v >> 2) + 4 * lhi + (v & 3);
        if (r < row_end && c < M2) Ts[(r - row_begin) * (int64_t)M2 + c] = acc[rb][cb][v];
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

int split_segments(const InstDev &d) { return (int)((d.Npad + kSplitSegLen - 1) / kSplitSegLen); }

size_t split_bits_bytes(const InstDev &d, int64_t chunk_rows) { return (size_t)chunk_rows * (size_t)(d.Npad / 32) * 4; }

hipError_t launch_row_pass_split(const InstDev &d, int32_t S, int64_t row_begin, int64_t row_end, float2 *T,
                                 int64_t seg_stride, uint32_t *bits, hipStream_t st) {
  (void)S;
  const int64_t rows = row_end - row_begin;
  if (rows <= 0) return hipSuccess;
  const int W = (int)(d.Npad / 32);
  {
    const int64_t grid = rows < 65536 ? rows : 65536;
    hipLaunchKernelGGL(k_mask_bits, dim3((unsigned)grid), dim3(256), 0, st, d, row_begin, row_end, W, bits);
  }
  const int n_rt = (int)((rows + kTR - 1) / kTR);
  const int n_ct = (2 * d.M + kTC - 1) / kTC;
  const int n_seg = split_segments(d);
  const int64_t G = (int64_t)n_rt * n_ct * n_seg;
  const int64_t grid = (G + 7) / 8 * 8;
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e =
        hipFuncSetAttribute((const void *)k_row_pass_split, hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBytes);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  hipLaunchKernelGGL(k_row_pass_split, dim3((unsigned)grid), dim3(kThreads), kLdsBytes, st, d, row_begin, row_end,
                     n_rt, n_ct, n_seg, (const uint32_t *)bits, W, (float *)T, 2 * seg_stride);
  return hipGetLastError();
}

}  // namespace fzp
