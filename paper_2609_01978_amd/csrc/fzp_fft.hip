// Float64 blocked-Bluestein chirp-z passes (Sec. 2.6, Eqs. 9-10), the stripe
// generator of the binary zone plate (Sec. 2.2, Eq. 4), the output factor of
// Eq. 2 and the device tables they use.
//
// One 1-D pass evaluates, for a line of samples g[i] on [i_start, i_end),
//   Y[q] = sum_i g[i] exp(2 pi i (beta c_i^2 / 2 - alpha c_i d_q)),
//   c_i = i - (N-1)/2,  d_q = q - M/2 + s,
// which is the Fresnel kernel of Eq. 2 along one axis in units of turns
// (beta = dx^2/(lambda z), alpha = dx dx_out/(lambda z)).  The line is cut into
// blocks of B = L - M + 1 samples; for a block starting at i0 (c0 = c_{i0},
// i = i0 + n) Bluestein's identity n d = (n^2 + d^2 - (d - n)^2)/2 gives
//   Y_block[q] = e^{2 pi i (beta c0^2/2 - alpha c0 d_q)} e^{-i pi alpha d_q^2}
//                sum_n u[n] h[q - n],
//   u[n] = g[i0 + n] e^{2 pi i beta c0 n} e^{i pi (beta - alpha) n^2},
//   h[k] = e^{i pi alpha (k - M/2 + s)^2},
// a linear convolution of length B + M - 1 = L taken by one forward FFT, a
// product with the precomputed spectrum H = FFT(h)/L and one inverse FFT, all
// inside LDS (L = 4096 float64 complex = 64 KiB).  The paper's engine instead
// pads each whole row to 2^nextpow2(N + M - 1) (Fig. 18 stage 2); blocking
// keeps every transform on chip whatever N is.
//
// The row pass generates g from the zone mask (times the crease phase screen
// and nothing else: the x chirp is part of the kernel above) and writes
// T[j][q]; the column pass runs the same operator down each ROI column of T,
// applies the Eq. 2 output factor and adds into the float64 ROI.

#include "fzp_device.h"
#include "fzp_internal.h"

namespace fzp {

namespace {


__device__ __forceinline__ double frac_turns(double t) { return t - rint(t); }

// Chord of aperture row j inside the disc K <= kmax: columns [i_start, i_end).
__device__ __forceinline__ void row_chord(int64_t N, double kmax, double bj, int64_t &i_start,
                                          int64_t &i_end) {
  const double rem = kmax - bj;
  if (rem < 0.0) {
    i_start = i_end = 0;
    return;
  }
  int64_t m = (int64_t)sqrt(rem);
  while ((double)(m + 1) * (double)(m + 1) <= rem) ++m;
  while (m > 0 && (double)m * (double)m > rem) --m;
  // |2i - N + 1| <= m  <=>  (N-1-m)/2 <= i <= (N-1+m)/2
  const int64_t lo2 = N - 1 - m, hi2 = N - 1 + m;
  int64_t a = lo2 >= 0 ? (lo2 + 1) / 2 : -((-lo2) / 2);
  int64_t b = hi2 >= 0 ? hi2 / 2 : -((-hi2 + 1) / 2);
  if (a < 0) a = 0;
  if (b > N - 1) b = N - 1;
  i_start = a;
  i_end = b + 1 > a ? b + 1 : a;
}

__global__ void k_zero(double *buf, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    buf[i] = 0.0;
}

// Block 0: Hx, block 1: Hy (h transformed by the same LDS FFT), block 2: Dt, Qx, Qy.
__global__ __launch_bounds__(kFftThreads) void k_build_tables(InstDev d, double2 *Hx, double2 *Hy,
                                                               double2 *Dt, double2 *Qx, double2 *Qy) {
  __shared__ double2 s_lds[kLdsN];
  const int t = threadIdx.x;
  const int M = d.M;
  const Tw tw = fft_twiddles();
  if (blockIdx.x < 2) {
    const double s = blockIdx.x == 0 ? d.sx : d.sy;
    double2 v[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int k = t + 256 * r;
      const int kk = k < M ? k : k - kFftLen;  // circular layout of k = -(B-1) .. M-1
      const double e = (double)kk - 0.5 * (double)M + s;
      v[r] = cexp_turns(0.5 * d.alpha * e * e);
    }
    fft4096<-1>(v, s_lds, tw);
    double2 *H = blockIdx.x == 0 ? Hx : Hy;
#pragma unroll
    for (int r = 0; r < 16; ++r) H[t + 256 * r] = cscale(v[r], 1.0 / (double)kFftLen);
  } else {
    const double ba = 0.5 * (d.beta - d.alpha);
    for (int n = t; n < kFftLen; n += blockDim.x) {
      const double nn = (double)n;
      Dt[n] = cexp_turns(ba * nn * nn);
    }
    for (int q = t; q < M; q += blockDim.x) {
      const double ex = (double)q - 0.5 * (double)M + d.sx;
      const double ey = (double)q - 0.5 * (double)M + d.sy;
      Qx[q] = cexp_turns(-0.5 * d.alpha * ex * ex);
      Qy[q] = cexp_turns(-0.5 * d.alpha * ey * ey);
    }
  }
}

// Opaque zero: keeps the compiler from hoisting table loads out of the block
// loop (hoisted, the 4096-entry spectrum would pin 64 registers per lane).
__device__ __forceinline__ int opaque_zero() {
  int z;
  asm volatile("s_mov_b32 %0, 0" : "=s"(z));
  return z;
}

// A loader either returns one sample, load(i), or, when it declares kBlock,
// fills a whole block at once: load.block(i0, cnt, v) sets v[r] = g[i0 + n]
// for n = threadIdx.x + 256 r < cnt and 0 otherwise (all of a block's loads can
// then be in flight together).
template <typename L, typename = void>
struct IsBlockLoader : std::false_type {};
template <typename L>
struct IsBlockLoader<L, std::void_t<decltype(L::kBlock)>> : std::true_type {};

// Blocked Bluestein over one line, shared by the row and column passes.
// load(i) returns g[i] (only called for i in [i_start, i_end)).
// The input chirp of block sample n = t + 256 r,
//   e^{2 pi i (lin n + gam n^2)},  lin = beta c0,  gam = (beta - alpha)/2,
// is advanced over r by a second-order phasor recurrence (16 steps), so no
// table is needed for it.
template <int NQ, typename Load>
__device__ __forceinline__ void bluestein_line(const InstDev &d, const double2 *__restrict__ H, double s_out,
                                               int64_t i_start, int64_t i_end, double2 *s_lds, const Tw &tw,
                                               double2 acc[NQ], Load load) {
  const int t = threadIdx.x;
  const int M = d.M, B = d.B;
  const double halfN = 0.5 * (double)(d.N - 1);
  const double gam = 0.5 * (d.beta - d.alpha);
  const double tt = (double)t;
  // e^{2 pi i gam (t^2 + 2 256 t r + 256^2 r^2)}: the parts that do not depend on the block
  const double g0 = frac_turns(gam * tt * tt);
  const double g1 = frac_turns(gam * 512.0 * tt + gam * 65536.0);
  const double2 dd = cexp_turns(frac_turns(gam * 131072.0));  // second difference
#pragma unroll
  for (int r = 0; r < NQ; ++r) acc[r] = make_double2(0.0, 0.0);
  for (int64_t i0 = i_start; i0 < i_end; i0 += B) {
    const double c0 = (double)i0 - halfN;
    const double lin = frac_turns(d.beta * c0);  // turns per sample
    double2 ph = cexp_turns(frac_turns(lin * tt) + g0);
    double2 dl = cexp_turns(frac_turns(lin * 256.0) + g1);
    double2 v[16];
    if constexpr (IsBlockLoader<Load>::value) {
      load.block(i0, i_end - i0 < (int64_t)B ? i_end - i0 : (int64_t)B, v);
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        v[r] = cmul(v[r], ph);
        ph = cmul(ph, dl);
        dl = cmul(dl, dd);
      }
    } else {
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int n = t + 256 * r;
        const int64_t i = i0 + n;
        double2 g = make_double2(0.0, 0.0);
        if (n < B && i < i_end) g = load(i);
        v[r] = cmul(g, ph);
        ph = cmul(ph, dl);
        dl = cmul(dl, dd);
      }
    }
    fft4096<-1>(v, s_lds, tw);
    const double2 *__restrict__ Hb = H + opaque_zero();
#pragma unroll
    for (int r = 0; r < 16; ++r) v[r] = cmul(v[r], Hb[t + 256 * r]);
    fft4096<+1>(v, s_lds, tw);
    const double p0 = frac_turns(0.5 * d.beta * (c0 * c0));
    const double ac0 = d.alpha * c0;
#pragma unroll
    for (int r = 0; r < NQ; ++r) {
      const int q = t + 256 * r;
      if (q < M) {
        const double dq = (double)q - 0.5 * (double)M + s_out;
        acc[r] = cadd(acc[r], cmul(v[r], cexp_turns(p0 - frac_turns(ac0 * dq))));
      }
    }
  }
}

// Row-pass input of a deformed plate for a whole block: the zone mask times
// the crease phase screen exp(2 pi i sum_k (H_k/lambda) exp(-d_k^2/(2 sigma_k^2))),
// d_k = x cos(theta_k) + y sin(theta_k) - rho_k, along one aperture row.  The
// thread's samples n = t + 256 r lie 256 samples apart, so along r each
// ridge's distance grows by D = 256 dx cos(theta) and its Gaussian
// g = exp(-a d^2) follows g(r+1) = g(r) R(r), R(r+1) = R(r) Q with
// R(0) = exp(-a (2 d0 D + D^2)), Q = exp(-2 a D^2): three exponentials per
// ridge per block instead of sixteen, in float64.  A ridge whose term stays
// below 2^-52 turns at the nearest of the thread's samples is skipped.
struct CreasedRow {
  static constexpr bool kBlock = true;
  const InstDev *d;
  double bj, y;
  __device__ __forceinline__ void block(int64_t i0, int64_t cnt, double2 v[16]) const {
    const int t = threadIdx.x;
    const int64_t N = d->N;
    const double c0 = (double)(2 * (i0 + t) - N + 1);
    const double x0 = 0.5 * c0 * d->dx;
    bool open[16];
    double turns[16];
    if (d->levels != 0 && d->n_creases == 0) {
      // L-level phase plate without creases: the level's phasor from the table
      const int L = d->levels;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const double ci = c0 + 512.0 * r;
        const double K = ci * ci + bj;  // exact integer
        const int lv = (int)(K * d->kappa_l) % L;
        v[r] = t + 256 * r < cnt ? d->lev[lv] : make_double2(0.0, 0.0);
      }
      return;
    }
    if (d->levels != 0) {
      // L-level phase plate: every disc sample passes, with the lens phase
      // quantised to level l = floor(K kappa_L) mod L, -l/L turns
      const int L = d->levels;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const double ci = c0 + 512.0 * r;
        const double K = ci * ci + bj;  // exact integer
        const int lv = (int)(K * d->kappa_l) % L;
        open[r] = t + 256 * r < cnt;
        turns[r] = -(double)lv / (double)L;
      }
    } else {
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const double ci = c0 + 512.0 * r;
        const double K = ci * ci + bj;  // exact integer
        const int zone = (int)(K * d->kappa);
        open[r] = t + 256 * r < cnt && ((zone & 1) ^ d->centre_open) != 0;
        turns[r] = 0.0;
      }
    }
    for (int k = 0; k < d->n_creases; ++k) {
      const CreaseDev &cr = d->cr[k];
      const double a = cr.inv2s2, h = cr.h_over_lambda;
      const double d0 = fma(x0, cr.c, fma(y, cr.s, -cr.rho));
      const double D = 256.0 * d->dx * cr.c;
      const double d15 = fma(15.0, D, d0);
      const double dmin = (d0 > 0.0) == (d15 > 0.0) ? fmin(fabs(d0), fabs(d15)) : 0.0;
      if (a * dmin * dmin > log(fabs(h)) + 36.0436533891) continue;  // ln 2^52
      double g = exp(-a * d0 * d0);
      double R = exp(-a * (2.0 * d0 * D + D * D));
      const double Q = exp(-2.0 * a * D * D);
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        turns[r] = fma(h, g, turns[r]);
        g *= R;
        R *= Q;
      }
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) v[r] = open[r] ? cexp_turns(turns[r]) : make_double2(0.0, 0.0);
  }
};

// Row pass: one work-group per aperture row (grid-stride), T[row - row_begin][q].
template <int NQ, bool DEFORM>
__global__ __launch_bounds__(kFftThreads, 2) void k_row_pass_fp64(InstDev d, int64_t row_begin, int64_t row_end,
                                                                  double2 *__restrict__ T) {
  __shared__ double2 s_lds[kLdsN];
  const int t = threadIdx.x;
  const Tw tw = fft_twiddles();
  const int64_t N = d.N;
  const int M = d.M;
  for (int64_t row = row_begin + blockIdx.x; row < row_end; row += gridDim.x) {
    const double cj = (double)(2 * row - N + 1);
    const double bj = cj * cj;
    int64_t i_start, i_end;
    row_chord(N, d.kmax, bj, i_start, i_end);
    const double y = 0.5 * cj * d.dx;
    double2 acc[NQ];
    if constexpr (DEFORM) {
      bluestein_line<NQ>(d, d.Hx, d.sx, i_start, i_end, s_lds, tw, acc, CreasedRow{&d, bj, y});
    } else {
      bluestein_line<NQ>(d, d.Hx, d.sx, i_start, i_end, s_lds, tw, acc, [&](int64_t i) -> double2 {
        const double ci = (double)(2 * i - N + 1);
        const double K = ci * ci + bj;  // exact integer
        const int zone = (int)(K * d.kappa);
        const bool open = ((zone & 1) ^ d.centre_open) != 0;
        return make_double2(open ? 1.0 : 0.0, 0.0);
      });
    }
    double2 *Trow = T + (row - row_begin) * (int64_t)M;
#pragma unroll
    for (int r = 0; r < NQ; ++r) {
      const int q = t + 256 * r;
      if (r * 256 < M && q < M) Trow[q] = cmul(acc[r], d.Qx[q]);
    }
  }
}

// Column pass of the FP64 path: one work-group per ROI column q (grid-stride)
// over the chunk's T[j][q] (complex float64, row-major).  Adds
// F[p,q] Qy[p] sum_blocks(...) into roi[p][q]; each ROI element is owned by one
// work-group, so the float64 sum over chunks is a fixed-order sequence.
template <int NQ>
__global__ __launch_bounds__(kFftThreads, 2) void k_col_pass(InstDev d, int64_t row_begin, int64_t row_end,
                                                             const double2 *__restrict__ T,
                                                             double2 *__restrict__ roi) {
  __shared__ double2 s_lds[kLdsN];
  const int t = threadIdx.x;
  const Tw tw = fft_twiddles();
  const int M = d.M;
  // Work-groups are dealt to the 8 XCDs round robin; with one work-group per
  // column, XCD x takes the contiguous columns [x M/8, (x+1) M/8), so the
  // work-groups sharing an XCD's L2 read adjacent elements of each T row.
  int q0 = blockIdx.x;
  if (gridDim.x == (unsigned)M && (M & 7) == 0) q0 = (q0 & 7) * (M >> 3) + (q0 >> 3);
  for (int q = q0; q < M; q += gridDim.x) {
    double2 acc[NQ];
    bluestein_line<NQ>(d, d.Hy, d.sy, row_begin, row_end, s_lds, tw, acc,
                       [&](int64_t j) -> double2 { return T[(j - row_begin) * (int64_t)M + q]; });
    const double xq = d.x0 + ((double)q - 0.5 * (double)M) * d.dx_out;
#pragma unroll
    for (int r = 0; r < NQ; ++r) {
      const int p = t + 256 * r;
      if (r * 256 < M && p < M) {
        const double yp = d.y0 + ((double)p - 0.5 * (double)M) * d.dx_out;
        const double2 F = cscale(cexp_turns(d.kz_turns + (xq * xq + yp * yp) * d.inv2lz), d.scale);
        const double2 val = cmul(F, cmul(acc[r], d.Qy[p]));
        double2 *o = roi + (int64_t)p * M + q;
        *o = cadd(*o, val);
      }
    }
  }
}

// Row pass over stored rows (the CZT zoom of the non-paraxial variant): row
// `row` of a field of d.N x d.N samples (its chirp is part of the kernel), all
// d.N samples, into T[row - row_begin][q].
struct StoredRow {
  static constexpr bool kBlock = true;
  const double2 *row;
  __device__ __forceinline__ void block(int64_t i0, int64_t cnt, double2 v[16]) const {
    const int t = threadIdx.x;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int64_t n = t + 256 * r;
      v[r] = n < cnt ? row[i0 + n] : make_double2(0.0, 0.0);
    }
  }
};

template <int NQ>
__global__ __launch_bounds__(kFftThreads, 2) void k_row_pass_stored(InstDev d, const double2 *__restrict__ U,
                                                                    int64_t row_begin, int64_t row_end,
                                                                    double2 *__restrict__ T) {
  __shared__ double2 s_lds[kLdsN];
  const int t = threadIdx.x;
  const Tw tw = fft_twiddles();
  const int M = d.M;
  for (int64_t row = row_begin + blockIdx.x; row < row_end; row += gridDim.x) {
    double2 acc[NQ];
    bluestein_line<NQ>(d, d.Hx, d.sx, 0, d.N, s_lds, tw, acc, StoredRow{U + row * d.N});
    double2 *Trow = T + (row - row_begin) * (int64_t)M;
#pragma unroll
    for (int r = 0; r < NQ; ++r) {
      const int q = t + 256 * r;
      if (r * 256 < M && q < M) Trow[q] = cmul(acc[r], d.Qx[q]);
    }
  }
}

int grid_for(int64_t work, int per_cu) {
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0) cus = v;
  }
  const int64_t cap = (int64_t)cus * per_cu * 64;
  return (int)(work < cap ? (work > 0 ? work : 1) : cap);
}

}  // namespace

hipError_t launch_zero(double *buf, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_zero, dim3((unsigned)blocks), dim3(256), 0, st, buf, n);
  return hipGetLastError();
}

hipError_t launch_build_tables(const Plan &p, const InstHost &ih, char *ws, hipStream_t st) {
  (void)p;
  hipLaunchKernelGGL(k_build_tables, dim3(3), dim3(kFftThreads), 0, st, ih.dev, (double2 *)(ws + ih.off_Hx),
                     (double2 *)(ws + ih.off_Hy), (double2 *)(ws + ih.off_Dt), (double2 *)(ws + ih.off_Qx),
                     (double2 *)(ws + ih.off_Qy));
  return hipGetLastError();
}

hipError_t launch_row_pass_fp64(const InstDev &d, int64_t row_begin, int64_t row_end, double2 *T, hipStream_t st) {
  const int64_t rows = row_end - row_begin;
  if (rows <= 0) return hipSuccess;
  const int grid = grid_for(rows, 2);
  const bool def = d.n_creases > 0 || d.levels != 0;  // complex aperture samples
#define FZP_ROW(NQ)                                                                                          \
  if (def)                                                                                                   \
    hipLaunchKernelGGL((k_row_pass_fp64<NQ, true>), dim3(grid), dim3(kFftThreads), 0, st, d, row_begin, row_end, T); \
  else                                                                                                       \
    hipLaunchKernelGGL((k_row_pass_fp64<NQ, false>), dim3(grid), dim3(kFftThreads), 0, st, d, row_begin, row_end, T);
  if (d.M <= 256) {
    FZP_ROW(1)
  } else if (d.M <= 512) {
    FZP_ROW(2)
  } else if (d.M <= 1024) {
    FZP_ROW(4)
  } else {
    FZP_ROW(8)
  }
#undef FZP_ROW
  return hipGetLastError();
}

hipError_t launch_row_pass_stored(const InstDev &d, const double2 *U, int64_t row_begin, int64_t row_end,
                                  double2 *T, hipStream_t st) {
  const int64_t rows = row_end - row_begin;
  if (rows <= 0) return hipSuccess;
  const int grid = grid_for(rows, 2);
#define FZP_ROWS(NQ) \
  hipLaunchKernelGGL((k_row_pass_stored<NQ>), dim3(grid), dim3(kFftThreads), 0, st, d, U, row_begin, row_end, T);
  if (d.M <= 256) {
    FZP_ROWS(1)
  } else if (d.M <= 512) {
    FZP_ROWS(2)
  } else if (d.M <= 1024) {
    FZP_ROWS(4)
  } else {
    FZP_ROWS(8)
  }
#undef FZP_ROWS
  return hipGetLastError();
}

hipError_t launch_col_pass(const InstDev &d, int64_t row_begin, int64_t row_end, const double2 *T, double2 *roi,
                           hipStream_t st) {
  if (row_end <= row_begin) return hipSuccess;
  const int grid = d.M;
#define FZP_COL(NQ) \
  hipLaunchKernelGGL((k_col_pass<NQ>), dim3(grid), dim3(kFftThreads), 0, st, d, row_begin, row_end, T, roi);
  if (d.M <= 256) {
    FZP_COL(1)
  } else if (d.M <= 512) {
    FZP_COL(2)
  } else if (d.M <= 1024) {
    FZP_COL(4)
  } else {
    FZP_COL(8)
  }
#undef FZP_COL
  return hipGetLastError();
}

}  // namespace fzp
