// Focal-spot metrics on the device (shared metric extractor: Sec. 3.3 stage 4,
// Fig. 18 stage 5): intensity, brightest sample, main-lobe power (DE), FWHM
// from a not-a-knot cubic spline through the row and column of the brightest
// sample, and the MTF at half the cutoff from |FFT2(I)|.  All reductions run in
// a fixed order (no atomics), so the results are reproducible.

#include <cmath>
#include <string>

#include "fzp_device.h"
#include "fzp_internal.h"

namespace fzp {

namespace {

constexpr int kPartWG = 256;     // work-groups of the first reduction stage
constexpr int kRedThreads = 256;
constexpr int kSplineMax = 4096;

struct Part {
  double vmax;
  int64_t imax;
  double lobe;
  double pad;
};

// Scratch layout (bytes from the scratch base).
__host__ __device__ inline size_t sc_I(int) { return 0; }
__host__ __device__ inline size_t sc_F(int M) { return (size_t)M * M * sizeof(double); }
__host__ __device__ inline size_t sc_part(int M) { return sc_F(M) + (size_t)M * M * sizeof(double2); }
__host__ __device__ inline size_t sc_res(int M) { return sc_part(M) + kPartWG * sizeof(Part); }
__host__ __device__ inline size_t sc_end(int M) { return sc_res(M) + 16 * sizeof(double); }

__device__ __forceinline__ bool better(double v, int64_t i, double bv, int64_t bi) {
  return v > bv || (v == bv && i < bi);
}

// Stage 1: I = |U|^2, per-work-group max (first index on ties) and lobe sum.
__global__ __launch_bounds__(kRedThreads) void k_intensity(InstDev d, const double2 *__restrict__ roi,
                                                           double *__restrict__ I, Part *parts, double rnull2) {
  const int M = d.M;
  const int64_t n = (int64_t)M * M;
  const int64_t per = (n + gridDim.x - 1) / gridDim.x;
  const int64_t b = blockIdx.x * per;
  const int64_t e = b + per < n ? b + per : n;
  double vmax = -1.0, lobe = 0.0;
  int64_t imax = INT64_MAX;
  for (int64_t k = b + threadIdx.x; k < e; k += blockDim.x) {
    const double2 u = roi[k];
    const double v = u.x * u.x + u.y * u.y;
    I[k] = v;
    if (better(v, k, vmax, imax)) {
      vmax = v;
      imax = k;
    }
    const int p = (int)(k / M), q = (int)(k % M);
    const double rx = ((double)q - 0.5 * (double)M) * d.dx_out;
    const double ry = ((double)p - 0.5 * (double)M) * d.dx_out;
    if (rx * rx + ry * ry <= rnull2) lobe += v;
  }
  __shared__ double s_v[kRedThreads], s_l[kRedThreads];
  __shared__ int64_t s_i[kRedThreads];
  s_v[threadIdx.x] = vmax;
  s_i[threadIdx.x] = imax;
  s_l[threadIdx.x] = lobe;
  __syncthreads();
  for (int w = kRedThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      const int o = threadIdx.x + w;
      if (better(s_v[o], s_i[o], s_v[threadIdx.x], s_i[threadIdx.x])) {
        s_v[threadIdx.x] = s_v[o];
        s_i[threadIdx.x] = s_i[o];
      }
      s_l[threadIdx.x] += s_l[o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) parts[blockIdx.x] = Part{s_v[0], s_i[0], s_l[0], 0.0};
}

// Not-a-knot cubic spline (unit spacing) second derivatives m[0..n-1] of y.
// Interior equations m[i-1] + 4 m[i] + m[i+1] = 6 (y[i-1] - 2 y[i] + y[i+1]);
// the not-a-knot conditions m[0] = 2 m[1] - m[2], m[n-1] = 2 m[n-2] - m[n-3]
// turn the first and last of them into 6 m[1] = r[1], 6 m[n-2] = r[n-2].
__device__ void spline_m(const double *y, int64_t stride, int n, double *m, double *cp) {
  auto Y = [&](int i) { return y[(int64_t)i * stride]; };
  auto R = [&](int i) { return 6.0 * (Y(i - 1) - 2.0 * Y(i) + Y(i + 1)); };
  m[1] = R(1) / 6.0;
  m[n - 2] = R(n - 2) / 6.0;
  if (n >= 5) {
    const int a = 2, b = n - 3;  // unknowns m[a..b]
    // Thomas algorithm, sub/super diagonal 1, diagonal 4
    double dprev = 0.0, cprev = 0.0;
    for (int i = a; i <= b; ++i) {
      double rhs = R(i);
      if (i == a) rhs -= m[1];
      if (i == b) rhs -= m[n - 2];
      const double den = 4.0 - (i == a ? 0.0 : cprev);
      const double c = 1.0 / den;
      const double dd = (rhs - (i == a ? 0.0 : dprev)) * c;
      cp[i] = c;
      m[i] = dd;
      cprev = c;
      dprev = dd;
    }
    for (int i = b - 1; i >= a; --i) m[i] = m[i] - cp[i] * m[i + 1];
  }
  m[0] = 2.0 * m[1] - m[2];
  m[n - 1] = 2.0 * m[n - 2] - m[n - 3];
}

struct Cubic {
  double a, b, c, d;  // a t^3 + b t^2 + c t + d on [i, i+1]
};

__device__ Cubic piece(const double *y, int64_t stride, const double *m, int i) {
  const double yi = y[(int64_t)i * stride], yj = y[(int64_t)(i + 1) * stride];
  return Cubic{(m[i + 1] - m[i]) / 6.0, 0.5 * m[i], (yj - yi) - (2.0 * m[i] + m[i + 1]) / 6.0, yi};
}

__device__ __forceinline__ double ev(const Cubic &c, double t) { return ((c.a * t + c.b) * t + c.c) * t + c.d; }

// FWHM in samples of the profile y[0..n-1] (stride), or NaN; with `frac` the
// full width at that fraction of the spline peak instead of one half.
__device__ double fwhm_profile(const double *y, int64_t stride, int n, double *m, double *cp, double frac = 0.5) {
  int k = 0;
  double best = y[0];
  for (int i = 1; i < n; ++i) {
    const double v = y[(int64_t)i * stride];
    if (v > best) {
      best = v;
      k = i;
    }
  }
  if (k == 0 || k == n - 1 || n < 5) return NAN;
  spline_m(y, stride, n, m, cp);
  double peak = best;
  for (int lo = k - 1; lo <= k; ++lo) {
    const Cubic c = piece(y, stride, m, lo);
    // roots of 3a t^2 + 2b t + c on [0, 1]
    const double A = 3.0 * c.a, Bq = 2.0 * c.b, C = c.c;
    double roots[2];
    int nr = 0;
    if (A != 0.0) {
      const double disc = Bq * Bq - 4.0 * A * C;
      if (disc >= 0.0) {
        const double sq = sqrt(disc);
        const double qq = -0.5 * (Bq + (Bq >= 0.0 ? sq : -sq));
        if (qq != 0.0) {
          roots[nr++] = qq / A;
          roots[nr++] = C / qq;
        } else {
          roots[nr++] = 0.0;
        }
      }
    } else if (Bq != 0.0) {
      roots[nr++] = -C / Bq;
    }
    for (int r = 0; r < nr; ++r)
      if (roots[r] >= 0.0 && roots[r] <= 1.0) {
        const double v = ev(c, roots[r]);
        if (v > peak) peak = v;
      }
  }
  const double half = frac * peak;
  int left = k, right = k;
  while (left >= 0 && y[(int64_t)left * stride] >= half) --left;
  while (right < n && y[(int64_t)right * stride] >= half) ++right;
  if (left < 0 || right >= n) return NAN;
  auto bisect = [&](int i, bool rising) {
    const Cubic c = piece(y, stride, m, i);
    double lo = (double)i, hi = (double)(i + 1);
    for (int it = 0; it < 200; ++it) {
      const double mid = 0.5 * (lo + hi);
      if (mid == lo || mid == hi) break;
      const bool above = ev(c, mid - (double)i) >= half;
      if (above == rising)
        hi = mid;
      else
        lo = mid;
    }
    return 0.5 * (lo + hi);
  };
  const double xl = bisect(left, true);
  const double xr = bisect(right - 1, false);
  return xr - xl;
}

// Stage 2: combine partials; FWHM along the row (x) and column (y) of the
// brightest sample; write max, lobe power and FWHM to res[].
__global__ __launch_bounds__(64) void k_reduce_fwhm(InstDev d, const double *__restrict__ I, const Part *parts,
                                                    int nparts, double *res) {
  __shared__ double s_m[kSplineMax], s_c[kSplineMax];
  __shared__ int64_t s_best;
  if (threadIdx.x == 0) {
    double bv = -1.0, lobe = 0.0;
    int64_t bi = INT64_MAX;
    for (int w = 0; w < nparts; ++w) {
      if (better(parts[w].vmax, parts[w].imax, bv, bi)) {
        bv = parts[w].vmax;
        bi = parts[w].imax;
      }
      lobe += parts[w].lobe;
    }
    s_best = bi;
    if (blockIdx.x == 0) {
      res[0] = bv;
      res[1] = lobe;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int M = d.M;
    const int64_t bi = s_best;
    const int p = (int)(bi / M), q = (int)(bi % M);
    double w;
    if (blockIdx.x == 0)
      w = fwhm_profile(I + (int64_t)p * M, 1, M, s_m, s_c);
    else
      w = fwhm_profile(I + q, M, M, s_m, s_c);
    res[2 + blockIdx.x] = w * d.dx_out;
  }
}

// Batched FWHM of log-intensity maps y = ln(I / I0 + floor) (the surrogate's
// form), one work-group per map: the brightest sample (first index on ties),
// the FWHM along its row (spline, as fwhm_profile), and two conditioning
// numbers that do not need the true map:
//   cond  = (w(1/2 - delta) - w(1/2 + delta)) / (2 delta w(1/2)), the relative
//           change of the width per unit change of the level (about 1.5 for an
//           Airy or Gaussian core; a shoulder or secondary peak near half the
//           maximum makes it jump);
//   ratio = the brightest sample farther than `excl` samples from the peak,
//           relative to the peak (a second spot that could take the peak over);
//   gap   = 1 - (brightest sample of the brighter neighbouring row) / peak, and
//   walt  = the FWHM along that neighbouring row: when the gap is small a
//           slightly different map can put its brightest sample there.
// A NaN width gives cond = +inf.  out[b][0..4] = (FWHM in samples, cond, ratio,
// gap, walt).
__global__ __launch_bounds__(kRedThreads) void k_fwhm_batch(const float *__restrict__ y, int M, double floor_,
                                                            double delta, double excl2, double *__restrict__ out) {
  extern __shared__ double s_row[];  // row, neighbour row, spline m, spline work: 4 M doubles
  __shared__ float s_v[kRedThreads];
  __shared__ int s_i[kRedThreads];
  const int b = blockIdx.x;
  const float *yb = y + (int64_t)b * M * M;
  const int MM = M * M;
  float bv = -INFINITY;
  int bi = INT32_MAX;
  for (int i = threadIdx.x; i < MM; i += kRedThreads)
    if (yb[i] > bv) {  // increasing i: the first index wins ties
      bv = yb[i];
      bi = i;
    }
  s_v[threadIdx.x] = bv;
  s_i[threadIdx.x] = bi;
  __syncthreads();
  for (int h = kRedThreads / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) {
      const float v = s_v[threadIdx.x + h];
      const int i = s_i[threadIdx.x + h];
      if (v > s_v[threadIdx.x] || (v == s_v[threadIdx.x] && i < s_i[threadIdx.x])) {
        s_v[threadIdx.x] = v;
        s_i[threadIdx.x] = i;
      }
    }
    __syncthreads();
  }
  const float ymax = s_v[0];
  const int pk = s_i[0];
  const int p = pk / M, q = pk % M;
  __syncthreads();
  // brightest sample outside the exclusion disc around the peak, and the
  // brightest samples of the rows above and below the peak's row
  float b2 = -INFINITY, up = -INFINITY, dn = -INFINITY;
  for (int i = threadIdx.x; i < MM; i += kRedThreads) {
    const int r = i / M;
    const double dp = (double)(r - p), dq = (double)(i % M - q);
    if (dp * dp + dq * dq > excl2 && yb[i] > b2) b2 = yb[i];
    if (r == p - 1 && yb[i] > up) up = yb[i];
    if (r == p + 1 && yb[i] > dn) dn = yb[i];
  }
  __shared__ float s_up[kRedThreads], s_dn[kRedThreads];
  s_v[threadIdx.x] = b2;
  s_up[threadIdx.x] = up;
  s_dn[threadIdx.x] = dn;
  for (int i = threadIdx.x; i < M; i += kRedThreads) s_row[i] = exp((double)yb[(int64_t)p * M + i]) - floor_;
  __syncthreads();
  for (int h = kRedThreads / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) {
      s_v[threadIdx.x] = fmaxf(s_v[threadIdx.x], s_v[threadIdx.x + h]);
      s_up[threadIdx.x] = fmaxf(s_up[threadIdx.x], s_up[threadIdx.x + h]);
      s_dn[threadIdx.x] = fmaxf(s_dn[threadIdx.x], s_dn[threadIdx.x + h]);
    }
    __syncthreads();
  }
  // the brighter neighbouring row (the row above on ties; none at the ROI edge)
  const int pn = s_up[0] >= s_dn[0] ? p - 1 : p + 1;
  const float yn = s_up[0] >= s_dn[0] ? s_up[0] : s_dn[0];
  const bool has_n = yn != -INFINITY;
  if (has_n)
    for (int i = threadIdx.x; i < M; i += kRedThreads) s_row[M + i] = exp((double)yb[(int64_t)pn * M + i]) - floor_;
  __syncthreads();
  if (threadIdx.x == 0) {
    double *m = s_row + 2 * M, *cp = s_row + 3 * M;
    const double w = fwhm_profile(s_row, 1, M, m, cp);
    const double wl = fwhm_profile(s_row, 1, M, m, cp, 0.5 - delta);
    const double wh = fwhm_profile(s_row, 1, M, m, cp, 0.5 + delta);
    double cond = (wl - wh) / (2.0 * delta * w);
    if (!(cond == cond)) cond = INFINITY;
    const double peak = exp((double)ymax) - floor_;
    const double sec = s_v[0] == -INFINITY ? 0.0 : exp((double)s_v[0]) - floor_;
    double *o = out + 5 * (int64_t)b;
    o[0] = w;
    o[1] = cond;
    o[2] = peak > 0.0 ? sec / peak : INFINITY;
    o[3] = has_n && peak > 0.0 ? 1.0 - (exp((double)yn) - floor_) / peak : 1.0;
    o[4] = has_n ? fwhm_profile(s_row + M, 1, M, m, cp) : NAN;
  }
}

// In-place radix-2 FFT of one line of length M (power of two, <= 4096) in LDS.
__device__ void fft_line(double2 *s, int M, int log2M, int dir) {
  for (int k = threadIdx.x; k < M; k += blockDim.x) {
    const int r = (int)(__brev((unsigned)k) >> (32 - log2M));
    if (r > k) {
      const double2 tmp = s[k];
      s[k] = s[r];
      s[r] = tmp;
    }
  }
  __syncthreads();
  for (int len = 2; len <= M; len <<= 1) {
    const int half = len >> 1;
    for (int b = threadIdx.x; b < M / 2; b += blockDim.x) {
      const int g = b / half, pos = b - g * half;
      const int i = g * len + pos, j = i + half;
      double sn, cs;
      sincospi(2.0 * (double)pos / (double)len, &sn, &cs);
      const double2 w = make_double2(cs, dir < 0 ? -sn : sn);
      const double2 u = s[i], v = cmul(s[j], w);
      s[i] = cadd(u, v);
      s[j] = csub(u, v);
    }
    __syncthreads();
  }
}

// 2-D FFT of I: pass 0 transforms rows of I into F, pass 1 transforms columns of F.
__global__ __launch_bounds__(256) void k_fft2_pass(const double *__restrict__ I, double2 *F, int M, int log2M,
                                                   int pass) {
  __shared__ double2 s[4096];
  for (int line = blockIdx.x; line < M; line += gridDim.x) {
    for (int k = threadIdx.x; k < M; k += blockDim.x)
      s[k] = pass == 0 ? make_double2(I[(int64_t)line * M + k], 0.0) : F[(int64_t)k * M + line];
    __syncthreads();
    fft_line(s, M, log2M, -1);
    for (int k = threadIdx.x; k < M; k += blockDim.x) {
      if (pass == 0)
        F[(int64_t)line * M + k] = s[k];
      else
        F[(int64_t)k * M + line] = s[k];
    }
    __syncthreads();
  }
}

// MTF at nu_cut/2: radial means of |F|/|F(0)| over bins round(|k|), linear
// interpolation at t = (nu_cut/2)/dnu between bins floor(t) and floor(t)+1.
__global__ __launch_bounds__(kRedThreads) void k_mtf(const double2 *__restrict__ F, int M, double t_bin, double *res) {
  const int b0 = (int)floor(t_bin);
  const int R = b0 + 2 < M / 2 ? b0 + 2 : M / 2;
  double s0 = 0.0, s1 = 0.0;
  int64_t n0 = 0, n1 = 0;
  // frequencies k in [-M/2, M/2) with |k| <= R
  const int klo = -R, khi = R < M / 2 ? R : M / 2 - 1;
  for (int ky = klo + (int)threadIdx.x; ky <= khi; ky += blockDim.x) {
    for (int kx = klo; kx <= khi; ++kx) {
      const double r = rint(sqrt((double)(kx * kx + ky * ky)));
      if (r != (double)b0 && r != (double)(b0 + 1)) continue;
      const double2 f = F[(int64_t)((ky + M) % M) * M + ((kx + M) % M)];
      const double a = sqrt(f.x * f.x + f.y * f.y);
      if (r == (double)b0) {
        s0 += a;
        ++n0;
      } else {
        s1 += a;
        ++n1;
      }
    }
  }
  __shared__ double a0[kRedThreads], a1[kRedThreads];
  __shared__ int64_t c0[kRedThreads], c1[kRedThreads];
  a0[threadIdx.x] = s0;
  a1[threadIdx.x] = s1;
  c0[threadIdx.x] = n0;
  c1[threadIdx.x] = n1;
  __syncthreads();
  for (int w = kRedThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      a0[threadIdx.x] += a0[threadIdx.x + w];
      a1[threadIdx.x] += a1[threadIdx.x + w];
      c0[threadIdx.x] += c0[threadIdx.x + w];
      c1[threadIdx.x] += c1[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double2 f00 = F[0];
    const double dc = sqrt(f00.x * f00.x + f00.y * f00.y);
    const double r0 = c0[0] ? a0[0] / (double)c0[0] / dc : NAN;
    if (c1[0] == 0 || t_bin == (double)b0)
      res[4] = r0;
    else {
      const double r1 = a1[0] / (double)c1[0] / dc;
      res[4] = r0 + (t_bin - (double)b0) * (r1 - r0);
    }
  }
}

__global__ void k_mtf_undefined(double *res) {
  if (threadIdx.x == 0) res[4] = NAN;
}

__global__ void k_finish(InstDev d, const double *res, double disc_samples, double R2_over_lz2,
                         fzp_metrics_t *out) {
  if (threadIdx.x != 0) return;
  const double p_in = disc_samples * d.dx * d.dx;
  const double p_lobe = res[1] * d.dx_out * d.dx_out;
  fzp_metrics_t m;
  m.fwhm_x = res[2];
  m.fwhm_y = res[3];
  m.de = p_lobe / p_in;
  m.mtf_half_cut = res[4];
  m.i_peak = res[0];
  m.strehl = res[0] / (M_PI * M_PI * R2_over_lz2);
  m.p_in = p_in;
  m.p_lobe = p_lobe;
  *out = m;
}

}  // namespace

hipError_t launch_fwhm_batch(const float *y, int32_t n, int32_t M, double floor_, double delta, double excl,
                             double *out, hipStream_t st) {
  hipLaunchKernelGGL(k_fwhm_batch, dim3((unsigned)n), dim3(kRedThreads), (size_t)4 * M * sizeof(double), st, y, M,
                     floor_, delta, excl * excl, out);
  return hipGetLastError();
}

size_t metrics_scratch_bytes(int32_t M) { return (sc_end(M) + 255) & ~(size_t)255; }

hipError_t launch_metrics(const InstDev &d, const double2 *roi, double disc_samples, char *scratch,
                          fzp_metrics_t *dev_out, hipStream_t st) {
  const int M = d.M;
  double *I = (double *)(scratch + sc_I(M));
  double2 *F = (double2 *)(scratch + sc_F(M));
  Part *parts = (Part *)(scratch + sc_part(M));
  double *res = (double *)(scratch + sc_res(M));
  hipLaunchKernelGGL(k_intensity, dim3(kPartWG), dim3(kRedThreads), 0, st, d, roi, I, parts, d.rnull2);
  hipLaunchKernelGGL(k_reduce_fwhm, dim3(2), dim3(64), 0, st, d, (const double *)I, (const Part *)parts, kPartWG,
                     res);
  int log2M = 0;
  while ((1 << log2M) < M) ++log2M;
  const bool pow2 = (1 << log2M) == M && M >= 8 && M <= 4096;
  if (pow2) {
    const int grid = M < 1024 ? M : 1024;
    hipLaunchKernelGGL(k_fft2_pass, dim3(grid), dim3(256), 0, st, (const double *)I, F, M, log2M, 0);
    hipLaunchKernelGGL(k_fft2_pass, dim3(grid), dim3(256), 0, st, (const double *)I, F, M, log2M, 1);
    hipLaunchKernelGGL(k_mtf, dim3(1), dim3(kRedThreads), 0, st, (const double2 *)F, M, d.t_mtf, res);
  } else {
    hipLaunchKernelGGL(k_mtf_undefined, dim3(1), dim3(64), 0, st, res);  // the MTF needs a power-of-two M
  }
  hipLaunchKernelGGL(k_finish, dim3(1), dim3(64), 0, st, d, (const double *)res, disc_samples, d.R2_over_lz2,
                     dev_out);
  return hipGetLastError();
}

}  // namespace fzp

extern "C" fzp_status_t fzp_fwhm_batch(const float *y_dev, int32_t n, int32_t M, double floor_, double level_delta,
                                       double exclusion_radius, double *out_dev, void *stream) {
  if (n < 0 || M < 5 || M > 2048 || !(floor_ > 0.0) || !std::isfinite(floor_) || !(level_delta > 0.0) ||
      !(level_delta < 0.25) || !(exclusion_radius >= 0.0) || !std::isfinite(exclusion_radius)) {
    fzp::set_last_error("fzp_fwhm_batch: bad argument");
    return FZP_E_INVAL;
  }
  if (n == 0) return FZP_OK;
  if (!y_dev || !out_dev) {
    fzp::set_last_error("fzp_fwhm_batch: NULL pointer");
    return FZP_E_INVAL;
  }
  const hipError_t e =
      fzp::launch_fwhm_batch(y_dev, n, M, floor_, level_delta, exclusion_radius, out_dev, (hipStream_t)stream);
  if (e != hipSuccess) {
    fzp::set_last_error(std::string("fzp_fwhm_batch: ") + hipGetErrorString(e));
    return FZP_E_DEVICE;
  }
  return FZP_OK;
}
