// Host side of the C ABI: argument validation, the grids and chirp-z
// parameters of each instance (Sec. 3.3 stage 1, Eq. 10; Fig. 18 stage 1),
// the workspace layout and the stripe/chunk schedule of a propagation.

#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <atomic>
#include <exception>
#include <fstream>
#include <sstream>
#include <limits>
#include <new>
#include <string>

#include "fzp_internal.h"

namespace {

thread_local std::string g_err;

fzp_status_t fail(fzp_status_t s, const std::string &msg) {
  g_err = msg;
  return s;
}

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

int64_t isqrt64(int64_t v) {
  if (v <= 0) return 0;
  int64_t m = (int64_t)std::sqrt((double)v);
  while (m > 0 && m * m > v) --m;
  while ((m + 1) * (m + 1) <= v) ++m;
  return m;
}

// Samples with K = (2i-N+1)^2 + (2j-N+1)^2 <= kmax (exact integers).
int64_t disc_count(int64_t N, int64_t kmax) {
  int64_t total = 0;
  for (int64_t j = 0; j < N; ++j) {
    const int64_t cj = 2 * j - N + 1;
    const int64_t rem = kmax - cj * cj;
    if (rem < 0) continue;
    int64_t m = isqrt64(rem);
    if (m > N - 1) m = N - 1;
    // c = 2i - N + 1 runs over integers of the parity of N - 1
    if ((N - 1) % 2 == 0)
      total += 2 * (m / 2) + 1;
    else
      total += 2 * ((m + 1) / 2);
  }
  return total;
}

}  // namespace

struct fzp_plan_s {
  fzp::Plan plan;
};

fzp::Plan::~Plan() {
  for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
  for (hipEvent_t e : lane_ev) (void)hipEventDestroy(e);
  for (hipStream_t t : lane_st) (void)hipStreamDestroy(t);
  for (hipEvent_t e : aux_ev) (void)hipEventDestroy(e);
  for (hipStream_t t : aux_st) (void)hipStreamDestroy(t);
}

namespace {

// Two events from the plan's pool (created on first use).
hipError_t take_events(fzp::Plan &p, hipEvent_t &a, hipEvent_t &b, size_t &first) {
  while (p.ev_pool.size() < p.ev_used + 2) {
    hipEvent_t e;
    hipError_t err = hipEventCreate(&e);
    if (err != hipSuccess) return err;
    p.ev_pool.push_back(e);
  }
  first = p.ev_used;
  a = p.ev_pool[p.ev_used];
  b = p.ev_pool[p.ev_used + 1];
  p.ev_used += 2;
  return hipSuccess;
}

// GEMM variant into every instance's kernel parameters: v % 8 the
// binary-stripe variant (0 .. 4), v / 8 the complex-stripe tile (0: 256
// columns, 1: 128 columns, 2: 128 columns with two work-groups per CU).
void set_variant(fzp::Plan &p, int32_t v) {
  const int32_t b = v % 8, c = v / 8;
  p.bin_variant = b;
  p.cplx_variant = c;
  for (auto &ih : p.inst) {
    ih.dev.bin_tile_rows = b == 1 ? 256 : 512;
    ih.dev.bin_ring = b >= 2 ? 8 : 4;
    ih.dev.bin_prefetch = b == 3 ? 1 : (b == 4 ? 2 : 0);
    ih.dev.cplx_tile = c;
  }
}

}  // namespace

using fzp::InstDev;
using fzp::InstHost;
using fzp::Plan;
using fzp::SaDev;

namespace {

bool smooth235(int64_t m) {
  for (int64_t f : {2, 3, 5})
    while (m % f == 0) m /= f;
  return m == 1;
}

// Radix stages of an LDS transform length (radices 8, 4, 2, 3, 5).
bool radices_of(int n, int32_t *r, int32_t &nst) {
  nst = 0;
  for (int f : {8, 4, 2, 3, 5})
    while (n % f == 0) {
      if (nst == fzp::kSaMaxStages) return false;
      r[nst++] = f;
      n /= f;
    }
  return n == 1;
}

// Non-paraxial variant (Sec. 3.6, Fig. 5): padded size Np = the smallest
// 2^a 3^b 5^c >= pad N with the parity of N (the aperture then sits on the
// padded grid's own sample positions), its factors n1 <= n2 <= 1024, and per
// instance the transfer-function constants (k_max = 2 k0 / 3, the two-point fit
// c = k0 / k_max, d = (sqrt(k0^2 - k_max^2) - k0) / k_max) and the zoom as a
// chirp-z pass with Z = 4 pi |d| z / k_max in place of lambda z.
fzp_status_t plan_sa(Plan &p, double pad) {
  const int64_t N = p.ap.N;
  int64_t Np = (int64_t)std::ceil(pad * (double)N);
  while (!(smooth235(Np) && (Np - N) % 2 == 0)) ++Np;
  int64_t n1 = 0;
  for (int64_t c = (int64_t)std::sqrt((double)Np) + 1; c >= 1; --c)
    if (Np % c == 0 && c * c <= Np && Np / c <= 1024) {
      n1 = c;
      break;
    }
  if (n1 == 0 || Np > (int64_t(1) << 20))
    return fail(FZP_E_UNSUPPORTED, "fzp_plan: padded grid of " + std::to_string(Np) + " samples per side is too large");
  const int64_t n2 = Np / n1;
  SaDev a;
  std::memset(&a, 0, sizeof(a));
  a.Np = Np;
  a.N = N;
  a.off = (Np - N) / 2;
  a.n1 = (int32_t)n1;
  a.n2 = (int32_t)n2;
  if (!radices_of(a.n1, a.rad1, a.nst1) || !radices_of(a.n2, a.rad2, a.nst2))
    return fail(FZP_E_UNSUPPORTED, "fzp_plan: padded grid does not factor into radices 2, 3, 5");
  a.radii_eq3 = (p.opt.flags & FZP_FLAG_PARAXIAL_RADII) ? 0 : 1;
  a.centre_open = p.ap.centre_open;
  a.kmax_disc = (double)p.kmax;
  a.c1 = p.dx * p.dx / (4.0 * p.ap.f0 * p.ap.f0);
  a.c2 = 2.0 * p.ap.f0 / p.ap.lambda0;
  a.kappa = p.kappa;
  a.dx = p.dx;
  a.inv_L2 = 1.0 / ((double)Np * p.dx * (double)Np * p.dx);
  a.norm = 1.0 / ((double)Np * (double)Np);
  const double k_fit = 2.0 / 3.0;
  for (auto &ih : p.inst) {
    SaDev s = a;
    const double lam = ih.lam, z = ih.z;
    const double k0 = 2.0 * M_PI / lam;
    const double kmx = k_fit * k0;
    const double d = (std::sqrt(k0 * k0 - kmx * kmx) - k0) / kmx;
    s.n_creases = ih.in.n_creases;
    s.inv_lam = 1.0 / lam;
    s.inv_lam2 = s.inv_lam * s.inv_lam;
    s.coef = d * lam / k_fit;
    s.z = z;
    ih.sa = s;
    ih.Z = 4.0 * M_PI * std::fabs(d) * z / kmx;
    // the zoom: a chirp-z pass over the Np x Np field with lambda z -> Z
    InstDev &dv = ih.dev;
    dv.N = Np;
    dv.alpha = p.dx * ih.dx_out / ih.Z;
    dv.beta = p.dx * p.dx / ih.Z;
    dv.scale = p.dx * p.dx / ih.Z;
    dv.inv2lz = 1.0 / (2.0 * ih.Z);
  }
  return FZP_OK;
}

}  // namespace

extern "C" const char *fzp_last_error(void) { return g_err.c_str(); }

void fzp::set_last_error(const std::string &msg) { g_err = msg; }

extern "C" fzp_status_t fzp_plan(const fzp_aperture_t *ap, const fzp_instance_t *inst, int32_t n_inst,
                                 const fzp_options_t *opt, fzp_plan_t *out) {
  try {
    if (!ap || !inst || !out || n_inst <= 0) return fail(FZP_E_INVAL, "fzp_plan: NULL argument or n_inst <= 0");
    *out = nullptr;
    fzp_options_t o{};
    if (opt) o = *opt;
    if (o.path != FZP_PATH_FP64_BLUESTEIN && o.path != FZP_PATH_SPLIT_BF16 && o.path != FZP_PATH_AUTO &&
        o.path != FZP_PATH_SA_CZT)
      return fail(FZP_E_INVAL, "fzp_plan: unknown path");
    if (!(std::isfinite(o.pad) && (o.pad == 0.0 || (o.pad >= 1.0 && o.pad <= 8.0))))
      return fail(FZP_E_INVAL, "fzp_plan: pad must be 0 (1.5) or in 1 .. 8");
    if (o.path == FZP_PATH_SA_CZT && ap->levels != 0)
      return fail(FZP_E_UNSUPPORTED, "fzp_plan: the non-paraxial path takes amplitude plates only");
    if (o.path == FZP_PATH_AUTO) {
      // the split GEMMs cost 8 M (binary), 16 M (2- and 4-level phase) or
      // 24 M (complex) flops per sample, the FP64 Bluestein path a few hundred
      // whatever M is: the measured crossovers on MI355X
      int mmax = 0;
      bool m16 = true, creased = false;
      for (int k = 0; k < n_inst; ++k) {
        mmax = inst[k].M > mmax ? inst[k].M : mmax;
        m16 = m16 && inst[k].M % 16 == 0;
        creased = creased || inst[k].n_creases > 0;
      }
      int limit = 128;
      if ((ap->levels == 0 || ap->levels == 2) && !creased) limit = 1024;  // binary GEMM
      else if (ap->levels == 0 || (ap->levels == 4 && !creased)) limit = 256;  // two binary GEMMs, or complex
      // the int8 row pass takes half the matrix-core time of the BF16 one
      if (o.flags & FZP_FLAG_SPLIT_INT8) limit *= 2;
      o.path = m16 && mmax <= limit ? FZP_PATH_SPLIT_BF16 : FZP_PATH_FP64_BLUESTEIN;
      if (o.path != FZP_PATH_SPLIT_BF16) o.flags &= ~FZP_FLAG_SPLIT_INT8;  // a form of the split path only
    }
    if (!finite_pos(ap->D) || !finite_pos(ap->f0) || !finite_pos(ap->lambda0))
      return fail(FZP_E_INVAL, "fzp_plan: D, f0 and lambda0 must be finite and positive");
    if (!(std::isfinite(ap->pitch) && ap->pitch >= 0.0)) return fail(FZP_E_INVAL, "fzp_plan: pitch must be >= 0");
    if (ap->N < 1 || ap->N > (int64_t(1) << 24)) return fail(FZP_E_INVAL, "fzp_plan: N must be in 1 .. 2^24");
    if (ap->centre_open != 0 && ap->centre_open != 1) return fail(FZP_E_INVAL, "fzp_plan: centre_open must be 0 or 1");
    if (ap->levels != 0 && (ap->levels < 2 || ap->levels > 64))
      return fail(FZP_E_INVAL, "fzp_plan: levels must be 0 (amplitude plate) or 2 .. 64 (phase plate)");
    if (ap->levels != 0 && ap->centre_open != 0)
      return fail(FZP_E_INVAL, "fzp_plan: centre_open applies to amplitude plates only");
    if (o.stripe_rows < 0 || o.chunk_rows < 0) return fail(FZP_E_INVAL, "fzp_plan: negative stripe or chunk rows");
    if (o.lanes < 0 || o.lanes > 8) return fail(FZP_E_INVAL, "fzp_plan: lanes must be in 0 .. 8");

    auto h = new (std::nothrow) fzp_plan_s;
    if (!h) return fail(FZP_E_NOMEM, "fzp_plan: out of host memory");
    Plan &p = h->plan;
    static std::atomic<uint64_t> next_serial{1};
    p.serial = next_serial.fetch_add(1, std::memory_order_relaxed);
    p.ap = *ap;
    p.opt = o;
    const int64_t N = ap->N;
    p.dx = ap->pitch > 0.0 ? ap->pitch : ap->D / (double)N;
    // the zone constant, one float64 expression: 4 r^2 / dx^2 = K  =>  r^2/(lambda0 f0) = K * kappa
    p.kappa = p.dx * p.dx / (4.0 * ap->lambda0 * ap->f0);
    if (ap->pitch > 0.0) {
      const double kk = std::floor(std::pow(ap->D / ap->pitch, 2.0));
      if (!(kk < 9.0e15)) {
        delete h;
        return fail(FZP_E_INVAL, "fzp_plan: D / pitch too large");
      }
      p.kmax = (int64_t)kk;
    } else {
      p.kmax = N * N;
    }
    // Eq. 6: dx <= lambda0 f0 / (2 D)
    if (!(o.flags & FZP_FLAG_ALLOW_UNDERSAMPLED) && p.dx > ap->lambda0 * ap->f0 / (2.0 * ap->D)) {
      delete h;
      return fail(FZP_E_SAMPLING, "fzp_plan: pitch exceeds the Nyquist limit lambda0 f0 / (2 D) of Eq. 6");
    }
    // zone (or phase-step) indices must fit int32 over the whole square grid
    const double kcorner = 2.0 * (double)(N - 1) * (double)(N - 1);
    const double step_scale = ap->levels != 0 ? 0.5 * (double)ap->levels : 1.0;
    if (!(kcorner * p.kappa * step_scale < 2.0e9)) {
      delete h;
      return fail(FZP_E_UNSUPPORTED, "fzp_plan: zone count beyond 2e9");
    }
    p.disc_samples = disc_count(N, p.kmax);

    p.inst.resize(n_inst);
    p.Mmax = 0;
    int64_t roi = 0;
    for (int k = 0; k < n_inst; ++k) {
      const fzp_instance_t &in = inst[k];
      InstHost &ih = p.inst[k];
      if (!finite_pos(in.lambda) || !(std::isfinite(in.z) && in.z >= 0.0) || !std::isfinite(in.x0) ||
          !std::isfinite(in.y0) || !(std::isfinite(in.half_width) && in.half_width >= 0.0)) {
        delete h;
        return fail(FZP_E_INVAL, "fzp_plan: instance " + std::to_string(k) + " has a bad lambda/z/x0/y0/half_width");
      }
      if (in.M < 2 || in.M > fzp::kMaxM) {
        delete h;
        return fail(FZP_E_INVAL, "fzp_plan: M must be in 2 .. 2048");
      }
      if (in.n_creases < 0 || in.n_creases > fzp::kMaxCreases || (in.n_creases > 0 && !in.creases)) {
        delete h;
        return fail(FZP_E_INVAL, "fzp_plan: n_creases must be in 0 .. 64 with a crease array");
      }
      ih.in = in;
      ih.in.creases = nullptr;
      ih.creases.assign(in.creases, in.creases + in.n_creases);
      for (const auto &c : ih.creases)
        if (!std::isfinite(c.theta) || !std::isfinite(c.offset) || !finite_pos(c.width) || !std::isfinite(c.height)) {
          delete h;
          return fail(FZP_E_INVAL, "fzp_plan: crease parameters must be finite with width > 0");
        }
      ih.lam = in.lambda;
      ih.z = in.z > 0.0 ? in.z : ap->f0 * ap->lambda0 / in.lambda;
      const double lz = ih.lam * ih.z;
      ih.hw = in.half_width > 0.0 ? in.half_width : 8.0 * ih.lam * ih.z / ap->D;
      ih.dx_out = 2.0 * ih.hw / (double)in.M;
      InstDev &d = ih.dev;
      std::memset(&d, 0, sizeof(d));
      d.N = N;
      d.kappa = p.kappa;
      d.kmax = (double)p.kmax;
      d.centre_open = ap->centre_open;
      d.levels = ap->levels;
      d.kappa_l = p.kappa * (0.5 * (double)ap->levels);
      d.M = in.M;
      d.B = fzp::kFftLen - in.M + 1;
      d.n_creases = in.n_creases;
      d.dx = p.dx;
      // alpha = dx dx_out / (lambda z); at the default pitch (D/N) and ROI
      // (hw = 8 lambda z / D) it is 16 / (N M), formed from the integers (exact
      // when N M is a power of two), so the Bluestein chirp turns alpha k^2 / 2
      // carry no rounding of dx, dx_out or lambda z
      if (ap->pitch == 0.0 && in.half_width == 0.0)
        d.alpha = 16.0 / ((double)N * (double)in.M);
      else
        d.alpha = p.dx * ih.dx_out / lz;
      d.beta = p.dx * p.dx / lz;
      d.sx = in.x0 / ih.dx_out;
      d.sy = in.y0 / ih.dx_out;
      const double zl = ih.z / ih.lam;
      d.kz_turns = (zl - std::floor(zl)) - 0.25;
      d.scale = p.dx * p.dx / lz;
      d.x0 = in.x0;
      d.y0 = in.y0;
      d.dx_out = ih.dx_out;
      d.inv2lz = 1.0 / (2.0 * lz);
      const double j11 = 3.8317059702075125;
      const double rnull = j11 / M_PI * lz / ap->D;
      d.rnull2 = rnull * rnull;
      const double R = 0.5 * ap->D;
      d.R2_over_lz2 = (R * R / lz) * (R * R / lz);
      d.t_mtf = 0.5 * (ap->D / lz) * (double)in.M * ih.dx_out;
      ih.roi_off = roi;
      roi += (int64_t)in.M * in.M;
      if (in.M > p.Mmax) p.Mmax = in.M;
    }
    p.roi_elems = roi;

    // non-paraxial variant: the padded grid, its FFT factors and each
    // instance's transfer function and zoom
    const bool sa = o.path == FZP_PATH_SA_CZT;
    if (sa) {
      const fzp_status_t st = plan_sa(p, o.pad > 0.0 ? o.pad : 1.5);
      if (st != FZP_OK) {
        delete h;
        return st;
      }
    }

    // stripe and chunk schedule
    const bool split = o.path == FZP_PATH_SPLIT_BF16;
    p.S = o.stripe_rows > 0 ? o.stripe_rows : (split ? 128 : 64);
    if (split && p.S != 64 && p.S != 128 && p.S != 256) {
      delete h;
      return fail(FZP_E_INVAL, "fzp_plan: split path stripe_rows must be 64, 128 or 256");
    }
    // split path with complex stripes: creases, or a phase plate other than the
    // 2- and 4-level ones (which run on the binary kernels, see four_level_fast)
    bool cplx = false;
    if (split)
      for (const auto &ih : p.inst) {
        cplx = cplx || ih.in.n_creases > 0 || (ap->levels != 0 && ap->levels != 2 && ap->levels != 4);
        if (ap->levels == 4 && ih.in.n_creases == 0) p.mask_sets = 2;
      }
    if (o.flags & FZP_FLAG_SPLIT_INT8) {
      if (!split) {
        delete h;
        return fail(FZP_E_UNSUPPORTED, "fzp_plan: FZP_FLAG_SPLIT_INT8 needs the split path");
      }
      for (auto &ih : p.inst) ih.dev.i8 = 1;
    }
    if (split)
      for (const auto &ih : p.inst)
        if (ih.in.M % 16 != 0) {
          delete h;
          return fail(FZP_E_UNSUPPORTED, "fzp_plan: the split path needs M to be a multiple of 16");
        }
    // split path: K is cut into segments of seg_len columns, each summed in
    // float32 and the segments added in float64 by the column pass; about 8
    // segments per row (4096 .. 65536 columns) also gives the GEMM grid
    // enough independent tiles at small N
    int64_t seg_len = 4096;
    while (seg_len < 65536 && seg_len * 16 <= N) seg_len *= 2;
    p.seg_len = seg_len;
    p.bin_variant = (o.flags & FZP_FLAG_BIN_TILE_256) ? 1
                    : (o.flags & FZP_FLAG_BIN_SHALLOW) ? 0
                    : (o.flags & FZP_FLAG_BIN_PREFETCH) ? 3
                    : (o.flags & FZP_FLAG_BIN_DEEP) ? 2 : 4;
    p.cplx_variant = (o.flags & FZP_FLAG_CPLX_TILE_DUAL) ? 2 : (o.flags & FZP_FLAG_CPLX_TILE_128) ? 1 : 0;
    for (auto &ih : p.inst) ih.dev.seg_len = seg_len;
    set_variant(p, p.bin_variant + 8 * p.cplx_variant);
    p.lanes_max = o.lanes > 0 && !sa ? o.lanes : 1;  // the padded field is one buffer
    p.lanes = p.lanes_max;
    const int64_t nseg = split ? (N + seg_len - 1) / seg_len : 1;
    const size_t tbytes = split ? sizeof(float) * 2 * (size_t)nseg : sizeof(double) * 2;
    if (o.chunk_rows > 0) {
      // more rows than the aperture has only enlarge the buffers (and could
      // overflow the byte counts below): at most N
      p.chunk_rows = o.chunk_rows < N ? o.chunk_rows : N;
    } else {
      const size_t budget = (size_t)(split ? 1024 : 512) << 20;  // T buffer target
      int64_t c = (int64_t)(budget / ((size_t)p.Mmax * tbytes));
      c = c / p.S * p.S;
      if (c < p.S) c = p.S;
      p.chunk_rows = c < N ? c : N;
    }
    if (sa) {
      // the zoom runs over the rows of the padded grid
      const int64_t Np = p.inst[0].sa.Np;
      const int64_t c = o.chunk_rows > 0 ? o.chunk_rows
                                         : (int64_t)(((size_t)512 << 20) / ((size_t)p.Mmax * sizeof(double2)));
      p.chunk_rows = c < Np ? (c > 0 ? c : 1) : Np;
    }
    if (split && cplx && o.chunk_rows <= 0) {
      // the complex stripe planes (8 bytes per sample of a chunk) stay near
      // 2 GiB, or grow up to 8 GiB while the GEMM grid of the smallest ROI
      // (256-row x 256-column tiles times K segments) has fewer than 512 tiles
      const int64_t npad = (N + 63) / 64 * 64;
      const size_t per_row = (size_t)npad * 8;
      int64_t c = (int64_t)(((size_t)2 << 30) / per_row) / 256 * 256;
      if (c < 256) c = 256;
      int Mmin = p.Mmax;
      for (const auto &ih : p.inst) Mmin = ih.dev.M < Mmin ? ih.dev.M : Mmin;
      const int64_t n_ct = (2 * Mmin + 255) / 256;
      while ((c / 256) * n_ct * nseg < 512 && c < N && (size_t)(2 * c) * per_row <= ((size_t)8 << 30)) c *= 2;
      if (c < p.chunk_rows) p.chunk_rows = c;
    }
    if (split) p.chunk_rows = (p.chunk_rows + p.S - 1) / p.S * p.S;

    // workspace layout
    size_t off = 0;
    for (int k = 0; k < n_inst; ++k) {
      InstHost &ih = p.inst[k];
      ih.off_Hx = off;
      off = align256(off + fzp::kFftLen * sizeof(double2));
      ih.off_Hy = off;
      off = align256(off + fzp::kFftLen * sizeof(double2));
      ih.off_Dt = off;
      off = align256(off + fzp::kFftLen * sizeof(double2));
      ih.off_Qx = off;
      off = align256(off + (size_t)ih.in.M * sizeof(double2));
      ih.off_Qy = off;
      off = align256(off + (size_t)ih.in.M * sizeof(double2));
      ih.off_cr = off;  // crease constants, then the phase-level phasors
      off = align256(off + (size_t)(ih.creases.size() + 1) * sizeof(fzp::CreaseDev) + 64 * sizeof(double2));
      ih.table_owner = k;
      ih.col_owner = k;
      ih.off_A = 0;
      ih.off_By = 0;
      ih.off_S = 0;
    }
    if (split) {
      // K padded to the GEMM stage: 64 columns, 128 for the int8 row pass
      const int64_t kal = p.inst[0].dev.i8 ? 128 : 64;
      const int64_t npad = (N + kal - 1) / kal * kal;
      for (int k = 0; k < n_inst; ++k) {
        InstHost &ih = p.inst[k];
        // instances with the same ROI grid and lambda z share one operand table
        for (int k2 = 0; k2 < k; ++k2) {
          const InstHost &o2 = p.inst[k2];
          if (o2.table_owner == k2 && o2.dev.M == ih.dev.M && o2.dev.alpha == ih.dev.alpha &&
              o2.dev.beta == ih.dev.beta && o2.dev.sx == ih.dev.sx) {
            ih.table_owner = k2;
            ih.off_A = o2.off_A;
            break;
          }
        }
        if (ih.table_owner == k) {
          ih.off_A = off;
          off = align256(off + (size_t)2 * 2 * ih.in.M * npad * sizeof(uint16_t));
          if (ap->levels == 2 || ap->levels == 4) {  // 2- and 4-level plates: prefix sums of the same kernel
            ih.off_S = off;
            off = align256(off + fzp::prefix_table_bytes(ih.in.M, npad));
          }
        } else {
          ih.off_S = p.inst[ih.table_owner].off_S;
        }
        // the column pass's kernel matrix B_y: shared on the same terms, with the y shift
        for (int k2 = 0; k2 < k; ++k2) {
          const InstHost &o2 = p.inst[k2];
          if (o2.col_owner == k2 && o2.dev.M == ih.dev.M && o2.dev.alpha == ih.dev.alpha &&
              o2.dev.beta == ih.dev.beta && o2.dev.sy == ih.dev.sy) {
            ih.col_owner = k2;
            ih.off_By = o2.off_By;
            break;
          }
        }
        if (ih.col_owner == k) {
          ih.off_By = off;
          off = align256(off + fzp::col_table_bytes(ih.in.M, npad));
        }
        ih.dev.Npad = npad;
      }
    }
    if (sa) {
      const SaDev &a = p.inst[0].sa;
      p.off_twNp = off;
      off = align256(off + (size_t)a.Np * sizeof(double2));
      p.off_tw1 = off;
      off = align256(off + (size_t)a.n1 * sizeof(double2));
      p.off_tw2 = off;
      off = align256(off + (size_t)a.n2 * sizeof(double2));
      p.off_U1 = off;
      off = align256(off + (size_t)a.Np * (size_t)a.Np * sizeof(double2));
    }
    p.T_bytes = align256((size_t)p.chunk_rows * p.Mmax * tbytes);
    if (split) {
      p.bits_bytes = align256(fzp::split_bits_bytes(p.inst[0].dev, p.chunk_rows));
      if (cplx) p.G_bytes = align256(fzp::split_stripe_bytes(p.inst[0].dev, p.chunk_rows));
      for (const auto &ih : p.inst) {
        p.Tb_bytes = std::max(p.Tb_bytes, align256(fzp::col_operand_bytes(ih.in.M, p.chunk_rows)));
        p.C_bytes = std::max(p.C_bytes, align256(fzp::col_partial_bytes(ih.in.M, p.chunk_rows)));
      }
    }
    for (int l = 0; l < p.lanes_max; ++l) {
      p.off_T.push_back(off);
      off += (size_t)p.mask_sets * p.T_bytes;
      // two operand buffers when chunk c+1's operand is made during chunk c
      const size_t nbuf = (o.flags & FZP_FLAG_OVERLAP_OPERAND) ? 2 : 1;
      p.off_bits.push_back(off);
      off += nbuf * (size_t)p.mask_sets * p.bits_bytes;
      p.off_G.push_back(off);
      off += nbuf * p.G_bytes;
      p.off_Tb.push_back(off);
      off += p.Tb_bytes;
      p.off_C.push_back(off);
      off += p.C_bytes;
    }
    p.off_scratch = off;
    // metric kernels' scratch, then one result record per instance (so that a
    // batch's metrics come back in one copy)
    p.scratch_bytes = fzp::metrics_scratch_bytes(p.Mmax) + align256(p.inst.size() * sizeof(fzp_metrics_t));
    off += p.scratch_bytes;
    p.ws_bytes = off;
    if (o.workspace_limit > 0 && p.ws_bytes > o.workspace_limit) {
      const size_t need = p.ws_bytes;
      delete h;
      return fail(FZP_E_NOMEM, "fzp_plan: workspace of " + std::to_string(need) + " bytes exceeds the limit");
    }
    *out = h;
    return FZP_OK;
  } catch (const std::bad_alloc &) {
    return fail(FZP_E_NOMEM, "fzp_plan: out of host memory");
  } catch (const std::exception &e) {
    return fail(FZP_E_INVAL, std::string("fzp_plan: ") + e.what());
  } catch (...) {
    return fail(FZP_E_INVAL, "fzp_plan: unknown error");
  }
}

extern "C" fzp_status_t fzp_plan_workspace_size(fzp_plan_t p, size_t *bytes) {
  if (!p || !bytes) return fail(FZP_E_INVAL, "fzp_plan_workspace_size: NULL argument");
  *bytes = p->plan.ws_bytes;
  return FZP_OK;
}

extern "C" fzp_status_t fzp_roi_elements(fzp_plan_t p, int64_t *n) {
  if (!p || !n) return fail(FZP_E_INVAL, "fzp_roi_elements: NULL argument");
  *n = p->plan.roi_elems;
  return FZP_OK;
}

extern "C" fzp_status_t fzp_roi_offset(fzp_plan_t p, int32_t k, int64_t *off) {
  if (!p || !off || k < 0 || k >= (int32_t)p->plan.inst.size()) return fail(FZP_E_INVAL, "fzp_roi_offset: bad argument");
  *off = p->plan.inst[k].roi_off;
  return FZP_OK;
}

extern "C" fzp_status_t fzp_plan_info(fzp_plan_t p, int32_t *fft_len, int32_t *block, int64_t *chunk_rows,
                                      int32_t *stripe_rows, int32_t *path, int64_t *disc_samples, double *kappa) {
  if (!p) return fail(FZP_E_INVAL, "fzp_plan_info: NULL plan");
  const Plan &pl = p->plan;
  if (fft_len) *fft_len = fzp::kFftLen;
  if (block) *block = pl.inst[0].dev.B;
  if (chunk_rows) *chunk_rows = pl.chunk_rows;
  if (stripe_rows) *stripe_rows = pl.S;
  if (path) *path = pl.opt.path;
  if (disc_samples) *disc_samples = pl.disc_samples;
  if (kappa) *kappa = pl.kappa;
  return FZP_OK;
}

extern "C" fzp_status_t fzp_grid_for_element(double D, double f0, double lambda0, int32_t levels, int32_t s_samp,
                                             double *pitch, int64_t *N) {
  if (!pitch || !N) return fail(FZP_E_INVAL, "fzp_grid_for_element: NULL output");
  if (!finite_pos(D) || !finite_pos(f0) || !finite_pos(lambda0) || levels < 0 || levels > 64 || s_samp < 0)
    return fail(FZP_E_INVAL, "fzp_grid_for_element: bad argument");
  const int32_t S = s_samp > 0 ? s_samp : 4;
  const int32_t L = levels > 2 ? levels : 2;
  const double edge = lambda0 * f0 / (0.5 * D);  // zone period at the rim
  const double dx = edge / ((double)S * (double)L);
  const double n = std::ceil(D / dx);
  if (!(n < 9.0e15)) return fail(FZP_E_INVAL, "fzp_grid_for_element: grid too large");
  int64_t nx = (int64_t)n;
  if (nx % 2 == 0) ++nx;
  *pitch = dx;
  *N = nx;
  return FZP_OK;
}

extern "C" fzp_status_t fzp_plan_geometry(fzp_plan_t h, int32_t k, fzp_geometry_t *out) {
  if (!h || !out || k < 0 || k >= (int32_t)h->plan.inst.size())
    return fail(FZP_E_INVAL, "fzp_plan_geometry: bad argument");
  const Plan &p = h->plan;
  // Eq. 3 at r = R: n = (2 / lambda0)(sqrt(f0^2 + R^2) - f0), without the cancellation
  const double R = 0.5 * p.ap.D, f = p.ap.f0;
  const double n = 2.0 * R * R / (p.ap.lambda0 * (std::sqrt(f * f + R * R) + f));
  std::memset(out, 0, sizeof(*out));
  out->zones_exact = n;
  out->total_zones = (int64_t)std::floor(n);
  if (p.opt.path == FZP_PATH_SA_CZT) {
    const InstHost &ih = p.inst[k];
    out->padded_n = ih.sa.Np;
    out->fft_n1 = ih.sa.n1;
    out->fft_n2 = ih.sa.n2;
    out->zoom_distance = ih.Z / ih.lam;
  }
  return FZP_OK;
}

extern "C" void fzp_destroy(fzp_plan_t p) { delete p; }

namespace {

fzp_status_t hip_fail(const char *what, hipError_t e) {
  return fail(FZP_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

// Device pointers of the tables of instance k inside workspace ws.
void bind_tables(Plan &p, char *ws) {
  for (auto &ih : p.inst) {
    ih.dev.Hx = (const double2 *)(ws + ih.off_Hx);
    ih.dev.Hy = (const double2 *)(ws + ih.off_Hy);
    ih.dev.Dt = (const double2 *)(ws + ih.off_Dt);
    ih.dev.Qx = (const double2 *)(ws + ih.off_Qx);
    ih.dev.Qy = (const double2 *)(ws + ih.off_Qy);
    ih.dev.cr = (const fzp::CreaseDev *)(ws + ih.off_cr);
    ih.dev.lev = (const double2 *)(ws + ih.off_cr + (ih.creases.size() + 1) * sizeof(fzp::CreaseDev));
    ih.dev.A = p.opt.path == FZP_PATH_SPLIT_BF16 ? (const uint16_t *)(ws + ih.off_A) : nullptr;
    ih.dev.By = p.opt.path == FZP_PATH_SPLIT_BF16 ? (const uint16_t *)(ws + ih.off_By) : nullptr;
    ih.dev.S = p.opt.path == FZP_PATH_SPLIT_BF16 && (p.ap.levels == 2 || p.ap.levels == 4)
                   ? (const double2 *)(ws + ih.off_S)
                   : nullptr;
    if (p.opt.path == FZP_PATH_SA_CZT) {
      ih.sa.cr = ih.dev.cr;
      ih.sa.twNp = (const double2 *)(ws + p.off_twNp);
      ih.sa.tw1 = (const double2 *)(ws + p.off_tw1);
      ih.sa.tw2 = (const double2 *)(ws + p.off_tw2);
    }
  }
}

}  // namespace

extern "C" fzp_status_t fzp_prepare(fzp_plan_t h, void *workspace, void *stream) {
  if (!h || !workspace) return fail(FZP_E_INVAL, "fzp_prepare: NULL argument");
  if (((uintptr_t)workspace & 255) != 0) return fail(FZP_E_INVAL, "fzp_prepare: workspace must be 256-byte aligned");
  try {
    Plan &p = h->plan;
    hipStream_t st = (hipStream_t)stream;
    char *ws = (char *)workspace;
    bind_tables(p, ws);
    for (size_t k = 0; k < p.inst.size(); ++k) {
      InstHost &ih = p.inst[k];
      // crease constants
      std::vector<fzp::CreaseDev> cd(ih.creases.size() + 1);
      for (size_t c = 0; c < ih.creases.size(); ++c) {
        const fzp_crease_t &cr = ih.creases[c];
        const double sigma = cr.width / (2.0 * std::sqrt(2.0 * std::log(2.0)));
        cd[c].c = std::cos(cr.theta);
        cd[c].s = std::sin(cr.theta);
        cd[c].rho = cr.offset;
        cd[c].inv2s2 = 1.0 / (2.0 * sigma * sigma);
        cd[c].h_over_lambda = cr.height / ih.lam;
      }
      hipError_t e = hipMemcpyAsync(ws + ih.off_cr, cd.data(), cd.size() * sizeof(fzp::CreaseDev),
                                    hipMemcpyHostToDevice, st);
      if (e != hipSuccess) return hip_fail("fzp_prepare: crease upload", e);
      // phase plates: the L level phasors exp(-2 pi i l / L) in float64
      std::vector<double2> lev(64, make_double2(0.0, 0.0));
      for (int l = 0; l < p.ap.levels; ++l) {
        const double a = -2.0 * M_PI * (double)l / (double)p.ap.levels;
        lev[l] = make_double2(std::cos(a), std::sin(a));
      }
      e = hipMemcpyAsync(ws + ih.off_cr + cd.size() * sizeof(fzp::CreaseDev), lev.data(), lev.size() * sizeof(double2),
                         hipMemcpyHostToDevice, st);
      if (e != hipSuccess) return hip_fail("fzp_prepare: level upload", e);
      // pageable source: make sure the copy has consumed cd before it goes out of scope
      e = hipStreamSynchronize(st);
      if (e != hipSuccess) return hip_fail("fzp_prepare: synchronize", e);
      e = fzp::launch_build_tables(p, ih, ws, st);
      if (e != hipSuccess) return hip_fail("fzp_prepare: table kernel", e);
      if (p.opt.path == FZP_PATH_SPLIT_BF16 && ih.table_owner == (int32_t)k) {
        e = ih.dev.i8 ? fzp::launch_build_i8_table(ih, ws, st) : fzp::launch_build_split_table(p, ih, ws, st);
        if (e != hipSuccess) return hip_fail("fzp_prepare: split table kernel", e);
        if (ih.dev.S) {
          e = fzp::launch_build_prefix_table(ih.dev, (double2 *)(ws + ih.off_S), st);
          if (e != hipSuccess) return hip_fail("fzp_prepare: prefix table kernel", e);
        }
      }
      if (p.opt.path == FZP_PATH_SPLIT_BF16 && ih.col_owner == (int32_t)k) {
        e = fzp::launch_build_col_table(ih.dev, (uint16_t *)(ws + ih.off_By), st);
        if (e != hipSuccess) return hip_fail("fzp_prepare: column table kernel", e);
      }
    }
    if (p.opt.path == FZP_PATH_SPLIT_BF16) {
      hipError_t e = fzp::init_split_attributes();
      if (e == hipSuccess && p.inst[0].dev.i8) e = fzp::init_i8_attributes();
      if (e != hipSuccess) return hip_fail("fzp_prepare: kernel attributes", e);
    }
    if (p.opt.path == FZP_PATH_SA_CZT) {
      hipError_t e = fzp::init_sa_attributes();
      if (e == hipSuccess)
        e = fzp::launch_sa_twiddles(p.inst[0].sa, (double2 *)(ws + p.off_twNp), (double2 *)(ws + p.off_tw1),
                                    (double2 *)(ws + p.off_tw2), st);
      if (e != hipSuccess) return hip_fail("fzp_prepare: padded-grid tables", e);
    }
    p.prepared_ws = workspace;
    return FZP_OK;
  } catch (const std::exception &e) {
    return fail(FZP_E_INVAL, std::string("fzp_prepare: ") + e.what());
  } catch (...) {
    return fail(FZP_E_INVAL, "fzp_prepare: unknown error");
  }
}

namespace {

// Internal lane streams and their fork/join events (created on first use).
hipError_t ensure_lanes(Plan &p) {
  if (p.lanes <= 1 || (int)p.lane_st.size() >= p.lanes_max) return hipSuccess;
  while ((int)p.lane_st.size() < p.lanes_max) {
    hipStream_t t;
    hipError_t e = hipStreamCreateWithFlags(&t, hipStreamNonBlocking);
    if (e != hipSuccess) return e;
    p.lane_st.push_back(t);
  }
  while ((int)p.lane_ev.size() < p.lanes_max + 1) {
    hipEvent_t ev;
    hipError_t e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e != hipSuccess) return e;
    p.lane_ev.push_back(ev);
  }
  return hipSuccess;
}

// Auxiliary stream and events of every lane (split path): the stripe operand
// of chunk c+1 is generated there while the GEMM of chunk c runs.
hipError_t ensure_aux(Plan &p) {
  while ((int)p.aux_st.size() < p.lanes_max) {
    hipStream_t t;
    hipError_t e = hipStreamCreateWithFlags(&t, hipStreamNonBlocking);
    if (e != hipSuccess) return e;
    p.aux_st.push_back(t);
  }
  while ((int)p.aux_ev.size() < 5 * p.lanes_max) {
    hipEvent_t ev;
    hipError_t e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e != hipSuccess) return e;
    p.aux_ev.push_back(ev);
  }
  return hipSuccess;
}

// Non-paraxial variant: the propagated padded field U1 of instance ih (seven
// FFT passes with the transfer function), then the chirp-z zoom over U1's
// rows in chunks of chunk_rows (row pass, then column pass into the ROI).
fzp_status_t enqueue_sa(Plan &p, InstHost &ih, char *ws, double2 *roi, hipStream_t st) {
  double2 *U1 = (double2 *)(ws + p.off_U1);
  double2 *T = (double2 *)(ws + p.off_T[0]);
  hipEvent_t ea = nullptr, eb = nullptr;
  size_t first = 0;
  auto mark = [&](int kind, bool begin) -> hipError_t {
    if (!p.profile) return hipSuccess;
    if (begin) {
      hipError_t pe = take_events(p, ea, eb, first);
      return pe == hipSuccess ? hipEventRecord(ea, st) : pe;
    }
    const hipError_t pe = hipEventRecord(eb, st);
    p.ev_marks.emplace_back(first, kind);
    return pe;
  };
  hipError_t e = mark(2, true);
  if (e == hipSuccess) e = fzp::launch_sa_field(ih.sa, U1, st);
  if (e == hipSuccess) e = mark(2, false);
  if (e != hipSuccess) return hip_fail("fzp_propagate_roi: padded field", e);
  const int64_t Np = ih.sa.Np;
  for (int64_t r0 = 0; r0 < Np; r0 += p.chunk_rows) {
    const int64_t r1 = r0 + p.chunk_rows < Np ? r0 + p.chunk_rows : Np;
    e = mark(0, true);
    if (e == hipSuccess) e = fzp::launch_row_pass_stored(ih.dev, U1, r0, r1, T, st);
    if (e == hipSuccess) e = mark(0, false);
    if (e != hipSuccess) return hip_fail("fzp_propagate_roi: zoom row pass", e);
    e = mark(1, true);
    if (e == hipSuccess) e = fzp::launch_col_pass(ih.dev, r0, r1, T, roi, st);
    if (e == hipSuccess) e = mark(1, false);
    if (e != hipSuccess) return hip_fail("fzp_propagate_roi: zoom column pass", e);
  }
  return FZP_OK;
}

// Rows [row_begin, row_end) of instance ih into its ROI, on stream st with the
// stripe buffers of `lane`.  On the split path the stripe operand (mask bits,
// or the complex stripe planes) of each chunk is generated on the lane's
// auxiliary stream into one of two buffers, one chunk ahead of the GEMM:
//   aux:  [wait GEMM(i-1)] stripe(i+1) -> buffer (i+1)%2, record m[(i+1)%2]
//   st:   wait m[i%2], GEMM(i) <- buffer i%2, record g[i%2], column pass(i)
fzp_status_t enqueue_instance(Plan &p, InstHost &ih, int lane, char *ws, double2 *roi, int64_t row_begin,
                              int64_t row_end, hipStream_t st) {
  const bool split = p.opt.path == FZP_PATH_SPLIT_BF16;
  // complex stripes: creases, or a phase plate other than the 2- and 4-level
  // ones (disc - 2 mask, disc - (1 - i) odd - (1 + i) half: binary kernels)
  const bool four = split && fzp::four_level_fast(ih.dev);
  const bool cplx = split && (ih.dev.n_creases > 0 ||
                              (ih.dev.levels != 0 && !fzp::two_level_fast(ih.dev) && !four));
  void *T = ws + p.off_T[lane];
  void *T2 = four ? ws + p.off_T[lane] + p.T_bytes : nullptr;  // the second mask's partial planes
  const size_t bits_set = (size_t)p.mask_sets * p.bits_bytes;   // one operand buffer
  hipError_t e;
  // the chunks (aligned to multiples of chunk_rows from row 0) with disc samples
  struct Chunk {
    int64_t r0, r1;
    int nseg;
  };
  std::vector<Chunk> chunks;
  for (int64_t c0 = row_begin / p.chunk_rows * p.chunk_rows; c0 < row_end; c0 += p.chunk_rows) {
    const int64_t r0 = c0 > row_begin ? c0 : row_begin;
    const int64_t r1 = c0 + p.chunk_rows < row_end ? c0 + p.chunk_rows : row_end;
    if (r1 <= r0) continue;
    int nseg = 1;
    if (split) {
      int sl, sh;
      fzp::split_seg_range(ih.dev, r0, r1, sl, sh);
      nseg = sh - sl;
      if (nseg <= 0) continue;  // no disc samples in these rows
    }
    chunks.push_back({r0, r1, nseg});
  }
  if (chunks.empty()) return FZP_OK;
  const int64_t seg_stride = p.chunk_rows * (int64_t)ih.dev.M;
  // each launch is bracketed by its own pair of events when profiling
  hipEvent_t ea = nullptr, eb = nullptr;
  size_t first = 0;
  auto begin_mark = [&](hipStream_t s) -> hipError_t {
    if (!p.profile) return hipSuccess;
    hipError_t pe = take_events(p, ea, eb, first);
    if (pe == hipSuccess) pe = hipEventRecord(ea, s);
    return pe;
  };
  auto end_mark = [&](int kind, hipStream_t s) -> hipError_t {
    if (!p.profile) return hipSuccess;
    hipError_t pe = hipEventRecord(eb, s);
    p.ev_marks.emplace_back(first, kind);
    return pe;
  };
  // Without FZP_FLAG_OVERLAP_OPERAND the operand is made on st itself, one
  // chunk at a time.
  const bool overlap = split && (p.opt.flags & FZP_FLAG_OVERLAP_OPERAND);
  if (overlap) {
    // the overlap is not supported under stream capture: a capture of it
    // (fzp_graph_create) ended in a host segmentation fault whose cause was
    // not found, so a capturing stream gets an error instead
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    e = hipStreamIsCapturing(st, &cs);
    if (e != hipSuccess) return hip_fail("fzp_propagate_roi_range: capture status", e);
    if (p.capturing || cs != hipStreamCaptureStatusNone)
      return fail(FZP_E_UNSUPPORTED, "fzp_propagate_roi_range: FZP_FLAG_OVERLAP_OPERAND under stream capture");
  }
  hipStream_t ax = st;
  hipEvent_t *ev = nullptr;  // [0] fork, [1 + b] stripe b ready, [3 + b] GEMM done with buffer b
  auto stripe = [&](size_t i) -> hipError_t {
    const int b = overlap ? (int)(i % 2) : 0;
    hipError_t pe = hipSuccess;
    if (overlap && i >= 2) pe = hipStreamWaitEvent(ax, ev[3 + b], 0);
    if (pe == hipSuccess) pe = begin_mark(ax);
    if (pe == hipSuccess)
      pe = cplx ? fzp::launch_stripe_cplx(ih.dev, chunks[i].r0, chunks[i].r1,
                                          (uint16_t *)(ws + p.off_G[lane] + b * p.G_bytes), ax)
                : (ih.dev.i8 ? fzp::launch_mask_bits_i8 : fzp::launch_mask_bits)(
                      ih.dev, chunks[i].r0, chunks[i].r1, (uint32_t *)(ws + p.off_bits[lane] + b * bits_set), ax,
                      four ? (uint32_t *)(ws + p.off_bits[lane] + b * bits_set + p.bits_bytes) : nullptr);
    if (pe == hipSuccess) pe = end_mark(2, ax);
    if (pe == hipSuccess && overlap) pe = hipEventRecord(ev[1 + b], ax);
    return pe;
  };
  if (overlap) {
    e = ensure_aux(p);
    if (e != hipSuccess) return hip_fail("fzp_propagate_roi_range: auxiliary stream", e);
    ax = p.aux_st[lane];
    ev = &p.aux_ev[5 * lane];
    // fork: the auxiliary stream starts after the work already on st
    e = hipEventRecord(ev[0], st);
    if (e == hipSuccess) e = hipStreamWaitEvent(ax, ev[0], 0);
    if (e == hipSuccess) e = stripe(0);
    if (e != hipSuccess) return hip_fail("fzp_propagate_roi_range: stripe operand", e);
  } else if (split) {
    e = stripe(0);
    if (e != hipSuccess) return hip_fail("fzp_propagate_roi_range: stripe operand", e);
  }
  for (size_t i = 0; i < chunks.size(); ++i) {
    const int64_t r0 = chunks[i].r0, r1 = chunks[i].r1;
    const int b = overlap ? (int)(i % 2) : 0;
    if (overlap) {
      e = i + 1 < chunks.size() ? stripe(i + 1) : hipSuccess;
      if (e == hipSuccess) e = hipStreamWaitEvent(st, ev[1 + b], 0);
      if (e != hipSuccess) return hip_fail("fzp_propagate_roi_range: stripe operand", e);
    } else if (split && i > 0) {
      e = stripe(i);
      if (e != hipSuccess) return hip_fail("fzp_propagate_roi_range: stripe operand", e);
    }
    e = begin_mark(st);
    if (e != hipSuccess) return hip_fail("fzp_propagate_roi_range: event", e);
    if (cplx && ih.dev.i8)
      e = fzp::launch_row_pass_i8_cplx(ih.dev, r0, r1, (float2 *)T, seg_stride, ws + p.off_G[lane] + b * p.G_bytes,
                                       st);
    else if (cplx)
      e = fzp::launch_row_pass_split_cplx(ih.dev, r0, r1, (float2 *)T, seg_stride,
                                          (const uint16_t *)(ws + p.off_G[lane] + b * p.G_bytes), st);
    else if (split) {
      const uint32_t *bits = (const uint32_t *)(ws + p.off_bits[lane] + b * bits_set);
      const uint32_t *bits2 = (const uint32_t *)(ws + p.off_bits[lane] + b * bits_set + p.bits_bytes);
      e = ih.dev.i8 ? fzp::launch_row_pass_i8(ih.dev, r0, r1, (float2 *)T, seg_stride, bits, st)
                    : fzp::launch_row_pass_split(ih.dev, p.S, r0, r1, (float2 *)T, seg_stride, bits, st);
      if (e == hipSuccess && four)
        e = ih.dev.i8 ? fzp::launch_row_pass_i8(ih.dev, r0, r1, (float2 *)T2, seg_stride, bits2, st)
                      : fzp::launch_row_pass_split(ih.dev, p.S, r0, r1, (float2 *)T2, seg_stride, bits2, st);
    }
    else
      e = fzp::launch_row_pass_fp64(ih.dev, r0, r1, (double2 *)T, st);
    if (e != hipSuccess) return hip_fail("fzp_propagate_roi_range: row pass", e);
    e = end_mark(0, st);
    if (e == hipSuccess && overlap) e = hipEventRecord(ev[3 + b], st);
    if (e == hipSuccess) e = begin_mark(st);
    if (e != hipSuccess) return hip_fail("fzp_propagate_roi_range: event", e);
    if (split)
      e = fzp::launch_col_pass_split(ih.dev, r0, r1, (const float2 *)T, chunks[i].nseg, seg_stride,
                                     (uint16_t *)(ws + p.off_Tb[lane]), (float *)(ws + p.off_C[lane]), roi, st,
                                     (const float2 *)T2);
    else
      e = fzp::launch_col_pass(ih.dev, r0, r1, (const double2 *)T, roi, st);
    if (e == hipSuccess) e = end_mark(1, st);
    if (e != hipSuccess) return hip_fail("fzp_propagate_roi_range: column pass", e);
  }
  // every stripe launch on the auxiliary stream was waited for by st
  return FZP_OK;
}

}  // namespace

extern "C" fzp_status_t fzp_propagate_roi_range(fzp_plan_t h, void *workspace, double *roi_dev, int64_t row_begin,
                                                int64_t row_end, int32_t accumulate, void *stream) {
  if (!h || !workspace || !roi_dev) return fail(FZP_E_INVAL, "fzp_propagate_roi_range: NULL argument");
  Plan &p = h->plan;
  if (row_begin < 0 || row_end < row_begin || row_end > p.ap.N)
    return fail(FZP_E_INVAL, "fzp_propagate_roi_range: need 0 <= row_begin <= row_end <= N");
  if (p.opt.path == FZP_PATH_SA_CZT && row_end > row_begin && (row_begin != 0 || row_end != p.ap.N))
    return fail(FZP_E_UNSUPPORTED, "fzp_propagate_roi_range: the non-paraxial path takes whole apertures only");
  if (p.prepared_ws != workspace) {
    const fzp_status_t s = fzp_prepare(h, workspace, stream);
    if (s != FZP_OK) return s;
  }
  hipStream_t st = (hipStream_t)stream;
  char *ws = (char *)workspace;
  hipError_t e;
  if (!accumulate) {
    e = fzp::launch_zero(roi_dev, 2 * p.roi_elems, st);
    if (e != hipSuccess) return hip_fail("fzp_propagate_roi_range: zero", e);
  }
  if (p.opt.path == FZP_PATH_SA_CZT) {
    // the angular spectrum needs the whole aperture at once
    if (row_end <= row_begin) return FZP_OK;
    if (row_begin != 0 || row_end != p.ap.N)
      return fail(FZP_E_UNSUPPORTED, "fzp_propagate_roi_range: the non-paraxial path takes whole apertures only");
    for (auto &ih : p.inst) {
      const fzp_status_t s = enqueue_sa(p, ih, ws, (double2 *)roi_dev + ih.roi_off, st);
      if (s != FZP_OK) return s;
    }
    return FZP_OK;
  }
  const int lanes = p.lanes < (int)p.inst.size() ? p.lanes : (int)p.inst.size();
  if (lanes <= 1) {
    for (auto &ih : p.inst) {
      const fzp_status_t s =
          enqueue_instance(p, ih, 0, ws, (double2 *)roi_dev + ih.roi_off, row_begin, row_end, st);
      if (s != FZP_OK) return s;
    }
    return FZP_OK;
  }
  // fork: every lane stream waits for the work already on st
  e = ensure_lanes(p);
  if (e == hipSuccess) e = hipEventRecord(p.lane_ev[0], st);
  for (int l = 0; l < lanes && e == hipSuccess; ++l) e = hipStreamWaitEvent(p.lane_st[l], p.lane_ev[0], 0);
  if (e != hipSuccess) return hip_fail("fzp_propagate_roi_range: fork", e);
  // instances dealt round robin to the lanes
  for (size_t k = 0; k < p.inst.size(); ++k) {
    InstHost &ih = p.inst[k];
    const int l = (int)(k % (size_t)lanes);
    const fzp_status_t s =
        enqueue_instance(p, ih, l, ws, (double2 *)roi_dev + ih.roi_off, row_begin, row_end, p.lane_st[l]);
    if (s != FZP_OK) return s;
  }
  // join: st waits for every lane
  for (int l = 0; l < lanes && e == hipSuccess; ++l) {
    e = hipEventRecord(p.lane_ev[1 + l], p.lane_st[l]);
    if (e == hipSuccess) e = hipStreamWaitEvent(st, p.lane_ev[1 + l], 0);
  }
  if (e != hipSuccess) return hip_fail("fzp_propagate_roi_range: join", e);
  return FZP_OK;
}

extern "C" fzp_status_t fzp_propagate_roi(fzp_plan_t h, void *workspace, double *roi_dev, void *stream) {
  if (!h) return fail(FZP_E_INVAL, "fzp_propagate_roi: NULL plan");
  return fzp_propagate_roi_range(h, workspace, roi_dev, 0, h->plan.ap.N, 0, stream);
}

uint64_t fzp::plan_serial(fzp_plan_t h) { return h->plan.serial; }

size_t fzp::plan_workspace_bytes(fzp_plan_t h) { return h->plan.ws_bytes; }

fzp_status_t fzp::propagate_fixed_workspace(fzp_plan_t h, char *ws, bool tables_current, double *roi_dev,
                                            hipStream_t stream) {
  Plan &p = h->plan;
  if (tables_current) {
    // the tables in ws are this plan's: only the device pointers are re-bound
    bind_tables(p, ws);
    p.prepared_ws = ws;
  } else {
    const fzp_status_t s = fzp_prepare(h, ws, stream);
    if (s != FZP_OK) return s;
  }
  // one lane on the caller's stream, no profiling events and no auxiliary
  // stream: nothing is created (lanes give the same bits as one lane)
  const int32_t lanes = p.lanes;
  const bool prof = p.profile;
  const int32_t flags = p.opt.flags;
  p.lanes = 1;
  p.profile = false;
  p.opt.flags &= ~FZP_FLAG_OVERLAP_OPERAND;
  const fzp_status_t s = fzp_propagate_roi_range(h, ws, roi_dev, 0, p.ap.N, 0, stream);
  p.lanes = lanes;
  p.profile = prof;
  p.opt.flags = flags;
  return s;
}

namespace {

// FNV-1a over everything that fixes the bits of a plan's ROI.
struct Fnv {
  uint64_t h = 1469598103934665603ull;
  void bytes(const void *p, size_t n) {
    const unsigned char *c = (const unsigned char *)p;
    for (size_t i = 0; i < n; ++i) h = (h ^ c[i]) * 1099511628211ull;
  }
  template <typename T> void put(const T &v) { bytes(&v, sizeof(v)); }
};

uint64_t plan_fingerprint(const Plan &p) {
  Fnv f;
  f.put(p.ap.D), f.put(p.ap.f0), f.put(p.ap.lambda0), f.put(p.ap.pitch), f.put(p.ap.N);
  f.put(p.ap.centre_open), f.put(p.ap.levels), f.put(p.opt.path), f.put(p.chunk_rows), f.put(p.seg_len);
  f.put(p.bin_variant), f.put(p.roi_elems), f.put(p.inst[0].dev.i8);
  for (const auto &ih : p.inst) {
    f.put(ih.in.lambda), f.put(ih.in.z), f.put(ih.in.x0), f.put(ih.in.y0), f.put(ih.in.half_width);
    f.put(ih.in.M), f.put(ih.in.n_creases);
    for (const auto &c : ih.creases) f.put(c.theta), f.put(c.offset), f.put(c.width), f.put(c.height);
  }
  return f.h;
}

constexpr char kCkptMagic[8] = {'F', 'Z', 'P', 'C', 'K', 'P', 'T', '1'};

struct CkptHeader {
  char magic[8];
  uint64_t fingerprint;
  int64_t roi_elems;  // complex elements
  int64_t next_row;
};

}  // namespace

extern "C" fzp_status_t fzp_propagate_resumable(fzp_plan_t h, void *workspace, double *roi_dev, const char *path,
                                                int64_t rows_per_checkpoint, int64_t max_rows, int32_t keep,
                                                int64_t *next_row, void *stream) {
  if (!h || !workspace || !roi_dev || !path) return fail(FZP_E_INVAL, "fzp_propagate_resumable: NULL argument");
  if (rows_per_checkpoint < 0 || max_rows < 0)
    return fail(FZP_E_INVAL, "fzp_propagate_resumable: negative row count");
  try {
    Plan &p = h->plan;
    const int64_t N = p.ap.N;
    // the non-paraxial path runs the whole aperture as one block
    const int64_t chunk = p.opt.path == FZP_PATH_SA_CZT ? N : (p.chunk_rows > 0 ? p.chunk_rows : N);
    int64_t block = rows_per_checkpoint > 0 ? rows_per_checkpoint : chunk;
    block = (block + chunk - 1) / chunk * chunk;
    hipStream_t st = (hipStream_t)stream;
    const uint64_t fp = plan_fingerprint(p);
    const size_t nbytes = (size_t)p.roi_elems * 2 * sizeof(double);
    std::vector<double> host((size_t)p.roi_elems * 2);
    int64_t row = 0;
    bool have_roi = false;
    if (FILE *f = std::fopen(path, "rb")) {
      CkptHeader hd;
      const bool ok = std::fread(&hd, sizeof(hd), 1, f) == 1 && std::memcmp(hd.magic, kCkptMagic, 8) == 0 &&
                      hd.roi_elems == p.roi_elems && hd.next_row >= 0 && hd.next_row <= N &&
                      (hd.next_row % chunk == 0 || hd.next_row == N) &&
                      std::fread(host.data(), 1, nbytes, f) == nbytes;
      std::fclose(f);
      if (!ok) return fail(FZP_E_INVAL, std::string("fzp_propagate_resumable: malformed checkpoint ") + path);
      if (hd.fingerprint != fp)
        return fail(FZP_E_INVAL, std::string("fzp_propagate_resumable: ") + path + " belongs to another plan");
      hipError_t e = hipMemcpyAsync(roi_dev, host.data(), nbytes, hipMemcpyHostToDevice, st);
      if (e == hipSuccess) e = hipStreamSynchronize(st);
      if (e != hipSuccess) return hip_fail("fzp_propagate_resumable: restore", e);
      row = hd.next_row;
      have_roi = true;
    }
    const std::string tmp = std::string(path) + ".tmp";
    int64_t done = 0;
    while (row < N && (max_rows == 0 || done < max_rows)) {
      const int64_t r1 = row + block < N ? row + block : N;
      fzp_status_t s = fzp_propagate_roi_range(h, workspace, roi_dev, row, r1, have_roi ? 1 : 0, stream);
      if (s != FZP_OK) return s;
      have_roi = true;
      done += r1 - row;
      row = r1;
      hipError_t e = hipMemcpyAsync(host.data(), roi_dev, nbytes, hipMemcpyDeviceToHost, st);
      if (e == hipSuccess) e = hipStreamSynchronize(st);
      if (e != hipSuccess) return hip_fail("fzp_propagate_resumable: checkpoint copy", e);
      CkptHeader hd;
      std::memcpy(hd.magic, kCkptMagic, 8);
      hd.fingerprint = fp;
      hd.roi_elems = p.roi_elems;
      hd.next_row = row;
      FILE *f = std::fopen(tmp.c_str(), "wb");
      bool ok = f && std::fwrite(&hd, sizeof(hd), 1, f) == 1 && std::fwrite(host.data(), 1, nbytes, f) == nbytes;
      if (f) ok = (std::fclose(f) == 0) && ok;
      if (!ok || std::rename(tmp.c_str(), path) != 0)
        return fail(FZP_E_DEVICE, std::string("fzp_propagate_resumable: cannot write ") + path);
    }
    if (!have_roi) {  // an aperture with no rows to run: the ROI is zero
      const hipError_t e = fzp::launch_zero(roi_dev, 2 * p.roi_elems, st);
      if (e != hipSuccess) return hip_fail("fzp_propagate_resumable: zero", e);
    }
    if (next_row) *next_row = row;
    if (row >= N && !keep) std::remove(path);
    return FZP_OK;
  } catch (const std::bad_alloc &) {
    return fail(FZP_E_NOMEM, "fzp_propagate_resumable: out of host memory");
  } catch (const std::exception &e) {
    return fail(FZP_E_INVAL, std::string("fzp_propagate_resumable: ") + e.what());
  }
}

extern "C" fzp_status_t fzp_metrics(fzp_plan_t h, void *workspace, const double *roi_dev, fzp_metrics_t *out_host,
                                    void *stream) {
  if (!h || !workspace || !roi_dev || !out_host) return fail(FZP_E_INVAL, "fzp_metrics: NULL argument");
  Plan &p = h->plan;
  if (p.prepared_ws != workspace) {
    const fzp_status_t s = fzp_prepare(h, workspace, stream);
    if (s != FZP_OK) return s;
  }
  hipStream_t st = (hipStream_t)stream;
  char *ws = (char *)workspace;
  char *scratch = ws + p.off_scratch;
  // the instances' kernels run one after another on `st` (they share the
  // scratch); each writes its own result record, copied back in one transfer
  fzp_metrics_t *dev_out = (fzp_metrics_t *)(scratch + fzp::metrics_scratch_bytes(p.Mmax));
  for (size_t k = 0; k < p.inst.size(); ++k) {
    const InstHost &ih = p.inst[k];
    const hipError_t e = fzp::launch_metrics(ih.dev, (const double2 *)roi_dev + ih.roi_off,
                                             (double)p.disc_samples, scratch, dev_out + k, st);
    if (e != hipSuccess) return hip_fail("fzp_metrics: kernels", e);
  }
  hipError_t e = hipMemcpyAsync(out_host, dev_out, p.inst.size() * sizeof(fzp_metrics_t), hipMemcpyDeviceToHost, st);
  if (e != hipSuccess) return hip_fail("fzp_metrics: copy", e);
  e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail("fzp_metrics: synchronize", e);
  return FZP_OK;
}

extern "C" fzp_status_t fzp_profile_enable(fzp_plan_t h, int32_t on) {
  if (!h) return fail(FZP_E_INVAL, "fzp_profile_enable: NULL plan");
  h->plan.profile = on != 0;
  return FZP_OK;
}

extern "C" fzp_status_t fzp_profile_read(fzp_plan_t h, double *row_ms, int64_t *row_launches, double *col_ms,
                                         int64_t *col_launches, double *aux_ms, int64_t *aux_launches,
                                         int32_t reset) {
  if (!h) return fail(FZP_E_INVAL, "fzp_profile_read: NULL plan");
  Plan &p = h->plan;
  for (const auto &mk : p.ev_marks) {
    hipError_t e = hipEventSynchronize(p.ev_pool[mk.first + 1]);
    if (e != hipSuccess) return hip_fail("fzp_profile_read: synchronize", e);
    float ms = 0.0f;
    e = hipEventElapsedTime(&ms, p.ev_pool[mk.first], p.ev_pool[mk.first + 1]);
    if (e != hipSuccess) return hip_fail("fzp_profile_read: elapsed", e);
    if (mk.second == 0) {
      p.row_ms += ms;
      ++p.row_n;
    } else if (mk.second == 1) {
      p.col_ms += ms;
      ++p.col_n;
    } else {
      p.aux_ms += ms;
      ++p.aux_n;
    }
  }
  p.ev_marks.clear();
  p.ev_used = 0;
  if (row_ms) *row_ms = p.row_ms;
  if (row_launches) *row_launches = p.row_n;
  if (col_ms) *col_ms = p.col_ms;
  if (col_launches) *col_launches = p.col_n;
  if (aux_ms) *aux_ms = p.aux_ms;
  if (aux_launches) *aux_launches = p.aux_n;
  if (reset) {
    p.row_ms = p.col_ms = p.aux_ms = 0.0;
    p.row_n = p.col_n = p.aux_n = 0;
  }
  return FZP_OK;
}

// ---------------------------------------------------------------------------
// Graph capture of a whole propagation
// ---------------------------------------------------------------------------

struct fzp_graph_s {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  ~fzp_graph_s() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
  }
};

extern "C" fzp_status_t fzp_graph_create(fzp_plan_t h, void *workspace, double *roi_dev, fzp_graph_t *out) {
  if (!h || !workspace || !roi_dev || !out) return fail(FZP_E_INVAL, "fzp_graph_create: NULL argument");
  *out = nullptr;
  Plan &p = h->plan;
  // a capture with the operand overlap ended in a host segmentation fault
  // (cause not found): refused before any device call
  if (p.opt.path == FZP_PATH_SPLIT_BF16 && (p.opt.flags & FZP_FLAG_OVERLAP_OPERAND))
    return fail(FZP_E_UNSUPPORTED, "fzp_graph_create: FZP_FLAG_OVERLAP_OPERAND cannot be captured");
  hipStream_t cs = nullptr;
  hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
  if (e != hipSuccess) return hip_fail("fzp_graph_create: stream", e);
  // tables, kernel attributes and lane streams exist before the capture starts
  fzp_status_t s = fzp_prepare(h, workspace, cs);
  if (s == FZP_OK) {
    e = hipStreamSynchronize(cs);
    if (e == hipSuccess) e = ensure_lanes(p);
    if (e != hipSuccess) s = hip_fail("fzp_graph_create: prepare", e);
  }
  if (s != FZP_OK) {
    (void)hipStreamDestroy(cs);
    return s;
  }
  auto *g = new (std::nothrow) fzp_graph_s;
  if (!g) {
    (void)hipStreamDestroy(cs);
    return fail(FZP_E_NOMEM, "fzp_graph_create: out of host memory");
  }
  const bool prof = p.profile;
  p.profile = false;
  e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    p.capturing = true;
    s = fzp_propagate_roi_range(h, workspace, roi_dev, 0, p.ap.N, 0, cs);
    p.capturing = false;
    hipGraph_t graph = nullptr;
    const hipError_t e2 = hipStreamEndCapture(cs, &graph);
    g->graph = graph;
    if (s == FZP_OK && e2 != hipSuccess) s = hip_fail("fzp_graph_create: end capture", e2);
    if (s == FZP_OK) {
      e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
      if (e != hipSuccess) s = hip_fail("fzp_graph_create: instantiate", e);
    }
  } else {
    s = hip_fail("fzp_graph_create: begin capture", e);
  }
  p.profile = prof;
  (void)hipStreamDestroy(cs);
  if (s != FZP_OK) {
    delete g;
    return s;
  }
  *out = g;
  return FZP_OK;
}

extern "C" fzp_status_t fzp_graph_launch(fzp_graph_t g, void *stream) {
  if (!g || !g->exec) return fail(FZP_E_INVAL, "fzp_graph_launch: NULL graph");
  const hipError_t e = hipGraphLaunch(g->exec, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail("fzp_graph_launch", e);
  return FZP_OK;
}

extern "C" void fzp_graph_destroy(fzp_graph_t g) { delete g; }

// ---------------------------------------------------------------------------
// Autotuner
// ---------------------------------------------------------------------------

namespace {

void set_decomposition(Plan &p, int64_t seg_len, int32_t variant) {
  p.seg_len = seg_len;
  for (auto &ih : p.inst) ih.dev.seg_len = seg_len;
  set_variant(p, variant);
}

// Plan shape and device: what the best decomposition depends on.
std::string tune_key(const Plan &p) {
  std::ostringstream k;
  int dev = 0;
  hipDeviceProp_t prop;
  std::string arch = "unknown";
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) arch = prop.gcnArchName;
  for (char &c : arch)
    if (c == ' ' || c == ':') c = '_';
  k << "fzp1/" << arch << "/N" << p.ap.N << "/path" << p.opt.path << "/chunk" << p.chunk_rows << "/L"
    << p.lanes_max;
  if (p.ap.levels != 0) k << "/phase" << p.ap.levels;
  if (!p.inst.empty() && p.inst[0].dev.i8) k << "/i8";  // the int8 row pass times differently
  // the multiset of (M, deformed) over instances, in instance order
  for (const auto &ih : p.inst) k << "/" << ih.dev.M << (ih.dev.n_creases > 0 ? "c" : "f");
  return k.str();
}

bool cache_lookup(const char *path, const std::string &key, int64_t &seg_len, int32_t &lanes, int32_t &tile) {
  if (!path) return false;
  std::ifstream f(path);
  std::string line;
  bool found = false;
  while (std::getline(f, line)) {
    std::istringstream ls(line);
    std::string k;
    int64_t sl;
    int32_t ln, tl;
    if (ls >> k >> sl >> ln >> tl && k == key) {
      seg_len = sl;
      lanes = ln;
      tile = tl;
      found = true;  // the last entry wins
    }
  }
  return found;
}

}  // namespace

extern "C" fzp_status_t fzp_autotune(fzp_plan_t h, void *workspace, double *roi_dev, void *stream,
                                     const char *cache_path, int64_t *seg_len_out, int32_t *lanes_out,
                                     int32_t *variant_out, double *ms_out) {
  if (!h || !workspace || !roi_dev) return fail(FZP_E_INVAL, "fzp_autotune: NULL argument");
  try {
    Plan &p = h->plan;
    hipStream_t st = (hipStream_t)stream;
    const bool split = p.opt.path == FZP_PATH_SPLIT_BF16;
    const int64_t seg0 = p.seg_len;
    // candidates: the default segment and its doublings (fewer partial planes,
    // so they fit the plan's T buffers), both binary-stripe GEMM tiles, and
    // every lane count
    std::vector<int64_t> segs{seg0};
    const int32_t cur = p.bin_variant + 8 * p.cplx_variant;
    std::vector<int32_t> tiles{cur};
    if (split) {
      for (int64_t sl = 2 * seg0; sl <= 65536 && sl < 2 * p.ap.N; sl *= 2) segs.push_back(sl);
      // binary-stripe variants where a binary mask GEMM runs, complex-stripe
      // tiles where a complex stripe does
      bool binary = false, cplx = false;
      for (const auto &ih : p.inst) {
        const bool c = ih.dev.n_creases > 0 || (ih.dev.levels != 0 && ih.dev.levels != 2 && ih.dev.levels != 4);
        cplx = cplx || c;
        binary = binary || !c;
      }
      std::vector<int32_t> bs{p.bin_variant}, cs{p.cplx_variant};
      if (binary && !p.inst[0].dev.i8) bs = {0, 1, 2, 3, 4};  // the int8 row pass has one form
      if (cplx && !p.inst[0].dev.i8) cs = {0, 1, 2};  // the int8 complex row pass has one form
      tiles.clear();
      for (int32_t c : cs)
        for (int32_t b : bs) tiles.push_back(b + 8 * c);
    }
    const std::string key = tune_key(p);
    int64_t best_seg = seg0;
    int32_t best_lanes = p.lanes_max, best_tile = cur;
    double best_ms = 0.0;
    if (cache_lookup(cache_path, key, best_seg, best_lanes, best_tile) && best_lanes >= 1 &&
        best_lanes <= p.lanes_max && std::find(segs.begin(), segs.end(), best_seg) != segs.end() &&
        best_tile >= 0 && best_tile % 8 <= 4 && best_tile / 8 <= 2) {
      set_decomposition(p, best_seg, best_tile);
      p.lanes = best_lanes;
    } else {
      const bool prof = p.profile;
      p.profile = false;
      hipEvent_t a = nullptr, b = nullptr;
      hipError_t e = hipEventCreate(&a);
      if (e == hipSuccess) e = hipEventCreate(&b);
      fzp_status_t s = e == hipSuccess ? FZP_OK : hip_fail("fzp_autotune: events", e);
      best_ms = std::numeric_limits<double>::infinity();
      for (int32_t ln = 1; ln <= p.lanes_max && s == FZP_OK; ++ln) {
        for (int64_t sl : segs) {
          for (int32_t tl : tiles) {
            set_decomposition(p, sl, tl);
            p.lanes = ln;
            // one untimed run (first use of the lanes, caches), then one timed run
            s = fzp_propagate_roi(h, workspace, roi_dev, stream);
            if (s != FZP_OK) break;
            e = hipEventRecord(a, st);
            if (e != hipSuccess) {
              s = hip_fail("fzp_autotune: record", e);
              break;
            }
            s = fzp_propagate_roi(h, workspace, roi_dev, stream);
            if (s != FZP_OK) break;
            e = hipEventRecord(b, st);
            if (e == hipSuccess) e = hipEventSynchronize(b);
            float ms = 0.0f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
            if (e != hipSuccess) {
              s = hip_fail("fzp_autotune: timing", e);
              break;
            }
            if (ms < best_ms) {
              best_ms = ms;
              best_seg = sl;
              best_lanes = ln;
              best_tile = tl;
            }
          }
          if (s != FZP_OK) break;
        }
      }
      if (a) (void)hipEventDestroy(a);
      if (b) (void)hipEventDestroy(b);
      p.profile = prof;
      set_decomposition(p, best_seg, best_tile);
      p.lanes = best_lanes;
      if (s != FZP_OK) return s;
      if (cache_path) {
        std::ofstream f(cache_path, std::ios::app);
        if (f) f << key << " " << best_seg << " " << best_lanes << " " << best_tile << "\n";
      }
    }
    if (seg_len_out) *seg_len_out = best_seg;
    if (lanes_out) *lanes_out = best_lanes;
    if (variant_out) *variant_out = best_tile;
    if (ms_out) *ms_out = best_ms;
    return FZP_OK;
  } catch (const std::exception &ex) {
    return fail(FZP_E_INVAL, std::string("fzp_autotune: ") + ex.what());
  } catch (...) {
    return fail(FZP_E_INVAL, "fzp_autotune: unknown error");
  }
}
