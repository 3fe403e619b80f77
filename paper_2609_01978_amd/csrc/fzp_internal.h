// Internal structures shared by the host plan (fzp_plan.cpp) and the kernel
// launchers (*.hip).  Not part of the public ABI.
#pragma once

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include <hip/hip_runtime.h>

#include "fzp.h"

namespace fzp {

constexpr int kFftLen = 4096;     // Bluestein block FFT length (LDS resident)
constexpr int kFftThreads = 256;  // threads per FFT work-group
constexpr int kMaxCreases = 64;
constexpr int kMaxM = 2048;
// int8 split table: the kernel row in units of 1 / 16256, 16256 = 127 * 128 the
// largest scale whose two balanced int8 digits (v = 128 v0 + v1, v1 in
// [-64, 63]) keep v0 in [-127, 127]
constexpr double kI8Scale = 16256.0;

// Per-crease constants, precomputed on the host in float64:
// h_k(x,y) = H_k exp(-(x cos + y sin - rho)^2 * inv2s2)
struct CreaseDev {
  double c, s, rho, inv2s2, h_over_lambda;  // height / lambda (turns)
  double pad[3];
};

// Everything a kernel needs to know about one instance.
struct InstDev {
  // aperture
  int64_t N;
  double kappa;     // dx*dx / (4 lambda0 f0)
  double kmax;      // K_max, exact integer in float64
  int32_t centre_open;
  int32_t M;
  int32_t B;        // Bluestein block length (kFftLen - M + 1)
  int32_t n_creases;
  double dx;
  // CZT (Eq. 10) in turns: phase(i, q) = beta c_i^2 / 2 - alpha c_i d_q,
  // c_i = i - (N-1)/2, d_q = q - M/2 + s
  double alpha, beta;
  double sx, sy;
  // output factor e^{ikz}/(i lambda z) dx^2 e^{i pi (x'^2+y'^2)/(lambda z)}
  double kz_turns;  // frac(z / lambda) - 1/4
  double scale;     // dx^2 / (lambda z)
  double x0, y0, dx_out, inv2lz;  // inv2lz = 1 / (2 lambda z)
  // metrics: r_null^2, (R^2/(lambda z))^2, MTF read point in radial bins
  double rnull2, R2_over_lz2, t_mtf;
  // device tables (pointers into the workspace)
  const double2 *Hx, *Hy;  // FFT_L(h) / L, h[k] = e^{i pi alpha (k - M/2 + s)^2}
  const double2 *Dt;       // e^{i pi (beta - alpha) n^2}, n < L
  const double2 *Qx, *Qy;  // e^{-i pi alpha d^2}
  const CreaseDev *cr;
  const double2 *lev;      // phase plates: exp(-2 pi i l / L), l = 0 .. L-1
  const double2 *S;        // split path, 2-level plate: prefix sums over i of the row kernel,
                           // S[i][q] = sum_{i' < i} e^{2 pi i (beta c_i'^2/2 - alpha c_i' d_q)}, (Npad+1) x M
  const uint16_t *A;       // split path: [2 planes][2M cols][Npad] bf16
  const uint16_t *By;      // split path: column kernel matrix, [4 planes][Npad/16][M padded to 256][16] bf16
  int64_t Npad;
  int64_t seg_len;         // split path: K columns per float32 partial sum (power of two)
  int32_t bin_tile_rows;   // split path, binary stripes: GEMM tile rows (512 or 256)
  int32_t bin_ring;        // split path, binary stripes, 512-row tile: LDS pipeline stages (4 or 8)
  int32_t bin_prefetch;    // 8-stage variant: 1 next-stage operands one stage early, 2 interleaved expansion
  int32_t cplx_tile;       // split path, complex stripes: 0 the 256-column GEMM tile, 1 the 128-column tile,
                           // 2 the 128-column tile with a 2-stage ring, two work-groups per CU
  int32_t i8;              // split path, binary stripes on the int8 matrix cores (FZP_FLAG_SPLIT_INT8):
                           // table A as two int8 digit planes [2][Npad/64][2M][64]
  int32_t levels;          // 0: binary amplitude plate; L >= 2: L-level phase plate
  double kappa_l;          // phase plates: kappa * (L / 2); level = floor(K kappa_l) mod L
};

// Non-paraxial variant (fzp_sa.hip): the padded grid, its two FFT factors
// with their radix sequences, the aperture rule and the transfer function.
constexpr int kSaMaxStages = 12;
struct SaDev {
  int64_t Np;              // padded samples per side, Np = n1 n2
  int64_t N, off;          // aperture samples per side; its first sample in the padded grid
  int32_t n1, n2;          // LDS transform lengths (<= 1024)
  int32_t nst1, nst2;      // radix stages of n1 and n2
  int32_t rad1[kSaMaxStages], rad2[kSaMaxStages];
  int32_t radii_eq3;       // 1: sag-corrected radii (Eq. 3), 0: paraxial radii (Eq. 4)
  int32_t centre_open, n_creases;
  double kmax_disc;        // K_max of the aperture disc (exact integer)
  double c1, c2;           // Eq. 3 zone index floor(c2 q / (sqrt(1 + q) + 1)), q = K c1
  double kappa;            // Eq. 4 zone index floor(K kappa)
  double dx;
  double inv_lam, inv_lam2;  // 1 / lambda and its square
  double coef;             // d lambda / k_fit (the fitted quadratic's K^2 term, per rho^2)
  double z;                // propagation distance
  double inv_L2;           // 1 / (Np dx)^2: rho^2 per squared frequency index
  double norm;             // 1 / Np^2 (the unnormalised inverse transform)
  const CreaseDev *cr;
  const double2 *twNp, *tw1, *tw2;  // W_Np^m, W_n1^k, W_n2^k
};

struct InstHost {
  fzp_instance_t in;  // creases pointer cleared
  std::vector<fzp_crease_t> creases;
  double lam, z, hw, dx_out;
  InstDev dev;
  size_t off_Hx, off_Hy, off_Dt, off_Qx, off_Qy, off_cr, off_A, off_By, off_S;
  int64_t roi_off;     // complex elements
  SaDev sa;            // FZP_PATH_SA_CZT: the padded-grid pass parameters
  double Z = 0.0;      // FZP_PATH_SA_CZT: the zoom's lambda z
  int32_t table_owner; // instance whose split table this one shares (itself if none)
  int32_t col_owner;   // instance whose column table (B_y) this one shares (itself if none)
};

struct Plan {
  uint64_t serial = 0;  // unique per plan in the process (fzp_plan)
  fzp_aperture_t ap;
  fzp_options_t opt;
  double dx;
  double kappa;
  int64_t kmax;
  int64_t disc_samples;
  int32_t S;
  int64_t chunk_rows;
  int32_t Mmax;
  std::vector<InstHost> inst;
  int64_t roi_elems;
  // stripe buffers, one set per lane: row-pass result T, zone-mask bits and
  // complex stripe planes (split path)
  size_t T_bytes = 0, bits_bytes = 0, G_bytes = 0, Tb_bytes = 0, C_bytes = 0;
  int32_t mask_sets = 1;  // binary masks (mask bits and T planes) per chunk: 2 for 4-level plates
  std::vector<size_t> off_T, off_bits, off_G, off_Tb, off_C;
  int32_t lanes_max = 1, lanes = 1;
  int64_t seg_len = 0;  // split path K segment (all instances)
  int32_t cplx_variant = 0;  // split path complex-stripe GEMM tile (InstDev::cplx_tile)
  int32_t bin_variant = 4;  // split path binary-stripe GEMM: 0 512 rows, 1 256 rows, 2 512 rows deep ring,
                            // 3 deep ring with next-stage fragment prefetch, 4 deep ring interleaved
  std::vector<hipStream_t> lane_st;
  std::vector<hipEvent_t> lane_ev;  // [0] fork, [1 + l] join of lane l
  std::vector<hipStream_t> aux_st;  // split path: stripe-operand stream of each lane
  std::vector<hipEvent_t> aux_ev;   // 5 per lane: fork, operand ready x2, GEMM done x2
  bool capturing = false;           // inside fzp_graph_create's stream capture
  // FZP_PATH_SA_CZT: padded field U1 (Np^2 complex) and the twiddle tables
  size_t off_U1 = 0, off_twNp = 0, off_tw1 = 0, off_tw2 = 0;
  size_t off_scratch, scratch_bytes;
  size_t ws_bytes;
  const void *prepared_ws = nullptr;
  // kernel timing (fzp_profile_*)
  bool profile = false;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  std::vector<std::pair<size_t, int>> ev_marks;  // (first event index, 0 = row / 1 = column / 2 = mask bits)
  double row_ms = 0.0, col_ms = 0.0, aux_ms = 0.0;
  int64_t row_n = 0, col_n = 0, aux_n = 0;
  ~Plan();
};

// Thread-local text returned by fzp_last_error (fzp_plan.cpp).
void set_last_error(const std::string &msg);

// One whole propagation of the plan on one lane of `stream` with the workspace
// at `ws` (fzp_plan.cpp), for fzp_propagate_roi_static: the tables are built
// there unless `tables_current` says the last plan prepared in it was this one;
// no stream, event or device memory is created.
fzp_status_t propagate_fixed_workspace(fzp_plan_t h, char *ws, bool tables_current, double *roi_dev,
                                       hipStream_t stream);
uint64_t plan_serial(fzp_plan_t h);
size_t plan_workspace_bytes(fzp_plan_t h);

// ---- launchers (fzp_fft.hip, fzp_gemm.hip, fzp_metrics.hip) ----
hipError_t launch_build_tables(const Plan &p, const InstHost &ih, char *ws, hipStream_t st);
hipError_t launch_build_split_table(const Plan &p, const InstHost &ih, char *ws, hipStream_t st);
hipError_t init_split_attributes();  // kernel attributes of the split GEMMs (outside graph capture)
hipError_t init_cplx_attributes();   // the complex-stripe GEMM's part of it (fzp_cplx.hip)
hipError_t launch_zero(double *buf, int64_t n_doubles, hipStream_t st);
hipError_t launch_row_pass_fp64(const InstDev &d, int64_t row_begin, int64_t row_end, double2 *T,
                                hipStream_t st);
// Split row pass: writes split_segments(d) partial results, each chunk_rows x M
// complex float32, seg_stride complex elements apart.
int split_segments(const InstDev &d);
size_t split_bits_bytes(const InstDev &d, int64_t chunk_rows);  // zone-mask bit buffer of one chunk
// K segments [seg_lo, seg_hi) holding disc samples of rows [row_begin, row_end);
// the split row pass writes exactly these partials, the first at T.
void split_seg_range(const InstDev &d, int64_t row_begin, int64_t row_end, int &seg_lo, int &seg_hi);
// bits2 (4-level plates, see four_level_fast): both masks in one pass, the odd
// zones into bits and the levels 1 and 2 into bits2
hipError_t launch_mask_bits(const InstDev &d, int64_t row_begin, int64_t row_end, uint32_t *bits, hipStream_t st,
                            uint32_t *bits2 = nullptr);
// Deformed (complex) stripes on the split path: the BF16 hi/lo stripe planes of
// one chunk (split_stripe_bytes for chunk_rows rows), then the complex GEMM.
void split_chunk_chord(const InstDev &d, int64_t row_begin, int64_t row_end, int64_t &lo, int64_t &hi);
size_t split_stripe_bytes(const InstDev &d, int64_t chunk_rows);
hipError_t launch_stripe_cplx(const InstDev &d, int64_t row_begin, int64_t row_end, uint16_t *G, hipStream_t st);
hipError_t launch_row_pass_split_cplx(const InstDev &d, int64_t row_begin, int64_t row_end, float2 *T,
                                      int64_t seg_stride, const uint16_t *G, hipStream_t st);
hipError_t launch_row_pass_split(const InstDev &d, int32_t S, int64_t row_begin, int64_t row_end,
                                 float2 *T, int64_t seg_stride, const uint32_t *bits, hipStream_t st);
// Int8 form of the binary row pass (fzp_i8.hip, d.i8): the digit table in the
// split table's space, then the same partial planes as launch_row_pass_split,
// holding int32 sums in units of 1 / kI8Scale.
int64_t bits_rows_pad(int64_t rows);  // mask-bit rows of a chunk, padded to the 512-row tile
hipError_t launch_build_i8_table(const InstHost &ih, char *ws, hipStream_t st);
hipError_t init_i8_attributes();  // its LDS attribute (outside graph capture)
// the chunk's zone-mask bits in the int8 row pass's word order (Npad a multiple of 128)
hipError_t launch_mask_bits_i8(const InstDev &d, int64_t row_begin, int64_t row_end, uint32_t *bits, hipStream_t st,
                               uint32_t *bits2 = nullptr);
hipError_t launch_row_pass_i8(const InstDev &d, int64_t row_begin, int64_t row_end, float2 *T, int64_t seg_stride,
                              const uint32_t *bits, hipStream_t st);
// Complex stripes on the int8 matrix cores (launch_stripe_cplx writes their
// int8 digit planes when d.i8): partials laid out as launch_row_pass_split's,
// in units of 1 / kI8Scale^2.
void split_stripe_extent(const InstDev &d, int64_t row_begin, int64_t row_end, int64_t &rows_pad, int64_t &kb0,
                         int64_t &nkb);
hipError_t launch_row_pass_i8_cplx(const InstDev &d, int64_t row_begin, int64_t row_end, float2 *T,
                                   int64_t seg_stride, const void *G, hipStream_t st);
hipError_t launch_col_pass(const InstDev &d, int64_t row_begin, int64_t row_end, const double2 *T, double2 *roi,
                           hipStream_t st);  // FP64 path
// Split path column pass as a split-BF16 GEMM (fzp_cplx.hip): the column kernel
// matrix B_y (col_table_bytes, built once per workspace), the chunk's T as a
// BF16 hi/lo operand (col_operand_bytes per lane) and float32 partial planes
// of the product (col_partial_bytes per lane), added in float64 into the ROI.
size_t col_table_bytes(int M, int64_t Npad);
size_t col_operand_bytes(int M, int64_t chunk_rows);
size_t col_partial_bytes(int M, int64_t chunk_rows);
hipError_t launch_build_col_table(const InstDev &d, uint16_t *By, hipStream_t st);
// 2-level phase plates on the split path (fzp_cplx.hip): t = disc - 2 mask
// (mask = the odd zones), so T = T_disc - 2 T_mask with T_mask from the binary
// GEMM and T_disc = S[hi] - S[lo] over each row's disc chord from float64
// prefix sums of the row kernel (prefix_table_bytes, built once per workspace).
bool two_level_fast(const InstDev &d);
// 4-level phase plates without creases on the split path: with the level l of
// a disc sample, (-i)^l = 1 - (1 - i) [l in {2, 3}] - (1 + i) [l in {1, 2}], so
// T = T_disc - (1 - i) T_odd - (1 + i) T_half with two binary-stripe GEMMs (the
// odd zones, and levels 1 and 2) and T_disc from the same prefix sums.
bool four_level_fast(const InstDev &d);
size_t prefix_table_bytes(int M, int64_t Npad);
hipError_t launch_build_prefix_table(const InstDev &d, double2 *S, hipStream_t st);
// T2 (4-level plates): the partial planes of the second mask's GEMM, laid out as T.
hipError_t launch_col_pass_split(const InstDev &d, int64_t row_begin, int64_t row_end, const float2 *T, int nseg,
                                 int64_t seg_stride, uint16_t *Tb, float *C, double2 *roi, hipStream_t st,
                                 const float2 *T2 = nullptr);
// Non-paraxial variant (fzp_sa.hip, fzp_fft.hip): twiddle tables, the
// propagated padded field U1 by seven passes of LDS FFTs, and the CZT zoom's
// row pass over U1's rows (the column pass is launch_col_pass).
hipError_t launch_sa_twiddles(const SaDev &a, double2 *twNp, double2 *tw1, double2 *tw2, hipStream_t st);
hipError_t launch_sa_field(const SaDev &a, double2 *U1, hipStream_t st);
hipError_t init_sa_attributes();
hipError_t launch_row_pass_stored(const InstDev &d, const double2 *U1, int64_t row_begin, int64_t row_end,
                                  double2 *T, hipStream_t st);
hipError_t launch_metrics(const InstDev &d, const double2 *roi, double disc_samples, char *scratch,
                          fzp_metrics_t *dev_out, hipStream_t st);
size_t metrics_scratch_bytes(int32_t M);

}  // namespace fzp
