// Shared device/host descriptors of the polarizability build (gfx950).
//
// The build of one call is a sequence of passes; a pass holds a batch of
// jobs, one job being one (item, tau_j) pair.  Every kernel takes a small
// launch struct by value that points at device tables of these descriptors.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>
#include <vector>

namespace gw {

// compile-time loop: f(integral_constant<int, i>) for i in [B, E)
template <int B, int E, typename F>
__device__ __forceinline__ void sfor(F &&f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    sfor<B + 1, E>(f);
  }
}

enum Prec : int { P_FP64 = 0, P_FP32 = 1, P_BF16X3 = 2 };

// Grid points are padded to a multiple of this in every operand, so that GEMM
// tiles never need row bounds checks on their operand loads.
constexpr int kRowPad = 256;
// Bands are padded to a multiple of this (zero bands).
constexpr int kBandPad = 64;

// ---------------------------------------------------------------------------
// Per-item geometry: FFT grid and the plane-wave sphere tables.
// ---------------------------------------------------------------------------
struct Geo {
  int32_t n0, n1, n2;
  int32_t n_r;
  int32_t n_g;
  int32_t n_disk;          // distinct (k1, k2) pencils touched by the sphere
  int32_t cols;            // columns per plane-FFT block
  int32_t planes;          // i0-planes per plane-FFT block
  const int32_t *disk_i12; // [n_disk] k1*n2 + k2
  const int32_t *slot_of;  // [n_disk][n0] output slot of (pencil d, k0), or -1
  const int32_t *disk_of;  // [n1*n2] pencil d of (k1, k2), or -1
  // real input only (packed transforms): the disk is closed under negation
  const int32_t *disk_pair;  // [n_disk] pencil of (-k1, -k2)
  const int32_t *disk_canon; // [n_canon] pencils d with d <= disk_pair[d]
  int32_t n_canon;
  // half rows (see FftJob::half_rows)
  const int32_t *slot_half;  // [n_disk][n0] compact row of (pencil d, k0), or -1
  const int32_t *hrow;       // [n_half] sphere index of compact row h
  const int32_t *gneg;       // [n_g] sphere index of -G
  int32_t n_half;
};

// Packed real transforms: the plane-FFT block's C lines carry 2C real columns
// (column-grouped in groups of 2C); lines of a job with n real columns.
__host__ __device__ constexpr int packed_lines(int n_cols, int cols) {
  return (n_cols + 2 * cols - 1) / (2 * cols) * cols;
}

// ---------------------------------------------------------------------------
// Staging: FP64 weights and scaled operands in the working layout.
// ---------------------------------------------------------------------------
struct StageOp {            // one (item, occ|unocc) operand, all taus of the pass
  const double *phi;        // band-major [K][N_r] (x2 if complex), FP64
  const int32_t *perm;      // [K] source band of sorted band k
  const double *eps;        // [K] sorted eigenvalues
  double edge;              // HOMO (occ) or LUMO (unocc)
  double sign;              // +1 occ: w = exp((eps-edge) tau); -1 unocc: exp(-(eps-edge) tau)
  int32_t k;                // real band count
  int32_t k_pad;            // padded band count (row pitch in bands)
  int32_t n_r, n_r_pad;
  int32_t cplx;
  int32_t n_jobs;           // taus of this item in the pass
  const double *tau;        // [n_jobs]
  void *const *psi;         // [n_jobs] output operand per tau
};

struct StageLaunch {
  const StageOp *ops;
  const int4 *blocks;       // (op, r-tile, k-tile, 0)
  int32_t n_blocks;
  int32_t prec;
};

// ---------------------------------------------------------------------------
// Fused band contraction + Hadamard product.
// ---------------------------------------------------------------------------
struct GemmJob {
  const void *psi_o;        // [n_r_pad][ld_o] working layout
  const void *psi_u;
  int32_t ld_o, ld_u;       // row pitch in bands
  int32_t k_o, k_u;         // bands to contract, multiple of the K chunk
  int32_t n_r;
  int32_t s0, w;            // slab column range [s0, s0 + w)
  int32_t cg_shift;         // slab columns are grouped by 2^cg_shift
  void *slab;               // [w / 2^cg_shift][n_r][2^cg_shift]: chi out (polarizability),
                            // W~(r, r') in (self-energy), complex working precision
  // self-energy only: the states psi_n [n_states][ld_states] (complex working
  // precision) and this job's partial sums, [slot][n_states][2] (occupied,
  // unoccupied), the slot being the fourth field of a unit
  const void *states;
  int32_t n_states, ld_states;
  double *part;
};

// Work queues of a persistent launch: units [q_off[q], q_off[q + 1]) form
// queue q.  Workgroup b starts on queue b % n_queues (workgroups of a launch
// are dealt to the XCDs in turn, so each queue is served by one XCD and its
// tiles share operand panels in that XCD's L2) and moves on to the next queue
// when its own is empty.
constexpr int kGemmQueues = 8;

struct GemmLaunch {
  const GemmJob *jobs;
  const int4 *units;        // (job, r0, c0, 0)
  int32_t n_units;
  int32_t hermitian;        // 1: units are lower-triangle tiles; mask r >= c
  int32_t *counter;         // n_queues ticket counters, zero before the launch; null: grid stride
  int32_t n_queues;         // 1 .. kGemmQueues
  int32_t q_off[kGemmQueues + 1];
};

// ---------------------------------------------------------------------------
// Sphere FFT over the first index (columns of a slab) or the second
// (rows of chi(G, r')), in two launches:
//   planes : per block of `cols` columns and `planes` i0-planes, 2D FFT over
//            (i1, i2) and gather of the sphere's pencils into tmp;
//   pencils: per (pencil, 256 columns), FFT over i0 and scatter of the sphere
//            points to the output.
// ---------------------------------------------------------------------------
struct FftJob {
  const void *in;           // element (r, c) at in[r * s_r + c * s_col], or, when
  int64_t s_r, s_col;       // s_col == 0, column-grouped: in[((c / C) * n_r + r) * C + c % C]
  void *tmp;                // pencil buffer [(i0 * n_disk + d) * n_cols + c]
  void *out;                // out[slot * o_slot + (col0 + c) * o_col]
  int64_t o_slot, o_col;
  int32_t col0;             // absolute index of column 0 (slab start for the first index)
  int32_t n_cols;
  int32_t geo;
  int32_t unit0_planes;     // first plane-FFT block of this job in the launch
  int32_t unit0_pencils;    // first pencil block of this job in the launch
  // real orbitals with a sphere closed under G -> -G: only the rows G of one
  // half (Geo::hrow) are transformed over the second index.  First index:
  // output row = slot_half (compact row, -1 = not kept).  Second index:
  // column c is row hrow[c]; each result chi(G, G') is also written
  // conjugated at (-G, -G'), which is exact for a real chi(r, r').
  int32_t half_rows;
  // single-launch transform (FftLaunch::fused): output rows column-grouped in
  // groups of 2^o_gshift
  int32_t o_gshift;
};

struct FftLaunch {
  const FftJob *jobs;
  int32_t n_jobs;
  const Geo *geos;
  int32_t n_units_planes;
  int32_t n_units_pencils;
  int32_t in_real;          // input is real
  int32_t lower_only;       // column c holds only rows r >= col0 + c; others read as zero
  int32_t grouped;          // every job's input is column-grouped (s_col == 0)
  int32_t packed;           // real, column-grouped input in groups of 2 * cols: two
                            // real columns per complex transform (pencil units are
                            // (mirror pair, 256 lines))
  int32_t fused;            // single-launch first-index transform (complex FP32,
                            // cubic fft_fusable grids): units are columns, input
                            // column-major (column groups one column wide)
};

// Single-launch transform: sizes, i0-planes per LDS batch (one thread per
// line, 256 threads) and LDS bytes (FP32 points).  Every disk pencil is owned
// by one thread, so n_disk <= 256.
constexpr bool fft_fusable(int n) { return n == 12 || n == 16 || n == 18 || n == 20 || n == 24; }
// (at most 9 16-byte loads per thread and batch, for registers)
__host__ __device__ constexpr int fused_pb(int n) {
  return 256 / n < n ? (256 / n < 4608 / (n * n) ? 256 / n : 4608 / (n * n))
                     : (n < 4608 / (n * n) ? n : 4608 / (n * n));
}
// LDS: the linear stage of one batch (whole KB) and the padded work area
__host__ __device__ constexpr int fused_stage_bytes(int n) {
  return (fused_pb(n) * n * n * 8 + 1023) / 1024 * 1024;
}
constexpr int fused_lds_bytes(int n) { return fused_stage_bytes(n) + 8 * fused_pb(n) * n * (n + 1); }

// ---------------------------------------------------------------------------
// Cosine transform (FP64 accumulation) and norms.
// ---------------------------------------------------------------------------
struct CtItem {
  const void *x;            // [n_tau_x][n_g][n_g] transposed: x_j[g'][g] = chi(G, G', i tau_{j0+j})
  double *out;              // [n_omega][n_g][n_g] complex FP64
  const double *coef;       // [n_omega][n_tau] c'_kj including the edge factor
  int32_t n_g, n_tau, n_omega;
  int32_t j0, n_tau_x;      // taus held in x: j0 .. j0 + n_tau_x - 1
  int32_t hermitian;        // 1: x holds X with chi = X + X^H
  int32_t accumulate;       // 1: continue the sums already in out (taus before j0)
  int32_t item;             // index of the item in the call (norm tables)
  int32_t tile0;            // first output tile of this item in the launch
};

struct CtLaunch {
  const CtItem *items;
  int32_t n_items;
  int32_t n_tiles;          // sum over items of the output tiles
};

// ---------------------------------------------------------------------------
// Sphere-to-grid FFT (the self-energy's W~(G, G') -> W~(r, r')), two launches:
//   pencils: per (pencil d, 256 columns), the sphere points of the pencil
//            along k0 (zero elsewhere), transformed along axis 0 into tmp;
//   planes : per block of `cols` columns x `planes` i0-planes, the pencils
//            placed in their (k1, k2) plane (zero elsewhere), transformed
//            along axes 1 and 2, every grid point written to out.
// ---------------------------------------------------------------------------
struct SfftJob {
  const void *in;           // element (slot s, column c) at in[s * i_slot + (col0 + c) * i_col]
  int64_t i_slot, i_col;
  void *tmp;                // pencils [(i0 * n_disk + d) * n_cols + c]
  void *out;                // o_shift >= 0: column-grouped [c >> o_shift][n_r][1 << o_shift];
  int64_t o_col;            // o_shift < 0: out[c * o_col + r]
  int32_t o_shift;
  int32_t col0, n_cols, geo;
  int32_t unit0_pencils, unit0_planes;
};

struct SfftLaunch {
  const SfftJob *jobs;
  int32_t n_jobs;
  const Geo *geos;
  int32_t n_units_pencils, n_units_planes;
  int32_t in_f64;           // input complex FP64 (else the working precision)
  int32_t conj_in;          // read the complex conjugate of each input element
  int32_t lower_only;       // only rows r >= col0 + c of column c are wanted: plane blocks
                            // whose rows all lie above their first column are skipped
                            // (those rows of out are left unwritten)
};

// ---------------------------------------------------------------------------
// Self-energy reductions: per (job, state) the partial sums of the tiles, in
// slot order, into sums; then per item the tau-domain elements and the cosine
// and sine transforms.
// ---------------------------------------------------------------------------
struct SigmaRed {
  const double *part;       // [n_slots][n_states][2]
  int32_t n_slots, n_states;
  double *sum;              // sum[n * sum_stride + {0, 1}]
  int32_t sum_stride;
};

struct SigmaFin {
  const double *sum;        // [n_states][n_tau][2] quadratic forms of the edge-scaled G
  const double *ct, *st;    // [n_omega][n_tau]
  const double *edge_o, *edge_u;   // [n_tau] exp((HOMO - mu) tau_j), exp(-(LUMO - mu) tau_j)
  int32_t n_states, n_tau, n_omega;
  double *out;              // [n_states][n_omega] complex
  double *out_tau;          // [n_states][n_tau][2] (Sigma_und(-i tau), Sigma_bar(i tau)) or null
};

// Host-side launch wrappers (defined in the .hip files).
hipError_t launch_stage(const StageLaunch &L, int prec, hipStream_t s);
// grid <= 0: persistent (resident blocks x num_cu)
hipError_t launch_gemm(const GemmLaunch &L, int prec, int cplx, int tile, int grid, int num_cu,
                       hipStream_t s);
int gemm_tile_count(int prec, int cplx);
int gemm_tile_bm(int prec, int cplx, int tile);
int gemm_tile_bn(int prec, int cplx, int tile);
int gemm_tile_per_cu(int prec, int cplx, int tile);   // resident workgroups per CU
int gemm_tile_kc(int prec, int cplx, int tile);
const char *gemm_tile_name(int prec, int cplx, int tile);
hipError_t launch_fft(const FftLaunch &L, int dbl, int sign, int lds_bytes, int cubic_n,
                      hipStream_t s);
// sphere-to-grid transform; lds_bytes as fft_lds_bytes + 4 * n_disk for the block shape
hipError_t launch_sfft(const SfftLaunch &L, int dbl, int sign, int lds_bytes, int cubic,
                       hipStream_t s);
// self-energy: fused band contractions, products with W~ and the diagonal
// matrix elements (one tile shape per precision, complex orbitals)
hipError_t launch_gemm_sigma(const GemmLaunch &L, int prec, int grid, int num_cu, hipStream_t s);
int gemm_sigma_bm(int prec);
int gemm_sigma_bn(int prec);
int gemm_sigma_kc(int prec);
int gemm_sigma_per_cu(int prec);
// states psi_n in the working precision: out[n][r] for r < n_r_pad (zero past n_r)
hipError_t launch_sigma_states(const double *phi_o, const double *phi_u, const int32_t *states,
                               int n_states, int n_occ, int n_r, int n_r_pad, int dbl, void *out,
                               hipStream_t s);
hipError_t launch_sigma_reduce(const SigmaRed *jobs, int n_jobs, int max_states, hipStream_t s);
hipError_t launch_sigma_final(const SigmaFin *items, int n_items, int max_states, int max_omega,
                              hipStream_t s);

// Plane-FFT block shape, shared by the planner and the kernels: runs of
// 128 bytes of adjacent columns, about 256 line transforms per step, at most
// 80 KB of LDS (two blocks per CU).
constexpr int fft_lds_bytes(int n1, int n2, int cols, int planes, int elem) {
  return planes * n1 * n2 * (cols + 1) * elem;
}
// at least two blocks per CU
constexpr int fft_lds_budget(int elem) { return elem <= 8 ? 64 * 1024 : 80 * 1024; }
constexpr int fft_cols(int n1, int n2, int elem) {
  int cols = 128 / elem;
  while (cols > 1 && fft_lds_bytes(n1, n2, cols, 1, elem) > fft_lds_budget(elem)) cols /= 2;
  return cols;
}
constexpr int fft_planes(int n0, int n1, int n2, int elem) {
  const int cols = fft_cols(n1, n2, elem);
  int planes = 256 / (n1 * cols > 0 ? n1 * cols : 1);
  if (planes < 1) planes = 1;
  if (planes > n0) planes = n0;
  while (planes > 1 && fft_lds_bytes(n1, n2, cols, planes, elem) > fft_lds_budget(elem)) --planes;
  return planes;
}
// cubic grids with a specialised FFT kernel
constexpr bool fft_specialised(int n) {
  return n == 12 || n == 16 || n == 18 || n == 20 || n == 24 || n == 28 || n == 32;
}
// Plane-FFT block of the specialised cubic kernels (n^3 grid): `cols` adjacent
// columns x `planes` i0-planes, one thread per line (planes * n * cols <= 512
// threads), LDS of planes * n * n * cols elements (at most 80 KB), planes
// dividing n.
constexpr int fftc_lds_bytes(int n, int cols, int planes, int elem) {
  return planes * n * n * cols * elem;
}
constexpr int fftc_cols(int n, int elem) {
  int cols = 128 / elem;
  while (cols > 1 && (fftc_lds_bytes(n, cols, 1, elem) > 80 * 1024 || n * cols > 512)) cols /= 2;
  return cols;
}
constexpr int fftc_planes(int n, int elem) {
  const int cols = fftc_cols(n, elem);
  int planes = 1;
  while (2 * planes * n * cols <= 512 && fftc_lds_bytes(n, cols, 2 * planes, elem) <= 80 * 1024 &&
         n % (2 * planes) == 0)
    planes *= 2;
  return planes;
}
constexpr int fftc_threads(int n, int elem) {
  return fftc_planes(n, elem) * n * fftc_cols(n, elem);
}
int fft_supported(int n);
// hermitian = 1: x holds X with chi = X + X^H; 32x32 tiles on or below the
// block diagonal (T (T + 1) / 2 per item, T = ceil(n_g / 32)), each written
// with its mirror.  hermitian = 0: 32x16 tiles over the full matrix.
hipError_t launch_ct(const CtLaunch &L, int dbl, int max_omega, int hermitian, hipStream_t s);
// mode 0: |chi(tau_j)|_F^2 of the taus held in x; mode 1: |chi(i omega_k)|_F^2 of out.
// Matrix m's squared norm is left as kNormParts partial sums at
// norm[m * kNormParts + p], to be added in order by the caller.
constexpr int kNormParts = 64;
hipError_t launch_norms_impl(const CtLaunch &L, int dbl, int mode, double *norm_tau,
                             double *norm_omega, const int32_t *tau_off,
                             const int32_t *omega_off, int max_mats, hipStream_t s);
hipError_t launch_fill_zero(void *p, int64_t bytes, hipStream_t s);

// ---------------------------------------------------------------------------
// Screened interaction from chi (FP64): eps = I - s chi s, its inverse by a
// blocked Gauss-Jordan exchange of kWBlock pivots per step, then W~(i omega)
// and the inverse cosine transform.  Matrices [n_mat][n][n] complex.
// ---------------------------------------------------------------------------
constexpr int kWBlock = 64;
constexpr int kWMaxTau = 32;
hipError_t launch_w_eps(const void *chi, const double *s, void *a, int n, int n_mat,
                        hipStream_t st);
// The block-lower 64 x 64 tiles of an n x n matrix as (row tile, column tile)
// pairs, grouped by partition x = 0..7 at [off[x], off[x + 1]) (partition x,
// served by the workgroups b with b % 8 == x, owns the column tiles x,
// 15 - x, 16 + x, ...), row tile by row tile within a partition.
void w_tile_table(int n, std::vector<int32_t> &pairs, int32_t off[9]);
// one pivot block at P0: dinv [n_mat][kWBlock][kWBlock], rp [n_mat][kWBlock][n],
// cp [n_mat][n][kWBlock]; tiles / toff: the table of w_tile_table in device
// memory; *flag is set when a pivot is not positive
hipError_t launch_w_block(void *a, void *dinv, void *rp, void *cp, int n, int n_mat, int P0,
                          const int32_t *tiles, const int32_t *toff, int *flag, hipStream_t st);
// fills the tiles above the block diagonal of a from those below (Hermitian),
// then ict [n_tau][n_omega]; w_omega may be null; n_tau <= kWMaxTau
hipError_t launch_w_final(void *a, const double *s, const double *ict, void *w_tau,
                          void *w_omega, int n, int n_omega, int n_tau, hipStream_t st);

// ---------------------------------------------------------------------------
// Analytic continuation by Thiele's reciprocal differences (FP64): f
// [n_fun][n], z [n], w [m], coef [n_fun][n] (or null), out [n_fun][m], all
// complex device arrays; n <= kPadeMaxPoints.
// ---------------------------------------------------------------------------
constexpr int kPadeMaxPoints = 32;
hipError_t launch_pade(const void *f, int n_fun, int n, const void *z, const void *w, int m,
                       void *coef, void *out, hipStream_t st);

}  // namespace gw
