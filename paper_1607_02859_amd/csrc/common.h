// Shared device/host descriptors of the polarizability build (gfx950).
//
// The build of one call is a sequence of passes; a pass holds a batch of
// jobs, one job being one (item, tau_j) pair.  Every kernel takes a small
// launch struct by value that points at device tables of these descriptors.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gw {

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
  int32_t n_disk;          // distinct (k1, k2) columns touched by the sphere
  int32_t planes;          // planes per LDS group in the FFT kernel
  int32_t disk_in_lds;     // 1: pencil buffer in LDS, 0: in global scratch
  const int32_t *disk_i12; // [n_disk] k1*n2 + k2
  const int32_t *slot_dk;  // [n_g] d*n0 + k0 for output slot s
};

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
  void *slab;               // [w][n_r] output (column-major in r)
};

struct GemmLaunch {
  const GemmJob *jobs;
  const int4 *units;        // (job, r0, c0, 0)
  int32_t n_units;
  int32_t hermitian;        // 1: units are lower-triangle tiles; mask r >= c
};

// ---------------------------------------------------------------------------
// Sphere FFT over the first index (columns of a slab) or the second
// (rows of chi(G, r')).
// ---------------------------------------------------------------------------
struct FftJob {
  const void *in;           // column c of this job starts at in + c * in_col_stride
  int64_t in_col_stride;    // elements
  void *out;                // out[slot * out_slot_stride + (col0 + c) * out_col_stride]
  int64_t out_slot_stride;
  int64_t out_col_stride;
  int32_t col0;
  int32_t n_cols;
  int32_t geo;
  int32_t work0;            // first work index of this job in the launch
};

struct FftLaunch {
  const FftJob *jobs;
  int32_t n_jobs;
  int32_t n_work;           // total columns
  const Geo *geos;
  void *scratch;            // global pencil buffers, one slot per block
  int64_t scratch_slot;     // elements per slot
  int32_t in_real;          // input columns are real
  int32_t lower_only;       // column c holds only rows r >= col0 + c; others read as zero
};

// ---------------------------------------------------------------------------
// Cosine transform (FP64 accumulation) and norms.
// ---------------------------------------------------------------------------
struct CtItem {
  const void *x;            // [n_tau][n_g][n_g] chi(G, G', i tau_j), working precision
  double *out;              // [n_omega][n_g][n_g] complex FP64
  const double *coef;       // [n_omega][n_tau] c'_kj including the edge factor
  int32_t n_g, n_tau, n_omega;
  int32_t hermitian;        // 1: x holds X with chi = X + X^H
  int64_t elem0;            // first flat output element of this item in the launch
};

struct CtLaunch {
  const CtItem *items;
  int32_t n_items;
  int64_t n_elem;           // sum over items of n_g^2
};

// Host-side launch wrappers (defined in the .hip files).
hipError_t launch_stage(const StageLaunch &L, int prec, hipStream_t s);
hipError_t launch_gemm(const GemmLaunch &L, int prec, int cplx, int tile, int grid,
                       hipStream_t s);
int gemm_tile_count(int prec, int cplx);
int gemm_tile_bm(int prec, int cplx, int tile);
int gemm_tile_bn(int prec, int cplx, int tile);
int gemm_tile_kc(int prec, int cplx, int tile);
const char *gemm_tile_name(int prec, int cplx, int tile);
hipError_t launch_fft(const FftLaunch &L, int dbl, int sign, int grid, int lds_bytes,
                      hipStream_t s);
int fft_supported(int n);
hipError_t launch_ct(const CtLaunch &L, int dbl, int max_omega, hipStream_t s);
hipError_t launch_norms_impl(const CtLaunch &L, int dbl, double *norm_tau, double *norm_omega,
                             const int32_t *tau_off, const int32_t *omega_off, int max_mats,
                             hipStream_t s);
hipError_t launch_fill_zero(void *p, int64_t bytes, hipStream_t s);

}  // namespace gw
