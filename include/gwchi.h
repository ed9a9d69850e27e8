/*
 * gwchi.h -- imaginary-time polarizability chi(G, G', i omega) of the
 * cubic-scaling space-time GW method (Liu, Kaltak, Klimes, Kresse,
 * arXiv:1607.02859) on AMD MI355X (gfx950).
 *
 * What one build computes, per item and per imaginary time tau_j
 * (Sec. II.A.1 Eqs. (1)-(2); Sec. II.B Eqs. (14)-(15); Sec. II.C Eqs. (43)-(45)):
 *
 *   G_occ(r,r')   =  sum_i phi_i(r) conj(phi_i(r')) exp(+(eps_i - mu) tau_j)
 *   G_unocc(r,r') =  sum_a phi_a(r) conj(phi_a(r')) exp(-(eps_a - mu) tau_j)
 *   chi(r,r')     = -G_occ(r,r') * conj(G_unocc(r,r'))      (pointwise)
 *   chi(G,G')     =  sum_{r,r'} exp(-i G.r) chi(r,r') exp(+i G'.r')
 *   chi(G,G',i omega_k) = sum_j ct[k][j] chi(G,G', i tau_j)   (Eq. (4) / (45))
 *
 * The pointwise product is the tau < 0 branch of Eq. (15) (occupied and
 * unoccupied functions exchanged); for real orbitals both branches agree.
 * There is no 1/N_r, cell-volume or spin factor.  r runs over the grid
 * points (i0/n0, i1/n1, i2/n2) with flat index r = (i0*n1 + i1)*n2 + i2, and
 * a plane wave G is named by its flat FFT index (k0*n1 + k1)*n2 + k2 with
 * k_d = m_d mod n_d.
 *
 * Conventions for every entry point:
 *  - All buffers are owned by the caller.  The library keeps no pointer to
 *    them after the call returns (device variant: after the enqueued work
 *    completes).  The context owns its device scratch and HIP objects.
 *  - No C++ exception crosses this interface.  On any status other than
 *    GWCHI_OK the contents of chi_out are unspecified and
 *    gwchi_last_error(ctx) describes the failure.
 *  - Precision: GWCHI_FP64 computes every step in FP64.  GWCHI_FP32 and
 *    GWCHI_BF16X3 compute the weights and the cosine transform in FP64 and
 *    the band contractions, products and FFTs in FP32; GWCHI_BF16X3 runs the
 *    band contractions as split-BF16 (hi + lo parts, three products
 *    hi*hi + hi*lo + lo*hi) on MFMA with FP32 accumulation.
 */
#ifndef GWCHI_H
#define GWCHI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gwchi_ctx gwchi_ctx;

typedef enum {
  GWCHI_OK = 0,
  GWCHI_EINVAL = 1,   /* invalid argument (see gwchi_validate)                */
  GWCHI_ENOMEM = 2,   /* device memory: even the narrowest plan does not fit  */
  GWCHI_EDEVICE = 3,  /* HIP runtime error, or no usable gfx950 device        */
  GWCHI_ENOTSUP = 4,  /* grid size outside the supported FFT sizes            */
  GWCHI_ENUMERIC = 5  /* optional output check found NaN or Inf               */
} gwchi_status;

typedef enum {
  GWCHI_FP64 = 0,
  GWCHI_FP32 = 1,
  GWCHI_BF16X3 = 2
} gwchi_precision;

/* One independent problem: one k-point (complex orbitals on the unit-cell
 * grid; the q = 0 contribution of that k) or one Gamma-only system (real
 * orbitals).  Items of one call may differ in every size; they are all real or
 * all complex. */
typedef struct {
  int32_t n[3];          /* FFT grid n0, n1, n2; each 7-smooth and in [1, 32] (else ENOTSUP) */
  int32_t is_complex;    /* 0: real orbitals, 1: complex orbitals interleaved (re, im)      */
  int32_t n_occ;         /* >= 1 */
  int32_t n_unocc;       /* >= 1 */
  /* Orbitals, band-major: phi_occ[b*N_r + r] (real) or phi_occ[2*(b*N_r + r) + {0,1}]
   * (complex), N_r = n0*n1*n2, FP64.  Any normalisation is accepted; the
   * synthetic workloads use sum_r |phi(r)|^2 = 1.
   * gwchi_chi_build: host memory.  gwchi_chi_build_device: device memory. */
  const double *phi_occ;
  const double *phi_unocc;
  const double *eps_occ;    /* [n_occ]   eV, any order, host memory                       */
  const double *eps_unocc;  /* [n_unocc] eV, any order, host memory                       */
  double mu;                /* eV; max(eps_occ) < mu < min(eps_unocc) strictly            */
  int32_t n_tau;            /* >= 1 */
  int32_t n_omega;          /* >= 1 */
  const double *tau;        /* [n_tau] imaginary times > 0 (eV^-1), host memory           */
  const double *ct;         /* [n_omega][n_tau] row-major, ct[k][j] = gamma_kj cos(omega_k tau_j)
                               (Eq. (4)), host memory                                     */
  int32_t n_g;              /* >= 1 */
  const int32_t *g_index;   /* [n_g] distinct flat FFT indices in [0, N_r), output order; host */
  /* Output chi[k][g][g'] complex interleaved FP64, row index g (first index,
   * exp(-i G.r)), column g' (exp(+i G'.r')), shape [n_omega][n_g][n_g].
   * gwchi_chi_build: host memory.  gwchi_chi_build_device: device memory. */
  double *chi_out;
} gwchi_item;

/* Per-call measurements.  Phase times are GPU time between HIP events
 * recorded on the build stream around each launch of that phase, summed. */
typedef struct {
  double ms_total;          /* stream time of the whole build                        */
  double ms_stage;          /* weights (FP64) + scaled operand staging               */
  double ms_gemm;           /* fused band contractions + Hadamard product             */
  double ms_fft_r;          /* FFT over r with sphere gather                          */
  double ms_fft_rp;         /* FFT over r' with sphere gather                         */
  double ms_ct;             /* cosine transform (FP64 accumulation)                   */
  int32_t n_gemm_launches;  /* launches that make up ms_gemm                          */
  int32_t n_fft_launches;   /* launches that make up ms_fft_r + ms_fft_rp             */
  double alg_flops;         /* 8 N_r^2 K (complex) or 2 N_r^2 K (real) per tau, summed */
  double mfma_flops;        /* flops issued on MFMA (split-BF16 counts 3 products)     */
  int32_t slab_width;       /* r' columns per slab used                                */
  int32_t tau_batch;        /* tau points processed per pass                           */
  int32_t tile_id;          /* GEMM tile configuration used                            */
  int32_t graph_replayed;   /* 1 if the build ran as a replay of a cached hipGraph     */
  double kappa_F_max;       /* max_k sum_j |c'_kj| ||chi(tau_j)||_F / ||chi(i w_k)||_F,
                               or -1 when not computed                                 */
} gwchi_report;

/* Context options.  gwchi_create sets the defaults noted below;
 * gwchi_set_options replaces every field. */
typedef struct {
  int32_t slab_width;        /* r' columns per slab, multiple of 256; 0 = planner
                                (2048, narrowed until the plan fits)                  */
  int32_t tau_batch;         /* (item, tau) jobs per pass; 0 = planner (all that fit)   */
  int32_t tile_id;           /* GEMM tile: 0 = tuned if cached, else the first of the
                                menu; t >= 1 = menu entry t-1 (default 0)              */
  int32_t use_graph;         /* 1 = capture the build into a hipGraph and replay it
                                (default 1)                                             */
  int32_t check_output;      /* 1 = scan chi_out for NaN/Inf (ENUMERIC), host build only
                                (default 0)                                             */
  int32_t timing;            /* 1 = fill the per-phase times of gwchi_report (default 0) */
  int32_t skip_zero_bands;   /* 1 = drop bands whose scaled orbitals are exactly zero in
                                the working precision; never on FP64 (default 0)       */
  int32_t hermitian;         /* 1 = compute only the lower block triangle of chi(r,r')
                                and complete by Hermiticity (default 1)                 */
  int32_t persistent;        /* 1 = band-GEMM launches are persistent (resident
                                workgroups take tiles by atomic ticket from per-XCD
                                queues of tile groups, most bands first); 0 = one
                                workgroup per tile (default 1)                          */
  int32_t kappa;             /* 1 = when a report is requested, also compute the
                                norms behind kappa_F_max (default 1); 0 = report
                                kappa_F_max = -1 and skip that pass                     */
  int64_t max_device_bytes;  /* cap on the context's scratch; 0 = 60% of free memory   */
} gwchi_options;

/* Create a context on HIP device device_id (must be gfx950).
 * tune_cache_path: JSON file written by gwchi_autotune, or NULL. */
gwchi_status gwchi_create(gwchi_ctx **ctx, int32_t device_id, const char *tune_cache_path);

/* Release every device buffer, stream, event and graph the context owns. */
gwchi_status gwchi_destroy(gwchi_ctx *ctx);

gwchi_status gwchi_set_options(gwchi_ctx *ctx, const gwchi_options *opt);
gwchi_status gwchi_get_options(const gwchi_ctx *ctx, gwchi_options *opt);

/* Host-only check of items (no device is touched).  EINVAL on: null
 * pointer, n_d <= 0, n_occ or n_unocc < 1, n_tau or n_omega or n_g < 1,
 * non-finite eps / mu / tau / ct (and non-finite orbitals when orbital
 * pointers are host memory: check_orbitals != 0), tau <= 0, mu not strictly
 * inside the gap, g_index out of range or duplicated, items of one call that
 * mix real and complex orbitals.  ENOTSUP when a grid size is not 7-smooth or
 * exceeds 32. */
gwchi_status gwchi_validate(const gwchi_item *items, int32_t n_items, int32_t check_orbitals);

/* Build chi(G,G',i omega) for every item; host buffers in and out.
 * Blocking: returns after chi_out is written.  report may be NULL. */
gwchi_status gwchi_chi_build(gwchi_ctx *ctx, const gwchi_item *items, int32_t n_items,
                             gwchi_precision prec, gwchi_report *report);

/* Same with phi_occ, phi_unocc and chi_out in device memory of the
 * context's device; all other arrays in host memory.  The work is enqueued
 * on hip_stream (a hipStream_t; NULL = the context's own stream).  Returns
 * once enqueued unless report is non-NULL, in which case it waits for the
 * stream and fills the report. */
gwchi_status gwchi_chi_build_device(gwchi_ctx *ctx, const gwchi_item *items, int32_t n_items,
                                    gwchi_precision prec, void *hip_stream,
                                    gwchi_report *report);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * build as gwchi_chi_build_device (device orbitals and output, host
 * eigenvalues, grids and plane waves, enqueued on hip_stream, NULL = the
 * context's stream), with every scratch buffer -- scaled operands, slabs,
 * chi(G, r'), pencils, chi(tau), ticket counters and launch tables -- carved
 * from one fixed device array of 96 MiB that each device holds for the life
 * of the process.  The call allocates no device or pinned host memory (its
 * planner uses the C++ heap for host-side tables) and captures no graph of
 * its own; no report and no kappa_F are produced.  The planner narrows the
 * r' slab and splits the (item, tau) jobs into passes until they fit; when
 * one job with a 256-column slab does not (grids of about 28^3 and larger, or
 * very many bands), or the launch tables exceed their 4 MiB region, the call
 * returns GWCHI_ENOMEM with the sizes in gwchi_last_error.  Every call on one
 * device shares the array and finds the previous call's contents in it (the
 * kernels clear what must start at zero); calls that overlap in time on one
 * device -- from two contexts, or on streams that are not ordered -- race on
 * it.  Results equal those of gwchi_chi_build_device with the same options
 * (the same kernels; pass and slab splits do not change the arithmetic). */
gwchi_status gwchi_chi_build_device_noalloc(gwchi_ctx *ctx, const gwchi_item *items,
                                            int32_t n_items, gwchi_precision prec,
                                            void *hip_stream);

/* Time every GEMM tile configuration on these items (host memory, as for
 * gwchi_chi_build; chi_out is not written): each tile runs a warm-up build
 * and a timed one, eagerly, with HIP events around every band-GEMM launch,
 * whatever the context's timing and graph options.  The tile with the
 * smallest summed GEMM time is kept in the context under the key
 * "<arch>/<precision>/<r|c>" (e.g. "gfx950/fp32/c") and the tune cache file
 * is rewritten.  Later builds of that family with tile_id = 0 use it. */
gwchi_status gwchi_autotune(gwchi_ctx *ctx, const gwchi_item *items, int32_t n_items,
                            gwchi_precision prec);

/* The GEMM times (ms, summed over the launches of one build) that the last
 * gwchi_autotune of this context measured for each tile of the (prec,
 * is_complex) family: ms[t] for menu entry t + 1, t < n (-1 past the menu),
 * and *chosen (may be NULL) = the index t that was kept.  EINVAL when this
 * context has not tuned that family. */
gwchi_status gwchi_autotune_times(const gwchi_ctx *ctx, gwchi_precision prec, int32_t is_complex,
                                  double *ms, int32_t n, int32_t *chosen);

/* ------------------------------------------------------------------------
 * Screened interaction W~ from chi (Sec. II.C steps (iii)-(iv)), FP64.
 *
 * For one k-point, every imaginary frequency omega_k and the symmetric
 * Coulomb kernel v(G, G') = s(G) s(G') of Eq. (47):
 *
 *   eps(G,G')        = delta_GG' - v(G,G') chi(G,G',i omega_k)        (Eq. (48))
 *   W~(G,G',i w_k)   = v(G,G') (eps^-1(G,G') - delta_GG')   (Eqs. (46), (49):
 *                      W minus its bare Coulomb part v(G) delta_GG')
 *   W~(G,G',i tau_j) = sum_k xi_jk cos(tau_j omega_k) W~(G,G',i omega_k)  (Eq. (50))
 *
 * where the matrix xi cos(tau omega) is the inverse of the forward cosine
 * matrix ct[k][j] = gamma_kj cos(omega_k tau_j) (Eq. (6)); the library
 * inverts ct on the host in FP64.  eps must be Hermitian positive definite,
 * which holds when chi(i omega) is Hermitian negative semidefinite (as the
 * build above returns it; with its default Hermitian completion exactly so);
 * it is inverted without pivoting.  chi is taken as Hermitian: only its
 * 64 x 64 tiles on or below the block diagonal are read, the others being
 * their conjugate transposes.
 * ------------------------------------------------------------------------ */
typedef struct {
  int32_t n_g;              /* >= 1, at most 65535                                       */
  int32_t n_omega;          /* >= 1                                                      */
  int32_t n_tau;            /* == n_omega (square grid), at most 32                      */
  /* chi[k][g][g'] complex interleaved FP64, [n_omega][n_g][n_g] (the chi_out
   * layout of the polarizability build).  gwchi_w_build: host memory;
   * gwchi_w_build_device: device memory.  Read only. */
  const double *chi;
  const double *sqrt_v;     /* [n_g] s(G) = sqrt(4 pi e^2) / |k + G| >= 0, finite; 0 drops the
                               plane wave (e.g. G = 0 at k = 0); host memory               */
  const double *ct;         /* [n_omega][n_tau] row-major, as gwchi_item.ct; host memory   */
  /* Outputs, complex interleaved FP64, same memory kind as chi:
   * w_tau_out [n_tau][n_g][n_g] (required), w_omega_out [n_omega][n_g][n_g]
   * (W~(i omega_k); may be NULL). */
  double *w_tau_out;
  double *w_omega_out;
} gwchi_w_item;

typedef struct {
  double ms_total;          /* stream time of the whole call                            */
  double ms_eps;            /* dielectric matrices                                      */
  double ms_invert;         /* blocked Gauss-Jordan inversion                           */
  double ms_final;          /* W~(i omega) and the inverse cosine transform             */
  double alg_flops;         /* 8 n_g^3 per matrix (complex inversion), summed           */
  int32_t n_launches;       /* kernel launches of the call                              */
} gwchi_w_report;

/* Host-only check of W items (no device is touched): the EINVAL cases of
 * gwchi_w_build below. */
gwchi_status gwchi_w_validate(const gwchi_w_item *items, int32_t n_items);

/* W~(i tau) (and optionally W~(i omega)) for every item; host buffers in and
 * out.  Blocking.  EINVAL on null pointers, n_g < 1 or > 65535, n_tau !=
 * n_omega, n_tau > 32, negative or non-finite sqrt_v, non-finite or singular
 * ct; ENUMERIC when a pivot of eps is not positive (eps not positive
 * definite; outputs unspecified).  report may be NULL. */
gwchi_status gwchi_w_build(gwchi_ctx *ctx, const gwchi_w_item *items, int32_t n_items,
                           gwchi_w_report *report);

/* Same with chi, w_tau_out and w_omega_out in device memory of the context's
 * device; sqrt_v and ct in host memory.  Enqueued on hip_stream (NULL = the
 * context's stream); returns once enqueued unless report is non-NULL, in
 * which case it waits, fills the report and checks the pivots (ENUMERIC). */
gwchi_status gwchi_w_build_device(gwchi_ctx *ctx, const gwchi_w_item *items, int32_t n_items,
                                  void *hip_stream, gwchi_w_report *report);

/* ------------------------------------------------------------------------
 * Analytic continuation by Thiele's reciprocal differences (Sec. II.E.1,
 * Eqs. (72)-(74)), FP64, for many functions known at the same N points:
 *
 *   g_1(z_j) = f_j,
 *   g_n(z_j) = (g_{n-1}(z_{n-1}) - g_{n-1}(z_j)) / ((z_j - z_{n-1}) g_{n-1}(z_j)),
 *   a_n      = g_n(z_n),
 *   P_N(w)   = a_1 / (1 + a_2 (w - z_1) / (1 + ... a_N (w - z_{N-1}) / 1)),
 *
 * the tail (w - z_N) g_{N+1}(w) of the last denominator dropped.  A zero
 * denominator in the recursion (a function already represented by fewer
 * levels, e.g. a constant) ends the fraction: that difference and every
 * deeper one are 0.  P_N(z_j) = f_j.  A denominator of zero in the
 * evaluation gives a non-finite value at that point.
 * ------------------------------------------------------------------------ */
typedef struct {
  int32_t n_points;         /* N, in [1, 32]                                             */
  const double *z;          /* [N] complex interleaved, distinct and finite; host memory */
  int32_t n_fun;            /* >= 1                                                       */
  /* f[fun][j] = f_fun(z_j), complex interleaved, [n_fun][N].  gwchi_pade: host
   * memory; gwchi_pade_device: device memory.  Read only. */
  const double *f;
  int32_t n_eval;           /* M >= 0                                                     */
  const double *w;          /* [M] complex interleaved, finite; host memory (NULL if M = 0) */
  /* Outputs, same memory kind as f: out[fun][p] = P_N(w_p), [n_fun][M] (NULL if
   * M = 0); coef[fun][n] = a_{n+1}, [n_fun][N], or NULL. */
  double *out;
  double *coef;
} gwchi_pade_item;

/* Host-only check of a continuation item (no device is touched): EINVAL on
 * NULL pointers, N outside [1, 32], n_fun < 1, n_eval < 0, non-finite or
 * repeated z, non-finite w. */
gwchi_status gwchi_pade_validate(const gwchi_pade_item *item);

/* Continuation with host buffers; blocking.  ms, if not NULL, receives the
 * kernel's stream time. */
gwchi_status gwchi_pade(gwchi_ctx *ctx, const gwchi_pade_item *item, double *ms);

/* Same with f, out and coef in device memory of the context's device (z and w
 * in host memory).  Enqueued on hip_stream (NULL = the context's stream);
 * returns once enqueued unless ms is not NULL, in which case it waits and
 * reports the kernel's stream time. */
gwchi_status gwchi_pade_device(gwchi_ctx *ctx, const gwchi_pade_item *item, void *hip_stream,
                               double *ms);

/* ------------------------------------------------------------------------
 * Correlation self-energy in space and imaginary time (Sec. II.D), diagonal
 * elements on the imaginary frequency axis, for Gamma-point items with
 * complex orbitals.  Per item and imaginary time tau_j > 0:
 *
 *   W~(r, r')           = sum_{G,G'} exp(+i G.r) W~(G, G', i tau_j) exp(-i G'.r')
 *                                                   (Eqs. (51)-(52) at k = 0)
 *   Gbar(r, r', i tau)  = -sum_a phi_a(r) conj(phi_a(r')) exp(-(eps_a - mu) tau)
 *   Gund(r, r', -i tau) = +sum_i phi_i(r) conj(phi_i(r')) exp(+(eps_i - mu) tau)
 *                                                   (Eqs. (1)-(2))
 *   Sigma_bar_nn(i tau)  = -sum_{r,r'} conj(psi_n(r)) Gbar(r,r') W~(r,r') psi_n(r')
 *   Sigma_und_nn(-i tau) = -sum_{r,r'} conj(psi_n(r)) Gund(r,r') W~(r,r') psi_n(r')
 *                                                   (Eq. (53); Sigma^(1) of Eqs. (55), (62))
 *   Sigma^c = (Sigma_bar + Sigma_und) / 2,  Sigma^s = (Sigma_bar - Sigma_und) / 2
 *                                                   (Eqs. (67)-(68))
 *   Sigma_nn(i omega_k) = sum_j ct[k][j] Sigma^c_j + i sum_j st[k][j] Sigma^s_j
 *                                                   (Eqs. (69)-(71))
 *
 * W~(i tau) is taken as Hermitian in (G, G') and even in tau (as the W~ step
 * returns it); then G o W~ is Hermitian in (r, r'), each tau-domain element is
 * real, and the library forms only the lower triangle r >= r' of the
 * products.  No 1/N_r or volume factor.  The band contractions run in the
 * requested precision (FP32 and split-BF16 as for the polarizability, with
 * W~(r, r') and the matrix-element sums of each tile in FP32); the weights,
 * the sums over tiles and the transforms are FP64 on every path.
 * ------------------------------------------------------------------------ */
typedef struct {
  int32_t n[3];             /* FFT grid, as gwchi_item                                     */
  int32_t is_complex;       /* must be 1 (real orbitals: ENOTSUP)                          */
  int32_t n_occ, n_unocc;   /* >= 1 each                                                   */
  /* orbitals, band-major complex FP64 as gwchi_item; gwchi_sigma_build: host,
   * gwchi_sigma_build_device: device memory */
  const double *phi_occ;
  const double *phi_unocc;
  const double *eps_occ;    /* [n_occ]   eV, host                                          */
  const double *eps_unocc;  /* [n_unocc] eV, host                                          */
  double mu;                /* strictly inside the gap                                     */
  int32_t n_tau, n_omega;   /* >= 1 each                                                   */
  const double *tau;        /* [n_tau] > 0, host                                           */
  const double *ct;         /* [n_omega][n_tau] gamma_kj cos(omega_k tau_j) (Eq. (4)), host  */
  const double *st;         /* [n_omega][n_tau] lambda_kj sin(omega_k tau_j) (Eq. (7)), host */
  int32_t n_g;              /* >= 1 */
  const int32_t *g_index;   /* [n_g] distinct flat FFT indices, host                       */
  /* W~(G, G', i tau_j), [n_tau][n_g][n_g] complex FP64 (row G, column G', the
   * layout of gwchi_w_item.w_tau_out); same memory kind as the orbitals */
  const double *w_tau;
  int32_t n_states;         /* in [1, 1024]                                                */
  const int32_t *states;    /* [n_states] host: b < n_occ is occupied band b, otherwise
                               unoccupied band b - n_occ (input order, as the orbitals)  */
  /* Outputs, same memory kind as the orbitals: sigma_out [n_states][n_omega]
   * complex interleaved (Sigma_nn(i omega_k)); sigma_tau_out [n_states][n_tau][2]
   * real (Sigma_und(-i tau_j), Sigma_bar(i tau_j)) or NULL */
  double *sigma_out;
  double *sigma_tau_out;
} gwchi_sigma_item;

typedef struct {
  double ms_total;          /* stream time of the whole call                           */
  double ms_stage;          /* weights, scaled operands and the states                 */
  double ms_fft;            /* W~(G, G') -> W~(r, r'), both transforms                 */
  double ms_gemm;           /* fused band contractions, products and matrix elements   */
  double ms_final;          /* sums over tiles, even/odd parts, cosine and sine        */
  int32_t n_gemm_launches;
  int32_t slab_width;
  int32_t tau_batch;        /* (item, tau) jobs per pass                               */
  double alg_flops;         /* 8 N_r^2 K per tau (the two Green's functions), summed   */
  double mfma_flops;        /* flops issued on MFMA by the band contractions           */
} gwchi_sigma_report;

/* Host-only check (no device is touched): the EINVAL cases of gwchi_validate
 * for the shared fields (orbitals checked when check_orbitals != 0), plus NULL
 * st / w_tau / states / sigma_out, non-finite st, n_states outside [1, 1024],
 * a state index outside [0, n_occ + n_unocc); ENOTSUP for real orbitals and
 * for the grid sizes gwchi_validate refuses. */
gwchi_status gwchi_sigma_validate(const gwchi_sigma_item *items, int32_t n_items,
                                  int32_t check_orbitals);

/* Diagonal self-energies for every item; host buffers in and out; blocking.
 * report may be NULL. */
gwchi_status gwchi_sigma_build(gwchi_ctx *ctx, const gwchi_sigma_item *items, int32_t n_items,
                               gwchi_precision prec, gwchi_sigma_report *report);

/* Same with phi_occ, phi_unocc, w_tau, sigma_out and sigma_tau_out in device
 * memory; enqueued on hip_stream (NULL = the context's stream); returns once
 * enqueued unless report is non-NULL (then it waits and fills the report). */
gwchi_status gwchi_sigma_build_device(gwchi_ctx *ctx, const gwchi_sigma_item *items,
                                      int32_t n_items, gwchi_precision prec, void *hip_stream,
                                      gwchi_sigma_report *report);

/* Message of the last failure on this context (never NULL). */
const char *gwchi_last_error(const gwchi_ctx *ctx);

/* Library version string. */
const char *gwchi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* GWCHI_H */
