// Screened interaction from the polarizability (gfx950), FP64 throughout.
//
// For one k-point and every imaginary frequency omega_k (Sec. II.C steps
// (iii)-(iv)), with v(G, G') = s(G) s(G') the symmetric Coulomb kernel of
// Eq. (47):
//   eps(G, G')   = delta_GG' - s(G) chi(G, G') s(G')             Eq. (48)
//   W~(G, G')    = s(G) (eps^-1(G, G') - delta_GG') s(G')       Eqs. (46), (49)
//   W~(i tau_j)  = sum_k ict[j][k] W~(i omega_k)                Eq. (50)
// ict being the inverse of the forward cosine matrix (Eq. (6)).
//
// eps is Hermitian positive definite for a Hermitian negative semidefinite
// chi (its eigenvalues are >= 1), so it is inverted in place by the
// Gauss-Jordan exchange (sweep) without pivoting, in blocks of kWBlock
// pivots.  Per block P = [P0, P0 + nb) of every matrix of the batch:
//   k_w_diag   D^-1 of the diagonal block (one workgroup per matrix, the
//              block in registers, pivot row and column through LDS);
//   k_w_panel  row panel R[p][j] = (D^-1 A[P, :])[p][j] for j outside P and
//              D^-1 on P; column panel C[i][p] = A[i][P0 + p] for i outside P;
//   k_w_update A[i][j] <- R[i - P0][j] for i in P, else
//              A[i][j] * [j outside P] - sum_p C[i][p] R[p][j]
//              (rank-nb update on FP64 MFMA; persistent, the next panel
//              chunks loaded while the MFMAs run).
// Only the block-lower 64 x 64 tiles are stored and updated: the sweep keeps
// the swept and unswept diagonal blocks Hermitian and the blocks between
// them anti-Hermitian, so a tile above the diagonal is the conjugate
// transpose of its mirror, negated when exactly one of its two blocks is
// swept (the panels read it so).  After the last block the block-lower tiles
// hold eps^-1; k_w_mirror fills the upper tiles (Hermitian), and k_w_final
// forms W~(i omega_k) and the inverse cosine transform in one pass.
#include <algorithm>
#include <type_traits>
#include <vector>

#include "common.h"

namespace gw {
namespace {

typedef double d4v __attribute__((ext_vector_type(4)));
typedef double d2v __attribute__((ext_vector_type(2)));

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

constexpr int NB = kWBlock;

// grid (ceil(n / 256), n, n_mat): a[m][g][h] = delta - s_g chi[m][g][h] s_h on
// the block-lower 64 x 64 tiles (the sweep reads no others; k_w_mirror fills
// the upper ones at the end)
__global__ __launch_bounds__(256) void k_w_eps(const double2 *__restrict__ chi,
                                               const double *__restrict__ s, double2 *__restrict__ a,
                                               int n) {
  const int h = blockIdx.x * 256 + threadIdx.x;
  const int g = blockIdx.y;
  if (h >= n || h / 64 > g / 64) return;
  const int64_t e = ((int64_t)blockIdx.z * n + g) * n + h;
  const double sg = s[g] * s[h];
  const double2 x = chi[e];
  double2 y = make_double2(-sg * x.x, -sg * x.y);
  if (g == h) y.x += 1.0;
  a[e] = y;
}

// one workgroup of 1024 threads per matrix: the exchange of the nb pivots of
// the diagonal block at P0; rows and columns past nb are the identity.  The
// block stays in registers (wave w holds rows w, w + 16, w + 32, w + 48, lane
// l column l); per pivot only the pivot row and column pass through LDS, in a
// double buffer: the owners of row and column p + 1 write them right after
// pivot p, so one barrier per pivot suffices.  A pivot whose real part is not
// positive and finite (eps not positive definite) sets *flag.
constexpr int DT = 1024;
constexpr int DR = NB * NB / DT;                 // rows per thread
static_assert(DT == 16 * NB && DR * 16 == NB, "k_w_diag maps 16 waves onto 64 rows");
__global__ __launch_bounds__(DT) void k_w_diag(const double2 *__restrict__ a,
                                               double2 *__restrict__ dinv, int n, int P0,
                                               int *flag) {
  __shared__ double2 rowb[2][NB], colb[2][NB];
  const int m = blockIdx.x;
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const double2 *A = a + (int64_t)m * n * n;
  const int nb = min(NB, n - P0);
  double2 r[DR];
#pragma unroll
  for (int k = 0; k < DR; ++k) {
    const int i = w + 16 * k;
    r[k] = (i < nb && l < nb) ? A[(int64_t)(P0 + i) * n + P0 + l]
                              : make_double2(i == l ? 1.0 : 0.0, 0.0);
  }
  if (w == 0) rowb[0][l] = r[0];
  if (l == 0) {
#pragma unroll
    for (int k = 0; k < DR; ++k) colb[0][w + 16 * k] = r[k];
  }
  __syncthreads();
  for (int p = 0; p < nb; ++p) {
    const int cur = p & 1, nxt = cur ^ 1;
    // every LDS read of the pivot first (one round trip), then the reciprocal
    const double2 dpp = rowb[cur][p];
    const double2 dpj = rowb[cur][l];
    double2 dip[DR];
#pragma unroll
    for (int k = 0; k < DR; ++k) dip[k] = colb[cur][w + 16 * k];
    if (threadIdx.x == 0 && !(dpp.x > 0.0 && dpp.x < 1.0e300)) atomicOr(flag, 1);
    const double q = 1.0 / (dpp.x * dpp.x + dpp.y * dpp.y);
    const double2 piv = make_double2(dpp.x * q, -dpp.y * q);
    // the pivot row scaled once per lane; on the pivot column (l == p) the
    // row entry is taken as 1 and the old value as 0, so that every element
    // off the pivot row takes the same update r - d_ip (piv d_pj): -d_ip piv
    // on the pivot column, and the pivot row becomes piv d_pj (piv at p)
    const double2 dps = l == p ? piv : cmul(piv, dpj);
#pragma unroll
    for (int k = 0; k < DR; ++k) {
      const double2 o = l == p ? make_double2(0.0, 0.0) : r[k];
      const double2 u =
          make_double2(__builtin_fma(-dip[k].x, dps.x, __builtin_fma(dip[k].y, dps.y, o.x)),
                       __builtin_fma(-dip[k].x, dps.y, __builtin_fma(-dip[k].y, dps.x, o.y)));
      r[k] = w + 16 * k == p ? dps : u;
    }
    const int p1 = p + 1;
    if (p1 < nb) {
#pragma unroll
      for (int k = 0; k < DR; ++k)
        if (w + 16 * k == p1) rowb[nxt][l] = r[k];
      if (l == p1) {
#pragma unroll
        for (int k = 0; k < DR; ++k) colb[nxt][w + 16 * k] = r[k];
      }
    }
    __syncthreads();
  }
  double2 *D = dinv + (int64_t)m * NB * NB;
#pragma unroll
  for (int k = 0; k < DR; ++k) D[(w + 16 * k) * NB + l] = r[k];
}

// grid (ceil(n / 64), n_mat): for the 64 columns j0 .. j0 + 63 the row panel
// rp[m][p][j] = (D^-1 A[P, :])[p][j] (D^-1 itself on the block's columns;
// layout [n_mat][NB][n]) on FP64 MFMA, and for the rows i of the same range
// the column panel cp[m][i][p] = A[i][P0 + p] (layout [n_mat][n][NB]); entries
// with p >= nb are zero.  Waves and lanes as in k_w_update below.
__global__ __launch_bounds__(256) void k_w_panel(const double2 *__restrict__ a,
                                                 const double2 *__restrict__ dinv,
                                                 double2 *__restrict__ rp, double2 *__restrict__ cp,
                                                 int n, int P0) {
  // the contraction over the block's 64 bands runs in NB / PH parts of PH
  // bands, so that three workgroups share a CU and the whole grid is resident
  // at once.  Every copy loop below issues all its loads before its first
  // store, so that they are in flight together.
  constexpr int PH = NB / 4;
  constexpr int PQ = 256 / PH;                 // rows per pass of a part
  constexpr int CPT = 64 * NB / 256;           // column-panel entries per thread
  constexpr int HPT = NB * PH / 256;           // part entries per thread
  static_assert(CPT == 16 && HPT == 4 && PQ == 16, "k_w_panel assumes 256 threads and 64-pivot blocks");
  __shared__ double2 sd[NB][PH + 1];
  __shared__ double2 sa[PH][64 + 1];
  const int m = blockIdx.y;
  const int j0 = blockIdx.x * 64;
  const int tile = (int)blockIdx.x, bp = P0 / 64;   // tile index, pivot block index
  const int nb = min(NB, n - P0);
  const double2 *A = a + (int64_t)m * n * n;
  const double2 *D = dinv + (int64_t)m * NB * NB;
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int tq = threadIdx.x / PH, lq = threadIdx.x % PH;
  // column panel for the rows of this tile below the pivot block (stored);
  // rows above it are written after the MFMAs, through LDS.  Thread entry t:
  // row j0 + w + 4 t, band l.
  if (tile >= bp) {
    double2 x[CPT];
#pragma unroll
    for (int t = 0; t < CPT; ++t) {
      const int i = j0 + w + 4 * t;
      const bool in_p = i >= P0 && i < P0 + nb;
      x[t] = (i < n && l < nb && !in_p) ? A[(int64_t)i * n + P0 + l] : make_double2(0.0, 0.0);
    }
    // full tiles store without per-row conditions (each conditional store
    // would get a wait for every store before it)
    double2 *Cp = cp + ((int64_t)m * n + j0 + w) * NB + l;
    if (j0 + 64 <= n) {
#pragma unroll
      for (int t = 0; t < CPT; ++t) Cp[4 * t * NB] = x[t];
    } else {
#pragma unroll
      for (int t = 0; t < CPT; ++t)
        if (j0 + w + 4 * t < n) Cp[4 * t * NB] = x[t];
    }
  }
  const int wr = w >> 1, wc = w & 1;
  d4v re[2][2], im[2][2];
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) re[bi][bj] = im[bi][bj] = d4v{0.0, 0.0, 0.0, 0.0};
  for (int h = 0; h < NB / PH; ++h) {
    const int q0 = h * PH;
    // D^-1 columns q0 .. q0 + PH - 1 (entry t: row tq + PQ t, column lq)
    // and M[P, j] for the bands of this part
    double2 xd[HPT], xa[HPT];
#pragma unroll
    for (int t = 0; t < HPT; ++t) xd[t] = D[(tq + PQ * t) * NB + q0 + lq];
    if (tile <= bp) {
      // M[P, j] is stored (block-lower): entry t band w + 4 t, column l
#pragma unroll
      for (int t = 0; t < HPT; ++t) {
        const int q = w + 4 * t, j = j0 + l;
        xa[t] = (q0 + q < nb && j < n) ? A[(int64_t)(P0 + q0 + q) * n + j] : make_double2(0.0, 0.0);
      }
    } else {
      // M[P, j] = conj(M[j, P]) above the diagonal: entry t row j0 + tq + PQ t,
      // band lq (reads along the row)
#pragma unroll
      for (int t = 0; t < HPT; ++t) {
        const int q = lq, j = j0 + tq + PQ * t;
        xa[t] = (q0 + q < nb && j < n) ? A[(int64_t)j * n + P0 + q0 + q] : make_double2(0.0, 0.0);
      }
    }
#pragma unroll
    for (int t = 0; t < HPT; ++t) sd[tq + PQ * t][lq] = xd[t];
    if (tile <= bp) {
#pragma unroll
      for (int t = 0; t < HPT; ++t) sa[w + 4 * t][l] = xa[t];
    } else {
#pragma unroll
      for (int t = 0; t < HPT; ++t) sa[lq][tq + PQ * t] = make_double2(xa[t].x, -xa[t].y);
    }
    __syncthreads();
#pragma unroll 4
    for (int k = 0; k < PH; k += 4) {
      double2 x[2], y[2];
#pragma unroll
      for (int bi = 0; bi < 2; ++bi) x[bi] = sd[wr * 32 + bi * 16 + (l & 15)][k + (l >> 4)];
#pragma unroll
      for (int bj = 0; bj < 2; ++bj) y[bj] = sa[k + (l >> 4)][wc * 32 + bj * 16 + (l & 15)];
#pragma unroll
      for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) {
          re[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(x[bi].x, y[bj].x, re[bi][bj], 0, 0, 0);
          re[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(-x[bi].y, y[bj].y, re[bi][bj], 0, 0, 0);
          im[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(x[bi].x, y[bj].y, im[bi][bj], 0, 0, 0);
          im[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(x[bi].y, y[bj].x, im[bi][bj], 0, 0, 0);
        }
    }
    __syncthreads();
  }
  // row panel: D^-1 itself on the block's own columns (only the tile at bp
  // has them), the product elsewhere
  double2 val[2][2][4];
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) {
      const int j = j0 + wc * 32 + bj * 16 + (l & 15);
      const bool in_p = j >= P0 && j < P0 + nb;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int p = wr * 32 + bi * 16 + (l >> 4) + 4 * v;
        double2 x = make_double2(0.0, 0.0);
        if (p < nb && j < n) x = in_p ? D[p * NB + (j - P0)] : make_double2(re[bi][bj][v], im[bi][bj][v]);
        val[bi][bj][v] = x;
      }
    }
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) {
      const int j = j0 + wc * 32 + bj * 16 + (l & 15);
      if (j0 + 64 <= n || j < n) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int p = wr * 32 + bi * 16 + (l >> 4) + 4 * v;
          rp[((int64_t)m * NB + p) * n + j] = val[bi][bj][v];
        }
      }
    }
  if (tile < bp) {
    // rows i of this tile lie above the pivot block: M[i, p] = -conj(M[p, i]),
    // M[p, i] stored; staged through LDS in parts so that reads and writes
    // run along rows
    for (int h = 0; h < NB / PH; ++h) {
      const int q0 = h * PH;
      double2 x[HPT];
#pragma unroll
      for (int t = 0; t < HPT; ++t) {
        const int q = w + 4 * t, i = j0 + l;
        x[t] = (q0 + q < nb && i < n) ? A[(int64_t)(P0 + q0 + q) * n + i] : make_double2(0.0, 0.0);
      }
#pragma unroll
      for (int t = 0; t < HPT; ++t) sa[w + 4 * t][l] = x[t];
      __syncthreads();
      double2 *Cp = cp + ((int64_t)m * n + j0 + tq) * NB + q0 + lq;
      if (j0 + 64 <= n) {
#pragma unroll
        for (int t = 0; t < HPT; ++t) {
          const double2 y = sa[lq][tq + PQ * t];
          Cp[PQ * t * NB] = make_double2(-y.x, y.y);
        }
      } else {
#pragma unroll
        for (int t = 0; t < HPT; ++t) {
          const double2 y = sa[lq][tq + PQ * t];
          if (j0 + tq + PQ * t < n) Cp[PQ * t * NB] = make_double2(-y.x, y.y);
        }
      }
      __syncthreads();
    }
  }
}

// Rank-nb update, persistent, on the block-lower tiles only (row tile >=
// column tile; T tiles per side): the sweep of a Hermitian matrix keeps the
// swept and unswept diagonal blocks Hermitian and the blocks between them
// anti-Hermitian, so the tiles above the diagonal follow from those below
// (the panels read them so, and k_w_mirror fills them at the end).
// Workgroups are dealt to the XCDs in turn: workgroup b serves partition
// b % 8, which owns the column tiles x, 15 - x, 16 + x, ... (a snake, so that
// the partitions get about equal numbers of lower tiles) of every matrix, so
// the panels its tiles read stay in that XCD's L2 while A streams through.
// The host lists each partition's lower tiles, row tile by row tile, in a
// table (w_tile_table); within a partition the tiles run matrix by matrix in
// that order, and its workgroups take every nk-th of them.
// Per tile: A[i][j] <- R[i - P0][j] for i in the pivot block P, else
// A[i][j] [j outside P] - sum_p C[i][p] R[p][j].
//
// The panels stream in chunks of UKC = 16 bands (NB / UKC per tile) through a
// two-stage LDS ring; each thread holds the next two chunks in registers,
// loaded while the MFMAs of the current chunk run, across tile boundaries,
// and the tile's current A values are loaded at its start, so that HBM and
// L2 traffic overlap the MFMAs.  Every load is issued from a clamped, valid
// address; out-of-range rows and columns only feed outputs never stored.
//   stage layout: C rows 64 x (UKC + 1) entries (padded: the 16 lanes reading
//   one band of 16 rows hit distinct banks), then R: UKC band rows x 64.
// Waves and lanes as in k_w_panel.
constexpr int UKC = 16;
constexpr int UCH = NB / UKC;                 // chunks per tile

struct UTile {
  int m, i0, j0;
};

// one chunk of panel values per thread: 4 C entries and 4 R entries
// (native vectors: arrays of them stay in registers across the tile loop)
__device__ __forceinline__ void uload(d2v (&hc)[4], d2v (&hr)[4], const double2 *__restrict__ rp,
                                      const double2 *__restrict__ cp, int n, const UTile &u,
                                      int kc) {
  const int k0 = kc * UKC;
  sfor<0, 4>([&](auto qq) {
    constexpr int q = decltype(qq)::value;
    const int e = threadIdx.x + 256 * q;       // C: row e / UKC, band e % UKC
    const int gi = min(u.i0 + e / UKC, n - 1);
    hc[q] = *reinterpret_cast<const d2v *>(cp + ((int64_t)u.m * n + gi) * NB + k0 + e % UKC);
    const int gj = min(u.j0 + e % 64, n - 1);  // R: band e / 64, column e % 64
    hr[q] = *reinterpret_cast<const d2v *>(rp + ((int64_t)u.m * NB + k0 + e / 64) * n + gj);
  });
}
__device__ __forceinline__ void ustore(const d2v (&hc)[4], const d2v (&hr)[4],
                                       double2 (*sc)[UKC + 1], double2 (*sr)[64]) {
  sfor<0, 4>([&](auto qq) {
    constexpr int q = decltype(qq)::value;
    const int e = threadIdx.x + 256 * q;
    *reinterpret_cast<d2v *>(&sc[e / UKC][e % UKC]) = hc[q];
    *reinterpret_cast<d2v *>(&sr[e / 64][e % 64]) = hr[q];
  });
}

__global__ __launch_bounds__(256, 2) void k_w_update(double2 *__restrict__ a,
                                                     const double2 *__restrict__ rp,
                                                     const double2 *__restrict__ cp, int n,
                                                     int P0, int n_mat,
                                                     const int2 *__restrict__ tl,
                                                     const int *__restrict__ toff) {
  __shared__ double2 sc0[64][UKC + 1], sc1[64][UKC + 1];
  __shared__ double2 sr0[UKC][64], sr1[UKC][64];
  const int nb = min(NB, n - P0);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int wr = w >> 1, wc = w & 1;
  const int G = gridDim.x;                     // at least 8
  const int x = (int)blockIdx.x % 8, k = (int)blockIdx.x / 8;
  const int nk = (G - x + 7) / 8;              // workgroups of partition x
  const int lo = toff[x], L = toff[x + 1] - lo;
  const int part_tiles = n_mat * L;
  const int my_tiles = part_tiles > k ? (part_tiles - k + nk - 1) / nk : 0;
  if (my_tiles == 0) return;                   // the whole workgroup leaves together
  const int n_chunks = my_tiles * UCH;
  // chunk c: local tile k + (c / UCH) nk, band chunk c % UCH; chunks past the
  // end load the last tile again (never used)
  auto chunk_tile = [&](int c) {
    const int q = k + min(c / UCH, my_tiles - 1) * nk;
    const int m = q / L;
    const int2 t = tl[lo + q - m * L];
    UTile u;
    u.m = m;
    u.i0 = t.x * 64;
    u.j0 = t.y * 64;
    return u;
  };
  // register sets X and Y: before chunk c, X holds chunk c + 1 and Y chunk
  // c + 2 for even c, the other way round for odd c
  d2v xc[4], xr[4], yc[4], yr[4];
  uload(xc, xr, rp, cp, n, chunk_tile(0), 0);
  ustore(xc, xr, sc0, sr0);
  uload(xc, xr, rp, cp, n, chunk_tile(1), 1 % UCH);
  uload(yc, yr, rp, cp, n, chunk_tile(2), 2 % UCH);
  __syncthreads();
  for (int it = 0; it < my_tiles; ++it) {
    const UTile u = chunk_tile(it * UCH);
    double2 *A = a + (int64_t)u.m * n * n;
    double2 old[2][2][4];
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
      for (int bj = 0; bj < 2; ++bj) {
        const int j = min(u.j0 + wc * 32 + bj * 16 + (l & 15), n - 1);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = min(u.i0 + wr * 32 + bi * 16 + (l >> 4) + 4 * v, n - 1);
          old[bi][bj][v] = A[(int64_t)i * n + j];
        }
      }
    d4v re[2][2], im[2][2];
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
      for (int bj = 0; bj < 2; ++bj) re[bi][bj] = im[bi][bj] = d4v{0.0, 0.0, 0.0, 0.0};
    sfor<0, UCH>([&](auto kk) {
      constexpr int kc = decltype(kk)::value;
      const int c = it * UCH + kc;
      // chunk c is in stage c % 2 (UCH is even, so stage kc % 2)
      double2(*sc)[UKC + 1] = (kc & 1) ? sc1 : sc0;
      double2(*sr)[64] = (kc & 1) ? sr1 : sr0;
#pragma unroll
      for (int k = 0; k < UKC; k += 4) {
        double2 x[2], y[2];
#pragma unroll
        for (int bi = 0; bi < 2; ++bi) x[bi] = sc[wr * 32 + bi * 16 + (l & 15)][k + (l >> 4)];
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) y[bj] = sr[k + (l >> 4)][wc * 32 + bj * 16 + (l & 15)];
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
          for (int bj = 0; bj < 2; ++bj) {
            re[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(x[bi].x, y[bj].x, re[bi][bj], 0, 0, 0);
            re[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(-x[bi].y, y[bj].y, re[bi][bj], 0, 0, 0);
            im[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(x[bi].x, y[bj].y, im[bi][bj], 0, 0, 0);
            im[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(x[bi].y, y[bj].x, im[bi][bj], 0, 0, 0);
          }
      }
      // chunk c + 1 into the other stage (last read by chunk c - 1, which
      // every wave finished before the previous barrier), then load c + 3
      if constexpr ((kc & 1) == 0) {
        if (c + 1 < n_chunks) ustore(xc, xr, sc1, sr1);
        uload(xc, xr, rp, cp, n, chunk_tile(c + 3), (kc + 3) % UCH);
      } else {
        if (c + 1 < n_chunks) ustore(yc, yr, sc0, sr0);
        uload(yc, yr, rp, cp, n, chunk_tile(c + 3), (kc + 3) % UCH);
      }
      __syncthreads();
    });
    // rows of the pivot block take the row panel (D^-1 on the block's columns)
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
      for (int bj = 0; bj < 2; ++bj) {
        const int j = u.j0 + wc * 32 + bj * 16 + (l & 15);
        const bool j_in_p = j >= P0 && j < P0 + nb;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = u.i0 + wr * 32 + bi * 16 + (l >> 4) + 4 * v;
          if (i >= n || j >= n) continue;
          const int64_t e = (int64_t)i * n + j;
          if (i >= P0 && i < P0 + nb) {
            A[e] = rp[((int64_t)u.m * NB + (i - P0)) * n + j];
          } else {
            const double2 o = j_in_p ? make_double2(0.0, 0.0) : old[bi][bj][v];
            A[e] = make_double2(o.x - re[bi][bj][v], o.y - im[bi][bj][v]);
          }
        }
      }
  }
}

// grid (T, T, n_mat): after the last pivot block A holds eps^-1 in its
// block-lower tiles; the tile (I, J) above the diagonal (I < J) becomes the
// conjugate transpose of tile (J, I), through LDS so that reads and writes run
// along rows.
__global__ __launch_bounds__(256) void k_w_mirror(double2 *__restrict__ a, int n) {
  const int I = blockIdx.y, J = blockIdx.x;
  if (I >= J) return;
  __shared__ double2 t[64][64 + 1];
  double2 *A = a + (int64_t)blockIdx.z * n * n;
  const int r0 = J * 64, c0 = I * 64;          // source tile (J, I)
  // all 16 loads of a thread in flight together, from clamped addresses (the
  // slots past n are never read back)
  {
    const int c = threadIdx.x & 63, rw = threadIdx.x >> 6;
    double2 x[16];
#pragma unroll
    for (int q = 0; q < 16; ++q)
      x[q] = A[(int64_t)min(r0 + rw + 4 * q, n - 1) * n + min(c0 + c, n - 1)];
#pragma unroll
    for (int q = 0; q < 16; ++q) t[rw + 4 * q][c] = x[q];
  }
  __syncthreads();
  for (int e = threadIdx.x; e < 64 * 64; e += 256) {
    const int r = e / 64, c = e % 64;          // target (c0 + r, r0 + c) = conj(source (r0 + c, c0 + r))
    if (c0 + r < n && r0 + c < n) {
      const double2 x = t[c][r];
      A[(int64_t)(c0 + r) * n + r0 + c] = make_double2(x.x, -x.y);
    }
  }
}

// grid (ceil(n / 256), n): per element (g, h), W~(i omega_k) = s_g s_h
// (A_k(g, h) - delta) for every k (written when w_omega is not null) and
// W~(i tau_j) = sum_k ict[j][k] W~(i omega_k), summed in increasing k, all
// taus in registers (n_tau <= MT).
template <int MT>
__global__ __launch_bounds__(256) void k_w_final(const double2 *__restrict__ a,
                                                 const double *__restrict__ s,
                                                 const double *__restrict__ ict,
                                                 double2 *__restrict__ w_tau,
                                                 double2 *__restrict__ w_omega, int n,
                                                 int n_omega, int n_tau) {
  const int h = blockIdx.x * 256 + threadIdx.x;
  const int g = blockIdx.y;
  if (h >= n) return;
  const int64_t nn = (int64_t)n * n;
  const int64_t e = (int64_t)g * n + h;
  const double ss = s[g] * s[h];
  double2 acc[MT];
#pragma unroll
  for (int j = 0; j < MT; ++j) acc[j] = make_double2(0.0, 0.0);
  for (int k = 0; k < n_omega; ++k) {
    double2 x = a[k * nn + e];
    if (g == h) x.x -= 1.0;
    const double2 wv = make_double2(ss * x.x, ss * x.y);
    if (w_omega) w_omega[k * nn + e] = wv;
#pragma unroll
    for (int j = 0; j < MT; ++j) {
      if (j < n_tau) {
        const double c = ict[j * n_omega + k];
        acc[j].x += c * wv.x;
        acc[j].y += c * wv.y;
      }
    }
  }
#pragma unroll
  for (int j = 0; j < MT; ++j)
    if (j < n_tau) w_tau[j * nn + e] = acc[j];
}

}  // namespace

hipError_t launch_w_eps(const void *chi, const double *s, void *a, int n, int n_mat,
                        hipStream_t st) {
  if (n < 1 || n_mat < 1) return hipSuccess;
  if (n > 65535 || n_mat > 65535) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_w_eps, dim3((n + 255) / 256, n, n_mat), dim3(256), 0, st,
                     (const double2 *)chi, s, (double2 *)a, n);
  return hipGetLastError();
}

void w_tile_table(int n, std::vector<int32_t> &pairs, int32_t off[9]) {
  const int T = (n + 63) / 64;
  pairs.clear();
  for (int x = 0; x < 8; ++x) {
    off[x] = (int32_t)(pairs.size() / 2);
    std::vector<int> cols;                     // snake: x, 15 - x, 16 + x, ... (increasing)
    for (int g = 0; g * 8 < T; ++g) {
      const int tj = (g & 1) ? g * 8 + 7 - x : g * 8 + x;
      if (tj < T) cols.push_back(tj);
    }
    for (int ti = 0; ti < T; ++ti)
      for (int tj : cols)
        if (tj <= ti) {
          pairs.push_back(ti);
          pairs.push_back(tj);
        }
  }
  off[8] = (int32_t)(pairs.size() / 2);
}

hipError_t launch_w_block(void *a, void *dinv, void *rp, void *cp, int n, int n_mat, int P0,
                          const int32_t *tile_list, const int32_t *toff, int *flag, hipStream_t st) {
  if (P0 < 0 || P0 >= n) return hipErrorInvalidValue;
  if (n_mat > 65535) return hipErrorInvalidValue;
  const int tiles = (n + 63) / 64;
  hipLaunchKernelGGL(k_w_diag, dim3(n_mat), dim3(DT), 0, st, (const double2 *)a,
                     (double2 *)dinv, n, P0, flag);
  hipLaunchKernelGGL(k_w_panel, dim3(tiles, n_mat), dim3(256), 0, st, (const double2 *)a,
                     (const double2 *)dinv, (double2 *)rp, (double2 *)cp, n, P0);
  // compute units of the device, queried once (initialisation is thread safe)
  static const int num_cu = [] {
    int dev = 0, cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cu <= 0)
      cu = 256;
    return cu;
  }();
  const int64_t n_tiles = (int64_t)tiles * (tiles + 1) / 2 * n_mat;   // block-lower tiles
  if (n_tiles > 0x7fffffff) return hipErrorInvalidValue;
  const int grid = (int)std::max<int64_t>(8, std::min<int64_t>(n_tiles, 2 * num_cu));
  hipLaunchKernelGGL(k_w_update, dim3(grid), dim3(256), 0, st, (double2 *)a, (const double2 *)rp,
                     (const double2 *)cp, n, P0, n_mat, (const int2 *)tile_list, toff);
  return hipGetLastError();
}

hipError_t launch_w_final(void *a, const double *s, const double *ict, void *w_tau,
                          void *w_omega, int n, int n_omega, int n_tau, hipStream_t st) {
  if (n > 65535) return hipErrorInvalidValue;
  const int tiles = (n + 63) / 64;
  if (tiles > 1)
    hipLaunchKernelGGL(k_w_mirror, dim3(tiles, tiles, n_omega), dim3(256), 0, st, (double2 *)a, n);
  const dim3 grid((n + 255) / 256, n), block(256);
  const double2 *A = (const double2 *)a;
  double2 *T = (double2 *)w_tau, *O = (double2 *)w_omega;
  if (n_tau <= 8)
    hipLaunchKernelGGL(k_w_final<8>, grid, block, 0, st, A, s, ict, T, O, n, n_omega, n_tau);
  else if (n_tau <= 16)
    hipLaunchKernelGGL(k_w_final<16>, grid, block, 0, st, A, s, ict, T, O, n, n_omega, n_tau);
  else if (n_tau <= 32)
    hipLaunchKernelGGL(k_w_final<32>, grid, block, 0, st, A, s, ict, T, O, n, n_omega, n_tau);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace gw
