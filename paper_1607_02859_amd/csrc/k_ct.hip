// Cosine transform from imaginary time to imaginary frequency (gfx950).
//
// Eq. (4), applied to chi as in Eq. (45):
//   chi(G, G', i omega_k) = sum_j c'_kj chi(G, G', i tau_j)
// with c'_kj = ct[k][j] * exp(-(eps_LUMO - eps_HOMO) tau_j): the caller's
// coefficient times the band-edge factor the staging step left out of the
// weights.  Inputs are read in the working precision and every product and
// sum is FP64; each output element sums j in increasing order.  With
// Hermitian completion the stored matrix is X and chi = X + X^H.
#include <type_traits>

#include "common.h"

namespace gw {
namespace {

template <typename T>
__device__ __forceinline__ double2 ld_x(const void *base, int64_t e) {
  if constexpr (sizeof(T) == 8) {
    return reinterpret_cast<const double2 *>(base)[e];
  } else {
    const float2 v = reinterpret_cast<const float2 *>(base)[e];
    return make_double2((double)v.x, (double)v.y);
  }
}

__device__ __forceinline__ int find_tile(const CtItem *items, int n, int t) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (items[mid].tile0 <= t) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// The cosine coefficients of a tile's frequencies, read through the constant
// address space: the index is the same in every lane, so they load as
// scalars (no vector registers, and no wait for them holds up the input
// loads in flight).
typedef __attribute__((address_space(4))) const double *ct_coef_ptr;

// One block per 32 (G) x 16 (G') output tile; thread (tx, ty) owns the two
// elements (a0 + ty + 16 i, b0 + tx), i = 0, 1, for CH frequencies.  The
// stored matrices are transposed, x_j[g'][g], so each tile of x_j is staged
// through LDS and read back transposed; output rows are written contiguously.
template <typename T, int CH>
__global__ __launch_bounds__(256) void k_ct(CtLaunch L, int k0) {
  __shared__ double2 t1[16][33];     // x_j[b0 + .][a0 + .]  = X[g][g'] transposed
  __shared__ double2 t2[32][17];     // x_j[a0 + .][b0 + .]  = X[g'][g] transposed
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;   // ty in [0, 16)
  for (int t = blockIdx.x; t < L.n_tiles; t += gridDim.x) {
    // the item index is the same in every lane: its fields load as scalars
    const CtItem it = L.items[__builtin_amdgcn_readfirstlane(find_tile(L.items, L.n_items, t))];
    if (k0 >= it.n_omega) continue;
    const int ng = it.n_g;
    const int ntb = (ng + 15) / 16;
    const int lt = t - it.tile0;
    const int a0 = (lt / ntb) * 32, b0 = (lt % ntb) * 16;
    const int64_t mat = (int64_t)ng * ng;
    double2 acc[2][CH];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int g = a0 + ty + 16 * i, gp = b0 + tx;
      const bool in = g < ng && gp < ng;
#pragma unroll
      for (int k = 0; k < CH; ++k)
        acc[i][k] = (it.accumulate && in && k0 + k < it.n_omega)
                        ? reinterpret_cast<const double2 *>(it.out)[(int64_t)(k0 + k) * mat +
                                                                    (int64_t)g * ng + gp]
                        : make_double2(0.0, 0.0);
    }
    for (int j = 0; j < it.n_tau_x; ++j) {
      const int64_t base = (int64_t)j * mat;
      // t1[gp][g] = x_j[b0 + gp][a0 + g]: 16 rows of 32
      for (int q = threadIdx.x; q < 16 * 32; q += 256) {
        const int r = q >> 5, c = q & 31;
        const int gp = b0 + r, g = a0 + c;
        t1[r][c] = (gp < ng && g < ng) ? ld_x<T>(it.x, base + (int64_t)gp * ng + g)
                                       : make_double2(0.0, 0.0);
      }
      if (it.hermitian) {
        // t2[g][gp] = x_j[a0 + g][b0 + gp]: 32 rows of 16
        for (int q = threadIdx.x; q < 32 * 16; q += 256) {
          const int r = q >> 4, c = q & 15;
          const int g = a0 + r, gp = b0 + c;
          t2[r][c] = (gp < ng && g < ng) ? ld_x<T>(it.x, base + (int64_t)g * ng + gp)
                                         : make_double2(0.0, 0.0);
        }
      }
      __syncthreads();
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const int gl = ty + 16 * i;       // 0..31
        double2 x = t1[tx][gl];           // X[g][g'] = x_j[g'][g]
        if (it.hermitian) {
          const double2 y = t2[gl][tx];   // X[g'][g] = x_j[g][g']
          x.x += y.x;
          x.y -= y.y;
        }
#pragma unroll
        for (int k = 0; k < CH; ++k) {
          if (k0 + k < it.n_omega) {
            const double c = it.coef[(int64_t)(k0 + k) * it.n_tau + it.j0 + j];
            acc[i][k].x += c * x.x;
            acc[i][k].y += c * x.y;
          }
        }
      }
      __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int g = a0 + ty + 16 * i, gp = b0 + tx;
      if (g < ng && gp < ng) {
#pragma unroll
        for (int k = 0; k < CH; ++k)
          if (k0 + k < it.n_omega)
            reinterpret_cast<double2 *>(it.out)[(int64_t)(k0 + k) * mat + (int64_t)g * ng + gp] =
                acc[i][k];
      }
    }
  }
}

// Hermitian completion: chi(i w_k) is Hermitian and out(b, a) = conj(out(a, b))^T
// holds exactly (the same sums with conjugated terms), so one block computes a
// 32x32 tile on or below the block diagonal and writes it and its mirror.
// 1024 threads, thread (tx, ty) owning element (a0 + ty, b0 + tx) for CH
// frequencies: one element per thread keeps the accumulators to 4 CH
// registers, so that four waves share each SIMD.  Per tau the thread needs
// X[g][g'] = x_j[g'][g] (the transposed tile, through LDS) and X[g'][g] =
// x_j[g][g'] (its own element, straight from its load).  The transposed tile
// alternates between two LDS buffers, so that one barrier per tau orders its
// writes and reads, and the input tiles of the next PD taus are in flight in
// registers while the current one is used.  The mirror tile is transposed
// through the same two buffers, one barrier per frequency.
template <typename T, int CH>
__global__ __launch_bounds__(1024, 4) void k_ct_herm(CtLaunch L, int k0) {
  constexpr int PD = sizeof(T) == 8 || CH > 16 ? 2 : 4;   // within 128 registers
  __shared__ double2 tt[2][32][33];  // tt[.][gp][g] = x_j[b0 + gp][a0 + g] = X[g][g']
  const int tid = threadIdx.x;
  const int tx = tid & 31, ty = tid >> 5;    // ty in [0, 32)
  typedef typename std::conditional<sizeof(T) == 8, double2, float2>::type V;
  for (int t = blockIdx.x; t < L.n_tiles; t += gridDim.x) {
    // the item index is the same in every lane: its fields load as scalars
    const CtItem it = L.items[__builtin_amdgcn_readfirstlane(find_tile(L.items, L.n_items, t))];
    if (k0 >= it.n_omega) continue;
    const int ng = it.n_g;
    const int lt = t - it.tile0;
    // lower-triangle tile index lt = ta (ta + 1) / 2 + tb, tb <= ta
    int ta = (int)((sqrt(8.0 * lt + 1.0) - 1.0) * 0.5);
    while ((ta + 1) * (ta + 2) / 2 <= lt) ++ta;
    while (ta * (ta + 1) / 2 > lt) --ta;
    const int tb = lt - ta * (ta + 1) / 2;
    const int a0 = ta * 32, b0 = tb * 32;
    const int64_t mat = (int64_t)ng * ng;
    const V *x = reinterpret_cast<const V *>(it.x);
    const int g = a0 + ty, gp = b0 + tx;
    const bool in = g < ng && gp < ng;
    double2 acc[CH];
#pragma unroll
    for (int k = 0; k < CH; ++k)
      acc[k] = (it.accumulate && in && k0 + k < it.n_omega)
                   ? reinterpret_cast<const double2 *>(it.out)[(int64_t)(k0 + k) * mat +
                                                               (int64_t)g * ng + gp]
                   : make_double2(0.0, 0.0);
    // those loads have landed: no wait for them stays in the tau loop (where
    // it would also wait for the input loads in flight)
    __builtin_amdgcn_s_waitcnt(0);
    // element (row ty, column tx) of each 32x32 input tile; the two tiles of
    // tau j + PD are fetched into register slot j % PD while tau j is used
    V r1[PD], r2[PD];
    const int g1 = a0 + tx, gp1 = b0 + ty;           // transposed tile: x_j[gp][g]
    const int g2 = a0 + ty, gp2 = b0 + tx;           // own element: x_j[g][gp]
    const bool ok1 = g1 < ng && gp1 < ng, ok2 = g2 < ng && gp2 < ng;
    auto fetch = [&](int j, V &q1, V &q2) {
      const int64_t base = (int64_t)j * mat;
      q1 = ok1 ? x[base + (int64_t)gp1 * ng + g1] : V{0, 0};
      q2 = ok2 ? x[base + (int64_t)g2 * ng + gp2] : V{0, 0};
    };
    const int nt = it.n_tau_x;
    const ct_coef_ptr cf = (ct_coef_ptr)(it.coef + (int64_t)k0 * it.n_tau + it.j0);
    sfor<0, PD>([&](auto ss) {
      constexpr int sl = decltype(ss)::value;
      if (sl < nt) fetch(sl, r1[sl], r2[sl]);
    });
    for (int jb = 0; jb < nt; jb += PD) {
      sfor<0, PD>([&](auto ss) {
        constexpr int sl = decltype(ss)::value;
        const int j = jb + sl;
        if (j < nt) {
          // buffer j % 2 was last read at tau j - 2, before the barrier of tau j - 1
          double2(*tb2)[33] = tt[j & 1];
          tb2[ty][tx] = make_double2((double)r1[sl].x, (double)r1[sl].y);
          const double wr = (double)r2[sl].x, wi = (double)r2[sl].y;
          __syncthreads();
          if (j + PD < nt) fetch(j + PD, r1[sl], r2[sl]);
          const double2 u = tb2[tx][ty];
          const double xr = u.x + wr, xi = u.y - wi;
#pragma unroll
          for (int k = 0; k < CH; ++k) {
            if (k0 + k < it.n_omega) {
              const double c = cf[(int64_t)k * it.n_tau + j];
              acc[k].x += c * xr;
              acc[k].y += c * xi;
            }
          }
        }
      });
    }
    double2 *out = reinterpret_cast<double2 *>(it.out);
    if (in) {
#pragma unroll
      for (int k = 0; k < CH; ++k)
        if (k0 + k < it.n_omega) out[(int64_t)(k0 + k) * mat + (int64_t)g * ng + gp] = acc[k];
    }
    // every read of the tau buffers is done before the mirror reuses them
    __syncthreads();
    if (ta != tb) {
      // mirror tile out[k][b0 + .][a0 + .] = conj(acc)^T, transposed through
      // LDS; frequency k uses buffer k % 2, last read at frequency k - 2,
      // before the barrier of frequency k - 1
#pragma unroll
      for (int k = 0; k < CH; ++k) {
        if (k0 + k >= it.n_omega) break;
        tt[k & 1][ty][tx] = acc[k];                  // [g_l][gp_l]
        __syncthreads();
        const double2 v = tt[k & 1][tx][ty];         // element (a0 + tx, b0 + ty)
        if (a0 + tx < ng && b0 + ty < ng)
          out[(int64_t)(k0 + k) * mat + (int64_t)(b0 + ty) * ng + a0 + tx] = make_double2(v.x, -v.y);
      }
      // the next tile's first tau writes buffer 0
      __syncthreads();
    }
  }
}

// FP32 inputs (the FP32 and split-BF16 paths): the same tiles, sums and
// mirror as k_ct_herm, with the input tiles of the coming taus loaded
// straight into a ring of R LDS stages instead of registers, so that R - 1
// taus (17 KB each) are in flight per block against the two of the register
// form.  A stage holds the transposed tile (rows x_j[b0 + r][a0 + .]) and the
// block's own tile (rows x_j[a0 + r][b0 + .]), 32 rows each of 32 complex
// values, one 256-byte wave load per row, rows padded to 272 bytes so that
// the column-wise reads of the transposed tile spread over the banks.  Rows
// and columns past n_g load a clamped valid address; they only feed outputs
// that are never stored.
// The loads are written out (global to LDS, 4 bytes per lane, M0 holding the
// wave's LDS row, written one wait state before the load) so that the
// compiler adds no wait of its own for them; the ring's waits order the
// stages: stage j is read after the vmcnt wait and barrier that cover its
// loads and refilled only after the barrier that follows its last reads.  No
// other code in this kernel reads M0.
#pragma clang diagnostic push
#pragma clang diagnostic ignored "-Winline-asm"
__device__ __forceinline__ void ct_dma4(const float *g, uint32_t lds) {
  asm volatile("s_mov_b32 m0, %1\n\ts_nop 0\n\tglobal_load_lds_dword %0, off"
               :
               : "v"(g), "s"(lds)
               : "memory", "m0");
}
#pragma clang diagnostic pop

// at most N vector-memory operations of this wave in flight, then the
// workgroup barrier (no fence: later stages' loads stay in flight)
template <int N>
__device__ __forceinline__ void ct_wait_barrier() {
  static_assert(N >= 0 && N < 64, "vmcnt has 6 bits");
  __builtin_amdgcn_sched_barrier(0);
  __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4) | (15 << 8));
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_sched_barrier(0);
}

template <int CH>
__global__ __launch_bounds__(1024, 4) void k_ct_herm_ring(CtLaunch L, int k0) {
  constexpr int R = 6;                       // stages
  constexpr int ROWB = 272;                  // 32 complex FP32 + 16 bytes of padding
  constexpr int STG = 64 * ROWB;             // transposed tile, then own tile
  constexpr int QW = 4;                      // row loads per wave per stage
  static_assert(R >= 2 && R - 2 <= 5 && QW * (R - 2) < 64, "waits cover the ring");
  __shared__ __attribute__((aligned(16))) char ring[R * STG];
  __shared__ double2 tt[2][32][33];          // mirror transposes
  const int tid = threadIdx.x;
  const int tx = tid & 31, ty = tid >> 5;    // ty in [0, 32)
  const int wv = tid >> 6, lane = tid & 63;
  const uint32_t lds_ring = __builtin_amdgcn_readfirstlane(
      (uint32_t)(uintptr_t)(__attribute__((address_space(3))) char *)ring);
  for (int t = blockIdx.x; t < L.n_tiles; t += gridDim.x) {
    // the item index is the same in every lane: its fields load as scalars
    const CtItem it = L.items[__builtin_amdgcn_readfirstlane(find_tile(L.items, L.n_items, t))];
    if (k0 >= it.n_omega) continue;
    const int ng = it.n_g;
    const int lt = t - it.tile0;
    int ta = (int)((sqrt(8.0 * lt + 1.0) - 1.0) * 0.5);
    while ((ta + 1) * (ta + 2) / 2 <= lt) ++ta;
    while (ta * (ta + 1) / 2 > lt) --ta;
    const int tb = lt - ta * (ta + 1) / 2;
    const int a0 = ta * 32, b0 = tb * 32;
    const int64_t mat = (int64_t)ng * ng;
    const int g = a0 + ty, gp = b0 + tx;
    const bool in = g < ng && gp < ng;
    double2 acc[CH];
#pragma unroll
    for (int k = 0; k < CH; ++k)
      acc[k] = (it.accumulate && in && k0 + k < it.n_omega)
                   ? reinterpret_cast<const double2 *>(it.out)[(int64_t)(k0 + k) * mat +
                                                               (int64_t)g * ng + gp]
                   : make_double2(0.0, 0.0);
    // those loads have landed: no wait for them stays in the tau loop (where
    // it would also wait for the input loads in flight)
    __builtin_amdgcn_s_waitcnt(0);
    // this wave's rows of a stage: q = 0, 1 transposed-tile rows 2 wv + q,
    // q = 2, 3 own-tile rows 2 wv + q - 2; lane = 2 * column + (re, im)
    // (offsets formed at each issue: registers go to the accumulators)
    const float *xf = reinterpret_cast<const float *>(it.x);
    const int nt = it.n_tau_x;
    const ct_coef_ptr cf = (ct_coef_ptr)(it.coef + (int64_t)k0 * it.n_tau + it.j0);
    auto issue = [&](int j) {
      const float *xj = xf + (int64_t)j * mat * 2;
      const uint32_t sb = lds_ring + (uint32_t)((j % R) * STG);
#pragma unroll
      for (int q = 0; q < QW; ++q) {
        const int r = 2 * wv + (q & 1);
        const bool own = q >= 2;
        const int row = min((own ? a0 : b0) + r, ng - 1);
        const int col = min((own ? b0 : a0) + (lane >> 1), ng - 1);
        const int64_t off = ((int64_t)row * ng + col) * 2 + (lane & 1);
        ct_dma4(xj + off, __builtin_amdgcn_readfirstlane(sb + (uint32_t)((own ? 32 + r : r) * ROWB)));
      }
    };
    for (int j = 0; j < R - 1 && j < nt; ++j) issue(j);
    for (int j = 0; j < nt; ++j) {
      // stage j has landed in every wave; the stages issued after it
      // (min(R - 2, nt - 1 - j) of them) may still be in flight
      switch (min(R - 2, nt - 1 - j)) {
        case 0: ct_wait_barrier<0>(); break;
        case 1: ct_wait_barrier<QW>(); break;
        case 2: ct_wait_barrier<2 * QW>(); break;
        case 3: ct_wait_barrier<3 * QW>(); break;
        default: ct_wait_barrier<4 * QW>(); break;
      }
      // refill the stage of tau j - 1, which every wave finished before this barrier
      if (j + R - 1 < nt) issue(j + R - 1);
      const char *st = ring + (j % R) * STG;
      const float2 u = *reinterpret_cast<const float2 *>(st + tx * ROWB + ty * 8);
      const float2 w = *reinterpret_cast<const float2 *>(st + (32 + ty) * ROWB + tx * 8);
      const double xr = (double)u.x + (double)w.x, xi = (double)u.y - (double)w.y;
#pragma unroll
      for (int k = 0; k < CH; ++k) {
        if (k0 + k < it.n_omega) {
          const double c = cf[(int64_t)k * it.n_tau + j];
          acc[k].x += c * xr;
          acc[k].y += c * xi;
        }
      }
    }
    double2 *out = reinterpret_cast<double2 *>(it.out);
    if (in) {
#pragma unroll
      for (int k = 0; k < CH; ++k)
        if (k0 + k < it.n_omega) out[(int64_t)(k0 + k) * mat + (int64_t)g * ng + gp] = acc[k];
    }
    // every read of the ring is done before the next tile refills it
    __syncthreads();
    if (ta != tb) {
      // mirror tile out[k][b0 + .][a0 + .] = conj(acc)^T through alternating buffers
#pragma unroll
      for (int k = 0; k < CH; ++k) {
        if (k0 + k >= it.n_omega) break;
        tt[k & 1][ty][tx] = acc[k];
        __syncthreads();
        const double2 v = tt[k & 1][tx][ty];
        if (a0 + tx < ng && b0 + ty < ng)
          out[(int64_t)(k0 + k) * mat + (int64_t)(b0 + ty) * ng + a0 + tx] = make_double2(v.x, -v.y);
      }
      __syncthreads();
    }
  }
}

// sum of |x|^2: mode 0 over the taus held in x (with Hermitian completion
// when set), mode 1 over the omegas of out.  Block x of the grid writes its
// partial sum of matrix m to slot [m][x] (kNormParts slots per matrix); the
// host adds the slots in order, so the result does not depend on the order
// in which blocks finish.
template <typename T>
__global__ __launch_bounds__(256) void k_norms(CtLaunch L, int mode, double *norm_tau,
                                               double *norm_omega, const int32_t *tau_off,
                                               const int32_t *omega_off) {
  __shared__ double red[4];
  const CtItem it = L.items[blockIdx.y];
  const int64_t mat = (int64_t)it.n_g * it.n_g;
  const int nm = mode == 0 ? it.n_tau_x : it.n_omega;
  for (int m = blockIdx.z; m < nm; m += gridDim.z) {
    double s = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < mat;
         e += (int64_t)gridDim.x * 256) {
      double2 x;
      if (mode == 0) {
        x = ld_x<T>(it.x, (int64_t)m * mat + e);
        if (it.hermitian) {
          const int64_t g = e / it.n_g, gp = e - g * it.n_g;
          const double2 y = ld_x<T>(it.x, (int64_t)m * mat + gp * it.n_g + g);
          x.x += y.x;
          x.y -= y.y;
        }
      } else {
        x = reinterpret_cast<const double2 *>(it.out)[(int64_t)m * mat + e];
      }
      s += x.x * x.x + x.y * x.y;
    }
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
      const double t = red[0] + red[1] + red[2] + red[3];
      const int64_t slot = mode == 0 ? tau_off[it.item] + it.j0 + m : omega_off[it.item] + m;
      (mode == 0 ? norm_tau : norm_omega)[slot * kNormParts + blockIdx.x] = t;
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void k_fill_zero(uint4 *p, int64_t n16, char *tail, int tail_n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride)
    p[i] = make_uint4(0, 0, 0, 0);
  if (blockIdx.x == 0 && (int)threadIdx.x < tail_n) tail[threadIdx.x] = 0;
}

template <typename T, int CH>
void launch_ct_herm_ch(const CtLaunch &L, int grid, int k0, hipStream_t s) {
  if constexpr (sizeof(T) == 4)
    hipLaunchKernelGGL((k_ct_herm_ring<CH>), dim3(grid), dim3(1024), 0, s, L, k0);
  else
    hipLaunchKernelGGL((k_ct_herm<T, CH>), dim3(grid), dim3(1024), 0, s, L, k0);
}

template <typename T>
hipError_t launch_ct_herm(const CtLaunch &L, int max_omega, hipStream_t s) {
  const int grid = L.n_tiles < 65536 ? L.n_tiles : 65536;
  int k0 = 0;
  while (k0 < max_omega) {
    const int left = max_omega - k0;
    if (left <= 4) launch_ct_herm_ch<T, 4>(L, grid, k0, s);
    else if (left <= 8) launch_ct_herm_ch<T, 8>(L, grid, k0, s);
    else if (left <= 12) launch_ct_herm_ch<T, 12>(L, grid, k0, s);
    else if (left <= 16) launch_ct_herm_ch<T, 16>(L, grid, k0, s);
    else launch_ct_herm_ch<T, 20>(L, grid, k0, s);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k0 += left <= 4 ? 4 : left <= 8 ? 8 : left <= 12 ? 12 : left <= 16 ? 16 : 20;
  }
  return hipSuccess;
}

}  // namespace

hipError_t launch_ct(const CtLaunch &L, int dbl, int max_omega, int hermitian, hipStream_t s) {
  if (L.n_tiles <= 0) return hipSuccess;
  if (hermitian) return dbl ? launch_ct_herm<double>(L, max_omega, s)
                            : launch_ct_herm<float>(L, max_omega, s);
  const int grid = L.n_tiles < 65536 ? L.n_tiles : 65536;
  constexpr int CH = 16;
  for (int k0 = 0; k0 < max_omega; k0 += CH) {
    if (dbl) hipLaunchKernelGGL((k_ct<double, CH>), dim3(grid), dim3(256), 0, s, L, k0);
    else hipLaunchKernelGGL((k_ct<float, CH>), dim3(grid), dim3(256), 0, s, L, k0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_norms_impl(const CtLaunch &L, int dbl, int mode, double *nt, double *nw,
                             const int32_t *toff, const int32_t *woff, int max_mats,
                             hipStream_t s) {
  if (L.n_items <= 0 || max_mats <= 0) return hipSuccess;
  dim3 grid(kNormParts, L.n_items, max_mats < 64 ? max_mats : 64);
  if (dbl) hipLaunchKernelGGL((k_norms<double>), grid, dim3(256), 0, s, L, mode, nt, nw, toff, woff);
  else hipLaunchKernelGGL((k_norms<float>), grid, dim3(256), 0, s, L, mode, nt, nw, toff, woff);
  return hipGetLastError();
}

hipError_t launch_fill_zero(void *p, int64_t bytes, hipStream_t s) {
  if (bytes <= 0) return hipSuccess;
  const int64_t n16 = bytes / 16;
  const int tail = (int)(bytes - n16 * 16);
  int64_t want = (n16 + 255) / 256;
  if (want < 1) want = 1;
  const int grid = (int)(want < 4096 ? want : 4096);
  hipLaunchKernelGGL(k_fill_zero, dim3(grid), dim3(256), 0, s, reinterpret_cast<uint4 *>(p), n16,
                     reinterpret_cast<char *>(p) + n16 * 16, tail);
  return hipGetLastError();
}

}  // namespace gw
