// Fused band contractions + Hadamard product on MFMA (gfx950).
//
// For one output tile (rows r of the grid, columns r' of the current slab)
// of one (item, tau) job:
//   acc_o(r, r') = sum_i Psi_o(r, i) conj(Psi_o(r', i))   = G_occ   / edge factor
//   acc_u(r, r') = sum_a Psi_u(r, a) conj(Psi_u(r', a))   = G_unocc / edge factor
//   chi(r, r')   = -acc_o(r, r') * conj(acc_u(r, r'))      (Eqs. (14)-(15))
// Neither Green's function leaves the registers: only chi is written, into
// the slab buffer grouped by columns, [column group][n_r][columns in group]
// with groups of 128 bytes, so that the lanes of one MFMA result row store
// contiguous runs and the FFT over r reads each group as one block.
//
// A complex product a * conj(b) is built from real MFMAs:
//   re += a.re b.re + a.im b.im,   im += a.im b.re - a.re b.im.
// Precisions:
//   FP64   v_mfma_f64_16x16x4_f64   (16x16 blocks, 4 bands per step)
//   FP32   v_mfma_f32_32x32x2_f32   (32x32 blocks, 2 bands per step)
//   BF16X3 v_mfma_f32_32x32x16_bf16 (32x32 blocks, 16 bands per step), each
//          real product as hi*hi + hi*lo + lo*hi with FP32 accumulation.
//
// A workgroup is WM x 2 waves; each wave owns WTM x WTN MFMA blocks.
// Operand chunks of KC bands are staged through LDS with a double buffer; the
// next chunk is fetched into registers while the current one feeds the MFMAs.
// The launch is persistent: as many workgroups as are resident take units
// with atomic tickets from per-XCD queues of compact tile groups (so that the
// tiles running together on one XCD share operand panels in its L2), or,
// without ticket counters, by grid stride.
#include <type_traits>

#include "common.h"

namespace gw {
namespace {

typedef float f4v __attribute__((ext_vector_type(4)));
typedef float f16v __attribute__((ext_vector_type(16)));
typedef double d4v __attribute__((ext_vector_type(4)));
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));

template <int P, bool C>
struct MM;

template <bool C>
struct MM<P_FP64, C> {
  static constexpr int MB = 16;         // block edge
  static constexpr int KS = 4;          // bands per MFMA step
  static constexpr int BPB = C ? 16 : 8;  // bytes per band element
  static constexpr int NACC = 4;
  typedef d4v acc_t;
  // the FP64 16x16 result interleaves rows: value v of lane l is row l/16 + 4v
  static __device__ __forceinline__ int acc_row(int l, int v) { return (l >> 4) + 4 * v; }
  static __device__ __forceinline__ int acc_col(int l) { return l & 15; }
  static __device__ __forceinline__ int frag_row(int l) { return l & 15; }
};

template <bool C>
struct MM<P_FP32, C> {
  static constexpr int MB = 32;
  static constexpr int KS = 2;
  static constexpr int BPB = C ? 8 : 4;
  static constexpr int NACC = 16;
  typedef f16v acc_t;
  static __device__ __forceinline__ int acc_row(int l, int v) {
    return 8 * (v >> 2) + 4 * (l >> 5) + (v & 3);
  }
  static __device__ __forceinline__ int acc_col(int l) { return l & 31; }
  static __device__ __forceinline__ int frag_row(int l) { return l & 31; }
};

template <bool C>
struct MM<P_BF16X3, C> {
  static constexpr int MB = 32;
  static constexpr int KS = 16;
  static constexpr int BPB = C ? 8 : 4;   // 2 B x (4 or 2) parts
  static constexpr int NACC = 16;
  typedef f16v acc_t;
  static __device__ __forceinline__ int acc_row(int l, int v) {
    return 8 * (v >> 2) + 4 * (l >> 5) + (v & 3);
  }
  static __device__ __forceinline__ int acc_col(int l) { return l & 31; }
  static __device__ __forceinline__ int frag_row(int l) { return l & 31; }
};

// compile-time loop: f(integral_constant<int, i>) for i in [B, E)
template <int B, int E, typename F>
__device__ __forceinline__ void sfor(F &&f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    sfor<B + 1, E>(f);
  }
}

__device__ __forceinline__ bf8v as_bf8(uint4 q) { return __builtin_bit_cast(bf8v, q); }
__device__ __forceinline__ uint4 neg_bf8(uint4 q) {
  q.x ^= 0x80008000u;
  q.y ^= 0x80008000u;
  q.z ^= 0x80008000u;
  q.w ^= 0x80008000u;
  return q;
}

template <int P, bool C, int WTM, int WTN, int KC, int WM>
struct Tile {
  typedef MM<P, C> M;
  static constexpr int NT = 128 * WM;            // threads: WM x 2 waves
  static constexpr int BM = WM * WTM * M::MB;
  static constexpr int BN = 2 * WTN * M::MB;
  static constexpr int ROWB = KC * M::BPB;        // bytes per operand row per chunk
  static constexpr int R16 = ROWB / 16;           // 16-B vectors per row
  static constexpr int PITCH = ROWB + 16;         // LDS row pitch (padding vs bank conflicts)
  static constexpr int NV = (BM + BN) * R16;      // vectors per chunk
  static constexpr int VPT = (NV + NT - 1) / NT;  // vectors per thread
  static constexpr int BUF = (BM + BN) * PITCH;   // bytes per LDS buffer
  static_assert(ROWB % 16 == 0, "row chunk must be 16-B aligned");
  static_assert(KC % M::KS == 0, "chunk must hold whole MFMA steps");
};

template <int P, bool C, int WTM, int WTN, int KC, int WM>
struct Gemm {
  typedef MM<P, C> M;
  typedef Tile<P, C, WTM, WTN, KC, WM> T;
  typedef typename M::acc_t acc_t;

  struct Acc {
    acc_t re[WTM][WTN];
    acc_t im[WTM][WTN];
  };

  static __device__ __forceinline__ void zero(Acc &a) {
    sfor<0, WTM>([&](auto ii) {
      sfor<0, WTN>([&](auto jj) {
        constexpr int i = decltype(ii)::value, j = decltype(jj)::value;
        a.re[i][j] = acc_t{};
        if constexpr (C) a.im[i][j] = acc_t{};
      });
    });
  }

  // global -> registers for chunk starting at band kc0
  // prefetch registers as one vector value, so that they stay in VGPRs
  typedef uint32_t regv_t __attribute__((ext_vector_type(4 * T::VPT)));
  struct Regs {
    regv_t v;
  };

  // global -> registers for the chunk starting at band kc0
  static __device__ __forceinline__ void fetch(Regs &reg, const char *base, int64_t pitchB,
                                               int r0, int c0, int kc0) {
    const int tid = threadIdx.x;
    sfor<0, T::VPT>([&](auto tt) {
      constexpr int t = decltype(tt)::value;
      const int v = tid + t * T::NT;
      if (T::NV % T::NT == 0 || v < T::NV) {
        const int row = v / T::R16, q = v % T::R16;
        const int grow = row < T::BM ? r0 + row : c0 + (row - T::BM);
        const char *p = base + (int64_t)grow * pitchB + (int64_t)kc0 * M::BPB + q * 16;
        const uint4 x = *reinterpret_cast<const uint4 *>(p);
        reg.v[4 * t + 0] = x.x;
        reg.v[4 * t + 1] = x.y;
        reg.v[4 * t + 2] = x.z;
        reg.v[4 * t + 3] = x.w;
      }
    });
  }

  static __device__ __forceinline__ void store(const Regs &reg, char *buf) {
    const int tid = threadIdx.x;
    sfor<0, T::VPT>([&](auto tt) {
      constexpr int t = decltype(tt)::value;
      const int v = tid + t * T::NT;
      if (T::NV % T::NT == 0 || v < T::NV) {
        const int row = v / T::R16, q = v % T::R16;
        *reinterpret_cast<uint4 *>(buf + row * T::PITCH + q * 16) =
            make_uint4(reg.v[4 * t + 0], reg.v[4 * t + 1], reg.v[4 * t + 2], reg.v[4 * t + 3]);
      }
    });
  }

  // one chunk of KC bands from LDS into the accumulators
  static __device__ __forceinline__ void compute(Acc &acc, const char *buf, int wr, int wc) {
    const int l = threadIdx.x & 63;
    const char *A = buf + (wr * WTM * M::MB) * T::PITCH;
    const char *B = buf + (T::BM + wc * WTN * M::MB) * T::PITCH;
    const int fr = M::frag_row(l);
#pragma unroll
    for (int kb = 0; kb < KC; kb += M::KS) {
      if constexpr (P == P_FP64) {
        const int band = kb + (l >> 4);
        if constexpr (C) {
          double2 a[WTM], b[WTN];
#pragma unroll
          for (int i = 0; i < WTM; ++i)
            a[i] = *reinterpret_cast<const double2 *>(A + (i * 16 + fr) * T::PITCH + band * 16);
#pragma unroll
          for (int j = 0; j < WTN; ++j)
            b[j] = *reinterpret_cast<const double2 *>(B + (j * 16 + fr) * T::PITCH + band * 16);
#pragma unroll
          for (int i = 0; i < WTM; ++i)
#pragma unroll
            for (int j = 0; j < WTN; ++j) {
              acc.re[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i].x, b[j].x, acc.re[i][j], 0, 0, 0);
              acc.re[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i].y, b[j].y, acc.re[i][j], 0, 0, 0);
              acc.im[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i].y, b[j].x, acc.im[i][j], 0, 0, 0);
              acc.im[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(-a[i].x, b[j].y, acc.im[i][j], 0, 0, 0);
            }
        } else {
          double a[WTM], b[WTN];
#pragma unroll
          for (int i = 0; i < WTM; ++i)
            a[i] = *reinterpret_cast<const double *>(A + (i * 16 + fr) * T::PITCH + band * 8);
#pragma unroll
          for (int j = 0; j < WTN; ++j)
            b[j] = *reinterpret_cast<const double *>(B + (j * 16 + fr) * T::PITCH + band * 8);
#pragma unroll
          for (int i = 0; i < WTM; ++i)
#pragma unroll
            for (int j = 0; j < WTN; ++j)
              acc.re[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc.re[i][j], 0, 0, 0);
        }
      } else if constexpr (P == P_FP32) {
        const int band = kb + (l >> 5);
        if constexpr (C) {
          float2 a[WTM], b[WTN];
#pragma unroll
          for (int i = 0; i < WTM; ++i)
            a[i] = *reinterpret_cast<const float2 *>(A + (i * 32 + fr) * T::PITCH + band * 8);
#pragma unroll
          for (int j = 0; j < WTN; ++j)
            b[j] = *reinterpret_cast<const float2 *>(B + (j * 32 + fr) * T::PITCH + band * 8);
#pragma unroll
          for (int i = 0; i < WTM; ++i)
#pragma unroll
            for (int j = 0; j < WTN; ++j) {
              acc.re[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[i].x, b[j].x, acc.re[i][j], 0, 0, 0);
              acc.re[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[i].y, b[j].y, acc.re[i][j], 0, 0, 0);
              acc.im[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[i].y, b[j].x, acc.im[i][j], 0, 0, 0);
              acc.im[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(-a[i].x, b[j].y, acc.im[i][j], 0, 0, 0);
            }
        } else {
          float a[WTM], b[WTN];
#pragma unroll
          for (int i = 0; i < WTM; ++i)
            a[i] = *reinterpret_cast<const float *>(A + (i * 32 + fr) * T::PITCH + band * 4);
#pragma unroll
          for (int j = 0; j < WTN; ++j)
            b[j] = *reinterpret_cast<const float *>(B + (j * 32 + fr) * T::PITCH + band * 4);
#pragma unroll
          for (int i = 0; i < WTM; ++i)
#pragma unroll
            for (int j = 0; j < WTN; ++j)
              acc.re[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[i], b[j], acc.re[i][j], 0, 0, 0);
        }
      } else {
        // split-BF16: 8-band group g, parts of 16 B each
        const int g = (kb >> 3) + (l >> 5);
        if constexpr (C) {
          uint4 a[WTM][4], b[WTN][4];
#pragma unroll
          for (int i = 0; i < WTM; ++i)
#pragma unroll
            for (int p = 0; p < 4; ++p)
              a[i][p] = *reinterpret_cast<const uint4 *>(A + (i * 32 + fr) * T::PITCH + g * 64 + p * 16);
#pragma unroll
          for (int j = 0; j < WTN; ++j)
#pragma unroll
            for (int p = 0; p < 4; ++p)
              b[j][p] = *reinterpret_cast<const uint4 *>(B + (j * 32 + fr) * T::PITCH + g * 64 + p * 16);
#pragma unroll
          for (int i = 0; i < WTM; ++i) {
            const bf8v arh = as_bf8(a[i][0]), arl = as_bf8(a[i][1]);
            const bf8v aih = as_bf8(a[i][2]), ail = as_bf8(a[i][3]);
            const bf8v nrh = as_bf8(neg_bf8(a[i][0])), nrl = as_bf8(neg_bf8(a[i][1]));
#pragma unroll
            for (int j = 0; j < WTN; ++j) {
              const bf8v brh = as_bf8(b[j][0]), brl = as_bf8(b[j][1]);
              const bf8v bih = as_bf8(b[j][2]), bil = as_bf8(b[j][3]);
              f16v &re = acc.re[i][j];
              f16v &im = acc.im[i][j];
              // re += a.re b.re + a.im b.im
              re = __builtin_amdgcn_mfma_f32_32x32x16_bf16(arl, brh, re, 0, 0, 0);
              re = __builtin_amdgcn_mfma_f32_32x32x16_bf16(arh, brl, re, 0, 0, 0);
              re = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ail, bih, re, 0, 0, 0);
              re = __builtin_amdgcn_mfma_f32_32x32x16_bf16(aih, bil, re, 0, 0, 0);
              re = __builtin_amdgcn_mfma_f32_32x32x16_bf16(arh, brh, re, 0, 0, 0);
              re = __builtin_amdgcn_mfma_f32_32x32x16_bf16(aih, bih, re, 0, 0, 0);
              // im += a.im b.re - a.re b.im
              im = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ail, brh, im, 0, 0, 0);
              im = __builtin_amdgcn_mfma_f32_32x32x16_bf16(aih, brl, im, 0, 0, 0);
              im = __builtin_amdgcn_mfma_f32_32x32x16_bf16(nrl, bih, im, 0, 0, 0);
              im = __builtin_amdgcn_mfma_f32_32x32x16_bf16(nrh, bil, im, 0, 0, 0);
              im = __builtin_amdgcn_mfma_f32_32x32x16_bf16(aih, brh, im, 0, 0, 0);
              im = __builtin_amdgcn_mfma_f32_32x32x16_bf16(nrh, bih, im, 0, 0, 0);
            }
          }
        } else {
          uint4 a[WTM][2], b[WTN][2];
#pragma unroll
          for (int i = 0; i < WTM; ++i)
#pragma unroll
            for (int p = 0; p < 2; ++p)
              a[i][p] = *reinterpret_cast<const uint4 *>(A + (i * 32 + fr) * T::PITCH + g * 32 + p * 16);
#pragma unroll
          for (int j = 0; j < WTN; ++j)
#pragma unroll
            for (int p = 0; p < 2; ++p)
              b[j][p] = *reinterpret_cast<const uint4 *>(B + (j * 32 + fr) * T::PITCH + g * 32 + p * 16);
#pragma unroll
          for (int i = 0; i < WTM; ++i)
#pragma unroll
            for (int j = 0; j < WTN; ++j) {
              f16v &re = acc.re[i][j];
              re = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf8(a[i][1]), as_bf8(b[j][0]), re, 0, 0, 0);
              re = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf8(a[i][0]), as_bf8(b[j][1]), re, 0, 0, 0);
              re = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf8(a[i][0]), as_bf8(b[j][0]), re, 0, 0, 0);
            }
        }
      }
    }
  }

  static __device__ __forceinline__ void phase(Acc &acc, char *lds, const void *psi, int ld,
                                               int k, int r0, int c0, int wr, int wc) {
    const int nchunks = k / KC;
    if (nchunks <= 0) return;
    const char *base = reinterpret_cast<const char *>(psi);
    const int64_t pitchB = (int64_t)ld * M::BPB;
    Regs reg;
    fetch(reg, base, pitchB, r0, c0, 0);
    store(reg, lds);
    __syncthreads();
    for (int c = 0; c < nchunks; ++c) {
      const bool more = c + 1 < nchunks;
      if (more) fetch(reg, base, pitchB, r0, c0, (c + 1) * KC);
      compute(acc, lds + (c & 1) * T::BUF, wr, wc);
      if (more) store(reg, lds + ((c + 1) & 1) * T::BUF);
      __syncthreads();
    }
  }

  // next unit: an atomic ticket on the workgroup's current queue, moving to
  // the following queues once it is empty (persistent grid), or the grid
  // stride.  *s_q holds the current queue; a return of n_units ends the loop.
  static __device__ __forceinline__ int next_unit(const GemmLaunch &L, int prev, int *s_u,
                                                  int *s_q) {
    if (L.counter == nullptr) return prev < 0 ? (int)blockIdx.x : prev + (int)gridDim.x;
    if (threadIdx.x == 0) {
      const int nq = L.n_queues;
      int q = prev < 0 ? (int)(blockIdx.x % (unsigned)nq) : *s_q;
      int u = L.n_units;
      for (int tries = 0; tries < nq; ++tries) {
        const int b = L.q_off[q], e = L.q_off[q + 1];
        if (b < e) {
          const int t = atomicAdd(L.counter + q, 1);
          if (t < e - b) {
            u = b + t;
            break;
          }
        }
        q = q + 1 == nq ? 0 : q + 1;
      }
      *s_q = q;
      *s_u = u;
    }
    __syncthreads();
    const int u = *s_u;
    __syncthreads();
    return u;
  }

  static __device__ __forceinline__ void run(const GemmLaunch &L, char *lds) {
    __shared__ int s_u, s_q;
    const int w = threadIdx.x >> 6;
    const int l = threadIdx.x & 63;
    const int wr = w >> 1, wc = w & 1;     // WM rows x 2 columns of waves
    for (int u = next_unit(L, -1, &s_u, &s_q); u < L.n_units;
         u = next_unit(L, u, &s_u, &s_q)) {
      const int4 unit = L.units[u];
      const GemmJob job = L.jobs[unit.x];
      const int r0 = unit.y, c0 = unit.z;
      Acc ao, au;
      zero(ao);
      zero(au);
      phase(ao, lds, job.psi_o, job.ld_o, job.k_o, r0, c0, wr, wc);
      phase(au, lds, job.psi_u, job.ld_u, job.k_u, r0, c0, wr, wc);
      // epilogue: chi = -acc_o * conj(acc_u), column-major slab
      const int n_r = job.n_r;
      const int cend = job.s0 + job.w;
      const bool herm = L.hermitian != 0;
      sfor<0, WTM>([&](auto ii) {
        constexpr int i = decltype(ii)::value;
        sfor<0, WTN>([&](auto jj) {
          constexpr int j = decltype(jj)::value;
          const int col = c0 + (wc * WTN + j) * M::MB + M::acc_col(l);
          const int cl = col - job.s0;
          const int sh = job.cg_shift;
          const int64_t cb = ((int64_t)(cl >> sh) * n_r << sh) + (cl & ((1 << sh) - 1));
          sfor<0, M::NACC>([&](auto vv) {
            constexpr int v = decltype(vv)::value;
            const int row = r0 + (wr * WTM + i) * M::MB + M::acc_row(l, v);
            const bool ok = col < cend && row < n_r && !(herm && row < col);
            const bool diag = herm && row == col;
            if constexpr (P == P_FP64) {
              const double ore = ao.re[i][j][v], ure = au.re[i][j][v];
              if constexpr (C) {
                const double oim = ao.im[i][j][v], uim = au.im[i][j][v];
                double2 x = make_double2(-(ore * ure + oim * uim), -(oim * ure - ore * uim));
                if (diag) x = make_double2(0.5 * x.x, 0.0);
                if (ok) reinterpret_cast<double2 *>(job.slab)[cb + ((int64_t)row << sh)] = x;
              } else {
                double x = -(ore * ure);
                if (diag) x *= 0.5;
                if (ok) reinterpret_cast<double *>(job.slab)[cb + ((int64_t)row << sh)] = x;
              }
            } else {
              const float ore = ao.re[i][j][v], ure = au.re[i][j][v];
              if constexpr (C) {
                const float oim = ao.im[i][j][v], uim = au.im[i][j][v];
                float2 x = make_float2(-(ore * ure + oim * uim), -(oim * ure - ore * uim));
                if (diag) x = make_float2(0.5f * x.x, 0.0f);
                if (ok) reinterpret_cast<float2 *>(job.slab)[cb + ((int64_t)row << sh)] = x;
              } else {
                float x = -(ore * ure);
                if (diag) x *= 0.5f;
                if (ok) reinterpret_cast<float *>(job.slab)[cb + ((int64_t)row << sh)] = x;
              }
            }
          });
        });
      });
    }
  }
};

// OCC: workgroups per CU the register allocation must allow; WM: rows of waves
template <int P, bool C, int WTM, int WTN, int KC, int OCC, int WM>
__global__ __launch_bounds__(128 * WM, OCC) void k_gemm(GemmLaunch L) {
  extern __shared__ __attribute__((aligned(16))) char lds[];
  Gemm<P, C, WTM, WTN, KC, WM>::run(L, lds);
}

struct TileCfg {
  int wtm, wtn, kc, wm;
  const char *name;
};

// Tile menus per (precision, complex).  Index 0 is the default.
// grid <= 0: persistent launch sized to the resident blocks of the device
// Resident workgroups per CU (occupancy query, once per tile; sets the LDS
// size attribute first).  0 on error.
template <int P, bool C, int WTM, int WTN, int KC, int OCC, int WM>
int per_cu_of() {
  typedef Tile<P, C, WTM, WTN, KC, WM> T;
  const int lds = 2 * T::BUF;
  auto kern = k_gemm<P, C, WTM, WTN, KC, OCC, WM>;
  static int per_cu = -1;
  if (per_cu < 0) {
    if (hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                            hipFuncAttributeMaxDynamicSharedMemorySize, lds) != hipSuccess)
      return 0;
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kern, T::NT, lds) != hipSuccess || n < 1)
      n = 1;
    per_cu = n;
  }
  return per_cu;
}

template <int P, bool C, int WTM, int WTN, int KC, int OCC, int WM>
hipError_t launch_one(const GemmLaunch &L, int grid, int num_cu, hipStream_t s) {
  typedef Tile<P, C, WTM, WTN, KC, WM> T;
  const int lds = 2 * T::BUF;
  const int per_cu = per_cu_of<P, C, WTM, WTN, KC, OCC, WM>();
  if (per_cu == 0) return hipErrorInvalidValue;
  if (grid <= 0) grid = per_cu * num_cu;
  if (grid > L.n_units) grid = L.n_units;
  hipLaunchKernelGGL((k_gemm<P, C, WTM, WTN, KC, OCC, WM>), dim3(grid), dim3(T::NT), lds, s, L);
  return hipGetLastError();
}

// (precision, complex, wave tile M, wave tile N, K chunk, workgroups per CU,
// rows of waves); entry 0 is the default.  Defaults come from timing every
// entry on the 24^3 complex and the 24^3 real workloads.
#define GW_TILES_FP64_C(X)                                                                     \
  X(P_FP64, true, 2, 2, 16, 2, 2) X(P_FP64, true, 1, 2, 16, 1, 4) X(P_FP64, true, 1, 2, 16, 2, 2) \
  X(P_FP64, true, 2, 1, 16, 2, 2) X(P_FP64, true, 2, 2, 8, 2, 2) X(P_FP64, true, 1, 1, 16, 2, 4)
#define GW_TILES_FP64_R(X)                                                                     \
  X(P_FP64, false, 2, 2, 16, 1, 4) X(P_FP64, false, 2, 2, 16, 3, 2) X(P_FP64, false, 2, 2, 32, 2, 2) \
  X(P_FP64, false, 4, 2, 16, 2, 2) X(P_FP64, false, 2, 4, 16, 1, 2) X(P_FP64, false, 1, 2, 32, 2, 4)
#define GW_TILES_FP32_C(X)                                                                     \
  X(P_FP32, true, 1, 2, 16, 1, 4) X(P_FP32, true, 2, 1, 16, 2, 2) X(P_FP32, true, 1, 2, 16, 2, 2) \
  X(P_FP32, true, 1, 2, 32, 1, 4) X(P_FP32, true, 2, 2, 16, 1, 2) X(P_FP32, true, 1, 1, 32, 2, 4)
#define GW_TILES_FP32_R(X)                                                                     \
  X(P_FP32, false, 2, 2, 16, 2, 2) X(P_FP32, false, 2, 2, 32, 2, 2) X(P_FP32, false, 2, 2, 16, 1, 4) \
  X(P_FP32, false, 1, 2, 32, 3, 2) X(P_FP32, false, 2, 4, 16, 1, 2) X(P_FP32, false, 1, 2, 32, 2, 4)
#define GW_TILES_BF16_C(X)                                                                     \
  X(P_BF16X3, true, 1, 2, 16, 1, 4) X(P_BF16X3, true, 2, 2, 16, 1, 2) X(P_BF16X3, true, 1, 2, 32, 1, 4) \
  X(P_BF16X3, true, 1, 2, 16, 2, 2) X(P_BF16X3, true, 2, 1, 16, 2, 2) X(P_BF16X3, true, 1, 1, 32, 2, 4)
#define GW_TILES_BF16_R(X)                                                                     \
  X(P_BF16X3, false, 2, 2, 32, 2, 2) X(P_BF16X3, false, 2, 2, 32, 1, 4) X(P_BF16X3, false, 1, 2, 32, 3, 2) \
  X(P_BF16X3, false, 2, 2, 16, 2, 2) X(P_BF16X3, false, 2, 4, 32, 1, 2) X(P_BF16X3, false, 1, 2, 32, 2, 4)

#define GW_COUNT(P, C, A, B, K, O, W) +1
#define GW_CFG(P, C, A, B, K, O, W) {A, B, K, W, #P "/" #C "/" #A "x" #B "/k" #K "/o" #O "/w" #W},

template <int P, bool C>
struct Menu;
#define GW_MENU(P, C, LIST)                                                   \
  template <>                                                                 \
  struct Menu<P, C> {                                                         \
    static constexpr int n = 0 LIST(GW_COUNT);                                \
    static const TileCfg *cfg() {                                             \
      static const TileCfg c[] = {LIST(GW_CFG)};                              \
      return c;                                                               \
    }                                                                         \
  };
GW_MENU(P_FP64, true, GW_TILES_FP64_C)
GW_MENU(P_FP64, false, GW_TILES_FP64_R)
GW_MENU(P_FP32, true, GW_TILES_FP32_C)
GW_MENU(P_FP32, false, GW_TILES_FP32_R)
GW_MENU(P_BF16X3, true, GW_TILES_BF16_C)
GW_MENU(P_BF16X3, false, GW_TILES_BF16_R)

const TileCfg *menu(int prec, int cplx, int *n) {
#define GW_SEL(P, C)                    \
  if (prec == P && (cplx != 0) == C) {  \
    *n = Menu<P, C>::n;                 \
    return Menu<P, C>::cfg();           \
  }
  GW_SEL(P_FP64, true) GW_SEL(P_FP64, false) GW_SEL(P_FP32, true) GW_SEL(P_FP32, false)
  GW_SEL(P_BF16X3, true) GW_SEL(P_BF16X3, false)
#undef GW_SEL
  *n = 0;
  return nullptr;
}

int mb_of(int prec) { return prec == P_FP64 ? 16 : 32; }

}  // namespace

int gemm_tile_count(int prec, int cplx) {
  int n = 0;
  menu(prec, cplx, &n);
  return n;
}
int gemm_tile_bm(int prec, int cplx, int tile) {
  int n = 0;
  const TileCfg *c = menu(prec, cplx, &n);
  return (c && tile >= 0 && tile < n) ? c[tile].wm * c[tile].wtm * mb_of(prec) : 0;
}
int gemm_tile_bn(int prec, int cplx, int tile) {
  int n = 0;
  const TileCfg *c = menu(prec, cplx, &n);
  return (c && tile >= 0 && tile < n) ? 2 * c[tile].wtn * mb_of(prec) : 0;
}
int gemm_tile_kc(int prec, int cplx, int tile) {
  int n = 0;
  const TileCfg *c = menu(prec, cplx, &n);
  return (c && tile >= 0 && tile < n) ? c[tile].kc : 0;
}
const char *gemm_tile_name(int prec, int cplx, int tile) {
  int n = 0;
  const TileCfg *c = menu(prec, cplx, &n);
  return (c && tile >= 0 && tile < n) ? c[tile].name : "?";
}

int gemm_tile_per_cu(int prec, int cplx, int tile) {
  int idx = 0;
#define GW_TRY(P, C, A, B, K, O, W)                           \
  if (prec == P && (cplx != 0) == C) {                        \
    if (idx == tile) return per_cu_of<P, C, A, B, K, O, W>(); \
    ++idx;                                                    \
  }
  GW_TILES_FP64_C(GW_TRY)
  GW_TILES_FP64_R(GW_TRY)
  GW_TILES_FP32_C(GW_TRY)
  GW_TILES_FP32_R(GW_TRY)
  GW_TILES_BF16_C(GW_TRY)
  GW_TILES_BF16_R(GW_TRY)
#undef GW_TRY
  return 0;
}

hipError_t launch_gemm(const GemmLaunch &L, int prec, int cplx, int tile, int grid, int num_cu,
                       hipStream_t s) {
  if (L.n_units <= 0) return hipSuccess;
  int idx = 0;
#define GW_TRY(P, C, A, B, K, O, W)                                  \
  if (prec == P && (cplx != 0) == C) {                               \
    if (idx == tile) return launch_one<P, C, A, B, K, O, W>(L, grid, num_cu, s); \
    ++idx;                                                           \
  }
  GW_TILES_FP64_C(GW_TRY)
  GW_TILES_FP64_R(GW_TRY)
  GW_TILES_FP32_C(GW_TRY)
  GW_TILES_FP32_R(GW_TRY)
  GW_TILES_BF16_C(GW_TRY)
  GW_TILES_BF16_R(GW_TRY)
#undef GW_TRY
  return hipErrorInvalidValue;
}

}  // namespace gw
