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
// Operand chunks of KC bands go from global memory straight into a ring of
// LDS stages (direct loads, swizzled 16-byte slots), several chunks ahead of
// the MFMAs.
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
  static constexpr int KR = C ? 4 : 8;  // bands per read round (16-byte slots)
  static constexpr int NACC = 4;
  typedef d4v acc_t;
  // the FP64 16x16 result interleaves rows: value v of lane l is row l/16 + 4v
  static constexpr int acc_row(int l, int v) { return (l >> 4) + 4 * v; }
  static constexpr int acc_col(int l) { return l & 15; }
  static constexpr int frag_row(int l) { return l & 15; }
};

template <bool C>
struct MM<P_FP32, C> {
  static constexpr int MB = 32;
  static constexpr int KS = 2;
  static constexpr int BPB = C ? 8 : 4;
  static constexpr int KR = C ? 4 : 8;
  static constexpr int NACC = 16;
  typedef f16v acc_t;
  static constexpr int acc_row(int l, int v) {
    return 8 * (v >> 2) + 4 * (l >> 5) + (v & 3);
  }
  static constexpr int acc_col(int l) { return l & 31; }
  static constexpr int frag_row(int l) { return l & 31; }
};

template <bool C>
struct MM<P_BF16X3, C> {
  static constexpr int MB = 32;
  static constexpr int KS = 16;
  static constexpr int BPB = C ? 8 : 4;   // 2 B x (4 or 2) parts
  static constexpr int KR = 16;
  static constexpr int NACC = 16;
  typedef f16v acc_t;
  static constexpr int acc_row(int l, int v) {
    return 8 * (v >> 2) + 4 * (l >> 5) + (v & 3);
  }
  static constexpr int acc_col(int l) { return l & 31; }
  static constexpr int frag_row(int l) { return l & 31; }
};


__device__ __forceinline__ bf8v as_bf8(uint4 q) { return __builtin_bit_cast(bf8v, q); }
__device__ __forceinline__ uint4 neg_bf8(uint4 q) {
  q.x ^= 0x80008000u;
  q.y ^= 0x80008000u;
  q.z ^= 0x80008000u;
  q.w ^= 0x80008000u;
  return q;
}

// A record every lane reads at the same index, through the constant address
// space, word by word: it loads as scalars (no vector registers held, and no
// vector-memory wait for it also waits for the previous tile's stores).
template <typename R>
__device__ __forceinline__ R ld_c(const R *p, int64_t i) {
  static_assert(sizeof(R) % 4 == 0, "whole words");
  typedef const __attribute__((address_space(4))) uint32_t cw;
  cw *w = (cw *)(p + i);
  R r;
  uint32_t *d = reinterpret_cast<uint32_t *>(&r);
#pragma unroll
  for (int k = 0; k < (int)(sizeof(R) / 4); ++k) d[k] = w[k];
  return r;
}

// Workgroup tile: WM x 2 waves, each owning WTM x WTN MFMA blocks; K is
// consumed in chunks of KC bands.  The operand rows of one chunk (BM rows of
// the tile, then BN rows of its columns) sit in LDS as rows of ROWB bytes made
// of 16-byte slots; slot s of row r is stored at slot s ^ swz(r), so that the
// lanes reading one slot of 16 consecutive rows fall on distinct banks.  The LDS
// holds a ring of ST chunks, filled by direct global-to-LDS loads (1 KB per
// wave instruction) ST - 1 chunks ahead of the MFMAs.
template <int P, bool C, int WTM, int WTN, int KC, int WM, int OCC>
struct Tile {
  typedef MM<P, C> M;
  static constexpr int NW = 2 * WM;                // waves
  static constexpr int NT = 64 * NW;               // threads
  static constexpr int BM = WM * WTM * M::MB;
  static constexpr int BN = 2 * WTN * M::MB;
  static constexpr int ROWB = KC * M::BPB;         // bytes per operand row per chunk
  static constexpr int SPR = ROWB / 16;            // 16-byte slots per row
  static constexpr int BUF = (BM + BN) * ROWB;     // bytes per stage
  static constexpr int NB = BUF / 1024;            // 1 KB wave loads per stage
  static constexpr int LPW = NB / NW;              // of which each wave issues
  // stages: as many as fit the workgroup's share of the CU's 160 KB, at most 4
  static constexpr int WG_PER_CU = (2 * OCC) / WM > 1 ? (2 * OCC) / WM : 1;
  static constexpr int ST0 = (160 * 1024 / WG_PER_CU) / BUF;
  static constexpr int ST = ST0 > 4 ? 4 : ST0;
  static_assert(ROWB % 16 == 0 && BUF % 1024 == 0 && NB % NW == 0,
                "a stage must split into whole 1 KB loads per wave");
  static_assert(ST >= 2, "two stages must fit");
  static_assert(KC % M::KR == 0, "chunk must hold whole read rounds");
  static_assert(SPR == 1 || SPR == 2 || SPR == 4 || SPR == 8 || SPR % 16 == 0,
                "row of 1, 2, 4, 8 or 16k slots");
  // A 16-byte LDS read serves 16 lanes per cycle from a 256-byte bank window;
  // the 16 lanes read one logical slot of 16 consecutive rows, so the swizzle
  // gives those rows 16 distinct slot positions within the window.
  static __device__ __forceinline__ int swz(int r) {
    if constexpr (SPR >= 16) return r & 15;
    else if constexpr (SPR == 8) return (r >> 1) & 7;
    else if constexpr (SPR == 4) return (r >> 2) & 3;
    else if constexpr (SPR == 2) return (r >> 3) & 1;
    else return 0;
  }
  // byte offset of (row, logical slot) in a stage
  static __device__ __forceinline__ int at(int r, int s) { return r * ROWB + ((s ^ swz(r)) << 4); }
};

template <typename R>
__device__ __forceinline__ R wave_sum(R v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// SIG: the self-energy epilogue (products with W~ and the diagonal matrix
// elements) instead of the polarizability's Hadamard product.
template <int P, bool C, int WTM, int WTN, int KC, int WM, int OCC, bool SIG = false>
struct Gemm {
  typedef MM<P, C> M;
  typedef Tile<P, C, WTM, WTN, KC, WM, OCC> T;
  typedef typename M::acc_t acc_t;

  struct Acc {
    acc_t re[WTM][WTN];
    acc_t im[WTM][WTN];
  };

  // The unoccupied-band pass (the long one) of the FP64 and FP32 complex
  // polarizability and of the FP64 self-energy forms the sum of a * conj(b)
  // with three real products instead of four (the FP32 self-energy kernel,
  // short of registers for its epilogue, measured no faster with three):
  //   S1 += a.re b.re,  S2 += a.im b.im,  S3 += (a.re + a.im)(b.re - b.im),
  //   re = S1 + S2,     im = S3 - S1 + S2.
  // S1 and S2 sit in Acc.re and Acc.im, S3 in an Acc3; the pass ends by
  // combining them, so that two accumulator sets are live in the other pass.
  static constexpr bool G3 = C && (P == P_FP64 || (P == P_FP32 && !SIG));
  struct Acc3 {
    acc_t x[WTM][WTN];
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

  // Direct global -> LDS loads: wave w issues the 1 KB blocks w, w + NW, ...
  // of a stage; lane l of block b fills bytes 16 l .. 16 l + 15 of it, which
  // hold logical slot ((16 l) % ROWB / 16) ^ swz(row) of that row.  From one
  // load of a lane to its next the row advances by DR = NW KB / ROWB, a
  // multiple of 16 (so the slot and its swizzle stay the same), and the tile's
  // BM rows of A and BN rows of B are whole numbers of DR: load t of every
  // lane lies in A when t DR < BM, else in B.  A lane keeps only its first
  // row and slot byte (row0, sb0); the rest is per load and the same for all
  // lanes.
  static constexpr int DR = T::NW * 1024 / T::ROWB;
  static_assert((T::NW * 1024) % T::ROWB == 0 && DR % 16 == 0 && T::BM % DR == 0 &&
                    T::BN % DR == 0 && T::LPW * DR == T::BM + T::BN,
                "loads advance by whole swizzle periods and split at the A/B boundary");
  static __device__ __forceinline__ void dma_lane(uint32_t &row0, uint32_t &sb0) {
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int byte = w * 1024 + l * 16;
    const int row = byte / T::ROWB, p = (byte % T::ROWB) >> 4;
    row0 = (uint32_t)row;
    sb0 = (uint32_t)((p ^ T::swz(row)) << 4);
  }
  // the loads of one chunk: base points at the chunk's first band of row 0,
  // pitchB is the operand's row pitch in bytes (row offsets in 64 bits: an
  // operand can exceed 4 GB)
  //
  // The DMA instruction is written out rather than taken from the compiler's
  // builtin: the compiler cannot tell which stage a builtin DMA writes, so it
  // waits for every DMA in flight before the next LDS read, the prefetch of a
  // later chunk included, and the ring degenerates to load-then-compute.  The
  // ring's own waits (wait_then_barrier) are what order the stages: a stage is
  // read only after the vmcnt wait and barrier that cover its loads, and is
  // refilled only after the barrier that follows its last reads.  M0 holds the
  // wave's LDS destination (16 bytes per lane from there); it must be written
  // one wait state before the load.
  // (M0 is reserved to the compiler, which sets it before each of its own
  // uses; no other code in these kernels reads it.)
#pragma clang diagnostic push
#pragma clang diagnostic ignored "-Winline-asm"
  static __device__ __forceinline__ void dma16(const char *g, uint32_t lds) {
    asm volatile("s_mov_b32 m0, %1\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %0, off"
                 :
                 : "v"(g), "s"(lds)
                 : "memory", "m0");
  }
#pragma clang diagnostic pop
  // operand row of load t: r0 + row (A) or c0 + row - BM (B), row = row0 + t DR
  static __device__ __forceinline__ void issue(const char *base, uint32_t pitchB, int r0, int c0,
                                               uint32_t row0, uint32_t sb0, char *buf) {
    const int w = threadIdx.x >> 6;
    const uint32_t lds0 = __builtin_amdgcn_readfirstlane(
        (uint32_t)(uintptr_t)(__attribute__((address_space(3))) char *)(buf + w * 1024));
    const char *lane = base + sb0;
    sfor<0, T::LPW>([&](auto tt) {
      constexpr int t = decltype(tt)::value;
      const uint32_t g = (uint32_t)((t * DR < T::BM ? r0 : c0 - T::BM) + t * DR) + row0;
      dma16(lane + (uint64_t)g * pitchB, lds0 + t * T::NW * 1024);
    });
  }

  template <typename V>
  static __device__ __forceinline__ V ld(const char *buf, int r, int s) {
    return *reinterpret_cast<const V *>(buf + T::at(r, s));
  }

  // One chunk of KC bands from LDS into the accumulators.  Every lane reads
  // whole 16-byte slots; a slot holding several bands feeds as many MFMA steps
  // (the MFMA's k index is the lane group, and A and B use the same
  // band-to-(step, group) assignment, so every band enters the sum once).
  // The MFMA section runs at raised wave priority, so that of the waves
  // sharing a SIMD the one holding its operands keeps the matrix core busy
  // while the others issue their LDS reads (measured: +3 % on split-BF16,
  // neutral on FP32, none for FP64).
  static __device__ __forceinline__ void compute3(Acc &acc, Acc3 &x, const char *buf, int wr,
                                                  int wc) {
    if constexpr (P != P_FP64) __builtin_amdgcn_s_setprio(1);
    const int l = threadIdx.x & 63;
    const int ra = wr * WTM * M::MB + M::frag_row(l);
    const int rb = T::BM + wc * WTN * M::MB + M::frag_row(l);
#pragma unroll 4
    for (int kb = 0; kb < KC; kb += M::KR) {
      if constexpr (P == P_FP64) {
        const int s = kb + (l >> 4);           // one band per slot
        double2 a[WTM], b[WTN];
        double as[WTM], bd[WTN];
#pragma unroll
        for (int i = 0; i < WTM; ++i) {
          a[i] = ld<double2>(buf, ra + i * 16, s);
          as[i] = a[i].x + a[i].y;
        }
#pragma unroll
        for (int j = 0; j < WTN; ++j) {
          b[j] = ld<double2>(buf, rb + j * 16, s);
          bd[j] = b[j].x - b[j].y;
        }
#pragma unroll
        for (int i = 0; i < WTM; ++i)
#pragma unroll
          for (int j = 0; j < WTN; ++j) {
            acc.re[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i].x, b[j].x, acc.re[i][j], 0, 0, 0);
            acc.im[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i].y, b[j].y, acc.im[i][j], 0, 0, 0);
            x.x[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(as[i], bd[j], x.x[i][j], 0, 0, 0);
          }
      } else {
        const int s = (kb >> 1) + (l >> 5);    // two bands (re, im, re, im) per slot
        float4 a[WTM], b[WTN];
        float as[WTM][2], bd[WTN][2];
#pragma unroll
        for (int i = 0; i < WTM; ++i) {
          a[i] = ld<float4>(buf, ra + i * 32, s);
          as[i][0] = a[i].x + a[i].y;
          as[i][1] = a[i].z + a[i].w;
        }
#pragma unroll
        for (int j = 0; j < WTN; ++j) {
          b[j] = ld<float4>(buf, rb + j * 32, s);
          bd[j][0] = b[j].x - b[j].y;
          bd[j][1] = b[j].z - b[j].w;
        }
#pragma unroll
        for (int i = 0; i < WTM; ++i)
#pragma unroll
          for (int j = 0; j < WTN; ++j) {
            f16v &s1 = acc.re[i][j];
            f16v &s2 = acc.im[i][j];
            f16v &s3 = x.x[i][j];
            s1 = __builtin_amdgcn_mfma_f32_32x32x2f32(a[i].x, b[j].x, s1, 0, 0, 0);
            s2 = __builtin_amdgcn_mfma_f32_32x32x2f32(a[i].y, b[j].y, s2, 0, 0, 0);
            s3 = __builtin_amdgcn_mfma_f32_32x32x2f32(as[i][0], bd[j][0], s3, 0, 0, 0);
            s1 = __builtin_amdgcn_mfma_f32_32x32x2f32(a[i].z, b[j].z, s1, 0, 0, 0);
            s2 = __builtin_amdgcn_mfma_f32_32x32x2f32(a[i].w, b[j].w, s2, 0, 0, 0);
            s3 = __builtin_amdgcn_mfma_f32_32x32x2f32(as[i][1], bd[j][1], s3, 0, 0, 0);
          }
      }
    }
    if constexpr (P != P_FP64) __builtin_amdgcn_s_setprio(0);
  }

  static __device__ __forceinline__ void zero3(Acc3 &x) {
    sfor<0, WTM>([&](auto ii) {
      sfor<0, WTN>([&](auto jj) { x.x[decltype(ii)::value][decltype(jj)::value] = acc_t{}; });
    });
  }
  // re = S1 + S2, im = S3 - S1 + S2: the end of a three-product pass
  static __device__ __forceinline__ void combine3(Acc &acc, const Acc3 &x) {
    sfor<0, WTM>([&](auto ii) {
      constexpr int i = decltype(ii)::value;
      sfor<0, WTN>([&](auto jj) {
        constexpr int j = decltype(jj)::value;
        const acc_t s1 = acc.re[i][j], s2 = acc.im[i][j];
        acc.re[i][j] = s1 + s2;
        acc.im[i][j] = x.x[i][j] - s1 + s2;
      });
    });
  }

  static __device__ __forceinline__ void compute(Acc &acc, const char *buf, int wr, int wc) {
    if constexpr (P != P_FP64) __builtin_amdgcn_s_setprio(1);
    compute_body(acc, buf, wr, wc);
    if constexpr (P != P_FP64) __builtin_amdgcn_s_setprio(0);
  }
  static __device__ __forceinline__ void compute_body(Acc &acc, const char *buf, int wr, int wc) {
    const int l = threadIdx.x & 63;
    const int ra = wr * WTM * M::MB + M::frag_row(l);
    const int rb = T::BM + wc * WTN * M::MB + M::frag_row(l);
#pragma unroll
    for (int kb = 0; kb < KC; kb += M::KR) {
      if constexpr (P == P_FP64) {
        const int g = l >> 4;
        if constexpr (C) {
          // one band per slot: 4 bands, one step
          const int s = kb + g;
          double2 a[WTM], b[WTN];
#pragma unroll
          for (int i = 0; i < WTM; ++i) a[i] = ld<double2>(buf, ra + i * 16, s);
#pragma unroll
          for (int j = 0; j < WTN; ++j) b[j] = ld<double2>(buf, rb + j * 16, s);
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
          // two bands per slot: 8 bands, two steps
          const int s = (kb >> 1) + g;
          double2 a[WTM], b[WTN];
#pragma unroll
          for (int i = 0; i < WTM; ++i) a[i] = ld<double2>(buf, ra + i * 16, s);
#pragma unroll
          for (int j = 0; j < WTN; ++j) b[j] = ld<double2>(buf, rb + j * 16, s);
#pragma unroll
          for (int i = 0; i < WTM; ++i)
#pragma unroll
            for (int j = 0; j < WTN; ++j) {
              acc.re[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i].x, b[j].x, acc.re[i][j], 0, 0, 0);
              acc.re[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i].y, b[j].y, acc.re[i][j], 0, 0, 0);
            }
        }
      } else if constexpr (P == P_FP32) {
        const int g = l >> 5;
        if constexpr (C) {
          // two bands (re, im, re, im) per slot: 4 bands, two steps
          const int s = (kb >> 1) + g;
          float4 a[WTM], b[WTN];
#pragma unroll
          for (int i = 0; i < WTM; ++i) a[i] = ld<float4>(buf, ra + i * 32, s);
#pragma unroll
          for (int j = 0; j < WTN; ++j) b[j] = ld<float4>(buf, rb + j * 32, s);
#pragma unroll
          for (int i = 0; i < WTM; ++i)
#pragma unroll
            for (int j = 0; j < WTN; ++j) {
              f16v &re = acc.re[i][j];
              f16v &im = acc.im[i][j];
              re = __builtin_amdgcn_mfma_f32_32x32x2f32(a[i].x, b[j].x, re, 0, 0, 0);
              re = __builtin_amdgcn_mfma_f32_32x32x2f32(a[i].y, b[j].y, re, 0, 0, 0);
              im = __builtin_amdgcn_mfma_f32_32x32x2f32(a[i].y, b[j].x, im, 0, 0, 0);
              im = __builtin_amdgcn_mfma_f32_32x32x2f32(-a[i].x, b[j].y, im, 0, 0, 0);
              re = __builtin_amdgcn_mfma_f32_32x32x2f32(a[i].z, b[j].z, re, 0, 0, 0);
              re = __builtin_amdgcn_mfma_f32_32x32x2f32(a[i].w, b[j].w, re, 0, 0, 0);
              im = __builtin_amdgcn_mfma_f32_32x32x2f32(a[i].w, b[j].z, im, 0, 0, 0);
              im = __builtin_amdgcn_mfma_f32_32x32x2f32(-a[i].z, b[j].w, im, 0, 0, 0);
            }
        } else {
          // four bands per slot: 8 bands, four steps
          const int s = (kb >> 2) + g;
          float4 a[WTM], b[WTN];
#pragma unroll
          for (int i = 0; i < WTM; ++i) a[i] = ld<float4>(buf, ra + i * 32, s);
#pragma unroll
          for (int j = 0; j < WTN; ++j) b[j] = ld<float4>(buf, rb + j * 32, s);
#pragma unroll
          for (int i = 0; i < WTM; ++i)
#pragma unroll
            for (int j = 0; j < WTN; ++j) {
              f16v &re = acc.re[i][j];
              re = __builtin_amdgcn_mfma_f32_32x32x2f32(a[i].x, b[j].x, re, 0, 0, 0);
              re = __builtin_amdgcn_mfma_f32_32x32x2f32(a[i].y, b[j].y, re, 0, 0, 0);
              re = __builtin_amdgcn_mfma_f32_32x32x2f32(a[i].z, b[j].z, re, 0, 0, 0);
              re = __builtin_amdgcn_mfma_f32_32x32x2f32(a[i].w, b[j].w, re, 0, 0, 0);
            }
        }
      } else {
        // split-BF16: 8-band group grp, parts of one 16-byte slot each
        const int grp = (kb >> 3) + (l >> 5);
        if constexpr (C) {
          uint4 a[WTM][4], b[WTN][4];
#pragma unroll
          for (int i = 0; i < WTM; ++i)
#pragma unroll
            for (int p = 0; p < 4; ++p) a[i][p] = ld<uint4>(buf, ra + i * 32, 4 * grp + p);
#pragma unroll
          for (int j = 0; j < WTN; ++j)
#pragma unroll
            for (int p = 0; p < 4; ++p) b[j][p] = ld<uint4>(buf, rb + j * 32, 4 * grp + p);
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
            for (int p = 0; p < 2; ++p) a[i][p] = ld<uint4>(buf, ra + i * 32, 2 * grp + p);
#pragma unroll
          for (int j = 0; j < WTN; ++j)
#pragma unroll
            for (int p = 0; p < 2; ++p) b[j][p] = ld<uint4>(buf, rb + j * 32, 2 * grp + p);
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

  // wait until at most N vector-memory operations of this wave are in flight
  // (the LDS writes of direct loads count until they land), then the
  // workgroup barrier; no fence, so later stages' loads stay in flight
  template <int N>
  static __device__ __forceinline__ void wait_then_barrier() {
    static_assert(N >= 0 && N < 64, "vmcnt has 6 bits");
    __builtin_amdgcn_sched_barrier(0);
    __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4) | (15 << 8));
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_sched_barrier(0);
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
    // the same for every lane: keeps the unit's job fields in scalar registers
    const int u = __builtin_amdgcn_readfirstlane(*s_u);
    __syncthreads();
    return u;
  }

  // Self-energy epilogue (complex orbitals), Sec. II.D: with acc_o and acc_u
  // the edge-scaled Green's functions of the tile,
  //   M(r, r') = acc(r, r') W~(r, r')      on r >= r' (diagonal halved), 0 above,
  // and for every state n the tile's share of
  //   Re sum_{r, r'} conj(psi_n(r)) M(r, r') psi_n(r'),
  // so that, M being Hermitian, twice the sum over the lower tiles is the
  // diagonal element <n| G o W~ |n>.  The states pass through LDS NSC at a
  // time; each (state, occ|unocc) sum is reduced over the lanes, then over the
  // waves in order, and written to the tile's slot of job.part.
  static __device__ __forceinline__ void sigma_epilogue(const GemmJob &job, int r0, int c0,
                                                        int slot, Acc &ao, Acc &au, char *lds) {
    static_assert(C, "the self-energy epilogue is for complex orbitals");
    typedef typename std::conditional<P == P_FP64, double, float>::type R;
    typedef typename std::conditional<P == P_FP64, double2, float2>::type R2;
    constexpr int NSC = 8;
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int wr = w >> 1, wc = w & 1;
    const int n_r = job.n_r;
    const int cend = job.s0 + job.w;
    // W~ slab columns are grouped by 128 bytes (SH fixed per precision), so the
    // rows of one MFMA block sit at constant offsets from one base per block
    constexpr int SH = sizeof(R2) == 16 ? 3 : 4;
    const R2 *wsl = reinterpret_cast<const R2 *>(job.slab);
    // 1. products with W~ (read in the layout the chi epilogue writes)
    sfor<0, WTM>([&](auto ii) {
      constexpr int i = decltype(ii)::value;
      sfor<0, WTN>([&](auto jj) {
        constexpr int j = decltype(jj)::value;
        const int col = c0 + (wc * WTN + j) * M::MB + M::acc_col(l);
        const int cl = col - job.s0;
        const int row0 = r0 + (wr * WTM + i) * M::MB + M::acc_row(l, 0);
        const R2 *base = wsl + (((int64_t)(cl >> SH) * n_r + row0) << SH) + (cl & ((1 << SH) - 1));
        sfor<0, M::NACC>([&](auto vv) {
          constexpr int v = decltype(vv)::value;
          constexpr int dr = M::acc_row(0, v) - M::acc_row(0, 0);   // same for every lane
          const int row = row0 + dr;
          const bool ok = col < cend && row < n_r && row >= col;
          R2 x = ok ? base[dr << SH] : R2{(R)0, (R)0};
          if (row == col) x = R2{(R)0.5 * x.x, (R)0.5 * x.y};
          const R ore = ao.re[i][j][v], oim = ao.im[i][j][v];
          ao.re[i][j][v] = ore * x.x - oim * x.y;
          ao.im[i][j][v] = ore * x.y + oim * x.x;
          const R ure = au.re[i][j][v], uim = au.im[i][j][v];
          au.re[i][j][v] = ure * x.x - uim * x.y;
          au.im[i][j][v] = ure * x.y + uim * x.x;
        });
      });
    });
    // 2. the states, NSC at a time: rows of the tile, then its columns
    R2 *srow = reinterpret_cast<R2 *>(lds);                 // [BM][NSC]
    R2 *scol = srow + T::BM * NSC;                          // [BN][NSC]
    R *red = reinterpret_cast<R *>(scol + T::BN * NSC);     // [NW][NSC][2]
    const R2 *psi = reinterpret_cast<const R2 *>(job.states);
    for (int n0 = 0; n0 < job.n_states; n0 += NSC) {
      __syncthreads();
      for (int q = threadIdx.x; q < (T::BM + T::BN) * NSC; q += T::NT) {
        const int k = q / (T::BM + T::BN), rr = q - k * (T::BM + T::BN);
        const int g = rr < T::BM ? r0 + rr : c0 + (rr - T::BM);
        const R2 v = n0 + k < job.n_states ? psi[(int64_t)(n0 + k) * job.ld_states + g]
                                           : R2{(R)0, (R)0};
        if (rr < T::BM) srow[rr * NSC + k] = v;
        else scol[(rr - T::BM) * NSC + k] = v;
      }
      __syncthreads();
      // one state at a time (a run-time loop keeps the register set small)
#pragma unroll 1
      for (int k = 0; k < NSC; ++k) {
        R so = (R)0, su = (R)0;
        sfor<0, WTN>([&](auto jj) {
          constexpr int j = decltype(jj)::value;
          R tor = 0, toi = 0, tur = 0, tui = 0;
          sfor<0, WTM>([&](auto ii) {
            constexpr int i = decltype(ii)::value;
            sfor<0, M::NACC>([&](auto vv) {
              constexpr int v = decltype(vv)::value;
              const R2 p = srow[((wr * WTM + i) * M::MB + M::acc_row(l, v)) * NSC + k];
              // conj(p) * M
              tor += p.x * ao.re[i][j][v] + p.y * ao.im[i][j][v];
              toi += p.x * ao.im[i][j][v] - p.y * ao.re[i][j][v];
              tur += p.x * au.re[i][j][v] + p.y * au.im[i][j][v];
              tui += p.x * au.im[i][j][v] - p.y * au.re[i][j][v];
            });
          });
          const R2 q = scol[((wc * WTN + j) * M::MB + M::acc_col(l)) * NSC + k];
          so += tor * q.x - toi * q.y;
          su += tur * q.x - tui * q.y;
        });
        so = wave_sum(so);
        su = wave_sum(su);
        if (l == 0) {
          red[(w * NSC + k) * 2 + 0] = so;
          red[(w * NSC + k) * 2 + 1] = su;
        }
      }
      __syncthreads();
      if ((int)threadIdx.x < 2 * NSC) {
        const int k = threadIdx.x >> 1, side = threadIdx.x & 1;
        double a = 0.0;
        for (int ww = 0; ww < T::NW; ++ww) a += (double)red[(ww * NSC + k) * 2 + side];
        if (n0 + k < job.n_states)
          job.part[((int64_t)slot * job.n_states + n0 + k) * 2 + side] = a;
      }
    }
    // every wave is done with LDS before the next unit's loads refill it
    __syncthreads();
  }

  static __device__ __forceinline__ void run(const GemmLaunch &L) {
    // one LDS array per stage, so that the compiler sees which stage each
    // access touches and lets loads into other stages stay in flight
    __shared__ __attribute__((aligned(1024))) char st0[T::BUF], st1[T::BUF];
    __shared__ __attribute__((aligned(1024))) char st2[T::ST > 2 ? T::BUF : 16];
    __shared__ __attribute__((aligned(1024))) char st3[T::ST > 3 ? T::BUF : 16];
    auto stage = [&](auto ss) -> char * {
      constexpr int s = decltype(ss)::value;
      if constexpr (s == 0) return st0;
      else if constexpr (s == 1) return st1;
      else if constexpr (s == 2) return st2;
      else return st3;
    };
    __shared__ int s_u, s_q;
    const int w = threadIdx.x >> 6;
    const int l = threadIdx.x & 63;
    const int wr = w >> 1, wc = w & 1;     // WM rows x 2 columns of waves
    constexpr int ST = T::ST;
    for (int u = next_unit(L, -1, &s_u, &s_q); u < L.n_units;
         u = next_unit(L, u, &s_u, &s_q)) {
      const int4 unit = ld_c(L.units, u);
      const GemmJob job = ld_c(L.jobs, unit.x);
      const int r0 = unit.y, c0 = unit.z;
      uint32_t row0, sb0;
      dma_lane(row0, sb0);
      // one pipelined pass over the n chunks of an operand into acc
      // three: the three-product form (Acc3 x holds S3), else x is unused
      auto pipe = [&](auto three, Acc &acc, Acc3 &x, const void *psi, int ld, int n) {
        constexpr int CB = KC * M::BPB;      // bytes per chunk in a row
        const char *base = reinterpret_cast<const char *>(psi);
        const uint32_t pitch = (uint32_t)ld * M::BPB;
        sfor<0, ST - 1>([&](auto ss) {
          if (decltype(ss)::value < n)
            issue(base + (size_t)decltype(ss)::value * CB, pitch, r0, c0, row0, sb0, stage(ss));
        });
        for (int cb = 0; cb < n; cb += ST) {
          sfor<0, ST>([&](auto ss) {
            constexpr int s = decltype(ss)::value;
            const int c = cb + s;
            if (c < n) {
              // chunk c has landed in every wave (later chunks may be in flight)
              if (c + ST - 2 < n) wait_then_barrier<T::LPW * (ST - 2)>();
              else wait_then_barrier<0>();
              // refill the stage of chunk c - 1, which every wave has finished
              if (c + ST - 1 < n)
                issue(base + (size_t)(c + ST - 1) * CB, pitch, r0, c0, row0, sb0,
                      stage(std::integral_constant<int, (s + ST - 1) % ST>{}));
              if constexpr (decltype(three)::value) compute3(acc, x, stage(ss), wr, wc);
              else compute(acc, stage(ss), wr, wc);
            }
          });
        }
        // every wave is done with the stages before the next prologue refills them
        __syncthreads();
      };
      Acc ao, au;
      if constexpr (G3) {
        // the unoccupied pass first: its third accumulator set is free while
        // the occupied accumulators are not yet live
        zero(au);
        {
          Acc3 x;
          zero3(x);
          pipe(std::true_type{}, au, x, job.psi_u, job.ld_u, job.k_u / KC);
          combine3(au, x);
        }
        zero(ao);
        Acc3 unused;
        pipe(std::false_type{}, ao, unused, job.psi_o, job.ld_o, job.k_o / KC);
      } else {
        Acc3 unused;
        zero(ao);
        zero(au);
        pipe(std::false_type{}, ao, unused, job.psi_o, job.ld_o, job.k_o / KC);
        pipe(std::false_type{}, au, unused, job.psi_u, job.ld_u, job.k_u / KC);
      }
      if constexpr (SIG) {
        sigma_epilogue(job, r0, c0, unit.w, ao, au, st0);
        continue;
      }
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
          if constexpr (P != P_FP64 && C) {
            if (sh == 0) {
              // one-column groups: a lane's values v and v + 1 are adjacent rows of
              // one column, so they go out as one 16-byte store when both are kept
              auto val = [&](int v, int row) {
                const float ore = ao.re[i][j][v], ure = au.re[i][j][v];
                const float oim = ao.im[i][j][v], uim = au.im[i][j][v];
                float2 x = make_float2(-(ore * ure + oim * uim), -(oim * ure - ore * uim));
                if (herm && row == col) x = make_float2(0.5f * x.x, 0.0f);
                return x;
              };
              sfor<0, M::NACC / 2>([&](auto vv) {
                constexpr int v = 2 * decltype(vv)::value;
                const int row = r0 + (wr * WTM + i) * M::MB + M::acc_row(l, v);
                static_assert(M::acc_row(0, v + 1) == M::acc_row(0, v) + 1, "adjacent rows");
                const bool ok0 = col < cend && row < n_r && !(herm && row < col);
                const bool ok1 = col < cend && row + 1 < n_r && !(herm && row + 1 < col);
                const float2 x0 = val(v, row), x1 = val(v + 1, row + 1);
                float2 *dst = reinterpret_cast<float2 *>(job.slab) + cb + row;
                if (ok0 && ok1) {
                  *reinterpret_cast<float4 *>(dst) = make_float4(x0.x, x0.y, x1.x, x1.y);
                } else {
                  if (ok0) dst[0] = x0;
                  if (ok1) dst[1] = x1;
                }
              });
              return;
            }
          }
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

// OCC: minimum waves per SIMD the register allocation must allow; WM: rows
// of waves
template <int P, bool C, int WTM, int WTN, int KC, int OCC, int WM>
__global__ __launch_bounds__(128 * WM, OCC) void k_gemm(GemmLaunch L) {
  Gemm<P, C, WTM, WTN, KC, WM, OCC>::run(L);
}

template <int P, int WTM, int WTN, int KC, int OCC, int WM>
__global__ __launch_bounds__(128 * WM, OCC) void k_gemm_sigma(GemmLaunch L) {
  Gemm<P, true, WTM, WTN, KC, WM, OCC, true>::run(L);
}

struct TileCfg {
  int wtm, wtn, kc, wm;
  const char *name;
};

// Tile menus per (precision, complex).  Index 0 is the default.
// grid <= 0: persistent launch sized to the resident blocks of the device
// Resident workgroups per CU (occupancy query, once per tile; at least 1).
template <int P, bool C, int WTM, int WTN, int KC, int OCC, int WM>
int per_cu_of() {
  typedef Tile<P, C, WTM, WTN, KC, WM, OCC> T;
  auto kern = k_gemm<P, C, WTM, WTN, KC, OCC, WM>;
  static int per_cu = -1;
  if (per_cu < 0) {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kern, T::NT, 0) != hipSuccess || n < 1)
      n = 1;
    per_cu = n;
  }
  return per_cu;
}

template <int P, bool C, int WTM, int WTN, int KC, int OCC, int WM>
hipError_t launch_one(const GemmLaunch &L, int grid, int num_cu, hipStream_t s) {
  typedef Tile<P, C, WTM, WTN, KC, WM, OCC> T;
  const int per_cu = per_cu_of<P, C, WTM, WTN, KC, OCC, WM>();
  if (grid <= 0) grid = per_cu * num_cu;
  if (grid > L.n_units) grid = L.n_units;
  hipLaunchKernelGGL((k_gemm<P, C, WTM, WTN, KC, OCC, WM>), dim3(grid), dim3(T::NT), 0, s, L);
  return hipGetLastError();
}

// (precision, complex, wave tile M, wave tile N, K chunk, minimum waves per SIMD,
// rows of waves); entry 0 is the default.  Defaults come from timing every
// entry on the 24^3 complex and the 24^3 real workloads.
#define GW_TILES_FP64_C(X)                                                                     \
  X(P_FP64, true, 2, 2, 16, 2, 2) X(P_FP64, true, 1, 2, 16, 1, 4) X(P_FP64, true, 1, 2, 16, 2, 2) \
  X(P_FP64, true, 2, 1, 16, 2, 2) X(P_FP64, true, 2, 2, 8, 2, 2) X(P_FP64, true, 1, 1, 16, 2, 4)
#define GW_TILES_FP64_R(X)                                                                     \
  X(P_FP64, false, 2, 2, 16, 3, 2) X(P_FP64, false, 4, 2, 16, 2, 2) X(P_FP64, false, 2, 2, 32, 2, 2) \
  X(P_FP64, false, 2, 4, 16, 1, 2) X(P_FP64, false, 2, 2, 16, 1, 4) X(P_FP64, false, 1, 2, 32, 2, 4)
#define GW_TILES_FP32_C(X)                                                                     \
  X(P_FP32, true, 1, 2, 32, 1, 4) X(P_FP32, true, 1, 2, 16, 2, 2) X(P_FP32, true, 1, 2, 16, 1, 4) \
  X(P_FP32, true, 2, 1, 16, 2, 2) X(P_FP32, true, 2, 2, 16, 1, 2) X(P_FP32, true, 1, 1, 32, 2, 4)
#define GW_TILES_FP32_R(X)                                                                     \
  X(P_FP32, false, 2, 2, 16, 2, 2) X(P_FP32, false, 2, 2, 32, 2, 2) X(P_FP32, false, 2, 2, 16, 1, 4) \
  X(P_FP32, false, 1, 2, 32, 3, 2) X(P_FP32, false, 2, 4, 16, 1, 2) X(P_FP32, false, 1, 2, 32, 2, 4)
#define GW_TILES_BF16_C(X)                                                                     \
  X(P_BF16X3, true, 1, 2, 32, 1, 4) X(P_BF16X3, true, 2, 1, 16, 2, 2) X(P_BF16X3, true, 1, 2, 16, 2, 2) \
  X(P_BF16X3, true, 1, 2, 16, 1, 4) X(P_BF16X3, true, 2, 2, 16, 1, 2) X(P_BF16X3, true, 1, 1, 32, 2, 4)
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

// Self-energy tiles, one per precision (complex orbitals): (wave tile M, wave
// tile N, K chunk, minimum waves per SIMD, rows of waves).
#define GW_SIGMA_TILES(X) \
  X(P_FP64, 2, 2, 16, 2, 2) X(P_FP32, 1, 2, 32, 1, 4) X(P_BF16X3, 1, 2, 32, 1, 4)

namespace {
template <int P, int WTM, int WTN, int KC, int OCC, int WM>
int sigma_per_cu() {
  typedef Tile<P, true, WTM, WTN, KC, WM, OCC> T;
  static int per_cu = -1;
  if (per_cu < 0) {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &n, k_gemm_sigma<P, WTM, WTN, KC, OCC, WM>, T::NT, 0) != hipSuccess || n < 1)
      n = 1;
    per_cu = n;
  }
  return per_cu;
}
}  // namespace

int gemm_sigma_bm(int prec) {
#define GW_SBM(P, A, B, K, O, W) if (prec == P) return W * A * (P == P_FP64 ? 16 : 32);
  GW_SIGMA_TILES(GW_SBM)
#undef GW_SBM
  return 0;
}
int gemm_sigma_bn(int prec) {
#define GW_SBN(P, A, B, K, O, W) if (prec == P) return 2 * B * (P == P_FP64 ? 16 : 32);
  GW_SIGMA_TILES(GW_SBN)
#undef GW_SBN
  return 0;
}
int gemm_sigma_kc(int prec) {
#define GW_SKC(P, A, B, K, O, W) if (prec == P) return K;
  GW_SIGMA_TILES(GW_SKC)
#undef GW_SKC
  return 0;
}
int gemm_sigma_per_cu(int prec) {
#define GW_SPC(P, A, B, K, O, W) if (prec == P) return sigma_per_cu<P, A, B, K, O, W>();
  GW_SIGMA_TILES(GW_SPC)
#undef GW_SPC
  return 0;
}

hipError_t launch_gemm_sigma(const GemmLaunch &L, int prec, int grid, int num_cu, hipStream_t s) {
  if (L.n_units <= 0) return hipSuccess;
#define GW_SL(P, A, B, K, O, W)                                                         \
  if (prec == P) {                                                                      \
    typedef Tile<P, true, A, B, K, W, O> T;                                             \
    int g = grid > 0 ? grid : sigma_per_cu<P, A, B, K, O, W>() * num_cu;                \
    if (g > L.n_units) g = L.n_units;                                                   \
    hipLaunchKernelGGL((k_gemm_sigma<P, A, B, K, O, W>), dim3(g), dim3(T::NT), 0, s, L); \
    return hipGetLastError();                                                           \
  }
  GW_SIGMA_TILES(GW_SL)
#undef GW_SL
  return hipErrorInvalidValue;
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
