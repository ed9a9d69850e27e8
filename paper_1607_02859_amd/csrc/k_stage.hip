// Weights and operand staging (gfx950).
//
// For one imaginary time tau the occupied and unoccupied Green's functions
// are G = Phi diag(w) Phi^H (Sec. II.A.1, Eqs. (1)-(2)).  Writing
// w = s^2 gives G = Psi Psi^H with Psi = Phi diag(s), so both GEMM operands
// come from one scaled matrix.  The weights are evaluated here in FP64,
// normalised to the band edge so that every s <= 1:
//   occupied:   s_i = exp(+0.5 (eps_i - eps_HOMO) tau)
//   unoccupied: s_a = exp(-0.5 (eps_a - eps_LUMO) tau)
// The edge factor exp(-(eps_LUMO - eps_HOMO) tau) that this leaves out of
// chi (mu cancels in the product of the two weights, the time dependence
// under Eq. (16)) is applied in FP64 by the cosine transform.
//
// Output layout per (item, tau, occ|unocc): row-major [n_r_pad][k_pad] in the
// working precision, bands contiguous, zero rows past n_r and zero bands past k:
//   FP64   : double2 (complex) / double (real)
//   FP32   : float2 / float
//   BF16X3 : per 8-band group, parts [re_hi][re_lo][im_hi][im_lo] x 8 bf16
//            (complex, 64 B) or [hi][lo] x 8 bf16 (real, 32 B), where, with
//            x the FP32 operand of the FP32 path, hi = bf16(x) and
//            lo = bf16(x - hi), both round-to-nearest-even (x - hi is exact
//            in FP32: hi keeps the leading 8 of x's 24 significand bits).
#include "common.h"

namespace gw {
namespace {

constexpr int kStageR = 64;   // grid points per block
constexpr int kStageK = 32;   // bands per block

__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float bf16_to_f32(uint16_t h) {
  return __uint_as_float(((uint32_t)h) << 16);
}

// split x into hi + lo, both bf16
__device__ __forceinline__ void split_bf16(float x, uint16_t &hi, uint16_t &lo) {
  hi = f32_to_bf16_rne(x);
  lo = f32_to_bf16_rne(x - bf16_to_f32(hi));
}

// A record every lane reads at the same index, through the constant address
// space, word by word: it loads as scalars, so no vector-memory wait for it
// (the wait counter being in order) also waits for the previous tau's stores.
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

__global__ __launch_bounds__(256) void k_stage(StageLaunch L) {
  __shared__ double2 tile[kStageK][kStageR + 1];
  __shared__ double sc[kStageK];
  const int tid = threadIdx.x;
  for (int b = blockIdx.x; b < L.n_blocks; b += gridDim.x) {
    const int4 blk = ld_c(L.blocks, b);
    const StageOp op = ld_c(L.ops, blk.x);
    const int r0 = blk.y * kStageR;
    const int k0 = blk.z * kStageK;
    // load Phi[perm[k]][r] for the tile, zero outside the real ranges
    for (int idx = tid; idx < kStageK * kStageR; idx += 256) {
      const int kk = idx / kStageR, rr = idx % kStageR;
      const int k = k0 + kk, r = r0 + rr;
      double2 v = make_double2(0.0, 0.0);
      if (k < op.k && r < op.n_r) {
        const int64_t src = (int64_t)op.perm[k] * op.n_r + r;
        if (op.cplx) {
          v = reinterpret_cast<const double2 *>(op.phi)[src];
        } else {
          v.x = op.phi[src];
        }
      }
      tile[kk][rr] = v;
    }
    // the band's eigenvalue once per block; per tau only scalar loads
    const double eps_k = (tid < kStageK && k0 + tid < op.k) ? op.eps[k0 + tid] : 0.0;
    for (int j = 0; j < op.n_jobs; ++j) {
      __syncthreads();
      const double tau_j = ld_c(op.tau, j);
      if (tid < kStageK) {
        const int k = k0 + tid;
        double s = 0.0;
        if (k < op.k) s = exp(0.5 * op.sign * (eps_k - op.edge) * tau_j);
        sc[tid] = s;
      }
      __syncthreads();
      char *out = reinterpret_cast<char *>(ld_c(op.psi, j));
      if (L.prec == P_FP64 || L.prec == P_FP32) {
        for (int idx = tid; idx < kStageK * kStageR; idx += 256) {
          const int rr = idx / kStageK, kk = idx % kStageK;
          const double2 v = tile[kk][rr];
          const double s = sc[kk];
          const int64_t e = (int64_t)(r0 + rr) * op.k_pad + (k0 + kk);
          if (L.prec == P_FP64) {
            if (op.cplx)
              reinterpret_cast<double2 *>(out)[e] = make_double2(v.x * s, v.y * s);
            else
              reinterpret_cast<double *>(out)[e] = v.x * s;
          } else {
            if (op.cplx)
              reinterpret_cast<float2 *>(out)[e] =
                  make_float2((float)(v.x * s), (float)(v.y * s));
            else
              reinterpret_cast<float *>(out)[e] = (float)(v.x * s);
          }
        }
      } else {
        // split-BF16: one thread per (row, 8-band group)
        constexpr int groups = kStageK / 8;
        const int parts = op.cplx ? 4 : 2;
        for (int idx = tid; idx < kStageR * groups; idx += 256) {
          const int rr = idx / groups, g = idx % groups;
          uint16_t hr[8], lr[8], hi_[8], li[8];
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            const double2 v = tile[g * 8 + e][rr];
            const double s = sc[g * 8 + e];
            split_bf16((float)(v.x * s), hr[e], lr[e]);
            split_bf16((float)(v.y * s), hi_[e], li[e]);
          }
          const int64_t row_bytes = (int64_t)op.k_pad * 2 * parts;   // 8 bands * 2 B * parts / 8
          char *dst = out + (int64_t)(r0 + rr) * row_bytes + (int64_t)((k0 / 8) + g) * 16 * parts;
          uint4 w[4];
          auto pack = [](const uint16_t *h) {
            uint4 q;
            q.x = h[0] | ((uint32_t)h[1] << 16);
            q.y = h[2] | ((uint32_t)h[3] << 16);
            q.z = h[4] | ((uint32_t)h[5] << 16);
            q.w = h[6] | ((uint32_t)h[7] << 16);
            return q;
          };
          w[0] = pack(hr);
          w[1] = pack(lr);
          w[2] = pack(hi_);
          w[3] = pack(li);
          // constant indices: w stays in registers (a run-time loop over the
          // parts put it in scratch memory, one load, wait and store per part)
          uint4 *d4 = reinterpret_cast<uint4 *>(dst);
          d4[0] = w[0];
          d4[1] = w[1];
          if (parts == 4) {
            d4[2] = w[2];
            d4[3] = w[3];
          }
        }
      }
    }
    __syncthreads();
  }
}

}  // namespace

hipError_t launch_stage(const StageLaunch &L, int prec, hipStream_t s) {
  if (L.n_blocks <= 0) return hipSuccess;
  (void)prec;
  const int grid = L.n_blocks < 8192 ? L.n_blocks : 8192;
  hipLaunchKernelGGL(k_stage, dim3(grid), dim3(256), 0, s, L);
  return hipGetLastError();
}

}  // namespace gw
