// Self-energy reductions and transforms (gfx950), Sec. II.D.
//
// The fused band-GEMM kernel leaves, per (item, tau_j) job, one partial sum
// per tile, state n and Green's function (occupied, unoccupied):
//   part[slot][n][side] = Re sum over the tile's lower-triangle points of
//                         conj(psi_n(r)) G~(r, r') W~(r, r') psi_n(r'),
// G~ being the Green's function scaled by its band-edge factor.  Here:
//   k_sigma_states : psi_n in the working precision, [n][r] zero-padded rows;
//   k_sigma_reduce : per (job, state) the sum of the slots in slot order
//                    (FP64, a fixed reduction tree: the result does not
//                    depend on the order in which tiles ran);
//   k_sigma_final  : per (item, state) the tau-domain elements
//                    Sigma_und(-i tau_j) = -2 e_o(tau_j) S_o,  Sigma_bar(i tau_j) = +2 e_u(tau_j) S_u
//                    (twice the lower-triangle sum is the Hermitian form), their
//                    even and odd parts (Eqs. (67)-(68)) and the cosine and
//                    sine transforms (Eqs. (69)-(71)), in FP64 with j increasing.
#include "common.h"

namespace gw {
namespace {

template <typename T2>
__global__ __launch_bounds__(256) void k_sigma_states(const double *phi_o, const double *phi_u,
                                                      const int32_t *states, int n_occ, int n_r,
                                                      int n_r_pad, T2 *out) {
  const int n = blockIdx.y;
  const int b = states[n];
  const double2 *src = reinterpret_cast<const double2 *>(b < n_occ ? phi_o : phi_u) +
                       (int64_t)(b < n_occ ? b : b - n_occ) * n_r;
  for (int r = blockIdx.x * 256 + threadIdx.x; r < n_r_pad; r += gridDim.x * 256) {
    const double2 v = r < n_r ? src[r] : make_double2(0.0, 0.0);
    out[(int64_t)n * n_r_pad + r] = T2{(decltype(T2{}.x))v.x, (decltype(T2{}.x))v.y};
  }
}

__global__ __launch_bounds__(256) void k_sigma_reduce(const SigmaRed *jobs) {
  __shared__ double r0[256], r1[256];
  const SigmaRed J = jobs[blockIdx.x];
  const int n = blockIdx.y;
  if (n >= J.n_states) return;
  const int t = threadIdx.x;
  double a0 = 0.0, a1 = 0.0;
  for (int s = t; s < J.n_slots; s += 256) {
    const double *p = J.part + ((int64_t)s * J.n_states + n) * 2;
    a0 += p[0];
    a1 += p[1];
  }
  r0[t] = a0;
  r1[t] = a1;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (t < h) {
      r0[t] += r0[t + h];
      r1[t] += r1[t + h];
    }
    __syncthreads();
  }
  if (t == 0) {
    J.sum[(int64_t)n * J.sum_stride + 0] = r0[0];
    J.sum[(int64_t)n * J.sum_stride + 1] = r1[0];
  }
}

__global__ __launch_bounds__(64) void k_sigma_final(const SigmaFin *items) {
  const SigmaFin F = items[blockIdx.x];
  const int n = blockIdx.y;
  if (n >= F.n_states) return;
  const double *sm = F.sum + (int64_t)n * F.n_tau * 2;
  for (int k = threadIdx.x; k < F.n_omega; k += blockDim.x) {
    double c = 0.0, s = 0.0;
    for (int j = 0; j < F.n_tau; ++j) {
      const double und = -2.0 * F.edge_o[j] * sm[2 * j];
      const double bar = 2.0 * F.edge_u[j] * sm[2 * j + 1];
      c += F.ct[(int64_t)k * F.n_tau + j] * (0.5 * (bar + und));
      s += F.st[(int64_t)k * F.n_tau + j] * (0.5 * (bar - und));
    }
    F.out[((int64_t)n * F.n_omega + k) * 2 + 0] = c;
    F.out[((int64_t)n * F.n_omega + k) * 2 + 1] = s;
  }
  if (F.out_tau)
    for (int j = threadIdx.x; j < F.n_tau; j += blockDim.x) {
      F.out_tau[((int64_t)n * F.n_tau + j) * 2 + 0] = -2.0 * F.edge_o[j] * sm[2 * j];
      F.out_tau[((int64_t)n * F.n_tau + j) * 2 + 1] = 2.0 * F.edge_u[j] * sm[2 * j + 1];
    }
}

}  // namespace

hipError_t launch_sigma_states(const double *phi_o, const double *phi_u, const int32_t *states,
                               int n_states, int n_occ, int n_r, int n_r_pad, int dbl, void *out,
                               hipStream_t s) {
  if (n_states <= 0) return hipSuccess;
  const int bx = (n_r_pad + 255) / 256 < 1024 ? (n_r_pad + 255) / 256 : 1024;
  dim3 grid(bx, n_states);
  if (dbl)
    hipLaunchKernelGGL(k_sigma_states<double2>, grid, dim3(256), 0, s, phi_o, phi_u, states,
                       n_occ, n_r, n_r_pad, reinterpret_cast<double2 *>(out));
  else
    hipLaunchKernelGGL(k_sigma_states<float2>, grid, dim3(256), 0, s, phi_o, phi_u, states,
                       n_occ, n_r, n_r_pad, reinterpret_cast<float2 *>(out));
  return hipGetLastError();
}

hipError_t launch_sigma_reduce(const SigmaRed *jobs, int n_jobs, int max_states, hipStream_t s) {
  if (n_jobs <= 0 || max_states <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_sigma_reduce, dim3(n_jobs, max_states), dim3(256), 0, s, jobs);
  return hipGetLastError();
}

hipError_t launch_sigma_final(const SigmaFin *items, int n_items, int max_states, int max_omega,
                              hipStream_t s) {
  (void)max_omega;
  if (n_items <= 0 || max_states <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_sigma_final, dim3(n_items, max_states), dim3(64), 0, s, items);
  return hipGetLastError();
}

}  // namespace gw
