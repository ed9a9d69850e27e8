// Analytic continuation by Thiele's reciprocal differences (gfx950), FP64.
//
// For each function f known at N points z_1..z_N (Sec. II.E.1, Eqs. (72)-(74)):
//   g_1(z_j) = f_j,  g_n(z_j) = (g_{n-1}(z_{n-1}) - g_{n-1}(z_j)) / ((z_j - z_{n-1}) g_{n-1}(z_j)),
//   a_n = g_n(z_n),
//   P_N(w) = a_1 / (1 + a_2 (w - z_1) / (1 + ... a_N (w - z_{N-1}) / 1)),
// the tail of the last denominator dropped; an exactly zero denominator in
// the recursion ends the fraction (that difference and every deeper one are 0).
//
// One wave per function: lane j holds g_n(z_j) through the recursion (updated
// in place, j >= n; a_{n-1} is broadcast from its lane at each level), then
// every lane takes all coefficients and the lanes share the evaluation points,
// so that the outputs of a function are written in contiguous runs.  The
// points z and w are shared by all functions.
//
// The fraction is evaluated from the innermost level out, with the tail
// t_k = 1 + c_k / t_{k+1} (c_k = a_k (w - z_{k-1}), t_N = 1) kept as a ratio
// P / Q: t_k = (P + c_k Q) / P, so every level is one complex product and one
// complex multiply-add, and P_N(w) = a_1 Q / P takes the only division.  P and
// Q are rescaled together by a power of two (exact) when P leaves
// [2^-400, 2^400].
#include <array>
#include <utility>

#include "common.h"

namespace gw {
namespace {

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// 1 / x: the hardware estimate refined by two Newton-Raphson steps
// r <- r (2 - x r) (each squares the relative error, so two steps reach full
// FP64 precision from the estimate); the exact division where x is zero, huge
// or not finite
__device__ __forceinline__ double recip(double x) {
  if (!(x > 1e-300 && x < 1e300)) return 1.0 / x;
  double r = __builtin_amdgcn_rcp(x);
  r = __builtin_fma(r, __builtin_fma(-x, r, 1.0), r);
  r = __builtin_fma(r, __builtin_fma(-x, r, 1.0), r);
  return r;
}
// the value of lane `lane` (a compile-time constant here) in every lane
__device__ __forceinline__ double2 bcast(double2 v, int lane) {
  const unsigned long long x = __builtin_bit_cast(unsigned long long, v.x);
  const unsigned long long y = __builtin_bit_cast(unsigned long long, v.y);
  const unsigned long long xb =
      ((unsigned long long)(unsigned)__builtin_amdgcn_readlane((int)(x >> 32), lane) << 32) |
      (unsigned)__builtin_amdgcn_readlane((int)(unsigned)x, lane);
  const unsigned long long yb =
      ((unsigned long long)(unsigned)__builtin_amdgcn_readlane((int)(y >> 32), lane) << 32) |
      (unsigned)__builtin_amdgcn_readlane((int)(unsigned)y, lane);
  return make_double2(__builtin_bit_cast(double, xb), __builtin_bit_cast(double, yb));
}
__device__ __forceinline__ double2 cdiv(double2 a, double2 b) {
  const double d = recip(b.x * b.x + b.y * b.y);
  return make_double2((a.x * b.x + a.y * b.y) * d, (a.y * b.x - a.x * b.y) * d);
}

// P_N at the U points p, p + 64, ..., p + 64 (U - 1) (interleaved, so that
// their chains overlap) from the coefficients g of one function
template <int NMAX, int U>
__device__ __forceinline__ void continue_points(const double2 *g, int n,
                                                const double2 *__restrict__ z,
                                                const double2 *__restrict__ w,
                                                double2 *__restrict__ O, int p) {
  constexpr double kHi = 0x1p400, kLo = 0x1p-400;
  double2 wp[U], P[U], Q[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    wp[u] = w[p + 64 * u];
    P[u] = Q[u] = make_double2(1.0, 0.0);
  }
#pragma unroll
  for (int k = NMAX - 1; k >= 1; --k) {
    if (k < n) {
      const double2 zk = z[k - 1];
      double mx[U];
      bool resc = false;
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const double2 c = cmul(g[k], make_double2(wp[u].x - zk.x, wp[u].y - zk.y));
        const double2 pn =
            make_double2(__builtin_fma(c.x, Q[u].x, __builtin_fma(-c.y, Q[u].y, P[u].x)),
                         __builtin_fma(c.x, Q[u].y, __builtin_fma(c.y, Q[u].x, P[u].y)));
        Q[u] = P[u];
        P[u] = pn;
        // Q is the previous level's P, already in range
        mx[u] = fmax(fabs(P[u].x), fabs(P[u].y));
        resc |= !(mx[u] > kLo && mx[u] < kHi);
      }
      if (resc) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const double sc = mx[u] >= kHi ? 0x1p-450 : (mx[u] <= kLo && mx[u] > 0.0 ? 0x1p450 : 1.0);
          P[u] = make_double2(P[u].x * sc, P[u].y * sc);
          Q[u] = make_double2(Q[u].x * sc, Q[u].y * sc);
        }
      }
    }
  }
#pragma unroll
  for (int u = 0; u < U; ++u) O[p + 64 * u] = cmul(g[0], cdiv(Q[u], P[u]));
}

// f [n_fun][n], z [n], w [m] complex; coef [n_fun][n] (or null), out [n_fun][m]
// one instantiation per number of points N (NMAX = N): the level loops are
// then fully unrolled with no run-time guards
template <int NMAX>
__global__ __launch_bounds__(256) void k_pade(const double2 *__restrict__ f, int n_fun,
                                              const double2 *__restrict__ z,
                                              const double2 *__restrict__ w, int m,
                                              double2 *__restrict__ coef,
                                              double2 *__restrict__ out) {
  constexpr int n = NMAX;
  const int fun = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int l = threadIdx.x & 63;
  if (fun >= n_fun) return;
  // the recursion with lane j holding g_k(z_j) (lanes j < n; the others idle):
  // at level k + 1 every lane j >= k takes a_k = g_k(z_k) from lane k - 1
  const double2 *F = f + (int64_t)fun * n;
  const int jl = min(l, n - 1);
  const double2 zj = z[jl];
  double2 gl = F[jl];
#pragma unroll
  for (int k = 1; k < NMAX; ++k) {
    const double2 prev = bcast(gl, k - 1);
    const double2 zk = z[k - 1];
    if (l >= k && l < n) {
      const double2 den = cmul(make_double2(zj.x - zk.x, zj.y - zk.y), gl);
      gl = (den.x == 0.0 && den.y == 0.0) ? make_double2(0.0, 0.0)
                                          : cdiv(make_double2(prev.x - gl.x, prev.y - gl.y), den);
    }
  }
  if (coef != nullptr && l < n) coef[(int64_t)fun * n + l] = gl;
  // every lane takes all coefficients a_j = g_j(z_j) from lane j
  double2 g[NMAX];
#pragma unroll
  for (int j = 0; j < NMAX; ++j) g[j] = bcast(gl, j);
  // evaluation, EU points per lane at a time, the last ones singly
  double2 *O = out + (int64_t)fun * m;
  constexpr int EU = 4;
  int p = l;
  for (; p + 64 * (EU - 1) < m; p += 64 * EU) continue_points<NMAX, EU>(g, n, z, w, O, p);
  for (; p < m; p += 64) continue_points<NMAX, 1>(g, n, z, w, O, p);
}

}  // namespace

template <int N>
void launch_pade_n(dim3 grid, hipStream_t st, const double2 *F, int n_fun, const double2 *Z,
                   const double2 *W, int m, double2 *C, double2 *O) {
  hipLaunchKernelGGL(k_pade<N>, grid, dim3(256), 0, st, F, n_fun, Z, W, m, C, O);
}

template <int... Ns>
constexpr auto pade_table(std::integer_sequence<int, Ns...>) {
  return std::array<decltype(&launch_pade_n<1>), sizeof...(Ns)>{&launch_pade_n<Ns + 1>...};
}

hipError_t launch_pade(const void *f, int n_fun, int n, const void *z, const void *w, int m,
                       void *coef, void *out, hipStream_t st) {
  if (n_fun < 1 || n < 1 || n > kPadeMaxPoints || m < 0) return hipErrorInvalidValue;
  const int64_t blocks = ((int64_t)n_fun + 3) / 4;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  static constexpr auto table = pade_table(std::make_integer_sequence<int, kPadeMaxPoints>{});
  table[n - 1](dim3((unsigned)blocks), st, (const double2 *)f, n_fun, (const double2 *)z,
               (const double2 *)w, m, (double2 *)coef, (double2 *)out);
  return hipGetLastError();
}

}  // namespace gw
