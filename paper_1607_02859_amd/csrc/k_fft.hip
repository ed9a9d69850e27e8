// Sphere-pruned 3D FFT of chi over one spatial index (gfx950).
//
// Sec. II.C step (i), Eqs. (43)-(44): chi is transformed to reciprocal space
// one index at a time and only plane waves inside the cutoff sphere are
// kept.  Here a "column" is one 3D field of N_r = n0*n1*n2 points:
//   first index  (sign -1): column r' of a slab of chi(r, r')  -> chi(G, r')
//   second index (sign +1): row G of chi(G, r')                -> chi(G, G')
// out(G) = sum_r exp(sign * 2 pi i (k0 i0/n0 + k1 i1/n1 + k2 i2/n2)) f(r),
// unnormalised, for the caller's list of plane waves.
//
// One workgroup transforms one column:
//   1. groups of i0-planes are loaded into LDS and transformed along i2 and
//      i1 (one thread per line, register FFT);
//   2. only the (k1, k2) pencils that the sphere touches are kept, in a
//      pencil buffer [d][i0] (LDS when it fits, else a per-block slot of
//      global scratch);
//   3. each pencil is transformed along i0 and the sphere points are
//      written in output-slot order.
// Line transforms are compile-time mixed-radix (4, 2, 3, 5, 7) decimation in
// time, with twiddles as compile-time constants (exact for quarter turns).
#include <type_traits>

#include "common.h"

namespace gw {
namespace {

// --- compile-time trigonometry (Taylor series on the reduced angle) --------
constexpr double kHalfPi = 1.57079632679489661923132169163975;

constexpr double ce_sin_red(double x) {   // |x| <= pi/2
  double x2 = x * x, term = x, sum = x;
  for (int n = 1; n < 16; ++n) {
    term *= -x2 / ((2.0 * n) * (2.0 * n + 1.0));
    sum += term;
  }
  return sum;
}
constexpr double ce_cos_red(double x) {
  double x2 = x * x, term = 1.0, sum = 1.0;
  for (int n = 1; n < 16; ++n) {
    term *= -x2 / ((2.0 * n - 1.0) * (2.0 * n));
    sum += term;
  }
  return sum;
}
// cos and sin of 2 pi e / n, by quadrant
constexpr double ce_cos2pi(int e, int n) {
  e = ((e % n) + n) % n;
  const int q = (4 * e) / n;
  const double th = kHalfPi * (double)(4 * e - q * n) / (double)n;
  const double c = ce_cos_red(th), s = ce_sin_red(th);
  return q == 0 ? c : q == 1 ? -s : q == 2 ? -c : s;
}
constexpr double ce_sin2pi(int e, int n) {
  e = ((e % n) + n) % n;
  const int q = (4 * e) / n;
  const double th = kHalfPi * (double)(4 * e - q * n) / (double)n;
  const double c = ce_cos_red(th), s = ce_sin_red(th);
  return q == 0 ? s : q == 1 ? c : q == 2 ? -s : -c;
}

template <typename T>
struct cx {
  T x, y;
};
template <typename T>
__device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) {
  return {a.x + b.x, a.y + b.y};
}

template <int B, int E, typename F>
__device__ __forceinline__ void sfor(F &&f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    sfor<B + 1, E>(f);
  }
}

// a * exp(SIGN * 2 pi i E / N)
template <int N, int E, int SIGN, typename T>
__device__ __forceinline__ cx<T> tw(cx<T> a) {
  constexpr int e = ((E % N) + N) % N;
  if constexpr (e == 0) {
    return a;
  } else if constexpr (2 * e == N) {
    return {-a.x, -a.y};
  } else if constexpr (4 * e == N) {
    if constexpr (SIGN > 0) return {-a.y, a.x};
    else return {a.y, -a.x};
  } else if constexpr (4 * e == 3 * N) {
    if constexpr (SIGN > 0) return {a.y, -a.x};
    else return {-a.y, a.x};
  } else {
    constexpr double c = ce_cos2pi(e, N);
    constexpr double s = SIGN * ce_sin2pi(e, N);
    return {a.x * (T)c - a.y * (T)s, a.x * (T)s + a.y * (T)c};
  }
}

constexpr int first_radix(int n) {
  return (n % 4 == 0) ? 4 : (n % 2 == 0) ? 2 : (n % 3 == 0) ? 3 : (n % 5 == 0) ? 5 : (n % 7 == 0) ? 7 : n;
}

// out[k] = sum_n in[n*S] exp(SIGN 2 pi i n k / N), decimation in time
template <int N, int SIGN, typename T, int S>
__device__ __forceinline__ void reg_fft(const cx<T> *in, cx<T> *out) {
  if constexpr (N == 1) {
    out[0] = in[0];
  } else {
    constexpr int R = first_radix(N);
    constexpr int M = N / R;
    cx<T> y[N];
    sfor<0, R>([&](auto n2) {
      reg_fft<M, SIGN, T, S * R>(in + decltype(n2)::value * S, y + decltype(n2)::value * M);
    });
    sfor<0, M>([&](auto k1) {
      constexpr int K1 = decltype(k1)::value;
      cx<T> t[R];
      sfor<0, R>([&](auto n2) {
        constexpr int N2 = decltype(n2)::value;
        t[N2] = tw<N, N2 * K1, SIGN>(y[N2 * M + K1]);
      });
      sfor<0, R>([&](auto k2) {
        constexpr int K2 = decltype(k2)::value;
        cx<T> s = t[0];
        sfor<1, R>([&](auto n2) {
          constexpr int N2 = decltype(n2)::value;
          s = s + tw<R, N2 * K2, SIGN>(t[N2]);
        });
        out[K1 + M * K2] = s;
      });
    });
  }
}

template <int N, int SIGN, typename T>
__device__ __forceinline__ void line_n(cx<T> *p, int stride) {
  cx<T> v[N], o[N];
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] = p[i * stride];
  reg_fft<N, SIGN, T, 1>(v, o);
#pragma unroll
  for (int i = 0; i < N; ++i) p[i * stride] = o[i];
}

#define GW_FFT_SIZES(X) \
  X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(12) X(14) X(15) X(16) X(18) X(20) X(21) \
  X(24) X(25) X(27) X(28) X(30) X(32)

// in-place transform of n values at p[0], p[stride], ...
template <int SIGN, typename T>
__device__ __noinline__ void line_fft(cx<T> *p, int stride, int n) {
  switch (n) {
#define GW_CASE(N)                    \
  case N:                             \
    line_n<N, SIGN, T>(p, stride);    \
    break;
    GW_FFT_SIZES(GW_CASE)
#undef GW_CASE
    default:
      break;
  }
}

template <typename T, int SIGN>
__global__ __launch_bounds__(256) void k_fft(FftLaunch L) {
  extern __shared__ __attribute__((aligned(16))) char smem[];
  const int tid = threadIdx.x;
  for (int w = blockIdx.x; w < L.n_work; w += gridDim.x) {
    int lo = 0, hi = L.n_jobs - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (L.jobs[mid].work0 <= w) lo = mid;
      else hi = mid - 1;
    }
    const FftJob J = L.jobs[lo];
    const int c = w - J.work0;
    const Geo G = L.geos[J.geo];
    const int n0 = G.n0, n1 = G.n1, n2 = G.n2;
    const int plane = n1 * n2, D = G.n_disk;
    cx<T> *pl = reinterpret_cast<cx<T> *>(smem);
    cx<T> *disk = G.disk_in_lds
                      ? pl + (int64_t)G.planes * plane
                      : reinterpret_cast<cx<T> *>(L.scratch) + (int64_t)blockIdx.x * L.scratch_slot;
    for (int p0 = 0; p0 < n0; p0 += G.planes) {
      const int np = min(G.planes, n0 - p0);
      // rows below this flat index are zero (lower-triangle storage of a Hermitian chi)
      const int rmin = L.lower_only ? (J.col0 + c) - p0 * plane : 0;
      if (L.in_real) {
        const T *in = reinterpret_cast<const T *>(J.in) + (int64_t)c * J.in_col_stride +
                      (int64_t)p0 * plane;
        for (int idx = tid; idx < np * plane; idx += 256)
          pl[idx] = idx >= rmin ? cx<T>{in[idx], (T)0} : cx<T>{(T)0, (T)0};
      } else {
        const cx<T> *in = reinterpret_cast<const cx<T> *>(J.in) + (int64_t)c * J.in_col_stride +
                          (int64_t)p0 * plane;
        for (int idx = tid; idx < np * plane; idx += 256)
          pl[idx] = idx >= rmin ? in[idx] : cx<T>{(T)0, (T)0};
      }
      __syncthreads();
      for (int ln = tid; ln < np * n1; ln += 256) line_fft<SIGN, T>(pl + ln * n2, 1, n2);
      __syncthreads();
      for (int ln = tid; ln < np * n2; ln += 256) {
        const int p = ln / n2, i2 = ln - p * n2;
        line_fft<SIGN, T>(pl + p * plane + i2, n2, n1);
      }
      __syncthreads();
      for (int idx = tid; idx < np * D; idx += 256) {
        const int p = idx / D, d = idx - p * D;
        disk[(int64_t)d * n0 + p0 + p] = pl[p * plane + G.disk_i12[d]];
      }
      __syncthreads();
    }
    for (int d = tid; d < D; d += 256) line_fft<SIGN, T>(disk + (int64_t)d * n0, 1, n0);
    __syncthreads();
    cx<T> *out = reinterpret_cast<cx<T> *>(J.out) + (int64_t)(J.col0 + c) * J.out_col_stride;
    for (int s = tid; s < G.n_g; s += 256) out[(int64_t)s * J.out_slot_stride] = disk[G.slot_dk[s]];
    __syncthreads();
  }
}

}  // namespace

int fft_supported(int n) {
  switch (n) {
#define GW_OK(N) case N:
    GW_FFT_SIZES(GW_OK)
#undef GW_OK
    return 1;
    default:
      return 0;
  }
}

hipError_t launch_fft(const FftLaunch &L, int dbl, int sign, int grid, int lds_bytes,
                      hipStream_t s) {
  if (L.n_work <= 0) return hipSuccess;
  const void *k;
  if (dbl) k = sign < 0 ? (const void *)k_fft<double, -1> : (const void *)k_fft<double, 1>;
  else k = sign < 0 ? (const void *)k_fft<float, -1> : (const void *)k_fft<float, 1>;
  hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
  if (e != hipSuccess) return e;
  if (dbl) {
    if (sign < 0) hipLaunchKernelGGL((k_fft<double, -1>), dim3(grid), dim3(256), lds_bytes, s, L);
    else hipLaunchKernelGGL((k_fft<double, 1>), dim3(grid), dim3(256), lds_bytes, s, L);
  } else {
    if (sign < 0) hipLaunchKernelGGL((k_fft<float, -1>), dim3(grid), dim3(256), lds_bytes, s, L);
    else hipLaunchKernelGGL((k_fft<float, 1>), dim3(grid), dim3(256), lds_bytes, s, L);
  }
  return hipGetLastError();
}

}  // namespace gw
