// Sphere-pruned 3D FFT of chi over one spatial index (gfx950).
//
// Sec. II.C step (i), Eqs. (43)-(44): chi is transformed to reciprocal space
// one index at a time and only plane waves inside the cutoff sphere are
// kept.  A "column" is one 3D field of N_r = n0*n1*n2 points:
//   first index  (sign -1): column r' of a slab of chi(r, r')  -> chi(G, r')
//   second index (sign +1): row G of chi(G, r')                -> chi(G, G')
// out(G) = sum_r exp(sign * 2 pi i (k0 i0/n0 + k1 i1/n1 + k2 i2/n2)) f(r),
// unnormalised, for the caller's list of plane waves.
//
// Two launches per transform:
//   k_fft_planes_c (cubic grids with a specialised size) / k_fft_planes (any
//                  grid): a block owns `cols` adjacent columns x `planes`
//                  i0-planes (columns innermost, so global reads and the tmp
//                  writes are contiguous runs of `cols` elements), transforms
//                  along i2 and i1 (one thread per line, register FFT) and
//                  keeps only the (k1, k2) pencils the sphere touches:
//                  tmp[(i0 * n_disk + d) * n_cols + c];
//   k_fft_pencils: a block owns one pencil d and 256 adjacent columns (one
//                  per thread), transforms along i0 in registers and writes
//                  the sphere points of that pencil; consecutive threads
//                  write consecutive columns.
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

// Loads and stores through global-address-space pointers: they compile to
// global (not flat) memory instructions, which the compiler keeps in flight
// across LDS accesses.
template <typename T>
__device__ __forceinline__ T ld_g(const T *p, int64_t i) {
  return ((const __attribute__((address_space(1))) T *)p)[i];
}
template <typename T>
__device__ __forceinline__ cx<T> ld_g(const cx<T> *p, int64_t i) {
  typedef T v2 __attribute__((ext_vector_type(2)));
  const v2 x = ((const __attribute__((address_space(1))) v2 *)p)[i];
  return cx<T>{x.x, x.y};
}
template <typename T>
__device__ __forceinline__ void st_g(cx<T> *p, int64_t i, cx<T> v) {
  typedef T v2 __attribute__((ext_vector_type(2)));
  ((__attribute__((address_space(1))) v2 *)p)[i] = v2{v.x, v.y};
}

// A record every lane reads at the same index, through the constant address
// space: it loads as scalars, so no vector-memory wait for it also waits for
// the loads of later data already in flight.
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

template <typename T>
__device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) {
  return {a.x + b.x, a.y + b.y};
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

template <typename T>
__device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) {
  return {a.x - b.x, a.y - b.y};
}
// a * (SIGN i)
template <int SIGN, typename T>
__device__ __forceinline__ cx<T> rot(cx<T> a) {
  if constexpr (SIGN > 0) return {-a.y, a.x};
  else return {a.y, -a.x};
}

// o[k] = sum_n t[n] exp(SIGN 2 pi i n k / R) for one small radix: the
// radix-2 and radix-4 butterflies, and for odd R the pairing of n with R - n:
//   o[k], o[R-k] = t[0] + sum_n (t[n] + t[R-n]) cos(2 pi n k / R)
//                  +- SIGN i sum_n (t[n] - t[R-n]) sin(2 pi n k / R),  n = 1 .. (R-1)/2
template <int R, int SIGN, typename T>
__device__ __forceinline__ void dft_small(const cx<T> (&t)[R], cx<T> (&o)[R]) {
  if constexpr (R == 1) {
    o[0] = t[0];
  } else if constexpr (R == 2) {
    o[0] = t[0] + t[1];
    o[1] = t[0] - t[1];
  } else if constexpr (R == 4) {
    const cx<T> a = t[0] + t[2], b = t[0] - t[2];
    const cx<T> c = t[1] + t[3], d = rot<SIGN>(t[1] - t[3]);
    o[0] = a + c;
    o[2] = a - c;
    o[1] = b + d;
    o[3] = b - d;
  } else {
    static_assert(R % 2 == 1, "odd radix");
    constexpr int H = (R - 1) / 2;
    cx<T> sp[H + 1], dm[H + 1];
    cx<T> o0 = t[0];
    sfor<1, H + 1>([&](auto nn) {
      constexpr int n = decltype(nn)::value;
      sp[n] = t[n] + t[R - n];
      dm[n] = t[n] - t[R - n];
      o0 = o0 + sp[n];
    });
    o[0] = o0;
    sfor<1, H + 1>([&](auto kk) {
      constexpr int k = decltype(kk)::value;
      cx<T> a = t[0], b = {(T)0, (T)0};
      sfor<1, H + 1>([&](auto nn) {
        constexpr int n = decltype(nn)::value;
        constexpr T c = (T)ce_cos2pi(n * k, R), sn = (T)ce_sin2pi(n * k, R);
        a = {a.x + sp[n].x * c, a.y + sp[n].y * c};
        b = {b.x + dm[n].x * sn, b.y + dm[n].y * sn};
      });
      const cx<T> ib = rot<SIGN>(b);
      o[k] = a + ib;
      o[R - k] = a - ib;
    });
  }
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
      cx<T> t[R], o[R];
      sfor<0, R>([&](auto n2) {
        constexpr int N2 = decltype(n2)::value;
        t[N2] = tw<N, N2 * K1, SIGN>(y[N2 * M + K1]);
      });
      dft_small<R, SIGN, T>(t, o);
      sfor<0, R>([&](auto k2) {
        constexpr int K2 = decltype(k2)::value;
        out[K1 + M * K2] = o[K2];
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

// LDS index of element (p, i1, i2, column cc) in a plane block: grid points
// in row-major order, each holding `cols` columns padded to cols + 1 elements,
// so that both column-contiguous and point-contiguous accesses spread over
// the LDS banks.
__device__ __forceinline__ int lds_idx(int p, int i1, int i2, int cc, int n1, int n2, int cols) {
  return ((p * n1 + i1) * n2 + i2) * (cols + 1) + cc;
}

__device__ __forceinline__ int find_job(const FftJob *jobs, int n, int u, bool pencils) {
  // u is the same in every lane: the table reads go through the constant
  // address space (scalar loads)
  const __attribute__((address_space(4))) FftJob *cj = (const __attribute__((address_space(4))) FftJob *)jobs;
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    const int u0 = pencils ? cj[mid].unit0_pencils : cj[mid].unit0_planes;
    if (u0 <= u) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Any grid: sizes and block shape from the geometry table, line lengths
// dispatched at run time.
template <typename T, int SIGN>
__global__ __launch_bounds__(256) void k_fft_planes(FftLaunch L) {
  extern __shared__ __attribute__((aligned(16))) char smem[];
  cx<T> *buf = reinterpret_cast<cx<T> *>(smem);
  const int tid = threadIdx.x;
  constexpr int EC = (int)sizeof(cx<T>);
  for (int u = blockIdx.x; u < L.n_units_planes; u += gridDim.x) {
    const FftJob J = ld_c(L.jobs, __builtin_amdgcn_readfirstlane(find_job(L.jobs, L.n_jobs, u, false)));
    const Geo G = ld_c(L.geos, J.geo);
    const int n0 = G.n0, n1 = G.n1, n2 = G.n2;
    const int C = G.cols;
    const int P = G.planes;
    const int D = G.n_disk;
    const int plane = n1 * n2;
    const int npg = (n0 + P - 1) / P;
    const int lu = u - J.unit0_planes;
    const int cg = lu / npg, pg = lu - cg * npg;
    const int c0 = cg * C, p0 = pg * P;
    const int np = min(P, n0 - p0);
    // packed real input: line cc of the block holds the real columns
    // ca = 2 c0 + cc (real part) and ca + C (imaginary part); tmp rows hold
    // n_pc packed lines
    const int c0r = L.packed ? 2 * c0 : c0;        // first real column of the block
    const int n_pc = L.packed ? packed_lines(J.n_cols, C) : J.n_cols;
    // lower-triangle storage: a block whose planes all lie above the first
    // stored row of its first column is zero; it is skipped and the pencil
    // pass reads those planes as zero (same test there)
    if (L.lower_only && (int64_t)(p0 + np) * plane <= (int64_t)J.col0 + c0r) continue;
    // the sphere's pencil table, kept in LDS for the gather
    int *s_i12 = reinterpret_cast<int *>(smem + fft_lds_bytes(n1, n2, C, P, EC));
    for (int d = tid; d < D; d += 256) s_i12[d] = G.disk_i12[d];
    // load np planes of C columns
    const int total = np * plane * C;
    // element idx of the block -> (global offset or -1, LDS index); packed:
    // e2 is the offset of the imaginary part's column
    auto locate = [&](int idx, int64_t &e, int64_t &e2, int &li) {
      int cc, rl;
      if (J.s_col == 0) {       // column-grouped input: one contiguous run
        cc = idx % C;
        rl = idx / C;
      } else {                  // each column contiguous in r
        const int span = np * plane;
        cc = idx / span;
        rl = idx - cc * span;
      }
      const int c = c0 + cc;
      const int64_t r = (int64_t)p0 * plane + rl;
      e = -1;
      e2 = -1;
      if (L.packed) {               // column-grouped, groups of 2C real columns
        const int ca = 2 * c0 + cc, cb = ca + C;
        const int64_t b = ((int64_t)cg * (n0 * plane) + r) * (2 * C) + cc;
        if (idx < total && ca < J.n_cols && !(L.lower_only && r < J.col0 + ca)) e = b;
        if (idx < total && cb < J.n_cols && !(L.lower_only && r < J.col0 + cb)) e2 = b + C;
      } else if (idx < total && c < J.n_cols && !(L.lower_only && r < J.col0 + c)) {
        e = J.s_col == 0 ? (int64_t)cg * (n0 * plane) * C + r * C + cc
                         : r * J.s_r + (int64_t)c * J.s_col;
      }
      const int p = rl / plane, q = rl - p * plane;
      const int i1 = q / n2, i2 = q - i1 * n2;
      li = lds_idx(p, i1, i2, cc, n1, n2, C);
    };
    auto fetch = [&](int64_t e, int64_t e2) -> cx<T> {
      cx<T> v = {(T)0, (T)0};
      if (L.packed) {
        if (e >= 0) v.x = reinterpret_cast<const T *>(J.in)[e];
        if (e2 >= 0) v.y = reinterpret_cast<const T *>(J.in)[e2];
      } else if (e >= 0) {
        if (L.in_real) v.x = reinterpret_cast<const T *>(J.in)[e];
        else v = reinterpret_cast<const cx<T> *>(J.in)[e];
      }
      return v;
    };
    for (int idx = tid; idx < total; idx += 256) {
      int64_t e, e2;
      int li;
      locate(idx, e, e2, li);
      buf[li] = fetch(e, e2);
    }
    __syncthreads();
    // along i2: lines (p, i1, cc), stride C
    for (int ln = tid; ln < np * n1 * C; ln += 256) {
      const int cc = ln % C, rest = ln / C;
      const int p = rest / n1, i1 = rest - p * n1;
      line_fft<SIGN, T>(buf + lds_idx(p, i1, 0, cc, n1, n2, C), C + 1, n2);
    }
    __syncthreads();
    // along i1: lines (p, i2, cc), stride one padded row
    for (int ln = tid; ln < np * n2 * C; ln += 256) {
      const int cc = ln % C, rest = ln / C;
      const int p = rest / n2, i2 = rest - p * n2;
      line_fft<SIGN, T>(buf + lds_idx(p, 0, i2, cc, n1, n2, C), n2 * (C + 1), n1);
    }
    __syncthreads();
    // keep the sphere's pencils
    cx<T> *tmp = reinterpret_cast<cx<T> *>(J.tmp);
    for (int idx = tid; idx < np * D * C; idx += 256) {
      const int cc = idx % C, rest = idx / C;
      const int p = rest / D, d = rest - p * D;
      const int c = c0 + cc;
      if ((L.packed ? 2 * c0 + cc : c) < J.n_cols) {
        const int i12 = s_i12[d];
        const int i1 = i12 / n2, i2 = i12 - i1 * n2;
        tmp[((int64_t)(p0 + p) * D + d) * n_pc + c] = buf[lds_idx(p, i1, i2, cc, n1, n2, C)];
      }
    }
    __syncthreads();
  }
}

// Specialised cubic grid NC^3.  A block of fftc_threads(NC) threads owns C
// adjacent columns x P planes:
//   step 1: one thread per line (p, i1, column) gets the NC values along i2
//           (column-grouped input: straight from global memory; input
//           contiguous along r: through a coalesced copy into LDS),
//           transforms them in registers and stores the result to LDS,
//           [p][i1][k2][column];
//   step 2: one thread per line (p, k2, column) reads the NC values along i1,
//           transforms them and writes the sphere's pencils (k1, k2) to tmp.
// Lanes run over adjacent columns first, so each group of lanes touches one
// contiguous run in global memory and in LDS.
// Register budget: two blocks per CU (waves per SIMD = 2 * threads / 256).
constexpr int fftc_min_waves(int nt) { return nt >= 128 ? (nt + 127) / 128 : 1; }
// GROUPED: every job's input is column-grouped (else contiguous along r with
// unit stride, s_r == 1).
template <typename T, int SIGN, int NC, bool GROUPED>
__global__ __launch_bounds__(fftc_threads(NC, (int)sizeof(cx<T>)),
                             fftc_min_waves(fftc_threads(NC, (int)sizeof(cx<T>))))
void k_fft_planes_c(FftLaunch L) {
  extern __shared__ __attribute__((aligned(16))) char smem[];
  cx<T> *buf = reinterpret_cast<cx<T> *>(smem);
  constexpr int EC = (int)sizeof(cx<T>);
  constexpr int C = fftc_cols(NC, EC);
  constexpr int P = fftc_planes(NC, EC);
  constexpr int plane = NC * NC;
  constexpr int npg = NC / P;
  const int tid = threadIdx.x;
  const int cc = tid % C, ln = tid / C;
  const int a = ln % NC, p = ln / NC;      // step 1: a = i1; step 2: a = k2
  for (int u = blockIdx.x; u < L.n_units_planes; u += gridDim.x) {
    const FftJob J = ld_c(L.jobs, __builtin_amdgcn_readfirstlane(find_job(L.jobs, L.n_jobs, u, false)));
    const Geo G = ld_c(L.geos, J.geo);
    const int D = G.n_disk;
    const int lu = u - J.unit0_planes;
    const int cg = lu / npg, pg = lu - cg * npg;
    const int c0 = cg * C, p0 = pg * P;
    // packed real input (column-grouped only): line cc holds the real columns
    // 2 c0 + cc (real part) and 2 c0 + cc + C (imaginary part)
    const bool packed = GROUPED && L.packed;
    const int c0r = packed ? 2 * c0 : c0;          // first real column of the block
    const int n_pc = packed ? packed_lines(J.n_cols, C) : J.n_cols;
    // lower-triangle storage: a block whose planes all lie above the first
    // stored row of its first column is zero; it is skipped and the pencil
    // pass reads those planes as zero (same test there)
    if (L.lower_only && (int64_t)(p0 + P) * plane <= (int64_t)J.col0 + c0r) continue;
    const int c = c0 + cc;
    const bool col_ok = (packed ? c0r + cc : c) < J.n_cols;
    const int64_t zlim = L.lower_only ? (int64_t)J.col0 + c : -1;
    // LDS element (grid point rl of the block, column k)
    auto li = [&](int rl, int k) { return rl * C + k; };
    // A thread's loads go out unconditionally at constant offsets from one
    // base (element 0 when its column is past the end), all NC in flight
    // together; masked values are replaced by zero afterwards.  Every row a
    // block touches lies inside the input buffer.
    auto load = [&](int64_t e) -> cx<T> {
      if (L.in_real) return cx<T>{ld_g(reinterpret_cast<const T *>(J.in), e), (T)0};
      return ld_g(reinterpret_cast<const cx<T> *>(J.in), e);
    };
    cx<T> v[NC], o[NC];
    const int rl0 = (p * NC + a) * NC;   // first point of this thread's i2 line
    if constexpr (GROUPED) {
      // column-grouped input (groups of C columns): a thread's line along i2
      // is a run of NC rows of one group, read straight into registers;
      // rows above the diagonal of lower-triangle storage read as zero
      const int64_t r0 = (int64_t)p0 * plane + rl0;
      if (packed) {
        // groups of 2C real columns; both columns of the line lie in one
        // group, which the slab holds whole
        const int ca = c0r + cc, cb = ca + C;
        const bool okb = cb < J.n_cols;
        const int64_t za = L.lower_only ? (int64_t)J.col0 + ca : -1;
        const int64_t zb = L.lower_only ? (int64_t)J.col0 + cb : -1;
        const int64_t e0 = col_ok ? ((int64_t)cg * G.n_r + r0) * (2 * C) + cc : 0;
        const T *in = reinterpret_cast<const T *>(J.in);
#pragma unroll
        for (int i = 0; i < NC; ++i) {
          const T xa = ld_g(in, e0 + i * (2 * C));
          const T xb = ld_g(in, e0 + i * (2 * C) + C);
          v[i] = cx<T>{(col_ok && r0 + i >= za) ? xa : (T)0, (okb && r0 + i >= zb) ? xb : (T)0};
        }
      } else {
        const int64_t e0 = col_ok ? ((int64_t)cg * G.n_r + r0) * C + cc : 0;
#pragma unroll
        for (int i = 0; i < NC; ++i) {
          const cx<T> x = load(e0 + i * C);
          v[i] = (col_ok && r0 + i >= zlim) ? x : cx<T>{(T)0, (T)0};
        }
      }
    } else {
      // each column contiguous in r with unit stride (element (r, c) at
      // r + c * s_col; never lower-triangle storage): the block's region is
      // copied to LDS, lanes over the C columns first and then over
      // consecutive points, so that a wave reads C runs of 64 / C points and
      // writes one LDS run; then each thread reads its line from LDS
      const int k = tid % C, rl1 = tid / C;
      const bool ok_k = c0 + k < J.n_cols;
      if constexpr (sizeof(T) == 4) {
        // complex FP32: two adjacent points per 16-byte load (n even, so the
        // column starts and the point pairs are 16-byte aligned)
        const int64_t e1 = ok_k ? (int64_t)p0 * plane + 2 * rl1 + (int64_t)(c0 + k) * J.s_col : 0;
        const float4 *in4 = reinterpret_cast<const float4 *>(reinterpret_cast<const cx<T> *>(J.in) + e1);
#pragma unroll
        for (int i = 0; i < NC / 2; ++i) {
          typedef float f4 __attribute__((ext_vector_type(4)));
          const f4 q = ((const __attribute__((address_space(1))) f4 *)in4)[i * (P * NC)];
          v[2 * i] = ok_k ? cx<T>{q.x, q.y} : cx<T>{(T)0, (T)0};
          v[2 * i + 1] = ok_k ? cx<T>{q.z, q.w} : cx<T>{(T)0, (T)0};
        }
#pragma unroll
        for (int i = 0; i < NC / 2; ++i) {
          const int rl = 2 * (rl1 + i * (P * NC));
          buf[li(rl, k)] = v[2 * i];
          buf[li(rl + 1, k)] = v[2 * i + 1];
        }
      } else {
        const int64_t e1 = ok_k ? (int64_t)p0 * plane + rl1 + (int64_t)(c0 + k) * J.s_col : 0;
#pragma unroll
        for (int i = 0; i < NC; ++i) {
          const cx<T> x = load(e1 + i * (P * NC));
          v[i] = ok_k ? x : cx<T>{(T)0, (T)0};
        }
#pragma unroll
        for (int i = 0; i < NC; ++i) buf[li(rl1 + i * (P * NC), k)] = v[i];
      }
      __syncthreads();
#pragma unroll
      for (int i = 0; i < NC; ++i) v[i] = buf[li(rl0 + i, cc)];
    }
    // step 1: line (p, i1 = a, column) along i2, kept in LDS as [p][i1][k2]
    reg_fft<NC, SIGN, T, 1>(v, o);
#pragma unroll
    for (int k = 0; k < NC; ++k) buf[li(rl0 + k, cc)] = o[k];
    __syncthreads();
    // step 2: line (p, k2 = a, c) along i1, then the sphere's pencils; the
    // pencil indices are loaded first, so that none waits behind a store
    {
      int dk[NC];
#pragma unroll
      for (int k = 0; k < NC; ++k) dk[k] = ld_g(G.disk_of, k * NC + a);
#pragma unroll
      for (int i = 0; i < NC; ++i) v[i] = buf[li((p * NC + i) * NC + a, cc)];
      reg_fft<NC, SIGN, T, 1>(v, o);
      if (col_ok) {
        cx<T> *tmp = reinterpret_cast<cx<T> *>(J.tmp) + (int64_t)(p0 + p) * D * n_pc + c;
#pragma unroll
        for (int k = 0; k < NC; ++k)
          if (dk[k] >= 0) st_g(tmp, (int64_t)dk[k] * n_pc, o[k]);
      }
    }
    __syncthreads();
  }
}

template <int N, int SIGN, typename T>
__device__ __forceinline__ void pencil_n(const FftJob &J, const Geo &G, int d, int c,
                                         int lower_only) {
  const cx<T> *tmp = reinterpret_cast<const cx<T> *>(J.tmp);
  // planes whose plane-FFT block was skipped as all-zero (see k_fft_planes)
  const int64_t plane = (int64_t)G.n1 * G.n2;
  const int64_t zlim = lower_only ? (int64_t)J.col0 + (c / G.cols) * G.cols : -1;
  // output slots first and every load unconditional (element 0 stands in for
  // the skipped planes), so that no load waits behind another or a store
  int so[N];
#pragma unroll
  for (int k = 0; k < N; ++k) so[k] = ld_g(G.slot_of, (int64_t)d * N + k);
  cx<T> v[N], o[N];
#pragma unroll
  for (int i = 0; i < N; ++i) {
    const int hi = min(N, (i / G.planes + 1) * G.planes);
    const bool ok = hi * plane > zlim;
    const cx<T> x = ld_g(tmp, ok ? ((int64_t)i * G.n_disk + d) * J.n_cols + c : 0);
    v[i] = ok ? x : cx<T>{(T)0, (T)0};
  }
  // FP32 with half rows: the mirror slots are loaded before the transform,
  // not one by one between the stores (each wait for one would also wait for
  // the stores); FP64 has no registers to spare for them
  constexpr int NS = sizeof(T) == 4 ? N : 1;
  int sn[NS];
  if constexpr (sizeof(T) == 4) {
    if (J.half_rows) {
#pragma unroll
      for (int k = 0; k < N; ++k) sn[k] = ld_g(G.gneg, (int64_t)(so[k] >= 0 ? so[k] : 0));
    }
  }
  reg_fft<N, SIGN, T, 1>(v, o);
  if (J.half_rows) {
    // column c is row g = hrow[c] of the kept half; chi(-G, -G') is the
    // conjugate of chi(G, G') (not written again for a row with -G = G)
    const int g = ld_g(G.hrow, (int64_t)c);
    const int gm = ld_g(G.gneg, (int64_t)g);
    cx<T> *out = reinterpret_cast<cx<T> *>(J.out);
#pragma unroll
    for (int k = 0; k < N; ++k) {
      if (so[k] >= 0) {
        st_g(out, (int64_t)so[k] * J.o_slot + (int64_t)g * J.o_col, o[k]);
        if (gm != g) {
          int m;
          if constexpr (sizeof(T) == 4) m = sn[k];
          else m = ld_g(G.gneg, (int64_t)so[k]);
          st_g(out, (int64_t)m * J.o_slot + (int64_t)gm * J.o_col, cx<T>{o[k].x, -o[k].y});
        }
      }
    }
    return;
  }
  cx<T> *out = reinterpret_cast<cx<T> *>(J.out) + (int64_t)(J.col0 + c) * J.o_col;
#pragma unroll
  for (int k = 0; k < N; ++k)
    if (so[k] >= 0) st_g(out, (int64_t)so[k] * J.o_slot, o[k]);
}

// Packed real input: line pc holds z = x_a + i x_b for the real columns ca
// and cb = ca + C, so that with Z its transform
//   X_a(G) = (Z(G) + conj Z(-G)) / 2,   X_b(G) = (Z(G) - conj Z(-G)) / (2 i).
// The thread owns pencil d = (k1, k2) and its mirror m = (-k1, -k2) (the disk
// is closed under negation), transforms both along i0 and writes the sphere
// points of both pencils for both columns; -G of (k0, d) is (-k0, m).
template <int N, int SIGN, typename T>
__device__ __forceinline__ void pencil_pk_n(const FftJob &J, const Geo &G, int d, int pc,
                                            int n_pc, int lower_only) {
  const cx<T> *tmp = reinterpret_cast<const cx<T> *>(J.tmp);
  const int C = G.cols;
  const int m = G.disk_pair[d];
  const int64_t plane = (int64_t)G.n1 * G.n2;
  const int ca = (pc / C) * (2 * C) + pc % C, cb = ca + C;
  // planes whose plane-FFT block was skipped as all-zero (first real column
  // of the block, as there)
  const int64_t zlim = lower_only ? (int64_t)J.col0 + (pc / C) * (2 * C) : -1;
  // output rows: sphere slots, or compact rows of the kept half
  const int32_t *tab = J.half_rows ? G.slot_half : G.slot_of;
  int sd[N], sm[N];
#pragma unroll
  for (int k = 0; k < N; ++k) {
    sd[k] = ld_g(tab, (int64_t)d * N + k);
    sm[k] = ld_g(tab, (int64_t)m * N + k);
  }
  auto pencil = [&](int dd, cx<T> (&z)[N]) {
    cx<T> v[N];
#pragma unroll
    for (int i = 0; i < N; ++i) {
      const int hi = min(N, (i / G.planes + 1) * G.planes);
      const bool ok = hi * plane > zlim;
      const cx<T> x = ld_g(tmp, ok ? ((int64_t)i * G.n_disk + dd) * n_pc + pc : 0);
      v[i] = ok ? x : cx<T>{(T)0, (T)0};
    }
    reg_fft<N, SIGN, T, 1>(v, z);
  };
  cx<T> zd[N], zm[N];
  pencil(d, zd);
  if (m != d) {
    pencil(m, zm);
  } else {
#pragma unroll
    for (int k = 0; k < N; ++k) zm[k] = zd[k];
  }
  cx<T> *out = reinterpret_cast<cx<T> *>(J.out);
  const bool oka = ca < J.n_cols, okb = cb < J.n_cols;
  const int64_t oa = (int64_t)(J.col0 + ca) * J.o_col, ob = (int64_t)(J.col0 + cb) * J.o_col;
  auto emit = [&](const cx<T> (&z)[N], const cx<T> (&w)[N], const int (&so)[N]) {
    sfor<0, N>([&](auto kk) {
      constexpr int k = decltype(kk)::value;
      if (so[k] >= 0) {
        const cx<T> g = z[k], q = w[(N - k) % N];      // Z(G), Z(-G)
        const cx<T> xa = {(T)0.5 * (g.x + q.x), (T)0.5 * (g.y - q.y)};
        const cx<T> xb = {(T)0.5 * (g.y + q.y), (T)0.5 * (q.x - g.x)};
        if (oka) st_g(out, (int64_t)so[k] * J.o_slot + oa, xa);
        if (okb) st_g(out, (int64_t)so[k] * J.o_slot + ob, xb);
      }
    });
  };
  emit(zd, zm, sd);
  if (m != d) emit(zm, zd, sm);
}

template <typename T, int SIGN, int NC>
__device__ __forceinline__ void fft_pencils_body(const FftLaunch &L) {
  for (int u = blockIdx.x; u < L.n_units_pencils; u += gridDim.x) {
    const FftJob J = ld_c(L.jobs, __builtin_amdgcn_readfirstlane(find_job(L.jobs, L.n_jobs, u, true)));
    const Geo G = ld_c(L.geos, J.geo);
    if (L.packed) {
      // units: (mirror pair q, 256 packed lines)
      const int n_pc = packed_lines(J.n_cols, G.cols);
      const int nch = (n_pc + 255) / 256;
      const int lu = u - J.unit0_pencils;
      const int q = lu / nch, ch = lu - q * nch;
      const int pc = ch * 256 + threadIdx.x;
      if (pc >= n_pc || (pc / G.cols) * (2 * G.cols) + pc % G.cols >= J.n_cols) continue;
      const int d = G.disk_canon[q];
      if constexpr (NC > 0) {
        pencil_pk_n<NC, SIGN, T>(J, G, d, pc, n_pc, L.lower_only);
      } else {
        switch (G.n0) {
#define GW_PEN(N)                                               \
  case N:                                                       \
    pencil_pk_n<N, SIGN, T>(J, G, d, pc, n_pc, L.lower_only);   \
    break;
          GW_FFT_SIZES(GW_PEN)
#undef GW_PEN
          default:
            break;
        }
      }
      continue;
    }
    const int nch = (J.n_cols + 255) / 256;
    const int lu = u - J.unit0_pencils;
    const int d = lu / nch, ch = lu - d * nch;
    const int c = ch * 256 + threadIdx.x;
    if (c >= J.n_cols) continue;
    if constexpr (NC > 0) {
      pencil_n<NC, SIGN, T>(J, G, d, c, L.lower_only);
    } else {
      switch (G.n0) {
#define GW_PEN(N)                             \
  case N:                                     \
    pencil_n<N, SIGN, T>(J, G, d, c, L.lower_only); \
    break;
        GW_FFT_SIZES(GW_PEN)
#undef GW_PEN
        default:
          break;
      }
    }
  }
}

template <typename T, int SIGN, int NC>
__global__ __launch_bounds__(256) void k_fft_pencils(FftLaunch L) {
  fft_pencils_body<T, SIGN, NC>(L);
}
// over r' (the scattered transposed stores of chi(tau)): at most two waves
// per SIMD, which measured faster there than more resident blocks
template <typename T, int NC>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 2)))
void k_fft_pencils_rp(FftLaunch L) {
  fft_pencils_body<T, 1, NC>(L);
}

// ---------------------------------------------------------------------------
// Single-launch first-index transform for small cubic grids (complex FP32
// input): one workgroup per column, whose n^3 points are contiguous in the
// slab (column groups one column wide).  The i0-planes pass through LDS in batches of
// PB: a batch arrives by direct global-to-LDS loads into a linear stage while
// the previous batch is being transformed (the last batch of a line prefetches
// the first stored batch of the workgroup's next column), is copied into a
// work area with rows padded to n + 1 points and masked to the stored lower
// triangle, and is transformed along i2 and i1 there; thread d then takes the
// values of disk pencil d = (k1, k2) into registers.  After the last batch
// each thread holds the n0 values of its pencil and transforms them along i0.
// The pencil scratch of the two-launch path never reaches memory.
// Output rows are column-grouped, out[((s / X) * n_r + c) * X + s % X] with
// X = 2^o_gshift, the layout the second-index transform reads.
// ---------------------------------------------------------------------------
// global -> LDS, 16 bytes per lane at lds + 16 * lane (lds wave-uniform); the
// instruction is written out so that the compiler adds no wait of its own for
// it (the barrier waits below order the stage).  M0 is written one wait state
// before the load; no other code in these kernels reads M0.
#pragma clang diagnostic push
#pragma clang diagnostic ignored "-Winline-asm"
__device__ __forceinline__ void fft_dma16(const char *g, uint32_t lds) {
  asm volatile("s_mov_b32 m0, %1\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %0, off"
               :
               : "v"(g), "s"(lds)
               : "memory", "m0");
}
#pragma clang diagnostic pop

// every load of this wave has landed (vmcnt 0), then the workgroup barrier
__device__ __forceinline__ void fft_wait_loads_barrier() {
  __builtin_amdgcn_sched_barrier(0);
  __builtin_amdgcn_s_waitcnt((7 << 4) | (15 << 8));
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_sched_barrier(0);
}

template <int NC, int SIGN>
__global__ __launch_bounds__(256, 2) void k_fft_fused(FftLaunch L) {
  typedef float T;
  extern __shared__ __attribute__((aligned(1024))) char smem[];
  constexpr int plane = NC * NC, RP = NC + 1, PP = NC * RP;
  constexpr int PB = fused_pb(NC), NB = (NC + PB - 1) / PB;
  constexpr int SB = fused_stage_bytes(NC);
  static_assert(NC % 2 == 0 && PB * NC <= 256, "two points per 16 bytes, one thread per line");
  typedef float f4 __attribute__((ext_vector_type(4)));
  const f4 *stage = reinterpret_cast<const f4 *>(smem);
  cx<T> *work = reinterpret_cast<cx<T> *>(smem + SB);
  const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
  const uint32_t lds_stage = __builtin_amdgcn_readfirstlane(
      (uint32_t)(uintptr_t)(__attribute__((address_space(3))) char *)smem);
  // a unit: its job, column, first stored row and first batch holding a
  // stored row (rows above the diagonal of lower-triangle storage read as zero)
  struct Unit {
    int job, line, b0;
    int64_t za;
  };
  auto unit = [&](int uu) -> Unit {
    Unit x;
    x.job = __builtin_amdgcn_readfirstlane(find_job(L.jobs, L.n_jobs, uu, false));
    const FftJob J = ld_c(L.jobs, x.job);
    x.line = uu - J.unit0_planes;
    x.za = L.lower_only ? (int64_t)J.col0 + x.line : 0;
    x.b0 = 0;
    while (x.b0 < NB - 1 && (int64_t)(x.b0 * PB + PB) * plane <= x.za) ++x.b0;
    return x;
  };
  // the loads of batch b of a column into the stage: 1 KB per wave
  // instruction; lanes past the batch read its first bytes again (their
  // stage bytes are never used)
  auto issue = [&](const Unit &x, int b) {
    const FftJob J = ld_c(L.jobs, x.job);
    const char *g = reinterpret_cast<const char *>(reinterpret_cast<const cx<T> *>(J.in) +
                                                    ((int64_t)x.line * ld_c(L.geos, J.geo).n_r +
                                                     (int64_t)b * PB * plane));
    const int np = NC - b * PB < PB ? NC - b * PB : PB;
    const int bytes = np * plane * (int)sizeof(cx<T>);
    for (int c = wv; c < SB / 1024; c += 4) {
      const int o = c * 1024 + lane * 16;
      fft_dma16(g + (o < bytes ? o : 0), __builtin_amdgcn_readfirstlane(lds_stage + c * 1024));
    }
  };
  int u = blockIdx.x;
  Unit cur;
  if (u < L.n_units_planes) {
    cur = unit(u);
    issue(cur, cur.b0);
  }
  for (; u < L.n_units_planes; u += gridDim.x) {
    const FftJob J = ld_c(L.jobs, cur.job);
    const Geo G = ld_c(L.geos, J.geo);
    const int un = u + (int)gridDim.x;
    const bool has_next = un < L.n_units_planes;
    const Unit nxt = has_next ? unit(un) : cur;
    // thread t owns disk pencil t = (k1, k2); its output slots are loaded
    // now, in flight with the column's first batch, and not one by one
    // between the stores at the end
    const bool own = tid < G.n_disk;
    const int i12 = ld_g(G.disk_i12, (int64_t)(own ? tid : 0));
    const int k1 = i12 / NC, k2 = i12 - k1 * NC;
    int slot[NC];
#pragma unroll
    for (int k = 0; k < NC; ++k) slot[k] = ld_g(G.slot_of, (int64_t)(own ? tid : 0) * NC + k);
    cx<T> zp[NC];
    sfor<0, NB>([&](auto bb) {
      constexpr int b = decltype(bb)::value;
      constexpr int p0 = b * PB;
      constexpr int np = NC - p0 < PB ? NC - p0 : PB;
      constexpr int npt = np * plane;
      if (b < cur.b0) {                                // all above the diagonal
        sfor<0, np>([&](auto pp) { zp[p0 + decltype(pp)::value] = cx<T>{(T)0, (T)0}; });
        return;
      }
      fft_wait_loads_barrier();                        // batch b is in the stage
      // stage -> work: padded rows, masked
      for (int e2 = tid; e2 < npt / 2; e2 += 256) {
        const int pt = 2 * e2;
        const int p = pt / plane, rem = pt - p * plane;
        const int i1 = rem / NC, i2 = rem - i1 * NC;
        const int64_t r = (int64_t)p0 * plane + pt;
        const f4 v = stage[e2];
        cx<T> *dst = work + p * PP + i1 * RP + i2;
        dst[0] = r >= cur.za ? cx<T>{v.x, v.y} : cx<T>{(T)0, (T)0};
        dst[1] = r + 1 >= cur.za ? cx<T>{v.z, v.w} : cx<T>{(T)0, (T)0};
      }
      __syncthreads();                                 // the stage is free again
      if (b + 1 < NB) issue(cur, b + 1);
      else if (has_next) issue(nxt, nxt.b0);
      if (tid < np * NC) {                             // along i2: line (p, i1)
        const int p = tid / NC, i1 = tid - p * NC;
        line_n<NC, SIGN, T>(work + p * PP + i1 * RP, 1);
      }
      __syncthreads();
      if (tid < np * NC) {                             // along i1: line (p, k2)
        const int p = tid / NC, kk2 = tid - p * NC;
        line_n<NC, SIGN, T>(work + p * PP + kk2, RP);
      }
      __syncthreads();
      if (own)
        sfor<0, np>([&](auto pp) {
          constexpr int p = decltype(pp)::value;
          zp[p0 + p] = work[p * PP + k1 * RP + k2];
        });
      __syncthreads();                                 // work is free again
    });
    // along i0
    cx<T> o[NC];
    reg_fft<NC, SIGN, T, 1>(zp, o);
    cx<T> *out = reinterpret_cast<cx<T> *>(J.out);
    const int gs = J.o_gshift;
    auto at = [&](int sl, int64_t col) -> int64_t {
      return ((((int64_t)(sl >> gs)) * G.n_r + col) << gs) + (sl & ((1 << gs) - 1));
    };
    if (own) {
#pragma unroll
      for (int k = 0; k < NC; ++k)
        if (slot[k] >= 0) st_g(out, at(slot[k], (int64_t)J.col0 + cur.line), o[k]);
    }
    cur = nxt;
  }
}

template <int SIGN>
hipError_t launch_fused_t(const FftLaunch &L, int lds_bytes, int n, hipStream_t s) {
  const void *k;
  switch (n) {
    case 12: k = (const void *)k_fft_fused<12, SIGN>; break;
    case 16: k = (const void *)k_fft_fused<16, SIGN>; break;
    case 18: k = (const void *)k_fft_fused<18, SIGN>; break;
    case 20: k = (const void *)k_fft_fused<20, SIGN>; break;
    case 24: k = (const void *)k_fft_fused<24, SIGN>; break;
    default: return hipErrorInvalidValue;
  }
  hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
  if (e != hipSuccess) return e;
  const int g = L.n_units_planes < 2048 ? L.n_units_planes : 2048;
  if (g <= 0) return hipSuccess;
  FftLaunch a = L;
  void *args[] = {&a};
  return hipLaunchKernel(k, dim3(g), dim3(256), args, lds_bytes, s);
}

template <typename T, int S, int NC>
hipError_t launch_fft_t(const FftLaunch &L, int lds_bytes, hipStream_t s) {
  // plane blocks: a grid of a few resident rounds that strides over the units
  // (a unit above the diagonal of lower-triangle storage exits at once)
  const int g1 = L.n_units_planes < 2048 ? L.n_units_planes : 2048;
  const int g2 = L.n_units_pencils < 65536 ? L.n_units_pencils : 65536;
  hipError_t e;
  if constexpr (NC > 0) {
    constexpr int EC = (int)sizeof(cx<T>);
    constexpr int lds = fftc_lds_bytes(NC, fftc_cols(NC, EC), fftc_planes(NC, EC), EC);
    (void)lds_bytes;
    auto kern = L.grouped ? k_fft_planes_c<T, S, NC, true> : k_fft_planes_c<T, S, NC, false>;
    e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (e != hipSuccess) return e;
    if (g1 > 0) hipLaunchKernelGGL(kern, dim3(g1), dim3(fftc_threads(NC, EC)), lds, s, L);
  } else {
    e = hipFuncSetAttribute((const void *)k_fft_planes<T, S>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
    if (e != hipSuccess) return e;
    if (g1 > 0) hipLaunchKernelGGL((k_fft_planes<T, S>), dim3(g1), dim3(256), lds_bytes, s, L);
  }
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (g2 > 0) {
    if constexpr (S > 0) hipLaunchKernelGGL((k_fft_pencils_rp<T, NC>), dim3(g2), dim3(256), 0, s, L);
    else hipLaunchKernelGGL((k_fft_pencils<T, S, NC>), dim3(g2), dim3(256), 0, s, L);
  }
  return hipGetLastError();
}

template <typename T, int S>
hipError_t launch_fft_n(const FftLaunch &L, int lds_bytes, int n, hipStream_t s) {
  switch (n) {
    case 12: return launch_fft_t<T, S, 12>(L, lds_bytes, s);
    case 16: return launch_fft_t<T, S, 16>(L, lds_bytes, s);
    case 18: return launch_fft_t<T, S, 18>(L, lds_bytes, s);
    case 20: return launch_fft_t<T, S, 20>(L, lds_bytes, s);
    case 24: return launch_fft_t<T, S, 24>(L, lds_bytes, s);
    case 28: return launch_fft_t<T, S, 28>(L, lds_bytes, s);
    case 32: return launch_fft_t<T, S, 32>(L, lds_bytes, s);
    default: return launch_fft_t<T, S, 0>(L, lds_bytes, s);
  }
}

// ---------------------------------------------------------------------------
// Sphere-to-grid transforms (the self-energy's W~(G, G') -> W~(r, r'), the
// two spatial transforms of Eqs. (51)-(52)): the reverse of the pipeline
// above.  Pencils first: the sphere points of pencil (k1, k2) along k0 are
// transformed along axis 0; then per i0-plane the pencils are placed in their
// (k1, k2) positions (zero elsewhere) and transformed along axes 1 and 2.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ cx<T> ld_in(const SfftLaunch &L, const SfftJob &J, int64_t e) {
  cx<T> v;
  if (L.in_f64) {
    const cx<double> d = ld_g(reinterpret_cast<const cx<double> *>(J.in), e);
    v = cx<T>{(T)d.x, (T)d.y};
  } else {
    v = ld_g(reinterpret_cast<const cx<T> *>(J.in), e);
  }
  if (L.conj_in) v.y = -v.y;
  return v;
}

__device__ __forceinline__ int find_sjob(const SfftJob *jobs, int n, int u, bool pencils) {
  // u is the same in every lane: scalar loads, as in find_job
  const __attribute__((address_space(4))) SfftJob *cj = (const __attribute__((address_space(4))) SfftJob *)jobs;
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    const int u0 = pencils ? cj[mid].unit0_pencils : cj[mid].unit0_planes;
    if (u0 <= u) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

template <int N, int SIGN, typename T>
__device__ __forceinline__ void spencil_n(const SfftLaunch &L, const SfftJob &J, const Geo &G,
                                          int d, int c) {
  // slots first, then every load (masked slots read element 0 and are zeroed)
  int so[N];
#pragma unroll
  for (int k = 0; k < N; ++k) so[k] = ld_g(G.slot_of, (int64_t)d * N + k);
  cx<T> v[N], o[N];
  const int64_t col = (int64_t)(J.col0 + c) * J.i_col;
  // all N loads out before any is used: one branch on the input type around
  // the whole batch (a branch per load made each conversion wait for its load)
  if (L.in_f64) {
    cx<double> xd[N];
#pragma unroll
    for (int k = 0; k < N; ++k)
      xd[k] = ld_g(reinterpret_cast<const cx<double> *>(J.in),
                   so[k] >= 0 ? (int64_t)so[k] * J.i_slot + col : col);
#pragma unroll
    for (int k = 0; k < N; ++k) v[k] = cx<T>{(T)xd[k].x, (T)xd[k].y};
  } else {
#pragma unroll
    for (int k = 0; k < N; ++k)
      v[k] = ld_g(reinterpret_cast<const cx<T> *>(J.in),
                  so[k] >= 0 ? (int64_t)so[k] * J.i_slot + col : col);
  }
#pragma unroll
  for (int k = 0; k < N; ++k) {
    if (L.conj_in) v[k].y = -v[k].y;
    if (so[k] < 0) v[k] = cx<T>{(T)0, (T)0};
  }
  reg_fft<N, SIGN, T, 1>(v, o);
  cx<T> *tmp = reinterpret_cast<cx<T> *>(J.tmp);
  // planes the plane pass skips (lower_only: every row of the plane block
  // above the block's first column) are not written
  const int64_t plane = (int64_t)G.n1 * G.n2;
  const int64_t zlim = L.lower_only ? (int64_t)J.col0 + (c / G.cols) * G.cols : -1;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    const int hi = min(N, (i / G.planes + 1) * G.planes);
    if (hi * plane > zlim) st_g(tmp, ((int64_t)i * G.n_disk + d) * J.n_cols + c, o[i]);
  }
}

template <typename T, int SIGN>
__global__ __launch_bounds__(256) void k_sfft_pencils(SfftLaunch L) {
  for (int u = blockIdx.x; u < L.n_units_pencils; u += gridDim.x) {
    const SfftJob J = ld_c(L.jobs, __builtin_amdgcn_readfirstlane(find_sjob(L.jobs, L.n_jobs, u, true)));
    const Geo G = ld_c(L.geos, J.geo);
    const int nch = (J.n_cols + 255) / 256;
    const int lu = u - J.unit0_pencils;
    const int d = lu / nch, ch = lu - d * nch;
    const int c = ch * 256 + threadIdx.x;
    if (c >= J.n_cols) continue;
    switch (G.n0) {
#define GW_SPEN(N)                              \
  case N:                                       \
    spencil_n<N, SIGN, T>(L, J, G, d, c);       \
    break;
      GW_FFT_SIZES(GW_SPEN)
#undef GW_SPEN
      default:
        break;
    }
  }
}

// A block owns C adjacent columns x P i0-planes (the plane-block shape of the
// forward transform), in LDS as [p][i1][i2][column] with padded columns.
// NC > 0: cubic NC^3 grid, line transforms inlined at compile-time length.
// The blocks are persistent over the units; the pencil values of a block's
// next unit (the first PF of each thread's share) are loaded into registers
// while the current unit's transforms and stores run.
template <typename T, int SIGN, int NC>
__global__ __launch_bounds__(256) void k_sfft_planes(SfftLaunch L) {
  extern __shared__ __attribute__((aligned(16))) char smem[];
  cx<T> *buf = reinterpret_cast<cx<T> *>(smem);
  const int tid = threadIdx.x;
  constexpr int EC = (int)sizeof(cx<T>);
  constexpr int PF = sizeof(T) == 8 ? 2 : 12;
  // unit u: job index, first column and plane, planes; false for a block
  // whose rows all lie above its first column (not wanted with lower_only)
  auto locate = [&](int u, int &ji, int &c0, int &p0, int &np) -> bool {
    ji = __builtin_amdgcn_readfirstlane(find_sjob(L.jobs, L.n_jobs, u, false));
    const SfftJob J = ld_c(L.jobs, ji);
    const Geo G = ld_c(L.geos, J.geo);
    const int plane = G.n1 * G.n2;
    const int npg = (G.n0 + G.planes - 1) / G.planes;
    const int lu = u - J.unit0_planes;
    const int cg = lu / npg, pg = lu - cg * npg;
    c0 = cg * G.cols;
    p0 = pg * G.planes;
    np = min(G.planes, G.n0 - p0);
    return !(L.lower_only && (int64_t)(p0 + np) * plane <= (int64_t)J.col0 + c0);
  };
  auto next_wanted = [&](int u) {
    int ji, c0, p0, np;
    while (u < L.n_units_planes && !locate(u, ji, c0, p0, np)) u += gridDim.x;
    return u;
  };
  // the first PF pencil values of this thread in unit u (entry idx = tid + 256 t:
  // column c0 + idx % C, plane p0 + idx / C / D, disk pencil idx / C % D)
  cx<T> pre[PF];
  auto prefetch = [&](int u) {
    if (u >= L.n_units_planes) return;
    int ji, c0, p0, np;
    locate(u, ji, c0, p0, np);
    const SfftJob J = ld_c(L.jobs, ji);
    const Geo G = ld_c(L.geos, J.geo);
    const int C = G.cols, D = G.n_disk;
    const cx<T> *tmp = reinterpret_cast<const cx<T> *>(J.tmp);
    const int n_cols = J.n_cols;
#pragma unroll
    for (int t = 0; t < PF; ++t) {
      // unconditional (element 0 stands in past the unit), so that no load
      // is waited for before the next goes out
      const int idx = tid + 256 * t;
      const int cc = idx % C, rest = idx / C;
      const int p = rest / D, d = rest - p * D;
      const int c = c0 + cc;
      const bool ok = idx < np * D * C && c < n_cols;
      pre[t] = ld_g(tmp, ok ? ((int64_t)(p0 + p) * D + d) * n_cols + c : 0);
    }
  };
  int u = next_wanted((int)blockIdx.x);
  prefetch(u);
  while (u < L.n_units_planes) {
    int ji, c0, p0, np;
    locate(u, ji, c0, p0, np);
    const SfftJob J = ld_c(L.jobs, ji);
    const Geo G = ld_c(L.geos, J.geo);
    const int n1 = G.n1, n2 = G.n2;
    const int C = G.cols, P = G.planes, D = G.n_disk;
    const int plane = n1 * n2;
    int *s_i12 = reinterpret_cast<int *>(smem + fft_lds_bytes(n1, n2, C, P, EC));
    for (int d = tid; d < D; d += 256) s_i12[d] = G.disk_i12[d];
    for (int idx = tid; idx < np * plane * (C + 1); idx += 256) buf[idx] = cx<T>{(T)0, (T)0};
    __syncthreads();
    // place the pencils of these planes: the prefetched ones, then any beyond
    const cx<T> *tmp = reinterpret_cast<const cx<T> *>(J.tmp);
#pragma unroll
    for (int t = 0; t < PF; ++t) {
      const int idx = tid + 256 * t;
      const int cc = idx % C, rest = idx / C;
      const int p = rest / D, d = rest - p * D;
      if (idx < np * D * C && c0 + cc < J.n_cols) {
        const int i12 = s_i12[d];
        const int k1 = i12 / n2, k2 = i12 - k1 * n2;
        buf[lds_idx(p, k1, k2, cc, n1, n2, C)] = pre[t];
      }
    }
    for (int idx = tid + 256 * PF; idx < np * D * C; idx += 256) {
      const int cc = idx % C, rest = idx / C;
      const int p = rest / D, d = rest - p * D;
      const int c = c0 + cc;
      if (c < J.n_cols) {
        const int i12 = s_i12[d];
        const int k1 = i12 / n2, k2 = i12 - k1 * n2;
        buf[lds_idx(p, k1, k2, cc, n1, n2, C)] =
            ld_g(tmp, ((int64_t)(p0 + p) * D + d) * J.n_cols + c);
      }
    }
    __syncthreads();
    // the next unit's pencils are in flight from here to its placement
    const int un = next_wanted(u + (int)gridDim.x);
    prefetch(un);
    // along axis 1: lines (p, k2, cc), stride one padded row
    for (int ln = tid; ln < np * n2 * C; ln += 256) {
      const int cc = ln % C, rest = ln / C;
      const int p = rest / n2, k2 = rest - p * n2;
      if constexpr (NC > 0) line_n<NC, SIGN, T>(buf + lds_idx(p, 0, k2, cc, n1, n2, C), n2 * (C + 1));
      else line_fft<SIGN, T>(buf + lds_idx(p, 0, k2, cc, n1, n2, C), n2 * (C + 1), n1);
    }
    __syncthreads();
    // along axis 2: lines (p, i1, cc), stride C + 1
    for (int ln = tid; ln < np * n1 * C; ln += 256) {
      const int cc = ln % C, rest = ln / C;
      const int p = rest / n1, i1 = rest - p * n1;
      if constexpr (NC > 0) line_n<NC, SIGN, T>(buf + lds_idx(p, i1, 0, cc, n1, n2, C), C + 1);
      else line_fft<SIGN, T>(buf + lds_idx(p, i1, 0, cc, n1, n2, C), C + 1, n2);
    }
    __syncthreads();
    // write every grid point of the block
    cx<T> *out = reinterpret_cast<cx<T> *>(J.out);
    const int total = np * plane * C;
    if (J.o_shift >= 0) {
      // column-grouped: columns of a group are contiguous, lanes over them first
      const int sh = J.o_shift;
      for (int idx = tid; idx < total; idx += 256) {
        const int cc = idx % C, rl = idx / C;
        const int c = c0 + cc;
        if (c < J.n_cols) {
          const int p = rl / plane, q = rl - p * plane;
          const int i1 = q / n2, i2 = q - i1 * n2;
          const int64_t r = (int64_t)(p0 + p) * plane + q;
          const int64_t e = (((int64_t)(c >> sh) * G.n_r + r) << sh) + (c & ((1 << sh) - 1));
          st_g(out, e, buf[lds_idx(p, i1, i2, cc, n1, n2, C)]);
        }
      }
    } else {
      // one row of out per column: lanes over consecutive grid points first
      const int span = np * plane;
      for (int idx = tid; idx < total; idx += 256) {
        const int cc = idx / span, rl = idx - cc * span;
        const int c = c0 + cc;
        if (c < J.n_cols) {
          const int p = rl / plane, q = rl - p * plane;
          const int i1 = q / n2, i2 = q - i1 * n2;
          const int64_t r = (int64_t)(p0 + p) * plane + q;
          st_g(out, (int64_t)c * J.o_col + r, buf[lds_idx(p, i1, i2, cc, n1, n2, C)]);
        }
      }
    }
    __syncthreads();
    u = un;
  }
}

template <typename T, int S, int NC>
hipError_t launch_sfft_planes(const SfftLaunch &L, int lds_bytes, int g2, hipStream_t s) {
  hipError_t e = hipFuncSetAttribute((const void *)k_sfft_planes<T, S, NC>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_sfft_planes<T, S, NC>), dim3(g2), dim3(256), lds_bytes, s, L);
  return hipGetLastError();
}

// cubic: the grid edge shared by every job's geometry (0 if they differ or a
// grid is not cubic)
template <typename T, int S>
hipError_t launch_sfft_t(const SfftLaunch &L, int lds_bytes, int cubic, hipStream_t s) {
  const int g1 = L.n_units_pencils < 65536 ? L.n_units_pencils : 65536;
  const int g2 = L.n_units_planes < 2048 ? L.n_units_planes : 2048;
  if (g1 > 0) hipLaunchKernelGGL((k_sfft_pencils<T, S>), dim3(g1), dim3(256), 0, s, L);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (g2 <= 0) return hipSuccess;
  switch (cubic) {
    case 12: return launch_sfft_planes<T, S, 12>(L, lds_bytes, g2, s);
    case 16: return launch_sfft_planes<T, S, 16>(L, lds_bytes, g2, s);
    case 18: return launch_sfft_planes<T, S, 18>(L, lds_bytes, g2, s);
    case 20: return launch_sfft_planes<T, S, 20>(L, lds_bytes, g2, s);
    case 24: return launch_sfft_planes<T, S, 24>(L, lds_bytes, g2, s);
    case 28: return launch_sfft_planes<T, S, 28>(L, lds_bytes, g2, s);
    case 32: return launch_sfft_planes<T, S, 32>(L, lds_bytes, g2, s);
    default: return launch_sfft_planes<T, S, 0>(L, lds_bytes, g2, s);
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

hipError_t launch_sfft(const SfftLaunch &L, int dbl, int sign, int lds_bytes, int cubic,
                       hipStream_t s) {
  if (!fft_specialised(cubic)) cubic = 0;
  if (dbl) return sign < 0 ? launch_sfft_t<double, -1>(L, lds_bytes, cubic, s)
                           : launch_sfft_t<double, 1>(L, lds_bytes, cubic, s);
  return sign < 0 ? launch_sfft_t<float, -1>(L, lds_bytes, cubic, s)
                  : launch_sfft_t<float, 1>(L, lds_bytes, cubic, s);
}

hipError_t launch_fft(const FftLaunch &L, int dbl, int sign, int lds_bytes, int cubic_n,
                      hipStream_t s) {
  if (cubic_n < 0) return hipErrorInvalidValue;   // layouts the planner never mixes
  if (L.fused) {
    if (dbl || sign > 0 || L.packed || !fft_fusable(cubic_n)) return hipErrorInvalidValue;
    return launch_fused_t<-1>(L, lds_bytes, cubic_n, s);
  }
  const int n = fft_specialised(cubic_n) ? cubic_n : 0;
  if (dbl) return sign < 0 ? launch_fft_n<double, -1>(L, lds_bytes, n, s)
                           : launch_fft_n<double, 1>(L, lds_bytes, n, s);
  return sign < 0 ? launch_fft_n<float, -1>(L, lds_bytes, n, s)
                  : launch_fft_n<float, 1>(L, lds_bytes, n, s);
}

}  // namespace gw
