// Host runtime behind the C ABI of gwchi.h: validation, planning, launch
// sequence, hipGraph cache, timing and report.
//
// One call is planned as a list of jobs, one per (item, tau_j), cut into
// passes that fit the device-memory budget.  Per pass:
//   stage (FP64 weights, scaled operands)                 - all jobs of the pass
//   for every r' slab: band GEMM + Hadamard, FFT over r   - one launch each, all jobs
//   FFT over r'                                           - one launch, all jobs
// and after the last pass one cosine-transform launch for all items.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <unordered_map>
#include <memory>
#include <mutex>
#include <numeric>
#include <sstream>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/gwchi.h"
#include "common.h"

using namespace gw;

// Fixed device scratch of the allocation-free entry point
// (gwchi_chi_build_device_noalloc).  Each device holds its own copy of this
// array for the life of the process.  In host code the name is only a
// stand-in: its device address comes from hipGetSymbolAddress, taken once per
// device (scratch_of_device) and kept in the context.
constexpr int64_t kNoAllocBytes = (int64_t)96 << 20;
static __device__ __align__(256) char g_noalloc_scratch[kNoAllocBytes];

namespace {

thread_local std::string g_tls_error;

// regions of the fixed scratch: the launch tables, the ticket counters, then
// the plan's buffers
constexpr int64_t kNoAllocTables = (int64_t)4 << 20;
constexpr int64_t kNoAllocCounters = (int64_t)64 << 10;

// Device address of the fixed scratch on `device` (which must be current):
// looked up once per device, nullptr if the lookup failed.
void *scratch_of_device(int device, std::string *why) {
  static std::mutex mu;
  static std::map<int, std::pair<void *, std::string>> addr;
  std::lock_guard<std::mutex> lock(mu);
  auto it = addr.find(device);
  if (it == addr.end()) {
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(g_noalloc_scratch));
    std::string msg;
    if (e != hipSuccess) {
      msg = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
      ptr = nullptr;
    }
    it = addr.emplace(device, std::make_pair(ptr, msg)).first;
  }
  if (why) *why = it->second.second;
  return it->second.first;
}

struct DevBuf {
  void *p = nullptr;
  size_t n = 0;
  hipError_t ensure(size_t bytes, bool *moved) {
    if (bytes <= n) return hipSuccess;
    if (p) {
      hipError_t e = hipFree(p);
      if (e != hipSuccess) return e;
      p = nullptr;
      n = 0;
    }
    size_t want = (bytes + 4095) / 4096 * 4096 + 4096;
    hipError_t e = hipMalloc(&p, want);
    if (e != hipSuccess) {
      p = nullptr;
      return e;
    }
    n = want;
    if (moved) *moved = true;
    return hipSuccess;
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
  }
};

struct HostPinned {
  void *p = nullptr;
  size_t n = 0;
  hipError_t ensure(size_t bytes) {
    if (bytes <= n) return hipSuccess;
    if (p) (void)hipHostFree(p);
    p = nullptr;
    n = 0;
    size_t want = bytes + bytes / 8 + 256;
    hipError_t e = hipHostMalloc(&p, want, hipHostMallocDefault);
    if (e != hipSuccess) {
      p = nullptr;
      return e;
    }
    n = want;
    return hipSuccess;
  }
  void release() {
    if (p) (void)hipHostFree(p);
    p = nullptr;
    n = 0;
  }
};

enum Phase { PH_STAGE = 0, PH_GEMM, PH_FFT_R, PH_FFT_RP, PH_CT, PH_NORM, PH_COUNT };

struct Launch {
  int phase;
  int kind;   // 0 stage, 1 gemm, 2 fft, 3 ct, 4 norms, 5 fill
  size_t off; // offset of the launch struct's tables in the table blob
  // typed payloads (device pointers patched in)
  StageLaunch stage;
  GemmLaunch gemm;
  FftLaunch fft;
  CtLaunch ct;
  int fft_sign = -1;
  int fft_lds = 0;
  int fft_cubic = 0;
  int gemm_grid = 0;
  int max_omega = 0;
  int max_mats = 0;
  void *fill_ptr = nullptr;
  int64_t fill_bytes = 0;
  int norm_mode = 0;
  const int32_t *toff = nullptr, *woff = nullptr;
};

}  // namespace

struct gwchi_ctx {
  int device = 0;
  int num_cu = 256;
  size_t lds_max = 65536;
  hipStream_t stream = nullptr;
  gwchi_options opt{};
  std::string err;
  std::string tune_path;
  std::string arch = "gfx950";       // device architecture, the first part of every tune key
  std::map<std::string, int> tune;   // key -> tile index
  std::map<std::string, std::vector<double>> tune_ms;   // key -> GEMM ms per tile, last autotune
  DevBuf b_phi, b_out, b_psi, b_slab, b_xr, b_x, b_tmp, b_tables, b_norm, b_ctr;
  // screened-interaction step: chi / outputs of the host entry, the matrices
  // being inverted, the pivot-block panels, the per-item tables, the pivot flag
  DevBuf b_wchi, b_wtau, b_womega, b_wa, b_wdinv, b_wrp, b_wcp, b_wtab, b_wflag;
  HostPinned h_wtab;
  // self-energy: states operands, per-(state, tau) sums, host-entry copies of
  // W~ and of the outputs
  DevBuf b_sstates, b_ssum, b_sw, b_sout, b_stau;
  // analytic continuation: host-entry copies of f / out / coef, the points z and w
  DevBuf b_pf, b_pout, b_pcoef, b_ptab;
  HostPinned h_ptab;
  HostPinned h_tables, h_norm;
  // allocation-free entry: device address of the fixed scratch on this
  // context's device (nullptr when unavailable, with the reason), and the
  // host copy of the last launch tables (read by the asynchronous upload)
  void *noalloc_scratch = nullptr;
  std::string noalloc_why;
  std::vector<char> noalloc_blob;
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  std::vector<hipEvent_t> ev_pool;
  // graph cache: one entry keyed by the structural signature of the plan
  std::string graph_key;
  hipGraphExec_t graph_exec = nullptr;
  hipGraph_t graph = nullptr;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> graph_evs;
};

namespace {

void set_err(gwchi_ctx *ctx, const std::string &m) {
  if (ctx) ctx->err = m;
  g_tls_error = m;
}

#define HIPCHK(call)                                                                  \
  do {                                                                                \
    hipError_t e_ = (call);                                                           \
    if (e_ != hipSuccess) {                                                           \
      set_err(ctx, std::string(#call) + ": " + hipGetErrorString(e_));               \
      return e_ == hipErrorOutOfMemory ? GWCHI_ENOMEM : GWCHI_EDEVICE;                \
    }                                                                                 \
  } while (0)

int64_t round_up(int64_t a, int64_t b) { return (a + b - 1) / b * b; }

bool finite_all(const double *p, int64_t n) {
  for (int64_t i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

gwchi_status validate_items(gwchi_ctx *ctx, const gwchi_item *items, int32_t n_items,
                            bool check_orbitals) {
  if (!items || n_items < 1) {
    set_err(ctx, "items is NULL or n_items < 1");
    return GWCHI_EINVAL;
  }
  for (int32_t t = 0; t < n_items; ++t) {
    const gwchi_item &it = items[t];
    std::string pre = "item " + std::to_string(t) + ": ";
    for (int d = 0; d < 3; ++d)
      if (it.n[d] < 1) {
        set_err(ctx, pre + "grid size must be >= 1");
        return GWCHI_EINVAL;
      }
    if (it.n_occ < 1 || it.n_unocc < 1) {
      set_err(ctx, pre + "n_occ and n_unocc must be >= 1");
      return GWCHI_EINVAL;
    }
    if (it.n_tau < 1 || it.n_omega < 1 || it.n_g < 1) {
      set_err(ctx, pre + "n_tau, n_omega and n_g must be >= 1");
      return GWCHI_EINVAL;
    }
    if (!it.phi_occ || !it.phi_unocc || !it.eps_occ || !it.eps_unocc || !it.tau || !it.ct ||
        !it.g_index || !it.chi_out) {
      set_err(ctx, pre + "NULL pointer");
      return GWCHI_EINVAL;
    }
    if (it.is_complex != 0 && it.is_complex != 1) {
      set_err(ctx, pre + "is_complex must be 0 or 1");
      return GWCHI_EINVAL;
    }
    for (int d = 0; d < 3; ++d)
      if (!fft_supported(it.n[d])) {
        set_err(ctx, pre + "grid size " + std::to_string(it.n[d]) +
                         " unsupported (7-smooth and <= 32 required)");
        return GWCHI_ENOTSUP;
      }
    const int64_t n_r = (int64_t)it.n[0] * it.n[1] * it.n[2];
    if (!finite_all(it.eps_occ, it.n_occ) || !finite_all(it.eps_unocc, it.n_unocc) ||
        !std::isfinite(it.mu) || !finite_all(it.tau, it.n_tau) ||
        !finite_all(it.ct, (int64_t)it.n_tau * it.n_omega)) {
      set_err(ctx, pre + "non-finite eigenvalue, mu, tau or ct");
      return GWCHI_EINVAL;
    }
    const double homo = *std::max_element(it.eps_occ, it.eps_occ + it.n_occ);
    const double lumo = *std::min_element(it.eps_unocc, it.eps_unocc + it.n_unocc);
    if (!(homo < it.mu && it.mu < lumo)) {
      set_err(ctx, pre + "mu must lie strictly between max(eps_occ) and min(eps_unocc)");
      return GWCHI_EINVAL;
    }
    for (int j = 0; j < it.n_tau; ++j)
      if (!(it.tau[j] > 0.0)) {
        set_err(ctx, pre + "tau must be > 0");
        return GWCHI_EINVAL;
      }
    std::vector<char> seen((size_t)n_r, 0);
    for (int g = 0; g < it.n_g; ++g) {
      const int32_t f = it.g_index[g];
      if (f < 0 || f >= n_r) {
        set_err(ctx, pre + "g_index out of range");
        return GWCHI_EINVAL;
      }
      if (seen[f]) {
        set_err(ctx, pre + "g_index has duplicates");
        return GWCHI_EINVAL;
      }
      seen[f] = 1;
    }
    if (check_orbitals) {
      const int64_t m = n_r * (it.is_complex ? 2 : 1);
      if (!finite_all(it.phi_occ, m * it.n_occ) || !finite_all(it.phi_unocc, m * it.n_unocc)) {
        set_err(ctx, pre + "non-finite orbital value");
        return GWCHI_EINVAL;
      }
    }
  }
  // one call runs one GEMM tile family: all real or all complex
  for (int32_t t = 1; t < n_items; ++t)
    if ((items[t].is_complex != 0) != (items[0].is_complex != 0)) {
      set_err(ctx, "items of one call must be all real or all complex");
      return GWCHI_EINVAL;
    }
  return GWCHI_OK;
}

// ----------------------------------------------------------------------------
// Plan
// ----------------------------------------------------------------------------

struct ItemPlan {
  int n0, n1, n2;
  int64_t n_r, n_r_pad;
  int cplx;
  int k_o, k_u, k_o_pad, k_u_pad;
  int n_tau, n_omega, n_g;
  double homo, lumo;
  std::vector<int32_t> perm_o, perm_u;
  std::vector<double> eps_o, eps_u;
  std::vector<int32_t> disk_i12, slot_of, disk_of;
  int n_disk = 0, planes = 1, cols = 16, fft_lds = 0;
  // real orbitals: the first-index transform packs two real columns into one
  // complex line (slab groups of 2 * cols columns); mirror pencils and the
  // canonical pencil of each mirror pair
  int pack = 0;
  std::vector<int32_t> disk_pair, disk_canon;
  // real orbitals, sphere closed under G -> -G: the second-index transform
  // runs over the rows of one half only (hrow), the first index keeps only
  // those rows (slot_half); gneg[g] is the sphere index of -G
  int half = 0;
  std::vector<int32_t> slot_half, hrow, gneg;
  // single-launch first-index transform (FP32 slab, small cubic grid, every
  // disk pencil owned by one of 256 threads); sgroup: slab column-group width
  int fused = 0, sgroup = 16;
  std::vector<double> coef;    // [n_omega][n_tau]
  std::vector<double> tau;
  const double *phi_o = nullptr, *phi_u = nullptr;
  double *out = nullptr;
  int job0 = 0;
};

struct JobPlan {
  int item, j;
  int k_o_eff, k_u_eff;
  int pass = 0;
  // byte offsets of this job's slots in the pass-local buffers
  int64_t o_psi = 0, o_slab = 0, o_xr = 0, o_tmp = 0, o_x = 0;
};

struct Plan {
  int prec = 0;
  int tile = 0, bm = 0, bn = 0, kc = 0;
  int slab_w = 2048;
  std::vector<ItemPlan> items;
  std::vector<JobPlan> jobs;
  std::vector<int> pass_begin;      // first job of each pass, plus the end
  // buffer sizes: maxima over passes of the packed job slots
  int64_t psi_bytes = 0, slab_bytes = 0, xr_bytes = 0, tmp_bytes = 0, x_bytes = 0;
  int max_jobs_pass = 0;
  int fft_lds = 0;
  double alg_flops = 0, mfma_flops = 0;
  int cplx_any = 0, real_any = 0;
};

int bpb_of(int prec, int cplx) {   // operand bytes per band element
  if (prec == P_FP64) return cplx ? 16 : 8;
  return cplx ? 8 : 4;
}
int elem_c(int prec) { return prec == P_FP64 ? 16 : 8; }            // complex working element
int elem_slab(int prec, int cplx) { return cplx ? elem_c(prec) : elem_c(prec) / 2; }

// tune-cache key: architecture / precision / real or complex, e.g. "gfx950/fp32/c"
std::string tune_key(const gwchi_ctx *ctx, int prec, int cplx) {
  return ctx->arch + "/" + (prec == P_FP64 ? "fp64" : prec == P_FP32 ? "fp32" : "bf16x3") +
         (cplx ? "/c" : "/r");
}

// arena_bytes > 0: the plan's buffers must fit in that many bytes of fixed
// scratch (the allocation-free entry); otherwise the context's budget applies.
// sigma_states > 0: plan a self-energy call (its own tile per precision; the
// slab holds complex W~(r, r') in groups of 128 bytes; the fifth buffer holds
// the per-tile partial sums of at most sigma_states states).
gwchi_status build_plan(gwchi_ctx *ctx, const gwchi_item *items, int n_items, int prec,
                        Plan &P, int64_t arena_bytes = 0, int sigma_states = 0) {
  P = Plan();
  P.prec = prec;
  // all items of one call use one (precision, complexity) tile family; items that mix
  // real and complex orbitals are rejected (validate_items reports it first)
  for (int t = 0; t < n_items; ++t) (items[t].is_complex ? P.cplx_any : P.real_any) = 1;
  if (P.cplx_any && P.real_any) {
    set_err(ctx, "items of one call must be all real or all complex");
    return GWCHI_EINVAL;
  }
  const int cplx = P.cplx_any;
  const int ntile = gemm_tile_count(prec, cplx);
  int tile = 0;
  if (ctx->opt.tile_id >= 1) {
    tile = ctx->opt.tile_id - 1;
    if (tile >= ntile) {
      set_err(ctx, "tile_id out of range");
      return GWCHI_EINVAL;
    }
  } else {
    auto it = ctx->tune.find(tune_key(ctx, prec, cplx));
    if (it != ctx->tune.end() && it->second >= 0 && it->second < ntile) tile = it->second;
  }
  P.tile = tile;
  P.bm = gemm_tile_bm(prec, cplx, tile);
  P.bn = gemm_tile_bn(prec, cplx, tile);
  P.kc = gemm_tile_kc(prec, cplx, tile);
  if (sigma_states > 0) {
    P.tile = 0;
    P.bm = gemm_sigma_bm(prec);
    P.bn = gemm_sigma_bn(prec);
    P.kc = gemm_sigma_kc(prec);
  }

  const int ec = elem_c(prec);
  const int es = elem_slab(prec, cplx);
  const int bpb = bpb_of(prec, cplx);
  P.items.resize(n_items);
  for (int t = 0; t < n_items; ++t) {
    const gwchi_item &it = items[t];
    ItemPlan &I = P.items[t];
    I.n0 = it.n[0];
    I.n1 = it.n[1];
    I.n2 = it.n[2];
    I.n_r = (int64_t)I.n0 * I.n1 * I.n2;
    I.n_r_pad = round_up(I.n_r, kRowPad);
    I.cplx = it.is_complex;
    I.k_o = it.n_occ;
    I.k_u = it.n_unocc;
    I.k_o_pad = (int)round_up(I.k_o, kBandPad);
    I.k_u_pad = (int)round_up(I.k_u, kBandPad);
    I.n_tau = it.n_tau;
    I.n_omega = it.n_omega;
    I.n_g = it.n_g;
    // sort bands: occupied by descending energy, unoccupied ascending (edge first)
    I.perm_o.resize(I.k_o);
    std::iota(I.perm_o.begin(), I.perm_o.end(), 0);
    std::stable_sort(I.perm_o.begin(), I.perm_o.end(),
                     [&](int a, int b) { return it.eps_occ[a] > it.eps_occ[b]; });
    I.perm_u.resize(I.k_u);
    std::iota(I.perm_u.begin(), I.perm_u.end(), 0);
    std::stable_sort(I.perm_u.begin(), I.perm_u.end(),
                     [&](int a, int b) { return it.eps_unocc[a] < it.eps_unocc[b]; });
    I.eps_o.resize(I.k_o);
    I.eps_u.resize(I.k_u);
    for (int k = 0; k < I.k_o; ++k) I.eps_o[k] = it.eps_occ[I.perm_o[k]];
    for (int k = 0; k < I.k_u; ++k) I.eps_u[k] = it.eps_unocc[I.perm_u[k]];
    I.homo = I.eps_o[0];
    I.lumo = I.eps_u[0];
    I.tau.assign(it.tau, it.tau + it.n_tau);
    // cosine coefficients with the band-edge factor exp(-(lumo - homo) tau_j), FP64
    I.coef.resize((size_t)I.n_omega * I.n_tau);
    for (int k = 0; k < I.n_omega; ++k)
      for (int j = 0; j < I.n_tau; ++j)
        I.coef[(size_t)k * I.n_tau + j] =
            it.ct[(size_t)k * I.n_tau + j] * std::exp(-(I.lumo - I.homo) * it.tau[j]);
    // sphere tables: pencils (k1, k2) in first-seen order, slot of (pencil, k0)
    std::map<int, int> dmap;
    std::vector<std::pair<int, int>> dk(I.n_g);
    for (int g = 0; g < I.n_g; ++g) {
      const int f = it.g_index[g];
      const int k0 = f / (I.n1 * I.n2);
      const int i12 = f - k0 * I.n1 * I.n2;
      auto ins = dmap.emplace(i12, (int)dmap.size());
      dk[g] = {ins.first->second, k0};
    }
    // real orbitals: the disk is closed under negation (pencils the sphere
    // does not touch are added without output slots), so that every pencil
    // of a packed transform finds its mirror
    I.pack = !I.cplx && sigma_states == 0;
    if (I.pack) {
      std::vector<int> have;
      for (auto &kv : dmap) have.push_back(kv.first);
      for (int i12 : have) {
        const int k1 = i12 / I.n2, k2 = i12 - k1 * I.n2;
        const int m = ((I.n1 - k1) % I.n1) * I.n2 + (I.n2 - k2) % I.n2;
        dmap.emplace(m, (int)dmap.size());
      }
    }
    I.n_disk = (int)dmap.size();
    I.disk_i12.resize(I.n_disk);
    for (auto &kv : dmap) I.disk_i12[kv.second] = kv.first;
    I.slot_of.assign((size_t)I.n_disk * I.n0, -1);
    for (int g = 0; g < I.n_g; ++g) I.slot_of[(size_t)dk[g].first * I.n0 + dk[g].second] = g;
    I.disk_of.assign((size_t)I.n1 * I.n2, -1);
    for (int d = 0; d < I.n_disk; ++d) I.disk_of[I.disk_i12[d]] = d;
    I.disk_pair.clear();
    I.disk_canon.clear();
    I.half = 0;
    I.slot_half.clear();
    I.hrow.clear();
    I.gneg.clear();
    if (I.pack) {
      // -G of every sphere point, if the sphere holds it
      std::unordered_map<int, int> gi;
      for (int g = 0; g < I.n_g; ++g) gi.emplace(it.g_index[g], g);
      I.gneg.assign(I.n_g, -1);
      bool closed = true;
      for (int g = 0; g < I.n_g && closed; ++g) {
        const int f = it.g_index[g];
        const int k0 = f / (I.n1 * I.n2), k1 = (f / I.n2) % I.n1, k2 = f % I.n2;
        const int fm = (((I.n0 - k0) % I.n0) * I.n1 + (I.n1 - k1) % I.n1) * I.n2 + (I.n2 - k2) % I.n2;
        auto q = gi.find(fm);
        if (q == gi.end()) closed = false;
        else I.gneg[g] = q->second;
      }
      if (closed) {
        I.half = 1;
        std::vector<int32_t> hidx(I.n_g, -1);
        for (int g = 0; g < I.n_g; ++g)
          if (g <= I.gneg[g]) {
            hidx[g] = (int32_t)I.hrow.size();
            I.hrow.push_back(g);
          }
        I.slot_half.assign(I.slot_of.size(), -1);
        for (size_t e = 0; e < I.slot_of.size(); ++e)
          if (I.slot_of[e] >= 0) I.slot_half[e] = hidx[I.slot_of[e]];
      } else {
        I.gneg.clear();
      }
    }
    if (I.pack) {
      I.disk_pair.resize(I.n_disk);
      for (int d = 0; d < I.n_disk; ++d) {
        const int k1 = I.disk_i12[d] / I.n2, k2 = I.disk_i12[d] - k1 * I.n2;
        I.disk_pair[d] = I.disk_of[((I.n1 - k1) % I.n1) * I.n2 + (I.n2 - k2) % I.n2];
        if (d <= I.disk_pair[d]) I.disk_canon.push_back(d);
      }
    }
    // plane-FFT block shape (same formula as the kernels)
    if (I.n0 == I.n1 && I.n1 == I.n2 && fft_specialised(I.n0)) {
      I.cols = fftc_cols(I.n0, ec);
      I.planes = fftc_planes(I.n0, ec);
      I.fft_lds = fftc_lds_bytes(I.n0, I.cols, I.planes, ec);
    } else {
      I.cols = fft_cols(I.n1, I.n2, ec);
      I.planes = fft_planes(I.n0, I.n1, I.n2, ec);
      I.fft_lds = fft_lds_bytes(I.n1, I.n2, I.cols, I.planes, ec) + 4 * I.n_disk;
    }
    // (complex orbitals only: for packed real columns the two-launch path
    // measures faster, its plane blocks skipping the zero triangle plane by
    // plane and its pencil pass spread over more threads)
    I.fused = prec != P_FP64 && sigma_states == 0 && !I.pack && I.n0 == I.n1 && I.n1 == I.n2 &&
              fft_fusable(I.n0) && I.n_disk <= 256;
    I.sgroup = I.fused ? 1 : I.cols * (I.pack ? 2 : 1);
    I.phi_o = it.phi_occ;
    I.phi_u = it.phi_unocc;
    I.out = it.chi_out;
    P.alg_flops += (I.cplx ? 8.0 : 2.0) * (double)I.n_r * (double)I.n_r * (I.k_o + I.k_u) * I.n_tau;
  }
  // jobs, with optional exact-zero band truncation
  const double thr = std::ldexp(1.0, -152);
  const bool skip = ctx->opt.skip_zero_bands && prec != P_FP64 && sigma_states == 0;
  for (int t = 0; t < n_items; ++t) {
    ItemPlan &I = P.items[t];
    I.job0 = (int)P.jobs.size();
    for (int j = 0; j < I.n_tau; ++j) {
      JobPlan J{t, j, I.k_o, I.k_u};
      if (skip) {
        int co = 0, cu = 0;
        for (int k = 0; k < I.k_o; ++k)
          if (std::exp(0.5 * (I.eps_o[k] - I.homo) * I.tau[j]) >= thr) co = k + 1;
        for (int k = 0; k < I.k_u; ++k)
          if (std::exp(-0.5 * (I.eps_u[k] - I.lumo) * I.tau[j]) >= thr) cu = k + 1;
        J.k_o_eff = std::max(co, 1);
        J.k_u_eff = std::max(cu, 1);
      }
      J.k_o_eff = (int)std::min<int64_t>(round_up(J.k_o_eff, P.kc), I.k_o_pad);
      J.k_u_eff = (int)std::min<int64_t>(round_up(J.k_u_eff, P.kc), I.k_u_pad);
      P.jobs.push_back(J);
    }
  }
  int lds_need = 0;
  for (auto &I : P.items) lds_need = std::max(lds_need, I.fft_lds);
  P.fft_lds = lds_need;
  // Pack jobs into passes.  Each job owns slots for its scaled operands, its
  // slab, chi(G, r'), the pencil scratch and chi(tau_j); consecutive jobs of
  // one item keep consecutive chi(tau) slots, which the cosine transform reads.
  size_t free_b = 0, total_b = 0;
  if (arena_bytes == 0 && hipMemGetInfo(&free_b, &total_b) != hipSuccess) free_b = (size_t)64 << 30;
  // scratch the context already holds is released before a larger plan allocates
  const size_t held = ctx->b_psi.n + ctx->b_slab.n + ctx->b_xr.n + ctx->b_x.n + ctx->b_tmp.n;
  const int64_t budget = arena_bytes > 0 ? arena_bytes
                         : ctx->opt.max_device_bytes > 0 ? ctx->opt.max_device_bytes
                                                         : (int64_t)((free_b + held) * 0.6);
  // the arena holds the five buffers only (each rounded up to 256 bytes)
  const int64_t fixed = arena_bytes > 0 ? 5 * 256 : (int64_t)64 << 20;
  const int n_jobs = (int)P.jobs.size();
  const int want = ctx->opt.tau_batch > 0 ? std::min(ctx->opt.tau_batch, n_jobs) : n_jobs;
  int W = ctx->opt.slab_width > 0 ? (int)round_up(ctx->opt.slab_width, 256) : 2048;
  for (;;) {
    auto sizes = [&](const ItemPlan &I, int64_t *b) {
      const int64_t wmax = std::min<int64_t>(W, I.n_r);
      b[0] = round_up(I.n_r_pad * (I.k_o_pad + I.k_u_pad) * bpb, 256);
      b[1] = sigma_states > 0 ? round_up(round_up(wmax, 128 / ec) * I.n_r * ec, 256)
                              : round_up(round_up(wmax, I.sgroup) * I.n_r * es, 256);
      b[2] = round_up(round_up(I.n_g, I.cols) * I.n_r * ec, 256);
      b[3] = round_up((int64_t)I.n0 * I.n_disk * std::max<int64_t>(wmax, I.n_g) * ec, 256);
      b[4] = (int64_t)I.n_g * I.n_g * ec;
      if (sigma_states > 0) {
        // tiles of one job over every slab, bounded by the full square
        const int64_t nrt = (I.n_r + P.bm - 1) / P.bm;
        const int64_t nct = (I.n_r + P.bn - 1) / P.bn + (I.n_r + W - 1) / W;
        b[4] = round_up(nrt * nct * sigma_states * 16, 256);
      }
    };
    bool ok = true;
    P.pass_begin.assign(1, 0);
    P.psi_bytes = P.slab_bytes = P.xr_bytes = P.tmp_bytes = P.x_bytes = 0;
    P.max_jobs_pass = 0;
    int64_t acc[5] = {0, 0, 0, 0, 0};
    int in_pass = 0;
    for (int q = 0; q < n_jobs && ok; ++q) {
      JobPlan &J = P.jobs[q];
      const ItemPlan &I = P.items[J.item];
      int64_t b[5];
      sizes(I, b);
      const int64_t job = b[0] + b[1] + b[2] + b[3] + b[4];
      const int64_t used = acc[0] + acc[1] + acc[2] + acc[3] + acc[4];
      // a new item's chi(tau) block starts 256-aligned
      const bool new_item = in_pass == 0 || P.jobs[q - 1].item != J.item;
      const int64_t xalign = new_item ? round_up(acc[4], 256) - acc[4] : 0;
      if (in_pass > 0 && (in_pass >= want || fixed + used + xalign + job > budget)) {
        P.pass_begin.push_back(q);
        for (int k = 0; k < 5; ++k) acc[k] = 0;
        in_pass = 0;
      }
      if (fixed + job > budget) {
        ok = false;
        break;
      }
      if (in_pass == 0 || P.jobs[q - 1].item != J.item) acc[4] = round_up(acc[4], 256);
      J.pass = (int)P.pass_begin.size() - 1;
      J.o_psi = acc[0];
      J.o_slab = acc[1];
      J.o_xr = acc[2];
      J.o_tmp = acc[3];
      J.o_x = acc[4];
      for (int k = 0; k < 5; ++k) acc[k] += b[k];
      ++in_pass;
      P.psi_bytes = std::max(P.psi_bytes, acc[0]);
      P.slab_bytes = std::max(P.slab_bytes, acc[1]);
      P.xr_bytes = std::max(P.xr_bytes, acc[2]);
      P.tmp_bytes = std::max(P.tmp_bytes, acc[3]);
      P.x_bytes = std::max(P.x_bytes, round_up(acc[4], 256));
      P.max_jobs_pass = std::max(P.max_jobs_pass, in_pass);
    }
    if (ok) {
      P.pass_begin.push_back(n_jobs);
      P.slab_w = W;
      break;
    }
    if (W <= 256 || ctx->opt.slab_width > 0) {
      if (arena_bytes > 0)
        set_err(ctx, "allocation-free build: one (item, tau) job with a 256-column slab needs more "
                     "than the fixed scratch of " + std::to_string(arena_bytes) + " bytes");
      else
        set_err(ctx, "device memory budget too small for one job with a 256-column slab");
      return GWCHI_ENOMEM;
    }
    W /= 2;
  }
  return GWCHI_OK;
}

// Blob of device tables, built on the host with offsets, then patched with the
// device base address and copied in one transfer.
struct Blob {
  std::vector<char> h;
  size_t add(const void *src, size_t bytes) {
    size_t off = round_up((int64_t)h.size(), 64);
    h.resize(off + bytes);
    if (bytes) std::memcpy(h.data() + off, src, bytes);
    return off;
  }
  template <typename T>
  size_t addv(const std::vector<T> &v) {
    return add(v.data(), v.size() * sizeof(T));
  }
};

// Device base addresses of a build's buffers.
struct Bases {
  char *psi = nullptr, *slab = nullptr, *xr = nullptr, *tmp = nullptr, *x = nullptr;
  double *norm = nullptr;
  int32_t *ctr = nullptr;
  char *tables = nullptr;
};

struct Built {
  int n_gemm = 0;             // GEMM launches (one ticket counter each)
  std::vector<Launch> launches;
  Blob blob;
  std::string key;     // structural signature for the graph cache
  int n_passes = 0;
  int64_t norm_tau_off = 0, norm_omega_off = 0;
  int n_norm_tau = 0, n_norm_omega = 0;
};

// Emit FFT launches for a set of jobs, one launch per distinct grid so that
// cubic grids run the kernels specialised for their size.
void emit_fft(Built &B, const Plan &P, std::vector<FftJob> &jobs, int phase, int sign,
              int in_real, int lower_only, size_t off_geos) {
  // key: grid and, for the first index, whether the items take the single launch
  std::map<std::tuple<int, int, int, int>, std::vector<FftJob>> groups;
  for (auto &f : jobs) {
    const ItemPlan &I = P.items[f.geo];
    groups[std::make_tuple(I.n0, I.n1, I.n2, phase == PH_FFT_R ? I.fused : 0)].push_back(f);
  }
  for (auto &kv : groups) {
    std::vector<FftJob> &fj = kv.second;
    const int fused = std::get<3>(kv.first);
    // real column-grouped input of packing items: two columns per transform
    bool packed = in_real != 0;
    for (auto &f : fj) packed = packed && f.s_col == 0 && P.items[f.geo].pack;
    int up = 0, un = 0, lds = 0;
    for (auto &f : fj) {
      const ItemPlan &I = P.items[f.geo];
      f.unit0_planes = up;
      f.unit0_pencils = un;
      if (fused) {
        up += f.n_cols;                                    // one unit per column
        lds = std::max(lds, fused_lds_bytes(I.n0));
        continue;
      }
      if (packed) {
        const int n_pc = packed_lines(f.n_cols, I.cols);
        up += (n_pc / I.cols) * ((I.n0 + I.planes - 1) / I.planes);
        un += (int)I.disk_canon.size() * ((n_pc + 255) / 256);
      } else {
        up += ((f.n_cols + I.cols - 1) / I.cols) * ((I.n0 + I.planes - 1) / I.planes);
        un += I.n_disk * ((f.n_cols + 255) / 256);
      }
      lds = std::max(lds, I.fft_lds);
    }
    const int n0 = std::get<0>(kv.first), n1 = std::get<1>(kv.first), n2 = std::get<2>(kv.first);
    Launch F{};
    F.phase = phase;
    F.kind = 2;
    F.fft.jobs = reinterpret_cast<const FftJob *>(B.blob.addv(fj));
    F.fft.n_jobs = (int)fj.size();
    F.fft.geos = reinterpret_cast<const Geo *>(off_geos);
    F.fft.n_units_planes = up;
    F.fft.n_units_pencils = un;
    F.fft.in_real = in_real;
    F.fft.packed = packed ? 1 : 0;
    F.fft.fused = fused;
    F.fft.lower_only = lower_only;
    // the jobs of a launch are all column-grouped or all contiguous along r
    // with unit stride (the two layouts the cubic kernels read; contiguous
    // input is complex, its columns start 16-byte aligned, so FP32 reads two
    // points at a time); anything else is refused at launch (fft_cubic = -1)
    F.fft.grouped = 1;
    for (auto &f : fj) F.fft.grouped &= f.s_col == 0 ? 1 : 0;
    bool layout_ok = true;
    for (auto &f : fj)
      if (!F.fft.grouped &&
          (f.s_col == 0 || f.s_r != 1 || lower_only || in_real || (f.s_col & 1) ||
           (reinterpret_cast<uintptr_t>(f.in) & 15)))
        layout_ok = false;
    F.fft_sign = sign;
    F.fft_lds = lds;
    F.fft_cubic = (n0 == n1 && n1 == n2) ? n0 : 0;
    if (!layout_ok && fft_specialised(F.fft_cubic)) F.fft_cubic = -1;
    B.launches.push_back(F);
  }
}

// The staging launch of jobs [jb, je) of a pass: one op per (item, occ|unocc)
// over all of the item's taus in the pass, blocks of 64 grid points x 32 bands.
// Table pointers are blob offsets (patched later); off_* are the per-item
// offsets of the band permutations and sorted eigenvalues.
StageLaunch make_stage(Blob &blob, const Plan &P, int jb, int je, char *psi_base,
                       const std::vector<size_t> &off_perm_o, const std::vector<size_t> &off_perm_u,
                       const std::vector<size_t> &off_eps_o, const std::vector<size_t> &off_eps_u) {
  const int cplx = P.cplx_any;
  std::vector<StageOp> ops;
  std::vector<int4> blocks;
  std::vector<std::vector<void *>> psi_lists;
  std::vector<std::vector<double>> tau_lists;
  int jj = jb;
  while (jj < je) {
    const int t = P.jobs[jj].item;
    int je2 = jj;
    while (je2 < je && P.jobs[je2].item == t) ++je2;
    const ItemPlan &I = P.items[t];
    for (int side = 0; side < 2; ++side) {
      StageOp op{};
      op.phi = side == 0 ? I.phi_o : I.phi_u;
      op.perm = reinterpret_cast<const int32_t *>(side == 0 ? off_perm_o[t] : off_perm_u[t]);
      op.eps = reinterpret_cast<const double *>(side == 0 ? off_eps_o[t] : off_eps_u[t]);
      op.edge = side == 0 ? I.homo : I.lumo;
      op.sign = side == 0 ? 1.0 : -1.0;
      op.k = side == 0 ? I.k_o : I.k_u;
      op.k_pad = side == 0 ? I.k_o_pad : I.k_u_pad;
      op.n_r = (int32_t)I.n_r;
      op.n_r_pad = (int32_t)I.n_r_pad;
      op.cplx = I.cplx;
      op.n_jobs = je2 - jj;
      std::vector<void *> pl;
      std::vector<double> tl;
      for (int q = jj; q < je2; ++q) {
        char *slot = psi_base + P.jobs[q].o_psi;
        const int64_t o_bytes = I.n_r_pad * I.k_o_pad * bpb_of(P.prec, cplx);
        pl.push_back(side == 0 ? slot : slot + o_bytes);
        tl.push_back(I.tau[P.jobs[q].j]);
      }
      psi_lists.push_back(pl);
      tau_lists.push_back(tl);
      const int opi = (int)ops.size();
      ops.push_back(op);
      const int rt = (int)(I.n_r_pad / 64), kt = op.k_pad / 32;
      for (int a = 0; a < rt; ++a)
        for (int b = 0; b < kt; ++b) blocks.push_back(make_int4(opi, a, b, 0));
    }
    jj = je2;
  }
  for (size_t i = 0; i < ops.size(); ++i) {
    ops[i].tau = reinterpret_cast<const double *>(blob.addv(tau_lists[i]));
    ops[i].psi = reinterpret_cast<void *const *>(blob.addv(psi_lists[i]));
  }
  StageLaunch S{};
  S.ops = reinterpret_cast<const StageOp *>(blob.addv(ops));
  S.blocks = reinterpret_cast<const int4 *>(blob.addv(blocks));
  S.n_blocks = (int)blocks.size();
  S.prec = P.prec;
  return S;
}

// Build every launch descriptor.  Pointers into the blob are stored as offsets
// and patched by patch_blob once the device address of the blob is known.
void build_launches(gwchi_ctx *ctx, Plan &P, bool want_norms, const Bases &D, Built &B) {
  B.launches.clear();
  B.blob.h.clear();
  const int cplx = P.cplx_any;
  const int ec = elem_c(P.prec);
  const int es = elem_slab(P.prec, cplx);
  const int n_items = (int)P.items.size();
  char *psi_base = D.psi;
  char *slab_base = D.slab;
  char *xr_base = D.xr;
  char *x_base = D.x;
  char *tmp_base = D.tmp;
  std::ostringstream key;
  key << "p" << P.prec << "t" << P.tile << "w" << P.slab_w << "h" << ctx->opt.hermitian << "n"
      << want_norms << "|";
  for (int b : P.pass_begin) key << b << ",";
  key << "|";
  // geometry tables
  std::vector<size_t> off_i12(n_items), off_sdk(n_items), off_dof(n_items), off_perm_o(n_items),
      off_perm_u(n_items), off_eps_o(n_items), off_eps_u(n_items), off_coef(n_items),
      off_pair(n_items, 0), off_canon(n_items, 0), off_shalf(n_items, 0), off_hrow(n_items, 0),
      off_gneg(n_items, 0);
  for (int t = 0; t < n_items; ++t) {
    const ItemPlan &I = P.items[t];
    off_i12[t] = B.blob.addv(I.disk_i12);
    off_sdk[t] = B.blob.addv(I.slot_of);
    off_dof[t] = B.blob.addv(I.disk_of);
    if (I.pack) {
      off_pair[t] = B.blob.addv(I.disk_pair);
      off_canon[t] = B.blob.addv(I.disk_canon);
    }
    if (I.half) {
      off_shalf[t] = B.blob.addv(I.slot_half);
      off_hrow[t] = B.blob.addv(I.hrow);
      off_gneg[t] = B.blob.addv(I.gneg);
    }
    off_perm_o[t] = B.blob.addv(I.perm_o);
    off_perm_u[t] = B.blob.addv(I.perm_u);
    off_eps_o[t] = B.blob.addv(I.eps_o);
    off_eps_u[t] = B.blob.addv(I.eps_u);
    off_coef[t] = B.blob.addv(I.coef);
    key << I.n0 << "," << I.n1 << "," << I.n2 << "," << I.cplx << "," << I.k_o << "," << I.k_u
        << "," << I.n_tau << "," << I.n_omega << "," << I.n_g << ";";
  }
  for (const auto &J : P.jobs) key << J.k_o_eff << "/" << J.k_u_eff << ",";
  // Geo entries hold device pointers: stored with offsets, patched later
  std::vector<Geo> geos(n_items);
  for (int t = 0; t < n_items; ++t) {
    const ItemPlan &I = P.items[t];
    Geo g{};
    g.n0 = I.n0;
    g.n1 = I.n1;
    g.n2 = I.n2;
    g.n_r = (int32_t)I.n_r;
    g.n_g = I.n_g;
    g.n_disk = I.n_disk;
    g.cols = I.cols;
    g.planes = I.planes;
    g.disk_i12 = reinterpret_cast<const int32_t *>(off_i12[t]);   // offset, patched
    g.slot_of = reinterpret_cast<const int32_t *>(off_sdk[t]);
    g.disk_of = reinterpret_cast<const int32_t *>(off_dof[t]);
    g.disk_pair = reinterpret_cast<const int32_t *>(off_pair[t]);
    g.disk_canon = reinterpret_cast<const int32_t *>(off_canon[t]);
    g.n_canon = (int32_t)I.disk_canon.size();
    g.slot_half = reinterpret_cast<const int32_t *>(off_shalf[t]);
    g.hrow = reinterpret_cast<const int32_t *>(off_hrow[t]);
    g.gneg = reinterpret_cast<const int32_t *>(off_gneg[t]);
    g.n_half = I.half ? (int32_t)I.hrow.size() : 0;
    geos[t] = g;
  }
  const size_t off_geos = B.blob.addv(geos);
  B.n_passes = (int)P.pass_begin.size() - 1;
  int max_slabs = 0;
  for (auto &I : P.items) max_slabs = std::max<int>(max_slabs, (int)((I.n_r + P.slab_w - 1) / P.slab_w));
  // norms: per-tau offsets (filled per pass), per-omega offsets (after the last pass)
  std::vector<int32_t> toff(n_items), woff(n_items);
  int nt = 0, nw = 0;
  for (int t = 0; t < n_items; ++t) {
    toff[t] = nt;
    woff[t] = nw;
    nt += P.items[t].n_tau;
    nw += P.items[t].n_omega;
  }
  B.n_norm_tau = nt;
  B.n_norm_omega = nw;
  const size_t off_toff = B.blob.addv(toff), off_woff = B.blob.addv(woff);
  if (want_norms) {
    Launch Z{};
    Z.phase = PH_NORM;
    Z.kind = 5;
    Z.fill_ptr = D.norm;
    Z.fill_bytes = (int64_t)(nt + nw) * kNormParts * 8;
    B.launches.push_back(Z);
  }
  for (int ps = 0; ps < B.n_passes; ++ps) {
    const int jb = P.pass_begin[ps], je = P.pass_begin[ps + 1];
    // ---- stage: one op per (item in pass, occ|unocc)
    {
      Launch L{};
      L.phase = PH_STAGE;
      L.kind = 0;
      L.stage = make_stage(B.blob, P, jb, je, psi_base, off_perm_o, off_perm_u, off_eps_o,
                           off_eps_u);
      B.launches.push_back(L);
    }
    // ---- per slab: gemm + fft over r
    // jobs with the most bands first, so that the persistent launch ends evenly
    std::vector<int> order;
    for (int q = jb; q < je; ++q) order.push_back(q);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
      return P.jobs[a].k_o_eff + P.jobs[a].k_u_eff > P.jobs[b].k_o_eff + P.jobs[b].k_u_eff;
    });
    // Tiles of a job form groups of about one XCD's resident workgroups,
    // gr x gc tiles (gc a power of two near the square root), so that the
    // tiles running together on one XCD share few operand panels.  Groups go,
    // in job order, to the least loaded of the per-XCD queues.
    const int per_cu = std::max(1, gemm_tile_per_cu(P.prec, cplx, P.tile));
    const int group = std::max(1, per_cu * ctx->num_cu / kGemmQueues);
    int gc_want = 1;
    while (gc_want * gc_want < group) gc_want *= 2;
    for (int s = 0; s < max_slabs; ++s) {
      std::vector<GemmJob> gj;
      std::vector<std::vector<int4>> qunits(kGemmQueues);
      std::vector<double> qwork(kGemmQueues, 0.0);
      std::vector<FftJob> fj;
      for (int q : order) {
        const JobPlan &J = P.jobs[q];
        const ItemPlan &I = P.items[J.item];
        const int64_t s0 = (int64_t)s * P.slab_w;
        if (s0 >= I.n_r) continue;
        const int w = (int)std::min<int64_t>(P.slab_w, I.n_r - s0);
        char *slot = psi_base + J.o_psi;
        GemmJob g{};
        g.psi_o = slot;
        g.psi_u = slot + I.n_r_pad * I.k_o_pad * bpb_of(P.prec, cplx);
        g.ld_o = I.k_o_pad;
        g.ld_u = I.k_u_pad;
        g.k_o = J.k_o_eff;
        g.k_u = J.k_u_eff;
        g.n_r = (int32_t)I.n_r;
        g.s0 = (int32_t)s0;
        g.w = w;
        g.cg_shift = 0;
        while ((1 << (g.cg_shift + 1)) <= I.sgroup) ++g.cg_shift;
        g.slab = slab_base + J.o_slab;
        const int gi = (int)gj.size();
        gj.push_back(g);
        const int nrt = (int)((I.n_r + P.bm - 1) / P.bm);
        const int nct = (w + P.bn - 1) / P.bn;
        const int gc = std::min(nct, gc_want);
        const int gr = std::max(1, (group + gc - 1) / gc);
        const double kk = (double)(J.k_o_eff + J.k_u_eff);
        for (int cb = 0; cb < nct; cb += gc) {
          for (int rb = 0; rb < nrt; rb += gr) {
            std::vector<int4> tiles;
            for (int rt = rb; rt < std::min(nrt, rb + gr); ++rt)
              for (int ct = cb; ct < std::min(nct, cb + gc); ++ct) {
                const int r0 = rt * P.bm, c0 = (int)s0 + ct * P.bn;
                if (ctx->opt.hermitian && r0 + P.bm <= c0) continue;
                tiles.push_back(make_int4(gi, r0, c0, 0));
              }
            if (tiles.empty()) continue;
            const int q = (int)(std::min_element(qwork.begin(), qwork.end()) - qwork.begin());
            qunits[q].insert(qunits[q].end(), tiles.begin(), tiles.end());
            qwork[q] += kk * (double)tiles.size();
            // complex FP64 / FP32 take three real products per band in the
            // unoccupied pass, four in the occupied one
            const double kmf = I.cplx ? (P.prec == P_BF16X3 ? 8.0 * kk
                                                             : 8.0 * J.k_o_eff + 6.0 * J.k_u_eff)
                                      : 2.0 * kk;
            P.mfma_flops += kmf * P.bm * P.bn * (P.prec == P_BF16X3 ? 3.0 : 1.0) *
                            (double)tiles.size();
          }
        }
        FftJob f{};
        f.in = g.slab;
        f.s_r = 1;
        f.s_col = 0;                       // column-grouped slab
        f.tmp = tmp_base + J.o_tmp;
        f.out = xr_base + J.o_xr;
        f.o_slot = I.n_r;
        f.o_col = 1;
        f.col0 = (int32_t)s0;
        f.n_cols = w;
        f.geo = J.item;
        f.half_rows = I.half;
        // single launch: rows of chi(G, r') column-grouped for the second index
        f.o_gshift = 0;
        while ((1 << (f.o_gshift + 1)) <= I.cols) ++f.o_gshift;
        fj.push_back(f);
      }
      if (gj.empty()) continue;
      Launch G{};
      G.phase = PH_GEMM;
      G.kind = 1;
      G.gemm.jobs = reinterpret_cast<const GemmJob *>(B.blob.addv(gj));
      std::vector<int4> units;
      G.gemm.n_queues = kGemmQueues;
      for (int q = 0; q < kGemmQueues; ++q) {
        G.gemm.q_off[q] = (int32_t)units.size();
        units.insert(units.end(), qunits[q].begin(), qunits[q].end());
      }
      G.gemm.q_off[kGemmQueues] = (int32_t)units.size();
      G.gemm.units = reinterpret_cast<const int4 *>(B.blob.addv(units));
      G.gemm.n_units = (int)units.size();
      G.gemm.hermitian = ctx->opt.hermitian;
      if (ctx->opt.persistent) {
        G.gemm.counter = D.ctr + B.n_gemm * kGemmQueues;
        G.gemm_grid = 0;
      } else {
        G.gemm.counter = nullptr;
        G.gemm_grid = (int)units.size();
      }
      ++B.n_gemm;
      B.launches.push_back(G);
      emit_fft(B, P, fj, PH_FFT_R, -1, cplx ? 0 : 1, ctx->opt.hermitian, off_geos);
    }
    // ---- fft over r': output stored transposed, x_j[g'][g]
    {
      std::vector<FftJob> fj;
      for (int q = jb; q < je; ++q) {
        const JobPlan &J = P.jobs[q];
        const ItemPlan &I = P.items[J.item];
        FftJob f{};
        f.in = xr_base + J.o_xr;
        f.s_r = 1;
        f.s_col = I.fused ? 0 : I.n_r;     // the single launch writes column groups
        f.tmp = tmp_base + J.o_tmp;
        f.out = x_base + J.o_x;
        f.o_slot = I.n_g;
        f.o_col = 1;
        f.col0 = 0;
        f.n_cols = I.half ? (int32_t)I.hrow.size() : I.n_g;
        f.half_rows = I.half;
        f.geo = J.item;
        fj.push_back(f);
      }
      emit_fft(B, P, fj, PH_FFT_RP, +1, 0, 0, off_geos);
    }
    // ---- cosine transform of this pass's taus, per item; an item whose taus
    // span passes continues its FP64 sums from the previous pass's output
    {
      std::vector<CtItem> cts;
      int tiles = 0, max_omega = 0, max_mats = 0;
      int jj = jb;
      while (jj < je) {
        const int t = P.jobs[jj].item;
        int je2 = jj;
        while (je2 < je && P.jobs[je2].item == t) ++je2;
        const ItemPlan &I = P.items[t];
        CtItem c{};
        c.x = x_base + P.jobs[jj].o_x;
        c.out = I.out;
        c.coef = reinterpret_cast<const double *>(off_coef[t]);
        c.n_g = I.n_g;
        c.n_tau = I.n_tau;
        c.j0 = P.jobs[jj].j;
        c.n_tau_x = je2 - jj;
        c.n_omega = I.n_omega;
        c.hermitian = ctx->opt.hermitian;
        c.accumulate = c.j0 > 0 ? 1 : 0;
        c.item = t;
        c.tile0 = tiles;
        const int tt = (I.n_g + 31) / 32;
        tiles += ctx->opt.hermitian ? tt * (tt + 1) / 2 : tt * ((I.n_g + 15) / 16);
        max_omega = std::max(max_omega, I.n_omega);
        max_mats = std::max(max_mats, je2 - jj);
        cts.push_back(c);
        jj = je2;
      }
      Launch C{};
      C.phase = PH_CT;
      C.kind = 3;
      C.ct.items = reinterpret_cast<const CtItem *>(B.blob.addv(cts));
      C.ct.n_items = (int)cts.size();
      C.ct.n_tiles = tiles;
      C.max_omega = max_omega;
      B.launches.push_back(C);
      if (want_norms) {
        Launch N{};
        N.phase = PH_NORM;
        N.kind = 4;
        N.ct = C.ct;
        N.norm_mode = 0;
        N.max_mats = max_mats;
        N.toff = reinterpret_cast<const int32_t *>(off_toff);
        N.woff = reinterpret_cast<const int32_t *>(off_woff);
        B.launches.push_back(N);
      }
    }
  }
  if (want_norms) {
    // norms of the finished outputs: one entry per item over its omegas
    std::vector<CtItem> cts;
    int max_omega = 0;
    for (int t = 0; t < n_items; ++t) {
      const ItemPlan &I = P.items[t];
      CtItem c{};
      c.out = I.out;
      c.n_g = I.n_g;
      c.n_tau = I.n_tau;
      c.n_omega = I.n_omega;
      c.item = t;
      cts.push_back(c);
      max_omega = std::max(max_omega, I.n_omega);
    }
    Launch N{};
    N.phase = PH_NORM;
    N.kind = 4;
    N.ct.items = reinterpret_cast<const CtItem *>(B.blob.addv(cts));
    N.ct.n_items = n_items;
    N.norm_mode = 1;
    N.max_mats = max_omega;
    N.toff = reinterpret_cast<const int32_t *>(off_toff);
    N.woff = reinterpret_cast<const int32_t *>(off_woff);
    B.launches.push_back(N);
  }
  // ticket counters of the persistent GEMM launches start at zero every build
  // (a fill kernel, which a captured graph replays correctly)
  if (B.n_gemm > 0 && ctx->opt.persistent) {
    Launch Z{};
    Z.phase = PH_STAGE;
    Z.kind = 5;
    Z.fill_ptr = D.ctr;
    Z.fill_bytes = (int64_t)B.n_gemm * kGemmQueues * 4;
    B.launches.insert(B.launches.begin(), Z);
  }
  key << "|persistent=" << ctx->opt.persistent;
  B.key = key.str();
}

// Replace blob offsets by device addresses.  Offsets are small integers
// (< blob size); every pointer field that refers to the blob was stored as an
// offset by build_launches, and every other pointer field holds a real device
// address, so the distinction is by construction, not by value.
template <typename T>
T *dev(const char *base, const T *off) {
  return reinterpret_cast<T *>(const_cast<char *>(base) + reinterpret_cast<uintptr_t>(off));
}

void patch_stage(StageLaunch &S, char *h, const char *base) {
  StageOp *ops = reinterpret_cast<StageOp *>(h + reinterpret_cast<uintptr_t>(S.ops));
  // the op count is implied by the blocks: walk the ops the blocks reference
  const int4 *blk = reinterpret_cast<const int4 *>(h + reinterpret_cast<uintptr_t>(S.blocks));
  int n_ops = 0;
  for (int i = 0; i < S.n_blocks; ++i) n_ops = std::max(n_ops, blk[i].x + 1);
  for (int i = 0; i < n_ops; ++i) {
    ops[i].perm = dev(base, ops[i].perm);
    ops[i].eps = dev(base, ops[i].eps);
    ops[i].tau = dev(base, ops[i].tau);
    ops[i].psi = dev(base, ops[i].psi);
  }
  S.ops = dev(base, S.ops);
  S.blocks = dev(base, S.blocks);
}

void patch_blob(Built &B, const char *base) {
  char *h = B.blob.h.data();
  for (auto &L : B.launches) {
    if (L.kind == 0) {
      patch_stage(L.stage, h, base);
    } else if (L.kind == 1) {
      L.gemm.jobs = dev(base, L.gemm.jobs);
      L.gemm.units = dev(base, L.gemm.units);
    } else if (L.kind == 2) {
      L.fft.jobs = dev(base, L.fft.jobs);
      L.fft.geos = dev(base, L.fft.geos);
    } else if (L.kind == 3 || L.kind == 4) {
      CtItem *cts = reinterpret_cast<CtItem *>(h + reinterpret_cast<uintptr_t>(L.ct.items));
      if (L.kind == 3)
        for (int i = 0; i < L.ct.n_items; ++i) cts[i].coef = dev(base, cts[i].coef);
      L.ct.items = dev(base, L.ct.items);
      if (L.kind == 4) {
        L.toff = dev(base, L.toff);
        L.woff = dev(base, L.woff);
      }
    }
  }
}

void patch_geos(Blob &blob, const char *base, size_t off_geos, int n_items) {
  Geo *g = reinterpret_cast<Geo *>(blob.h.data() + off_geos);
  for (int i = 0; i < n_items; ++i) {
    g[i].disk_i12 = dev(base, g[i].disk_i12);
    g[i].slot_of = dev(base, g[i].slot_of);
    g[i].disk_of = dev(base, g[i].disk_of);
    if (g[i].n_canon > 0) {
      g[i].disk_pair = dev(base, g[i].disk_pair);
      g[i].disk_canon = dev(base, g[i].disk_canon);
    }
    if (g[i].n_half > 0) {
      g[i].slot_half = dev(base, g[i].slot_half);
      g[i].hrow = dev(base, g[i].hrow);
      g[i].gneg = dev(base, g[i].gneg);
    }
  }
}

gwchi_status enqueue(gwchi_ctx *ctx, const Plan &P, Built &B, const Bases &D, bool timing,
                     std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> *evs) {
  hipStream_t s = ctx->stream;
  const int cplx = P.cplx_any;
  const int dbl = P.prec == P_FP64;
  size_t ev_i = 0;
  auto ev = [&](void) -> hipEvent_t {
    if (ev_i >= ctx->ev_pool.size()) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
      ctx->ev_pool.push_back(e);
    }
    return ctx->ev_pool[ev_i++];
  };
  for (auto &L : B.launches) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (timing) {
      e0 = ev();
      e1 = ev();
      if (!e0 || !e1) {
        set_err(ctx, "hipEventCreate failed");
        return GWCHI_EDEVICE;
      }
      HIPCHK(hipEventRecord(e0, s));
    }
    switch (L.kind) {
      case 0:
        HIPCHK(launch_stage(L.stage, P.prec, s));
        break;
      case 1:
        HIPCHK(launch_gemm(L.gemm, P.prec, cplx, P.tile, L.gemm_grid, ctx->num_cu, s));
        break;
      case 2:
        HIPCHK(launch_fft(L.fft, dbl, L.fft_sign, L.fft_lds, L.fft_cubic, s));
        break;
      case 3:
        HIPCHK(launch_ct(L.ct, dbl, L.max_omega, ctx->opt.hermitian, s));
        break;
      case 4:
        HIPCHK(launch_norms_impl(L.ct, dbl, L.norm_mode, D.norm,
                                 D.norm + (int64_t)B.n_norm_tau * kNormParts,
                                 L.toff, L.woff, L.max_mats, s));
        break;
      case 5:
        HIPCHK(launch_fill_zero(L.fill_ptr, L.fill_bytes, s));
        break;
    }
    if (timing) {
      HIPCHK(hipEventRecord(e1, s));
      evs->push_back({L.phase, {e0, e1}});
    }
  }
  return GWCHI_OK;
}

// noalloc: carve every buffer from the fixed device scratch instead of the
// context's allocations (no report, no graph, no kappa norms).
gwchi_status run_build(gwchi_ctx *ctx, const gwchi_item *items, int n_items, int prec,
                       gwchi_report *rep, bool noalloc = false) {
  Plan P;
  const int64_t arena = noalloc ? kNoAllocBytes - kNoAllocTables - kNoAllocCounters : 0;
  gwchi_status st = build_plan(ctx, items, n_items, prec, P, arena);
  if (st != GWCHI_OK) return st;
  // every buffer and table below may still be read by the previous build
  HIPCHK(hipStreamSynchronize(ctx->stream));
  const bool want_norms = !noalloc && rep != nullptr && ctx->opt.kappa != 0;
  int n_norm = 0;
  for (auto &I : P.items) n_norm += I.n_tau + I.n_omega;
  int max_slabs = 0;
  for (auto &I : P.items) max_slabs = std::max<int>(max_slabs, (int)((I.n_r + P.slab_w - 1) / P.slab_w));
  const size_t n_ctr = (size_t)((int)P.pass_begin.size() - 1) * max_slabs + 16;
  Bases D;
  bool moved = false;
  if (noalloc) {
    char *base = reinterpret_cast<char *>(ctx->noalloc_scratch);
    if ((int64_t)(n_ctr * kGemmQueues * 4) > kNoAllocCounters) {
      set_err(ctx, "allocation-free build: too many GEMM launches for the counter region");
      return GWCHI_ENOMEM;
    }
    D.tables = base;
    D.ctr = reinterpret_cast<int32_t *>(base + kNoAllocTables);
    char *p = base + kNoAllocTables + kNoAllocCounters;
    char **dst[5] = {&D.psi, &D.slab, &D.xr, &D.tmp, &D.x};
    const int64_t need[5] = {P.psi_bytes, P.slab_bytes, P.xr_bytes, P.tmp_bytes, P.x_bytes};
    for (int k = 0; k < 5; ++k) {
      *dst[k] = p;
      p += round_up(need[k], 256);
    }
    if (p > base + kNoAllocBytes) {       // the planner sized the buffers to fit
      set_err(ctx, "allocation-free build: plan exceeds the fixed scratch");
      return GWCHI_ENOMEM;
    }
  } else {
    // scratch for the plan; when any buffer must grow, drop all of them first so
    // that old and new never coexist
    DevBuf *bufs[5] = {&ctx->b_psi, &ctx->b_slab, &ctx->b_xr, &ctx->b_tmp, &ctx->b_x};
    const int64_t need[5] = {P.psi_bytes, P.slab_bytes, P.xr_bytes, P.tmp_bytes, P.x_bytes};
    bool grow = false;
    for (int k = 0; k < 5; ++k) grow |= (size_t)need[k] > bufs[k]->n;
    if (grow) {
      for (int k = 0; k < 5; ++k) bufs[k]->release();
      for (int k = 0; k < 5; ++k) HIPCHK(bufs[k]->ensure((size_t)need[k], nullptr));
    }
    HIPCHK(ctx->b_norm.ensure((size_t)n_norm * kNormParts * 8 + 64, &moved));
    HIPCHK(ctx->b_ctr.ensure(n_ctr * kGemmQueues * 4, &moved));
    D.psi = reinterpret_cast<char *>(ctx->b_psi.p);
    D.slab = reinterpret_cast<char *>(ctx->b_slab.p);
    D.xr = reinterpret_cast<char *>(ctx->b_xr.p);
    D.tmp = reinterpret_cast<char *>(ctx->b_tmp.p);
    D.x = reinterpret_cast<char *>(ctx->b_x.p);
    D.norm = reinterpret_cast<double *>(ctx->b_norm.p);
    D.ctr = reinterpret_cast<int32_t *>(ctx->b_ctr.p);
  }
  Built B;
  build_launches(ctx, P, want_norms, D, B);
  // geos offset: locate it as the table referenced by the first FFT launch
  size_t off_geos = 0;
  for (auto &L : B.launches)
    if (L.kind == 2) {
      off_geos = reinterpret_cast<uintptr_t>(L.fft.geos);
      break;
    }
  if (noalloc) {
    if ((int64_t)B.blob.h.size() > kNoAllocTables) {
      set_err(ctx, "allocation-free build: launch tables of " + std::to_string(B.blob.h.size()) +
                       " bytes exceed the " + std::to_string(kNoAllocTables) + "-byte table region");
      return GWCHI_ENOMEM;
    }
  } else {
    HIPCHK(ctx->b_tables.ensure(B.blob.h.size() + 64, &moved));
    D.tables = reinterpret_cast<char *>(ctx->b_tables.p);
  }
  patch_geos(B.blob, D.tables, off_geos, n_items);
  patch_blob(B, D.tables);
  if (noalloc) {
    // the host copy lives in the context until the next build (which first
    // waits for this one's stream), so the asynchronous copy may read it late
    ctx->noalloc_blob.assign(B.blob.h.begin(), B.blob.h.end());
    HIPCHK(hipMemcpyAsync(D.tables, ctx->noalloc_blob.data(), ctx->noalloc_blob.size(),
                          hipMemcpyHostToDevice, ctx->stream));
    return enqueue(ctx, P, B, D, false, nullptr);
  }
  HIPCHK(ctx->h_tables.ensure(B.blob.h.size() + 64));
  std::memcpy(ctx->h_tables.p, B.blob.h.data(), B.blob.h.size());
  HIPCHK(hipMemcpyAsync(D.tables, ctx->h_tables.p, B.blob.h.size(),
                        hipMemcpyHostToDevice, ctx->stream));
  const bool timing = ctx->opt.timing != 0;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> evs;
  hipEvent_t t0 = nullptr, t1 = nullptr;
  if (rep) {
    HIPCHK(hipEventCreate(&t0));
    HIPCHK(hipEventCreate(&t1));
    HIPCHK(hipEventRecord(t0, ctx->stream));
  }
  bool replayed = false;
  // HIP events recorded inside a captured graph cannot be timed, so the
  // per-launch timing mode runs the same launch list eagerly.
  const bool use_graph = ctx->opt.use_graph != 0 && !timing;
  if (use_graph) {
    std::ostringstream k;
    k << B.key << "|timing=" << timing << "|tables=" << ctx->b_tables.p << ",psi=" << ctx->b_psi.p
      << ",slab=" << ctx->b_slab.p << ",xr=" << ctx->b_xr.p << ",x=" << ctx->b_x.p << ",sc="
      << ctx->b_tmp.p << ",norm=" << ctx->b_norm.p;
    for (auto &I : P.items) k << "," << (const void *)I.phi_o << (const void *)I.phi_u << (void *)I.out;
    const std::string key = k.str();
    if (ctx->graph_exec && key == ctx->graph_key) {
      HIPCHK(hipGraphLaunch(ctx->graph_exec, ctx->stream));
      evs = ctx->graph_evs;
      replayed = true;
    } else {
      if (ctx->graph_exec) {
        (void)hipGraphExecDestroy(ctx->graph_exec);
        ctx->graph_exec = nullptr;
      }
      if (ctx->graph) {
        (void)hipGraphDestroy(ctx->graph);
        ctx->graph = nullptr;
      }
      ctx->graph_key.clear();
      HIPCHK(hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal));
      st = enqueue(ctx, P, B, D, false, nullptr);
      hipGraph_t g = nullptr;
      hipError_t ec = hipStreamEndCapture(ctx->stream, &g);
      if (st != GWCHI_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
      }
      if (ec != hipSuccess) {
        set_err(ctx, std::string("hipStreamEndCapture: ") + hipGetErrorString(ec));
        return GWCHI_EDEVICE;
      }
      hipGraphExec_t ex = nullptr;
      hipError_t ei = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
      if (ei != hipSuccess) {
        (void)hipGraphDestroy(g);
        set_err(ctx, std::string("hipGraphInstantiate: ") + hipGetErrorString(ei));
        return GWCHI_EDEVICE;
      }
      ctx->graph = g;
      ctx->graph_exec = ex;
      ctx->graph_key = key;
      ctx->graph_evs = evs;
      HIPCHK(hipGraphLaunch(ctx->graph_exec, ctx->stream));
    }
  } else {
    st = enqueue(ctx, P, B, D, timing, &evs);
    if (st != GWCHI_OK) return st;
  }
  if (rep) {
    HIPCHK(hipEventRecord(t1, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    std::memset(rep, 0, sizeof(*rep));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, t0, t1));
    rep->ms_total = ms;
    double ph[PH_COUNT] = {0};
    for (auto &e : evs) {
      float m = 0.f;
      HIPCHK(hipEventElapsedTime(&m, e.second.first, e.second.second));
      ph[e.first] += m;
      if (e.first == PH_GEMM) rep->n_gemm_launches++;
      if (e.first == PH_FFT_R || e.first == PH_FFT_RP) rep->n_fft_launches++;
    }
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    rep->ms_stage = ph[PH_STAGE];
    rep->ms_gemm = ph[PH_GEMM];
    rep->ms_fft_r = ph[PH_FFT_R];
    rep->ms_fft_rp = ph[PH_FFT_RP];
    rep->ms_ct = ph[PH_CT];
    rep->alg_flops = P.alg_flops;
    rep->mfma_flops = P.mfma_flops;
    rep->slab_width = P.slab_w;
    rep->tau_batch = P.max_jobs_pass;
    rep->tile_id = P.tile + 1;
    rep->graph_replayed = replayed ? 1 : 0;
    rep->kappa_F_max = -1.0;
  }
  if (rep && want_norms) {
    // kappa_F from the norms: each squared norm is the in-order sum of its partial slots
    std::vector<double> part((size_t)n_norm * kNormParts), nrm(n_norm, 0.0);
    HIPCHK(hipMemcpy(part.data(), D.norm, part.size() * 8, hipMemcpyDeviceToHost));
    for (int m = 0; m < n_norm; ++m)
      for (int p = 0; p < kNormParts; ++p) nrm[m] += part[(size_t)m * kNormParts + p];
    double kmax = 0.0;
    int ot = 0, ow = B.n_norm_tau;
    for (auto &I : P.items) {
      for (int k = 0; k < I.n_omega; ++k) {
        double num = 0.0;
        for (int j = 0; j < I.n_tau; ++j)
          num += std::fabs(I.coef[(size_t)k * I.n_tau + j]) * std::sqrt(nrm[ot + j]);
        const double den = std::sqrt(nrm[ow + k]);
        if (den > 0) kmax = std::max(kmax, num / den);
      }
      ot += I.n_tau;
      ow += I.n_omega;
    }
    rep->kappa_F_max = kmax;
  }
  return GWCHI_OK;
}

gwchi_status check_output(gwchi_ctx *ctx, const gwchi_item *items, int n_items) {
  for (int t = 0; t < n_items; ++t) {
    const int64_t n = (int64_t)items[t].n_omega * items[t].n_g * items[t].n_g * 2;
    if (!finite_all(items[t].chi_out, n)) {
      set_err(ctx, "output check: non-finite value in chi_out of item " + std::to_string(t));
      return GWCHI_ENUMERIC;
    }
  }
  return GWCHI_OK;
}

void load_tune(gwchi_ctx *ctx) {
  ctx->tune.clear();
  if (ctx->tune_path.empty()) return;
  std::ifstream f(ctx->tune_path);
  if (!f) return;
  // flat JSON object of "key": int
  std::string s((std::istreambuf_iterator<char>(f)), std::istreambuf_iterator<char>());
  size_t p = 0;
  while ((p = s.find('"', p)) != std::string::npos) {
    size_t q = s.find('"', p + 1);
    if (q == std::string::npos) break;
    std::string k = s.substr(p + 1, q - p - 1);
    size_t c = s.find(':', q);
    if (c == std::string::npos) break;
    int v = std::atoi(s.c_str() + c + 1);
    ctx->tune[k] = v;
    p = s.find_first_of(",}", c);
    if (p == std::string::npos) break;
  }
}

void save_tune(gwchi_ctx *ctx) {
  if (ctx->tune_path.empty()) return;
  std::ofstream f(ctx->tune_path);
  f << "{";
  bool first = true;
  for (auto &kv : ctx->tune) {
    f << (first ? "" : ", ") << "\"" << kv.first << "\": " << kv.second;
    first = false;
  }
  f << "}\n";
}


// Copy host orbitals into the context's device buffer and point a copy of the
// items at device orbitals and a device output buffer.
gwchi_status upload_items(gwchi_ctx *ctx, const gwchi_item *items, int n_items,
                          std::vector<gwchi_item> &dev_items) {
  int64_t in_bytes = 0, out_bytes = 0;
  std::vector<int64_t> in_off(n_items), out_off(n_items);
  for (int t = 0; t < n_items; ++t) {
    const gwchi_item &it = items[t];
    const int64_t n_r = (int64_t)it.n[0] * it.n[1] * it.n[2];
    const int64_t m = n_r * (it.is_complex ? 2 : 1) * 8;
    in_off[t] = in_bytes;
    in_bytes += round_up(m * (it.n_occ + it.n_unocc), 256);
    out_off[t] = out_bytes;
    out_bytes += round_up((int64_t)it.n_omega * it.n_g * it.n_g * 16, 256);
  }
  bool moved = false;
  if ((size_t)in_bytes > ctx->b_phi.n || (size_t)out_bytes > ctx->b_out.n)
    HIPCHK(hipStreamSynchronize(ctx->stream));
  HIPCHK(ctx->b_phi.ensure((size_t)in_bytes, &moved));
  HIPCHK(ctx->b_out.ensure((size_t)out_bytes, &moved));
  dev_items.assign(items, items + n_items);
  for (int t = 0; t < n_items; ++t) {
    const gwchi_item &it = items[t];
    const int64_t n_r = (int64_t)it.n[0] * it.n[1] * it.n[2];
    const int64_t m = n_r * (it.is_complex ? 2 : 1) * 8;
    char *base = reinterpret_cast<char *>(ctx->b_phi.p) + in_off[t];
    HIPCHK(hipMemcpy(base, it.phi_occ, m * it.n_occ, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(base + m * it.n_occ, it.phi_unocc, m * it.n_unocc, hipMemcpyHostToDevice));
    dev_items[t].phi_occ = reinterpret_cast<const double *>(base);
    dev_items[t].phi_unocc = reinterpret_cast<const double *>(base + m * it.n_occ);
    dev_items[t].chi_out =
        reinterpret_cast<double *>(reinterpret_cast<char *>(ctx->b_out.p) + out_off[t]);
  }
  return GWCHI_OK;
}

// ---------------------------------------------------------------------------
// Screened interaction W~ from chi (Sec. II.C steps (iii)-(iv)).
// ---------------------------------------------------------------------------

// Inverse of the n x n row-major matrix a by Gauss-Jordan elimination with
// partial pivoting, in FP64 (the inverse cosine matrix of Eq. (6)); false
// when a pivot falls below 1e-13 n max|a| (numerically singular) or the
// result is not finite.
bool invert_small(const double *a, int n, std::vector<double> &inv) {
  std::vector<double> m(a, a + (size_t)n * n);
  double scale = 0.0;
  for (double x : m) scale = std::max(scale, std::fabs(x));
  const double tiny = 1e-13 * n * scale;
  inv.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) inv[(size_t)i * n + i] = 1.0;
  for (int c = 0; c < n; ++c) {
    int piv = c;
    double best = std::fabs(m[(size_t)c * n + c]);
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(m[(size_t)r * n + c]) > best) {
        best = std::fabs(m[(size_t)r * n + c]);
        piv = r;
      }
    if (!(best > tiny) || !std::isfinite(best)) return false;
    if (piv != c)
      for (int k = 0; k < n; ++k) {
        std::swap(m[(size_t)c * n + k], m[(size_t)piv * n + k]);
        std::swap(inv[(size_t)c * n + k], inv[(size_t)piv * n + k]);
      }
    const double d = 1.0 / m[(size_t)c * n + c];
    for (int k = 0; k < n; ++k) {
      m[(size_t)c * n + k] *= d;
      inv[(size_t)c * n + k] *= d;
    }
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      const double f = m[(size_t)r * n + c];
      if (f == 0.0) continue;
      for (int k = 0; k < n; ++k) {
        m[(size_t)r * n + k] -= f * m[(size_t)c * n + k];
        inv[(size_t)r * n + k] -= f * inv[(size_t)c * n + k];
      }
    }
  }
  return finite_all(inv.data(), (int64_t)n * n);
}

// Host checks of the items; fills the inverse cosine matrix of each item.
gwchi_status validate_w_items(gwchi_ctx *ctx, const gwchi_w_item *items, int32_t n_items,
                              std::vector<std::vector<double>> &ict) {
  if (!items || n_items < 1) {
    set_err(ctx, "items is NULL or n_items < 1");
    return GWCHI_EINVAL;
  }
  ict.assign(n_items, {});
  for (int t = 0; t < n_items; ++t) {
    const gwchi_w_item &it = items[t];
    const std::string at = "w item " + std::to_string(t) + ": ";
    if (!it.chi || !it.sqrt_v || !it.ct || !it.w_tau_out) {
      set_err(ctx, at + "chi, sqrt_v, ct and w_tau_out must not be NULL");
      return GWCHI_EINVAL;
    }
    if (it.n_g < 1 || it.n_g > 65535) {
      set_err(ctx, at + "n_g must be in [1, 65535]");
      return GWCHI_EINVAL;
    }
    if (it.n_omega < 1 || it.n_tau != it.n_omega || it.n_tau > kWMaxTau) {
      set_err(ctx, at + "n_tau must equal n_omega, in [1, " + std::to_string(kWMaxTau) + "]");
      return GWCHI_EINVAL;
    }
    for (int g = 0; g < it.n_g; ++g)
      if (!(it.sqrt_v[g] >= 0.0) || !std::isfinite(it.sqrt_v[g])) {
        set_err(ctx, at + "sqrt_v must be finite and >= 0");
        return GWCHI_EINVAL;
      }
    if (!finite_all(it.ct, (int64_t)it.n_omega * it.n_tau)) {
      set_err(ctx, at + "ct is not finite");
      return GWCHI_EINVAL;
    }
    if (!invert_small(it.ct, it.n_tau, ict[t])) {
      set_err(ctx, at + "ct is singular");
      return GWCHI_EINVAL;
    }
  }
  return GWCHI_OK;
}

// Enqueue W~ for items whose chi and outputs are device pointers, on the
// context's stream.  With a report: wait, fill it and check the pivot flag.
gwchi_status run_w(gwchi_ctx *ctx, const gwchi_w_item *items, int n_items,
                   const std::vector<std::vector<double>> &ict, gwchi_w_report *rep) {
  hipStream_t st = ctx->stream;
  int64_t a_b = 0, p_b = 0, d_b = 0, tab = 0;
  std::vector<int64_t> toff(n_items), tile_off(n_items);
  std::vector<std::vector<int32_t>> tiles(n_items);   // per item: 9 offsets, then the pairs
  for (int t = 0; t < n_items; ++t) {
    const gwchi_w_item &it = items[t];
    const int64_t n = it.n_g, K = it.n_omega;
    a_b = std::max(a_b, K * n * n * 16);
    p_b = std::max(p_b, K * kWBlock * n * 16);
    d_b = std::max(d_b, K * kWBlock * kWBlock * 16);
    toff[t] = tab;
    tab += round_up(n + (int64_t)it.n_tau * it.n_omega, 32);
    std::vector<int32_t> pairs;
    int32_t off[9];
    w_tile_table((int)n, pairs, off);
    tiles[t].assign(off, off + 9);
    tiles[t].push_back(0);                       // the pairs start 8-byte aligned
    tiles[t].insert(tiles[t].end(), pairs.begin(), pairs.end());
    tile_off[t] = tab;
    tab += round_up(((int64_t)tiles[t].size() + 1) / 2, 32);   // in doubles
  }
  HIPCHK(ctx->b_wa.ensure(a_b, nullptr));
  HIPCHK(ctx->b_wrp.ensure(p_b, nullptr));
  HIPCHK(ctx->b_wcp.ensure(p_b, nullptr));
  HIPCHK(ctx->b_wdinv.ensure(d_b, nullptr));
  HIPCHK(ctx->b_wtab.ensure(tab * 8, nullptr));
  HIPCHK(ctx->b_wflag.ensure(256, nullptr));
  // the pinned staging buffer may still feed an earlier call's copy
  HIPCHK(hipStreamSynchronize(st));
  HIPCHK(ctx->h_wtab.ensure(tab * 8));
  double *h = reinterpret_cast<double *>(ctx->h_wtab.p);
  for (int t = 0; t < n_items; ++t) {
    const gwchi_w_item &it = items[t];
    std::memcpy(h + toff[t], it.sqrt_v, (size_t)it.n_g * 8);
    std::memcpy(h + toff[t] + it.n_g, ict[t].data(), ict[t].size() * 8);
    std::memcpy(h + tile_off[t], tiles[t].data(), tiles[t].size() * 4);
  }
  HIPCHK(hipMemcpyAsync(ctx->b_wtab.p, h, tab * 8, hipMemcpyHostToDevice, st));
  int *flag = reinterpret_cast<int *>(ctx->b_wflag.p);
  HIPCHK(launch_fill_zero(flag, 256, st));
  int launches = 1;
  std::vector<hipEvent_t> ev;
  auto mark = [&]() -> gwchi_status {
    if (!rep) return GWCHI_OK;
    hipEvent_t e;
    HIPCHK(hipEventCreate(&e));
    ev.push_back(e);
    HIPCHK(hipEventRecord(e, st));
    return GWCHI_OK;
  };
  auto cleanup = [&]() {
    for (auto e : ev) (void)hipEventDestroy(e);
  };
  gwchi_status s0 = mark();
  if (s0 != GWCHI_OK) return cleanup(), s0;
  double flops = 0.0;
  for (int t = 0; t < n_items; ++t) {
    const gwchi_w_item &it = items[t];
    const int n = it.n_g, K = it.n_omega;
    const double *s_dev = reinterpret_cast<const double *>(ctx->b_wtab.p) + toff[t];
    const double *ict_dev = s_dev + n;
    const int32_t *tile_dev =
        reinterpret_cast<const int32_t *>(reinterpret_cast<const double *>(ctx->b_wtab.p) + tile_off[t]);
    hipError_t e = launch_w_eps(it.chi, s_dev, ctx->b_wa.p, n, K, st);
    ++launches;
    if (e == hipSuccess && (s0 = mark()) != GWCHI_OK) return cleanup(), s0;
    for (int p0 = 0; e == hipSuccess && p0 < n; p0 += kWBlock) {
      e = launch_w_block(ctx->b_wa.p, ctx->b_wdinv.p, ctx->b_wrp.p, ctx->b_wcp.p, n, K, p0,
                         tile_dev + 10, tile_dev, flag, st);
      launches += 3;
    }
    if (e == hipSuccess && (s0 = mark()) != GWCHI_OK) return cleanup(), s0;
    if (e == hipSuccess)
      e = launch_w_final(ctx->b_wa.p, s_dev, ict_dev, it.w_tau_out, it.w_omega_out, n, K,
                         it.n_tau, st);
    ++launches;
    if (e != hipSuccess) {
      cleanup();
      set_err(ctx, std::string("W~ launch: ") + hipGetErrorString(e));
      return GWCHI_EDEVICE;
    }
    if ((s0 = mark()) != GWCHI_OK) return cleanup(), s0;
    flops += 8.0 * (double)n * n * n * K;
  }
  if (!rep) return GWCHI_OK;
  hipError_t e = hipStreamSynchronize(st);
  gwchi_w_report r{};
  r.alg_flops = flops;
  r.n_launches = launches;
  float ms = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev.front(), ev.back());
  r.ms_total = ms;
  for (int t = 0; t < n_items && e == hipSuccess; ++t) {
    float a = 0.f, b = 0.f, c = 0.f;
    e = hipEventElapsedTime(&a, ev[3 * t], ev[3 * t + 1]);
    if (e == hipSuccess) e = hipEventElapsedTime(&b, ev[3 * t + 1], ev[3 * t + 2]);
    if (e == hipSuccess) e = hipEventElapsedTime(&c, ev[3 * t + 2], ev[3 * t + 3]);
    r.ms_eps += a;
    r.ms_invert += b;
    r.ms_final += c;
  }
  int hflag = 0;
  if (e == hipSuccess) e = hipMemcpy(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost);
  cleanup();
  if (e != hipSuccess) {
    set_err(ctx, std::string("W~: ") + hipGetErrorString(e));
    return GWCHI_EDEVICE;
  }
  *rep = r;
  if (hflag) {
    set_err(ctx, "W~: a pivot of the dielectric matrix is not positive (eps is not positive definite)");
    return GWCHI_ENUMERIC;
  }
  return GWCHI_OK;
}

// ---------------------------------------------------------------------------
// Self-energy (Sec. II.D): diagonal elements on the imaginary axis.
//
// One call is planned like a polarizability build (jobs = (item, tau_j),
// passes sized to the device budget, r' slabs).  Per pass:
//   stage (weights, scaled operands)                      - all jobs
//   W~(G, G') -> W~(G, r') (sphere-to-grid over G')       - all jobs
//   for every r' slab: W~(G, r') -> W~(r, r'), then the fused band GEMM with
//   the products and the matrix elements                  - one launch each
//   sums over the tiles per (job, state)                  - one launch
// and after the last pass one launch for the even/odd parts and transforms.
// ---------------------------------------------------------------------------

constexpr int kSigmaMaxStates = 1024;
enum SPhase { SP_STAGE = 0, SP_FFT, SP_GEMM, SP_FINAL, SP_COUNT };

// The fields a self-energy item shares with a polarizability item, for the
// shared validation and planner (sigma_out stands in for chi_out; it is
// never written through this copy).
gwchi_item sigma_as_item(const gwchi_sigma_item &s) {
  gwchi_item it{};
  for (int d = 0; d < 3; ++d) it.n[d] = s.n[d];
  it.is_complex = s.is_complex;
  it.n_occ = s.n_occ;
  it.n_unocc = s.n_unocc;
  it.phi_occ = s.phi_occ;
  it.phi_unocc = s.phi_unocc;
  it.eps_occ = s.eps_occ;
  it.eps_unocc = s.eps_unocc;
  it.mu = s.mu;
  it.n_tau = s.n_tau;
  it.n_omega = s.n_omega;
  it.tau = s.tau;
  it.ct = s.ct;
  it.n_g = s.n_g;
  it.g_index = s.g_index;
  it.chi_out = s.sigma_out;
  return it;
}

gwchi_status validate_sigma_items(gwchi_ctx *ctx, const gwchi_sigma_item *items, int32_t n_items,
                                  bool check_orbitals) {
  if (!items || n_items < 1) {
    set_err(ctx, "items is NULL or n_items < 1");
    return GWCHI_EINVAL;
  }
  std::vector<gwchi_item> conv(n_items);
  for (int t = 0; t < n_items; ++t) {
    const gwchi_sigma_item &it = items[t];
    const std::string pre = "sigma item " + std::to_string(t) + ": ";
    if (!it.st || !it.w_tau || !it.states || !it.sigma_out) {
      set_err(ctx, pre + "st, w_tau, states and sigma_out must not be NULL");
      return GWCHI_EINVAL;
    }
    if (it.is_complex == 0) {
      set_err(ctx, pre + "real orbitals are not supported by the self-energy step");
      return GWCHI_ENOTSUP;
    }
    if (it.n_states < 1 || it.n_states > kSigmaMaxStates) {
      set_err(ctx, pre + "n_states must be in [1, " + std::to_string(kSigmaMaxStates) + "]");
      return GWCHI_EINVAL;
    }
    conv[t] = sigma_as_item(it);
  }
  gwchi_status st = validate_items(ctx, conv.data(), n_items, check_orbitals);
  if (st != GWCHI_OK) return st;
  for (int t = 0; t < n_items; ++t) {
    const gwchi_sigma_item &it = items[t];
    const std::string pre = "sigma item " + std::to_string(t) + ": ";
    if (!finite_all(it.st, (int64_t)it.n_tau * it.n_omega)) {
      set_err(ctx, pre + "st is not finite");
      return GWCHI_EINVAL;
    }
    for (int k = 0; k < it.n_states; ++k)
      if (it.states[k] < 0 || it.states[k] >= it.n_occ + it.n_unocc) {
        set_err(ctx, pre + "state index out of range");
        return GWCHI_EINVAL;
      }
  }
  return GWCHI_OK;
}

struct SLaunch {
  int phase = 0;
  int kind = 0;   // 0 stage, 5 fill, 6 states, 7 sphere-to-grid FFT, 8 GEMM, 9 reduce, 10 final
  StageLaunch stage{};
  SfftLaunch sfft{};
  int sign = 0;
  GemmLaunch gemm{};
  const double *phi_o = nullptr, *phi_u = nullptr;
  const int32_t *states = nullptr;
  int n_states = 0, n_occ = 0, n_r = 0, n_r_pad = 0;
  void *out = nullptr;
  const SigmaRed *red = nullptr;
  const SigmaFin *fin = nullptr;
  int n = 0, max_states = 0, max_omega = 0;
  int cubic = 0;                  // sphere-to-grid: shared cubic grid edge, or 0
  void *fill_ptr = nullptr;
  int64_t fill_bytes = 0;
};

// Unit counts of a sphere-to-grid launch: job prefix offsets and totals.
// units of a sphere-to-grid launch; returns the grid edge the jobs share when
// every grid is cubic and the same (the plane kernel then runs with
// compile-time line lengths), else 0
int sfft_units(std::vector<SfftJob> &jobs, const std::vector<Geo> &geos, SfftLaunch &L) {
  int up = 0, un = 0;
  int cubic = -1;
  for (auto &j : jobs) {
    const Geo &g = geos[j.geo];
    const int n = (g.n0 == g.n1 && g.n1 == g.n2) ? g.n0 : 0;
    cubic = cubic < 0 ? n : (cubic == n ? n : 0);
    j.unit0_pencils = un;
    j.unit0_planes = up;
    un += g.n_disk * ((j.n_cols + 255) / 256);
    up += ((j.n_cols + g.cols - 1) / g.cols) * ((g.n0 + g.planes - 1) / g.planes);
  }
  L.n_units_pencils = un;
  L.n_units_planes = up;
  return cubic < 0 ? 0 : cubic;
}

gwchi_status run_sigma(gwchi_ctx *ctx, const gwchi_sigma_item *items, int n_items, int prec,
                       gwchi_sigma_report *rep) {
  std::vector<gwchi_item> conv(n_items);
  int max_states = 0, max_omega = 0;
  for (int t = 0; t < n_items; ++t) {
    conv[t] = sigma_as_item(items[t]);
    max_states = std::max(max_states, items[t].n_states);
    max_omega = std::max(max_omega, items[t].n_omega);
  }
  Plan P;
  gwchi_status st = build_plan(ctx, conv.data(), n_items, prec, P, 0, max_states);
  if (st != GWCHI_OK) return st;
  HIPCHK(hipStreamSynchronize(ctx->stream));
  {
    DevBuf *bufs[5] = {&ctx->b_psi, &ctx->b_slab, &ctx->b_xr, &ctx->b_tmp, &ctx->b_x};
    const int64_t need[5] = {P.psi_bytes, P.slab_bytes, P.xr_bytes, P.tmp_bytes, P.x_bytes};
    bool grow = false;
    for (int k = 0; k < 5; ++k) grow |= (size_t)need[k] > bufs[k]->n;
    if (grow) {
      for (int k = 0; k < 5; ++k) bufs[k]->release();
      for (int k = 0; k < 5; ++k) HIPCHK(bufs[k]->ensure((size_t)need[k], nullptr));
    }
  }
  const int ec = elem_c(prec);
  const int dbl = prec == P_FP64 ? 1 : 0;
  const int sh = ec == 16 ? 3 : 4;           // W~ slab columns in groups of 128 bytes
  std::vector<int64_t> st_off(n_items), sum_off(n_items);
  int64_t st_bytes = 0, sum_n = 0;
  for (int t = 0; t < n_items; ++t) {
    st_off[t] = st_bytes;
    st_bytes += round_up((int64_t)items[t].n_states * P.items[t].n_r_pad * ec, 256);
    sum_off[t] = sum_n;
    sum_n += (int64_t)items[t].n_states * items[t].n_tau * 2;
  }
  HIPCHK(ctx->b_sstates.ensure((size_t)st_bytes + 256, nullptr));
  HIPCHK(ctx->b_ssum.ensure((size_t)sum_n * 8 + 64, nullptr));
  int max_slabs = 0;
  for (auto &I : P.items) max_slabs = std::max<int>(max_slabs, (int)((I.n_r + P.slab_w - 1) / P.slab_w));
  const int n_passes = (int)P.pass_begin.size() - 1;
  HIPCHK(ctx->b_ctr.ensure(((size_t)n_passes * max_slabs + 16) * kGemmQueues * 4, nullptr));
  char *psi_base = reinterpret_cast<char *>(ctx->b_psi.p);
  char *slab_base = reinterpret_cast<char *>(ctx->b_slab.p);
  char *xr_base = reinterpret_cast<char *>(ctx->b_xr.p);
  char *tmp_base = reinterpret_cast<char *>(ctx->b_tmp.p);
  char *x_base = reinterpret_cast<char *>(ctx->b_x.p);
  char *sst_base = reinterpret_cast<char *>(ctx->b_sstates.p);
  double *ssum = reinterpret_cast<double *>(ctx->b_ssum.p);
  int32_t *ctr = reinterpret_cast<int32_t *>(ctx->b_ctr.p);

  Blob blob;
  std::vector<SLaunch> L;
  // per-item tables
  std::vector<size_t> off_perm_o(n_items), off_perm_u(n_items), off_eps_o(n_items),
      off_eps_u(n_items), off_states(n_items), off_ct(n_items), off_st(n_items),
      off_eo(n_items), off_eu(n_items);
  std::vector<Geo> geos(n_items);
  int lds = 0;
  for (int t = 0; t < n_items; ++t) {
    const ItemPlan &I = P.items[t];
    const gwchi_sigma_item &it = items[t];
    off_perm_o[t] = blob.addv(I.perm_o);
    off_perm_u[t] = blob.addv(I.perm_u);
    off_eps_o[t] = blob.addv(I.eps_o);
    off_eps_u[t] = blob.addv(I.eps_u);
    off_states[t] = blob.add(it.states, (size_t)it.n_states * 4);
    off_ct[t] = blob.add(it.ct, (size_t)it.n_omega * it.n_tau * 8);
    off_st[t] = blob.add(it.st, (size_t)it.n_omega * it.n_tau * 8);
    std::vector<double> eo(it.n_tau), eu(it.n_tau);
    for (int j = 0; j < it.n_tau; ++j) {
      eo[j] = std::exp((I.homo - it.mu) * it.tau[j]);     // occupied edge factor at -tau
      eu[j] = std::exp(-(I.lumo - it.mu) * it.tau[j]);    // unoccupied edge factor at +tau
    }
    off_eo[t] = blob.addv(eo);
    off_eu[t] = blob.addv(eu);
    Geo g{};
    g.n0 = I.n0;
    g.n1 = I.n1;
    g.n2 = I.n2;
    g.n_r = (int32_t)I.n_r;
    g.n_g = I.n_g;
    g.n_disk = I.n_disk;
    g.cols = fft_cols(I.n1, I.n2, ec);
    g.planes = fft_planes(I.n0, I.n1, I.n2, ec);
    g.disk_i12 = reinterpret_cast<const int32_t *>(blob.addv(I.disk_i12));
    g.slot_of = reinterpret_cast<const int32_t *>(blob.addv(I.slot_of));
    g.disk_of = reinterpret_cast<const int32_t *>(blob.addv(I.disk_of));
    geos[t] = g;
    lds = std::max(lds, fft_lds_bytes(I.n1, I.n2, g.cols, g.planes, ec) + 4 * I.n_disk);
  }
  const size_t off_geos = blob.addv(geos);
  // ticket counters start at zero (fill kernel), then the states operands
  {
    SLaunch Z;
    Z.phase = SP_STAGE;
    Z.kind = 5;
    Z.fill_ptr = ctr;
    Z.fill_bytes = ((int64_t)n_passes * max_slabs + 16) * kGemmQueues * 4;
    L.push_back(Z);
  }
  for (int t = 0; t < n_items; ++t) {
    SLaunch S;
    S.phase = SP_STAGE;
    S.kind = 6;
    S.phi_o = items[t].phi_occ;
    S.phi_u = items[t].phi_unocc;
    S.states = reinterpret_cast<const int32_t *>(off_states[t]);
    S.n_states = items[t].n_states;
    S.n_occ = items[t].n_occ;
    S.n_r = (int)P.items[t].n_r;
    S.n_r_pad = (int)P.items[t].n_r_pad;
    S.out = sst_base + st_off[t];
    L.push_back(S);
  }
  const int per_cu = std::max(1, gemm_sigma_per_cu(prec));
  const int group = std::max(1, per_cu * ctx->num_cu / kGemmQueues);
  int gc_want = 1;
  while (gc_want * gc_want < group) gc_want *= 2;
  double mfma = 0.0;
  int n_gemm = 0;
  std::vector<int> job_slots(P.jobs.size(), 0);
  for (int ps = 0; ps < n_passes; ++ps) {
    const int jb = P.pass_begin[ps], je = P.pass_begin[ps + 1];
    {
      SLaunch S;
      S.phase = SP_STAGE;
      S.kind = 0;
      S.stage = make_stage(blob, P, jb, je, psi_base, off_perm_o, off_perm_u, off_eps_o, off_eps_u);
      L.push_back(S);
    }
    // W~(G, G') -> W~(G, r'): element (slot G', column G) = conj(W~(G', G)) by
    // Hermiticity, so consecutive columns are consecutive in memory
    {
      std::vector<SfftJob> fj;
      for (int q = jb; q < je; ++q) {
        const JobPlan &J = P.jobs[q];
        const ItemPlan &I = P.items[J.item];
        SfftJob f{};
        f.in = items[J.item].w_tau + (int64_t)J.j * I.n_g * I.n_g * 2;
        f.i_slot = I.n_g;
        f.i_col = 1;
        f.tmp = tmp_base + J.o_tmp;
        f.out = xr_base + J.o_xr;
        f.o_col = I.n_r;
        f.o_shift = -1;
        f.col0 = 0;
        f.n_cols = I.n_g;
        f.geo = J.item;
        fj.push_back(f);
      }
      SLaunch S;
      S.phase = SP_FFT;
      S.kind = 7;
      S.sign = -1;
      S.cubic = sfft_units(fj, geos, S.sfft);
      S.sfft.jobs = reinterpret_cast<const SfftJob *>(blob.addv(fj));
      S.sfft.n_jobs = (int)fj.size();
      S.sfft.geos = reinterpret_cast<const Geo *>(off_geos);
      S.sfft.in_f64 = 1;
      S.sfft.conj_in = 1;
      L.push_back(S);
    }
    std::vector<int> order;
    for (int q = jb; q < je; ++q) order.push_back(q);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
      return P.jobs[a].k_o_eff + P.jobs[a].k_u_eff > P.jobs[b].k_o_eff + P.jobs[b].k_u_eff;
    });
    for (int s = 0; s < max_slabs; ++s) {
      std::vector<SfftJob> fj;
      std::vector<GemmJob> gj;
      std::vector<std::vector<int4>> qunits(kGemmQueues);
      std::vector<double> qwork(kGemmQueues, 0.0);
      for (int q : order) {
        const JobPlan &J = P.jobs[q];
        const ItemPlan &I = P.items[J.item];
        const int64_t s0 = (int64_t)s * P.slab_w;
        if (s0 >= I.n_r) continue;
        const int w = (int)std::min<int64_t>(P.slab_w, I.n_r - s0);
        // W~(G, r') -> W~(r, r' in slab), columns grouped by 128 bytes
        SfftJob f{};
        f.in = xr_base + J.o_xr;
        f.i_slot = I.n_r;
        f.i_col = 1;
        f.tmp = tmp_base + J.o_tmp;
        f.out = slab_base + J.o_slab;
        f.o_col = 0;
        f.o_shift = sh;
        f.col0 = (int32_t)s0;
        f.n_cols = w;
        f.geo = J.item;
        fj.push_back(f);
        char *slot = psi_base + J.o_psi;
        GemmJob g{};
        g.psi_o = slot;
        g.psi_u = slot + I.n_r_pad * I.k_o_pad * bpb_of(prec, 1);
        g.ld_o = I.k_o_pad;
        g.ld_u = I.k_u_pad;
        g.k_o = J.k_o_eff;
        g.k_u = J.k_u_eff;
        g.n_r = (int32_t)I.n_r;
        g.s0 = (int32_t)s0;
        g.w = w;
        g.cg_shift = sh;
        g.slab = slab_base + J.o_slab;
        g.states = sst_base + st_off[J.item];
        g.n_states = items[J.item].n_states;
        g.ld_states = (int32_t)I.n_r_pad;
        g.part = reinterpret_cast<double *>(x_base + J.o_x);
        const int gi = (int)gj.size();
        gj.push_back(g);
        const int nrt = (int)((I.n_r + P.bm - 1) / P.bm);
        const int nct = (w + P.bn - 1) / P.bn;
        const int gc = std::min(nct, gc_want);
        const int gr = std::max(1, (group + gc - 1) / gc);
        const double kk = (double)(J.k_o_eff + J.k_u_eff);
        for (int cb = 0; cb < nct; cb += gc)
          for (int rb = 0; rb < nrt; rb += gr) {
            std::vector<int4> tiles;
            for (int rt = rb; rt < std::min(nrt, rb + gr); ++rt)
              for (int ct = cb; ct < std::min(nct, cb + gc); ++ct) {
                const int r0 = rt * P.bm, c0 = (int)s0 + ct * P.bn;
                if (r0 + P.bm <= c0) continue;          // lower triangle only
                tiles.push_back(make_int4(gi, r0, c0, job_slots[q]++));
              }
            if (tiles.empty()) continue;
            const int qq = (int)(std::min_element(qwork.begin(), qwork.end()) - qwork.begin());
            qunits[qq].insert(qunits[qq].end(), tiles.begin(), tiles.end());
            qwork[qq] += kk * (double)tiles.size();
            // FP64: three real products per band in the unoccupied pass
            mfma += (prec == P_FP64 ? 8.0 * J.k_o_eff + 6.0 * J.k_u_eff : 8.0 * kk) * P.bm * P.bn *
                    (prec == P_BF16X3 ? 3.0 : 1.0) * (double)tiles.size();
          }
      }
      if (gj.empty()) continue;
      {
        SLaunch S;
        S.phase = SP_FFT;
        S.kind = 7;
        S.sign = +1;
        S.cubic = sfft_units(fj, geos, S.sfft);
        S.sfft.jobs = reinterpret_cast<const SfftJob *>(blob.addv(fj));
        S.sfft.n_jobs = (int)fj.size();
        S.sfft.geos = reinterpret_cast<const Geo *>(off_geos);
        S.sfft.in_f64 = dbl;
        S.sfft.conj_in = 0;
        S.sfft.lower_only = 1;          // the GEMM reads rows r >= r' only
        L.push_back(S);
      }
      SLaunch G;
      G.phase = SP_GEMM;
      G.kind = 8;
      G.gemm.jobs = reinterpret_cast<const GemmJob *>(blob.addv(gj));
      std::vector<int4> units;
      G.gemm.n_queues = kGemmQueues;
      for (int q = 0; q < kGemmQueues; ++q) {
        G.gemm.q_off[q] = (int32_t)units.size();
        units.insert(units.end(), qunits[q].begin(), qunits[q].end());
      }
      G.gemm.q_off[kGemmQueues] = (int32_t)units.size();
      G.gemm.units = reinterpret_cast<const int4 *>(blob.addv(units));
      G.gemm.n_units = (int)units.size();
      G.gemm.hermitian = 1;
      G.gemm.counter = ctr + n_gemm * kGemmQueues;
      ++n_gemm;
      L.push_back(G);
    }
    // sums over the tiles of every job of the pass
    {
      std::vector<SigmaRed> red;
      for (int q = jb; q < je; ++q) {
        const JobPlan &J = P.jobs[q];
        SigmaRed r{};
        r.part = reinterpret_cast<const double *>(x_base + J.o_x);
        r.n_slots = job_slots[q];
        r.n_states = items[J.item].n_states;
        r.sum = ssum + sum_off[J.item] + (int64_t)J.j * 2;
        r.sum_stride = items[J.item].n_tau * 2;
        red.push_back(r);
      }
      SLaunch R;
      R.phase = SP_FINAL;
      R.kind = 9;
      R.red = reinterpret_cast<const SigmaRed *>(blob.addv(red));
      R.n = (int)red.size();
      R.max_states = max_states;
      L.push_back(R);
    }
  }
  {
    std::vector<SigmaFin> fin;
    for (int t = 0; t < n_items; ++t) {
      SigmaFin f{};
      f.sum = ssum + sum_off[t];
      f.ct = reinterpret_cast<const double *>(off_ct[t]);
      f.st = reinterpret_cast<const double *>(off_st[t]);
      f.edge_o = reinterpret_cast<const double *>(off_eo[t]);
      f.edge_u = reinterpret_cast<const double *>(off_eu[t]);
      f.n_states = items[t].n_states;
      f.n_tau = items[t].n_tau;
      f.n_omega = items[t].n_omega;
      f.out = items[t].sigma_out;
      f.out_tau = items[t].sigma_tau_out;
      fin.push_back(f);
    }
    SLaunch F;
    F.phase = SP_FINAL;
    F.kind = 10;
    F.fin = reinterpret_cast<const SigmaFin *>(blob.addv(fin));
    F.n = n_items;
    F.max_states = max_states;
    F.max_omega = max_omega;
    L.push_back(F);
  }
  // device tables: allocate, patch the blob offsets, upload
  bool moved = false;
  HIPCHK(ctx->b_tables.ensure(blob.h.size() + 64, &moved));
  const char *base = reinterpret_cast<const char *>(ctx->b_tables.p);
  char *h = blob.h.data();
  patch_geos(blob, base, off_geos, n_items);
  for (auto &S : L) {
    if (S.kind == 0) {
      patch_stage(S.stage, h, base);
    } else if (S.kind == 6) {
      S.states = dev(base, S.states);
    } else if (S.kind == 7) {
      S.sfft.jobs = dev(base, S.sfft.jobs);
      S.sfft.geos = dev(base, S.sfft.geos);
    } else if (S.kind == 8) {
      S.gemm.jobs = dev(base, S.gemm.jobs);
      S.gemm.units = dev(base, S.gemm.units);
    } else if (S.kind == 9) {
      S.red = dev(base, S.red);
    } else if (S.kind == 10) {
      SigmaFin *f = reinterpret_cast<SigmaFin *>(h + reinterpret_cast<uintptr_t>(S.fin));
      for (int t = 0; t < S.n; ++t) {
        f[t].ct = dev(base, f[t].ct);
        f[t].st = dev(base, f[t].st);
        f[t].edge_o = dev(base, f[t].edge_o);
        f[t].edge_u = dev(base, f[t].edge_u);
      }
      S.fin = dev(base, S.fin);
    }
  }
  HIPCHK(ctx->h_tables.ensure(blob.h.size() + 64));
  std::memcpy(ctx->h_tables.p, blob.h.data(), blob.h.size());
  HIPCHK(hipMemcpyAsync(ctx->b_tables.p, ctx->h_tables.p, blob.h.size(), hipMemcpyHostToDevice,
                        ctx->stream));
  // launches, each phase bracketed by events when a report is wanted
  hipStream_t sm = ctx->stream;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> evs;
  size_t ev_i = 0;
  auto ev = [&]() -> hipEvent_t {
    if (ev_i >= ctx->ev_pool.size()) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
      ctx->ev_pool.push_back(e);
    }
    return ctx->ev_pool[ev_i++];
  };
  for (auto &S : L) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (rep) {
      e0 = ev();
      e1 = ev();
      if (!e0 || !e1) {
        set_err(ctx, "hipEventCreate failed");
        return GWCHI_EDEVICE;
      }
      HIPCHK(hipEventRecord(e0, sm));
    }
    switch (S.kind) {
      case 0: HIPCHK(launch_stage(S.stage, prec, sm)); break;
      case 5: HIPCHK(launch_fill_zero(S.fill_ptr, S.fill_bytes, sm)); break;
      case 6:
        HIPCHK(launch_sigma_states(S.phi_o, S.phi_u, S.states, S.n_states, S.n_occ, S.n_r,
                                   S.n_r_pad, dbl, S.out, sm));
        break;
      case 7: HIPCHK(launch_sfft(S.sfft, dbl, S.sign, lds, S.cubic, sm)); break;
      case 8: HIPCHK(launch_gemm_sigma(S.gemm, prec, 0, ctx->num_cu, sm)); break;
      case 9: HIPCHK(launch_sigma_reduce(S.red, S.n, S.max_states, sm)); break;
      case 10: HIPCHK(launch_sigma_final(S.fin, S.n, S.max_states, S.max_omega, sm)); break;
    }
    if (rep) {
      HIPCHK(hipEventRecord(e1, sm));
      evs.push_back({S.phase, {e0, e1}});
    }
  }
  if (rep) {
    HIPCHK(hipStreamSynchronize(sm));
    gwchi_sigma_report r{};
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, evs.front().second.first, evs.back().second.second));
    r.ms_total = ms;
    double ph[SP_COUNT] = {0};
    for (auto &e : evs) {
      float m = 0.f;
      HIPCHK(hipEventElapsedTime(&m, e.second.first, e.second.second));
      ph[e.first] += m;
    }
    r.ms_stage = ph[SP_STAGE];
    r.ms_fft = ph[SP_FFT];
    r.ms_gemm = ph[SP_GEMM];
    r.ms_final = ph[SP_FINAL];
    r.n_gemm_launches = n_gemm;
    r.slab_width = P.slab_w;
    r.tau_batch = P.max_jobs_pass;
    r.alg_flops = P.alg_flops;
    r.mfma_flops = mfma;
    *rep = r;
  }
  return GWCHI_OK;
}

// ---------------------------------------------------------------------------
// Analytic continuation (Sec. II.E.1).
// ---------------------------------------------------------------------------

gwchi_status validate_pade(gwchi_ctx *ctx, const gwchi_pade_item *it) {
  if (!it || !it->z || !it->f || (it->n_eval > 0 && (!it->w || !it->out))) {
    set_err(ctx, "pade: item, z, f (and w, out when n_eval > 0) must not be NULL");
    return GWCHI_EINVAL;
  }
  if (it->n_points < 1 || it->n_points > kPadeMaxPoints || it->n_fun < 1 || it->n_eval < 0) {
    set_err(ctx, "pade: n_points must be in [1, " + std::to_string(kPadeMaxPoints) +
                     "], n_fun >= 1, n_eval >= 0");
    return GWCHI_EINVAL;
  }
  if (!finite_all(it->z, 2 * (int64_t)it->n_points) ||
      (it->n_eval > 0 && !finite_all(it->w, 2 * (int64_t)it->n_eval))) {
    set_err(ctx, "pade: z and w must be finite");
    return GWCHI_EINVAL;
  }
  for (int a = 0; a < it->n_points; ++a)
    for (int b = a + 1; b < it->n_points; ++b)
      if (it->z[2 * a] == it->z[2 * b] && it->z[2 * a + 1] == it->z[2 * b + 1]) {
        set_err(ctx, "pade: the points z must be distinct");
        return GWCHI_EINVAL;
      }
  return GWCHI_OK;
}

// Enqueue the continuation of an item whose f, out and coef are device
// pointers on the context's stream; with ms, wait and time it.
gwchi_status run_pade(gwchi_ctx *ctx, const gwchi_pade_item *it, double *ms) {
  hipStream_t st = ctx->stream;
  const int64_t nz = it->n_points, nw = it->n_eval;
  const int64_t tab = 2 * (nz + nw);
  HIPCHK(ctx->b_ptab.ensure(tab * 8, nullptr));
  HIPCHK(hipStreamSynchronize(st));      // the pinned staging may feed an earlier copy
  HIPCHK(ctx->h_ptab.ensure(tab * 8));
  double *h = reinterpret_cast<double *>(ctx->h_ptab.p);
  std::memcpy(h, it->z, nz * 16);
  if (nw > 0) std::memcpy(h + 2 * nz, it->w, nw * 16);
  HIPCHK(hipMemcpyAsync(ctx->b_ptab.p, h, tab * 8, hipMemcpyHostToDevice, st));
  const double *zd = reinterpret_cast<const double *>(ctx->b_ptab.p);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (ms) {
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    HIPCHK(hipEventRecord(e0, st));
  }
  hipError_t e = launch_pade(it->f, it->n_fun, it->n_points, zd, zd + 2 * nz, it->n_eval,
                             it->coef, it->out, st);
  if (e != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    set_err(ctx, std::string("pade launch: ") + hipGetErrorString(e));
    return GWCHI_EDEVICE;
  }
  if (ms) {
    float t = 0.f;
    e = hipEventRecord(e1, st);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess) {
      set_err(ctx, std::string("pade: ") + hipGetErrorString(e));
      return GWCHI_EDEVICE;
    }
    *ms = t;
  }
  return GWCHI_OK;
}

}  // namespace

// ============================================================================
// C ABI
// ============================================================================
extern "C" {

const char *gwchi_version(void) { return "gwchi 0.1.0 (gfx950)"; }

const char *gwchi_last_error(const gwchi_ctx *ctx) {
  return ctx ? ctx->err.c_str() : g_tls_error.c_str();
}

gwchi_status gwchi_validate(const gwchi_item *items, int32_t n_items, int32_t check_orbitals) {
  try {
    return validate_items(nullptr, items, n_items, check_orbitals != 0);
  } catch (...) {
    g_tls_error = "internal error in validation";
    return GWCHI_EINVAL;
  }
}

gwchi_status gwchi_create(gwchi_ctx **out, int32_t device_id, const char *tune_cache_path) {
  if (!out) {
    g_tls_error = "ctx is NULL";
    return GWCHI_EINVAL;
  }
  *out = nullptr;
  try {
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) {
      g_tls_error = "no HIP device";
      return GWCHI_EDEVICE;
    }
    if (device_id < 0 || device_id >= n) {
      g_tls_error = "device_id out of range";
      return GWCHI_EINVAL;
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device_id) != hipSuccess) {
      g_tls_error = "hipGetDeviceProperties failed";
      return GWCHI_EDEVICE;
    }
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
      g_tls_error = std::string("device is ") + prop.gcnArchName + ", libgwchi is compiled for gfx950 only";
      return GWCHI_EDEVICE;
    }
    std::unique_ptr<gwchi_ctx> ctx(new gwchi_ctx());
    ctx->device = device_id;
    ctx->arch = std::string(prop.gcnArchName).substr(0, 6);
    ctx->num_cu = prop.multiProcessorCount;
    ctx->lds_max = prop.sharedMemPerBlock;
    if (hipSetDevice(device_id) != hipSuccess ||
        hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&ctx->ev_in, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&ctx->ev_out, hipEventDisableTiming) != hipSuccess) {
      g_tls_error = "stream/event creation failed";
      return GWCHI_EDEVICE;
    }
    // the fixed scratch of the allocation-free entry, with this device current
    ctx->noalloc_scratch = scratch_of_device(device_id, &ctx->noalloc_why);
    ctx->opt.use_graph = 1;
    ctx->opt.hermitian = 1;
    ctx->opt.persistent = 1;
    ctx->opt.kappa = 1;
    if (tune_cache_path) ctx->tune_path = tune_cache_path;
    load_tune(ctx.get());
    *out = ctx.release();
    return GWCHI_OK;
  } catch (...) {
    g_tls_error = "internal error in gwchi_create";
    return GWCHI_EDEVICE;
  }
}

gwchi_status gwchi_destroy(gwchi_ctx *ctx) {
  if (!ctx) return GWCHI_OK;
  (void)hipSetDevice(ctx->device);
  if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
  if (ctx->graph_exec) (void)hipGraphExecDestroy(ctx->graph_exec);
  if (ctx->graph) (void)hipGraphDestroy(ctx->graph);
  for (auto e : ctx->ev_pool) (void)hipEventDestroy(e);
  if (ctx->ev_in) (void)hipEventDestroy(ctx->ev_in);
  if (ctx->ev_out) (void)hipEventDestroy(ctx->ev_out);
  for (DevBuf *b : {&ctx->b_phi, &ctx->b_out, &ctx->b_psi, &ctx->b_slab, &ctx->b_xr, &ctx->b_x,
                    &ctx->b_tmp, &ctx->b_tables, &ctx->b_norm, &ctx->b_ctr, &ctx->b_wchi,
                    &ctx->b_wtau, &ctx->b_womega, &ctx->b_wa, &ctx->b_wdinv, &ctx->b_wrp,
                    &ctx->b_wcp, &ctx->b_wtab, &ctx->b_wflag, &ctx->b_pf, &ctx->b_pout,
                    &ctx->b_pcoef, &ctx->b_ptab, &ctx->b_sstates, &ctx->b_ssum, &ctx->b_sw,
                    &ctx->b_sout, &ctx->b_stau})
    b->release();
  ctx->h_tables.release();
  ctx->h_wtab.release();
  ctx->h_ptab.release();
  ctx->h_norm.release();
  if (ctx->stream) (void)hipStreamDestroy(ctx->stream);
  delete ctx;
  return GWCHI_OK;
}

gwchi_status gwchi_set_options(gwchi_ctx *ctx, const gwchi_options *opt) {
  if (!ctx || !opt) return GWCHI_EINVAL;
  if (opt->slab_width < 0 || opt->tau_batch < 0 || opt->tile_id < 0 || opt->max_device_bytes < 0) {
    set_err(ctx, "negative option value");
    return GWCHI_EINVAL;
  }
  ctx->opt = *opt;
  return GWCHI_OK;
}

gwchi_status gwchi_get_options(const gwchi_ctx *ctx, gwchi_options *opt) {
  if (!ctx || !opt) return GWCHI_EINVAL;
  *opt = ctx->opt;
  return GWCHI_OK;
}

gwchi_status gwchi_chi_build_device(gwchi_ctx *ctx, const gwchi_item *items, int32_t n_items,
                                    gwchi_precision prec, void *hip_stream,
                                    gwchi_report *report) {
  if (!ctx) {
    g_tls_error = "ctx is NULL";
    return GWCHI_EINVAL;
  }
  try {
    if (prec != GWCHI_FP64 && prec != GWCHI_FP32 && prec != GWCHI_BF16X3) {
      set_err(ctx, "unknown precision");
      return GWCHI_EINVAL;
    }
    gwchi_status st = validate_items(ctx, items, n_items, false);
    if (st != GWCHI_OK) return st;
    HIPCHK(hipSetDevice(ctx->device));
    hipStream_t us = reinterpret_cast<hipStream_t>(hip_stream);
    // order after the caller's stream
    HIPCHK(hipEventRecord(ctx->ev_in, us));
    HIPCHK(hipStreamWaitEvent(ctx->stream, ctx->ev_in, 0));
    st = run_build(ctx, items, n_items, (int)prec, report);
    if (st != GWCHI_OK) return st;
    HIPCHK(hipEventRecord(ctx->ev_out, ctx->stream));
    HIPCHK(hipStreamWaitEvent(us, ctx->ev_out, 0));
    return GWCHI_OK;
  } catch (const std::bad_alloc &) {
    set_err(ctx, "host allocation failed");
    return GWCHI_ENOMEM;
  } catch (...) {
    set_err(ctx, "internal error");
    return GWCHI_EDEVICE;
  }
}

gwchi_status gwchi_chi_build_device_noalloc(gwchi_ctx *ctx, const gwchi_item *items,
                                            int32_t n_items, gwchi_precision prec,
                                            void *hip_stream) {
  if (!ctx) {
    g_tls_error = "ctx is NULL";
    return GWCHI_EINVAL;
  }
  try {
    if (prec != GWCHI_FP64 && prec != GWCHI_FP32 && prec != GWCHI_BF16X3) {
      set_err(ctx, "unknown precision");
      return GWCHI_EINVAL;
    }
    gwchi_status st = validate_items(ctx, items, n_items, false);
    if (st != GWCHI_OK) return st;
    if (!ctx->noalloc_scratch) {
      set_err(ctx, "allocation-free build: fixed scratch unavailable (" + ctx->noalloc_why + ")");
      return GWCHI_EDEVICE;
    }
    HIPCHK(hipSetDevice(ctx->device));
    hipStream_t us = reinterpret_cast<hipStream_t>(hip_stream);
    HIPCHK(hipEventRecord(ctx->ev_in, us));
    HIPCHK(hipStreamWaitEvent(ctx->stream, ctx->ev_in, 0));
    st = run_build(ctx, items, n_items, (int)prec, nullptr, true);
    if (st != GWCHI_OK) return st;
    HIPCHK(hipEventRecord(ctx->ev_out, ctx->stream));
    HIPCHK(hipStreamWaitEvent(us, ctx->ev_out, 0));
    return GWCHI_OK;
  } catch (const std::bad_alloc &) {
    set_err(ctx, "host allocation failed");
    return GWCHI_ENOMEM;
  } catch (...) {
    set_err(ctx, "internal error");
    return GWCHI_EDEVICE;
  }
}

gwchi_status gwchi_chi_build(gwchi_ctx *ctx, const gwchi_item *items, int32_t n_items,
                             gwchi_precision prec, gwchi_report *report) {
  if (!ctx) {
    g_tls_error = "ctx is NULL";
    return GWCHI_EINVAL;
  }
  try {
    if (prec != GWCHI_FP64 && prec != GWCHI_FP32 && prec != GWCHI_BF16X3) {
      set_err(ctx, "unknown precision");
      return GWCHI_EINVAL;
    }
    gwchi_status st = validate_items(ctx, items, n_items, true);
    if (st != GWCHI_OK) return st;
    HIPCHK(hipSetDevice(ctx->device));
    std::vector<gwchi_item> dev_items;
    st = upload_items(ctx, items, n_items, dev_items);
    if (st != GWCHI_OK) return st;
    st = run_build(ctx, dev_items.data(), n_items, (int)prec, report);
    if (st != GWCHI_OK) return st;
    HIPCHK(hipStreamSynchronize(ctx->stream));
    for (int t = 0; t < n_items; ++t) {
      const gwchi_item &it = items[t];
      HIPCHK(hipMemcpy(it.chi_out, dev_items[t].chi_out, (size_t)it.n_omega * it.n_g * it.n_g * 16,
                       hipMemcpyDeviceToHost));
    }
    if (ctx->opt.check_output) return check_output(ctx, items, n_items);
    return GWCHI_OK;
  } catch (const std::bad_alloc &) {
    set_err(ctx, "host allocation failed");
    return GWCHI_ENOMEM;
  } catch (...) {
    set_err(ctx, "internal error");
    return GWCHI_EDEVICE;
  }
}

gwchi_status gwchi_autotune(gwchi_ctx *ctx, const gwchi_item *items, int32_t n_items,
                            gwchi_precision prec) {
  if (!ctx) return GWCHI_EINVAL;
  try {
    if (prec != GWCHI_FP64 && prec != GWCHI_FP32 && prec != GWCHI_BF16X3) {
      set_err(ctx, "unknown precision");
      return GWCHI_EINVAL;
    }
    gwchi_status st = validate_items(ctx, items, n_items, true);
    if (st != GWCHI_OK) return st;
    HIPCHK(hipSetDevice(ctx->device));
    std::vector<gwchi_item> dev_items;
    st = upload_items(ctx, items, n_items, dev_items);
    if (st != GWCHI_OK) return st;
    const int cplx = items[0].is_complex;
    const int n = gemm_tile_count((int)prec, cplx);
    const gwchi_options saved = ctx->opt;
    // every tile runs the same eager launch list with per-launch events, so
    // that the band-GEMM time of each tile is measured (a warm-up build, then
    // the timed one)
    std::vector<double> ms(n, 0.0);
    double best = 1e300;
    int best_t = 0;
    for (int t = 0; t < n; ++t) {
      ctx->opt = saved;
      ctx->opt.tile_id = t + 1;
      ctx->opt.use_graph = 0;
      ctx->opt.timing = 1;
      gwchi_report rep;
      for (int rep_i = 0; rep_i < 2; ++rep_i) {
        st = run_build(ctx, dev_items.data(), n_items, (int)prec, &rep);
        if (st != GWCHI_OK) {
          ctx->opt = saved;
          return st;
        }
      }
      ms[t] = rep.ms_gemm;
      if (!(rep.ms_gemm > 0.0)) {
        ctx->opt = saved;
        set_err(ctx, "autotune: tile " + std::to_string(t + 1) + " measured no GEMM time");
        return GWCHI_EDEVICE;
      }
      if (rep.ms_gemm < best) {
        best = rep.ms_gemm;
        best_t = t;
      }
    }
    ctx->opt = saved;
    const std::string key = tune_key(ctx, (int)prec, cplx);
    ctx->tune[key] = best_t;
    ctx->tune_ms[key] = ms;
    save_tune(ctx);
    return GWCHI_OK;
  } catch (...) {
    set_err(ctx, "internal error");
    return GWCHI_EDEVICE;
  }
}

gwchi_status gwchi_autotune_times(const gwchi_ctx *ctx, gwchi_precision prec, int32_t is_complex,
                                  double *ms, int32_t n, int32_t *chosen) {
  if (!ctx || !ms || n < 0) return GWCHI_EINVAL;
  try {
    const std::string key = tune_key(ctx, (int)prec, is_complex ? 1 : 0);
    auto it = ctx->tune_ms.find(key);
    auto ch = ctx->tune.find(key);
    if (it == ctx->tune_ms.end() || ch == ctx->tune.end()) return GWCHI_EINVAL;
    for (int32_t t = 0; t < n; ++t) ms[t] = t < (int32_t)it->second.size() ? it->second[t] : -1.0;
    if (chosen) *chosen = ch->second;
    return GWCHI_OK;
  } catch (...) {
    return GWCHI_EINVAL;
  }
}

gwchi_status gwchi_w_validate(const gwchi_w_item *items, int32_t n_items) {
  try {
    std::vector<std::vector<double>> ict;
    return validate_w_items(nullptr, items, n_items, ict);
  } catch (...) {
    g_tls_error = "internal error";
    return GWCHI_EDEVICE;
  }
}

gwchi_status gwchi_w_build_device(gwchi_ctx *ctx, const gwchi_w_item *items, int32_t n_items,
                                  void *hip_stream, gwchi_w_report *report) {
  if (!ctx) {
    g_tls_error = "ctx is NULL";
    return GWCHI_EINVAL;
  }
  try {
    std::vector<std::vector<double>> ict;
    gwchi_status st = validate_w_items(ctx, items, n_items, ict);
    if (st != GWCHI_OK) return st;
    HIPCHK(hipSetDevice(ctx->device));
    hipStream_t us = reinterpret_cast<hipStream_t>(hip_stream);
    HIPCHK(hipEventRecord(ctx->ev_in, us));
    HIPCHK(hipStreamWaitEvent(ctx->stream, ctx->ev_in, 0));
    st = run_w(ctx, items, n_items, ict, report);
    if (st != GWCHI_OK) return st;
    HIPCHK(hipEventRecord(ctx->ev_out, ctx->stream));
    HIPCHK(hipStreamWaitEvent(us, ctx->ev_out, 0));
    return GWCHI_OK;
  } catch (const std::bad_alloc &) {
    set_err(ctx, "host allocation failed");
    return GWCHI_ENOMEM;
  } catch (...) {
    set_err(ctx, "internal error");
    return GWCHI_EDEVICE;
  }
}

gwchi_status gwchi_w_build(gwchi_ctx *ctx, const gwchi_w_item *items, int32_t n_items,
                           gwchi_w_report *report) {
  if (!ctx) {
    g_tls_error = "ctx is NULL";
    return GWCHI_EINVAL;
  }
  try {
    std::vector<std::vector<double>> ict;
    gwchi_status st = validate_w_items(ctx, items, n_items, ict);
    if (st != GWCHI_OK) return st;
    HIPCHK(hipSetDevice(ctx->device));
    gwchi_w_report total{};
    // one item at a time through the context's device buffers
    for (int t = 0; t < n_items; ++t) {
      const gwchi_w_item &it = items[t];
      const size_t in_b = (size_t)it.n_omega * it.n_g * it.n_g * 16;
      const size_t tau_b = (size_t)it.n_tau * it.n_g * it.n_g * 16;
      HIPCHK(ctx->b_wchi.ensure(in_b, nullptr));
      HIPCHK(ctx->b_wtau.ensure(tau_b, nullptr));
      if (it.w_omega_out) HIPCHK(ctx->b_womega.ensure(in_b, nullptr));
      HIPCHK(hipMemcpy(ctx->b_wchi.p, it.chi, in_b, hipMemcpyHostToDevice));
      gwchi_w_item d = it;
      d.chi = reinterpret_cast<const double *>(ctx->b_wchi.p);
      d.w_tau_out = reinterpret_cast<double *>(ctx->b_wtau.p);
      d.w_omega_out = it.w_omega_out ? reinterpret_cast<double *>(ctx->b_womega.p) : nullptr;
      std::vector<std::vector<double>> one(1, ict[t]);
      gwchi_w_report r{};
      st = run_w(ctx, &d, 1, one, &r);
      if (st != GWCHI_OK) return st;
      HIPCHK(hipMemcpy(it.w_tau_out, d.w_tau_out, tau_b, hipMemcpyDeviceToHost));
      if (it.w_omega_out) HIPCHK(hipMemcpy(it.w_omega_out, d.w_omega_out, in_b, hipMemcpyDeviceToHost));
      total.ms_total += r.ms_total;
      total.ms_eps += r.ms_eps;
      total.ms_invert += r.ms_invert;
      total.ms_final += r.ms_final;
      total.alg_flops += r.alg_flops;
      total.n_launches += r.n_launches;
    }
    if (report) *report = total;
    return GWCHI_OK;
  } catch (const std::bad_alloc &) {
    set_err(ctx, "host allocation failed");
    return GWCHI_ENOMEM;
  } catch (...) {
    set_err(ctx, "internal error");
    return GWCHI_EDEVICE;
  }
}

gwchi_status gwchi_sigma_validate(const gwchi_sigma_item *items, int32_t n_items,
                                  int32_t check_orbitals) {
  try {
    return validate_sigma_items(nullptr, items, n_items, check_orbitals != 0);
  } catch (...) {
    g_tls_error = "internal error in validation";
    return GWCHI_EINVAL;
  }
}

gwchi_status gwchi_sigma_build_device(gwchi_ctx *ctx, const gwchi_sigma_item *items,
                                      int32_t n_items, gwchi_precision prec, void *hip_stream,
                                      gwchi_sigma_report *report) {
  if (!ctx) {
    g_tls_error = "ctx is NULL";
    return GWCHI_EINVAL;
  }
  try {
    if (prec != GWCHI_FP64 && prec != GWCHI_FP32 && prec != GWCHI_BF16X3) {
      set_err(ctx, "unknown precision");
      return GWCHI_EINVAL;
    }
    gwchi_status st = validate_sigma_items(ctx, items, n_items, false);
    if (st != GWCHI_OK) return st;
    HIPCHK(hipSetDevice(ctx->device));
    hipStream_t us = reinterpret_cast<hipStream_t>(hip_stream);
    HIPCHK(hipEventRecord(ctx->ev_in, us));
    HIPCHK(hipStreamWaitEvent(ctx->stream, ctx->ev_in, 0));
    st = run_sigma(ctx, items, n_items, (int)prec, report);
    if (st != GWCHI_OK) return st;
    HIPCHK(hipEventRecord(ctx->ev_out, ctx->stream));
    HIPCHK(hipStreamWaitEvent(us, ctx->ev_out, 0));
    return GWCHI_OK;
  } catch (const std::bad_alloc &) {
    set_err(ctx, "host allocation failed");
    return GWCHI_ENOMEM;
  } catch (...) {
    set_err(ctx, "internal error");
    return GWCHI_EDEVICE;
  }
}

gwchi_status gwchi_sigma_build(gwchi_ctx *ctx, const gwchi_sigma_item *items, int32_t n_items,
                               gwchi_precision prec, gwchi_sigma_report *report) {
  if (!ctx) {
    g_tls_error = "ctx is NULL";
    return GWCHI_EINVAL;
  }
  try {
    if (prec != GWCHI_FP64 && prec != GWCHI_FP32 && prec != GWCHI_BF16X3) {
      set_err(ctx, "unknown precision");
      return GWCHI_EINVAL;
    }
    gwchi_status st = validate_sigma_items(ctx, items, n_items, true);
    if (st != GWCHI_OK) return st;
    HIPCHK(hipSetDevice(ctx->device));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    // device copies: orbitals, W~, outputs, packed per item
    int64_t phi_b = 0, w_b = 0, o_b = 0, ot_b = 0;
    std::vector<int64_t> phi_off(n_items), w_off(n_items), o_off(n_items), ot_off(n_items);
    for (int t = 0; t < n_items; ++t) {
      const gwchi_sigma_item &it = items[t];
      const int64_t n_r = (int64_t)it.n[0] * it.n[1] * it.n[2];
      phi_off[t] = phi_b;
      phi_b += round_up(n_r * 16 * (it.n_occ + it.n_unocc), 256);
      w_off[t] = w_b;
      w_b += round_up((int64_t)it.n_tau * it.n_g * it.n_g * 16, 256);
      o_off[t] = o_b;
      o_b += round_up((int64_t)it.n_states * it.n_omega * 16, 256);
      ot_off[t] = ot_b;
      ot_b += it.sigma_tau_out ? round_up((int64_t)it.n_states * it.n_tau * 16, 256) : 0;
    }
    HIPCHK(ctx->b_phi.ensure((size_t)phi_b, nullptr));
    HIPCHK(ctx->b_sw.ensure((size_t)w_b, nullptr));
    HIPCHK(ctx->b_sout.ensure((size_t)o_b, nullptr));
    HIPCHK(ctx->b_stau.ensure((size_t)ot_b + 256, nullptr));
    std::vector<gwchi_sigma_item> d(items, items + n_items);
    for (int t = 0; t < n_items; ++t) {
      const gwchi_sigma_item &it = items[t];
      const int64_t n_r = (int64_t)it.n[0] * it.n[1] * it.n[2];
      char *pb = reinterpret_cast<char *>(ctx->b_phi.p) + phi_off[t];
      HIPCHK(hipMemcpy(pb, it.phi_occ, n_r * 16 * it.n_occ, hipMemcpyHostToDevice));
      HIPCHK(hipMemcpy(pb + n_r * 16 * it.n_occ, it.phi_unocc, n_r * 16 * it.n_unocc,
                       hipMemcpyHostToDevice));
      char *wb = reinterpret_cast<char *>(ctx->b_sw.p) + w_off[t];
      HIPCHK(hipMemcpy(wb, it.w_tau, (size_t)it.n_tau * it.n_g * it.n_g * 16, hipMemcpyHostToDevice));
      d[t].phi_occ = reinterpret_cast<const double *>(pb);
      d[t].phi_unocc = reinterpret_cast<const double *>(pb + n_r * 16 * it.n_occ);
      d[t].w_tau = reinterpret_cast<const double *>(wb);
      d[t].sigma_out = reinterpret_cast<double *>(reinterpret_cast<char *>(ctx->b_sout.p) + o_off[t]);
      d[t].sigma_tau_out = it.sigma_tau_out
                               ? reinterpret_cast<double *>(reinterpret_cast<char *>(ctx->b_stau.p) + ot_off[t])
                               : nullptr;
    }
    st = run_sigma(ctx, d.data(), n_items, (int)prec, report);
    if (st != GWCHI_OK) return st;
    HIPCHK(hipStreamSynchronize(ctx->stream));
    for (int t = 0; t < n_items; ++t) {
      const gwchi_sigma_item &it = items[t];
      HIPCHK(hipMemcpy(it.sigma_out, d[t].sigma_out, (size_t)it.n_states * it.n_omega * 16,
                       hipMemcpyDeviceToHost));
      if (it.sigma_tau_out)
        HIPCHK(hipMemcpy(it.sigma_tau_out, d[t].sigma_tau_out, (size_t)it.n_states * it.n_tau * 16,
                         hipMemcpyDeviceToHost));
    }
    return GWCHI_OK;
  } catch (const std::bad_alloc &) {
    set_err(ctx, "host allocation failed");
    return GWCHI_ENOMEM;
  } catch (...) {
    set_err(ctx, "internal error");
    return GWCHI_EDEVICE;
  }
}

gwchi_status gwchi_pade_validate(const gwchi_pade_item *item) {
  try {
    return validate_pade(nullptr, item);
  } catch (...) {
    g_tls_error = "internal error";
    return GWCHI_EDEVICE;
  }
}

gwchi_status gwchi_pade_device(gwchi_ctx *ctx, const gwchi_pade_item *item, void *hip_stream,
                               double *ms) {
  if (!ctx) {
    g_tls_error = "ctx is NULL";
    return GWCHI_EINVAL;
  }
  try {
    gwchi_status st = validate_pade(ctx, item);
    if (st != GWCHI_OK) return st;
    HIPCHK(hipSetDevice(ctx->device));
    hipStream_t us = reinterpret_cast<hipStream_t>(hip_stream);
    HIPCHK(hipEventRecord(ctx->ev_in, us));
    HIPCHK(hipStreamWaitEvent(ctx->stream, ctx->ev_in, 0));
    st = run_pade(ctx, item, ms);
    if (st != GWCHI_OK) return st;
    HIPCHK(hipEventRecord(ctx->ev_out, ctx->stream));
    HIPCHK(hipStreamWaitEvent(us, ctx->ev_out, 0));
    return GWCHI_OK;
  } catch (const std::bad_alloc &) {
    set_err(ctx, "host allocation failed");
    return GWCHI_ENOMEM;
  } catch (...) {
    set_err(ctx, "internal error");
    return GWCHI_EDEVICE;
  }
}

gwchi_status gwchi_pade(gwchi_ctx *ctx, const gwchi_pade_item *item, double *ms) {
  if (!ctx) {
    g_tls_error = "ctx is NULL";
    return GWCHI_EINVAL;
  }
  try {
    gwchi_status st = validate_pade(ctx, item);
    if (st != GWCHI_OK) return st;
    HIPCHK(hipSetDevice(ctx->device));
    const size_t fb = (size_t)item->n_fun * item->n_points * 16;
    const size_t ob = (size_t)item->n_fun * item->n_eval * 16;
    HIPCHK(ctx->b_pf.ensure(fb, nullptr));
    if (ob > 0) HIPCHK(ctx->b_pout.ensure(ob, nullptr));
    if (item->coef) HIPCHK(ctx->b_pcoef.ensure(fb, nullptr));
    HIPCHK(hipMemcpy(ctx->b_pf.p, item->f, fb, hipMemcpyHostToDevice));
    gwchi_pade_item d = *item;
    d.f = reinterpret_cast<const double *>(ctx->b_pf.p);
    d.out = ob > 0 ? reinterpret_cast<double *>(ctx->b_pout.p) : nullptr;
    d.coef = item->coef ? reinterpret_cast<double *>(ctx->b_pcoef.p) : nullptr;
    double t = 0.0;
    st = run_pade(ctx, &d, &t);
    if (st != GWCHI_OK) return st;
    if (ob > 0) HIPCHK(hipMemcpy(item->out, d.out, ob, hipMemcpyDeviceToHost));
    if (item->coef) HIPCHK(hipMemcpy(item->coef, d.coef, fb, hipMemcpyDeviceToHost));
    if (ms) *ms = t;
    return GWCHI_OK;
  } catch (const std::bad_alloc &) {
    set_err(ctx, "host allocation failed");
    return GWCHI_ENOMEM;
  } catch (...) {
    set_err(ctx, "internal error");
    return GWCHI_EDEVICE;
  }
}

}  // extern "C"
