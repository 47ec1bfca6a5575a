// mci_api.hip -- host side of libmci: descriptor validation, plan construction (FP64
// channel-matrix inversion on the GPU, transform tables), and the C ABI of mci.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cmath>
#include <complex>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <new>
#include <string>
#include <vector>

#include "mci_2d.h"
#include "mci_fftlines.h"
#include "mci_fused.h"
#include "mci_host_util.h"
#include "mci_internal.h"
#include "mci_plan.h"

using namespace mci;

static thread_local std::string g_last_error;

namespace mci {
mci_status fail(mci_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}
}  // namespace mci

#define HIP_TRY(expr)                                                                    \
  do {                                                                                   \
    hipError_t _e = (expr);                                                              \
    if (_e != hipSuccess) return fail(MCI_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(_e)); \
  } while (0)

// ----------------------------------------------------------------- FFT planning (host)
static bool factor_7smooth(int64_t n, std::vector<int>& radices, int max_radix = 8) {
  radices.clear();
  if (n < 1) return false;
  int64_t m = n;
  while (max_radix >= 8 && m % 8 == 0) { radices.push_back(8); m /= 8; }
  while (max_radix < 8 && m % 4 == 0) { radices.push_back(4); m /= 4; }
  if (m % 4 == 0) { radices.push_back(4); m /= 4; }
  if (m % 2 == 0) { radices.push_back(2); m /= 2; }
  for (int p : {3, 5, 7})
    while (m % p == 0) { radices.push_back(p); m /= p; }
  return m == 1;
}

static int64_t next_7smooth(int64_t n) {
  for (int64_t c = std::max<int64_t>(n, 1);; ++c) {
    int64_t m = c;
    for (int p : {2, 3, 5, 7})
      while (m % p == 0) m /= p;
    if (m == 1) return c;
  }
}

int64_t mci::next_smooth_length(int64_t n) { return next_7smooth(n); }

template <typename C>
static void* upload(const std::vector<std::complex<double>>& v, hipError_t& err) {
  std::vector<C> h(v.size());
  for (size_t i = 0; i < v.size(); ++i) {
    h[i].x = (decltype(C::x))v[i].real();
    h[i].y = (decltype(C::x))v[i].imag();
  }
  void* d = nullptr;
  err = hipMalloc(&d, h.size() * sizeof(C));
  if (err != hipSuccess) return nullptr;
  err = hipMemcpy(d, h.data(), h.size() * sizeof(C), hipMemcpyHostToDevice);
  return d;
}

static void free_side(FftSide& f) {
  if (f.tw) (void)hipFree(f.tw);
  if (f.chirp) (void)hipFree(f.chirp);
  if (f.bhat) (void)hipFree(f.bhat);
  if (f.twA) (void)hipFree(f.twA);
  if (f.twB) (void)hipFree(f.twB);
  if (f.twL) (void)hipFree(f.twL);
  f.tw = f.chirp = f.bhat = f.twA = f.twB = f.twL = nullptr;
}

static mci_status build_side(FftSide& f, int64_t len, int sign, int prec, bool force_blue = false) {
  f.len = len;
  f.sign = sign;
  f.blue = !factor_7smooth(len, f.radices) || force_blue;
  f.lexec = f.blue ? next_7smooth(2 * len - 1) : len;
  if (f.blue && prec == MCI_F32) {
    // a Bluestein length the one- or two-pass LDS transform takes (2^a 3^b, also 7-smooth)
    const int64_t m = next_two_pass_length(2 * len - 1);
    if (m > 0) f.lexec = m;
  }
  factor_7smooth(f.lexec, f.radices8, 8);
  factor_7smooth(f.lexec, f.radices4, 4);
  f.radices = f.radices8;
  std::vector<std::complex<double>> tw(f.lexec);
  for (int64_t k = 0; k < f.lexec; ++k) tw[k] = root_of_unity(k, f.lexec);
  hipError_t e;
  f.tw = prec == MCI_F64 ? upload<double2>(tw, e) : upload<float2>(tw, e);
  if (!f.tw) return fail(MCI_E_OUT_OF_MEMORY, "twiddle table");
  if (e != hipSuccess) return fail(MCI_E_DEVICE, "twiddle upload");
  if (prec == MCI_F32 && two_pass_factors(f.lexec, f.fa, f.fb)) {
    for (int which = 0; which < 2; ++which) {
      const int n = which ? f.fb : f.fa;
      if (n <= 1) continue;
      std::vector<std::complex<double>> t(n);
      for (int k = 0; k < n; ++k) t[k] = root_of_unity(k, n);
      void* d = upload<float2>(t, e);
      if (!d || e != hipSuccess) return fail(MCI_E_DEVICE, "line twiddle upload");
      (which ? f.twB : f.twA) = d;
    }
    {
      std::vector<std::complex<double>> t(fl_twiddle_entries(f.lexec), 0.0);
      for (int64_t j = 0; j < std::min<int64_t>(f.lexec, kTwLo); ++j) t[j] = root_of_unity(j, f.lexec);
      for (int64_t i = 0; kTwLo * i < f.lexec; ++i) t[kTwLo + i] = root_of_unity(kTwLo * i, f.lexec);
      f.twL = upload<float2>(t, e);
      if (!f.twL || e != hipSuccess) return fail(MCI_E_DEVICE, "two-pass twiddle upload");
    }
    if ((e = prepare_two_pass(f.fa, f.fb)) != hipSuccess) return fail(MCI_E_DEVICE, "two-pass LDS attribute");
  } else {
    f.fa = f.fb = 0;
  }
  if (!f.blue) return MCI_OK;
  // chirp c[k] = e^{sign i pi k^2 / len}; k^2 reduced modulo 2 len exactly
  std::vector<std::complex<double>> c(len), b(f.lexec, 0.0);
  for (int64_t k = 0; k < len; ++k) {
    c[k] = chirp_value(k, len, sign);
  }
  for (int64_t m = 0; m < len; ++m) {
    b[m] = std::conj(c[m]);
    if (m) b[f.lexec - m] = std::conj(c[m]);
  }
  host_fft(b, f.radices, -1);
  for (auto& v : b) v /= (double)f.lexec;
  // stored zero-padded to lexec entries, so that a transform's output stage can apply it by position
  c.resize(f.lexec, 0.0);
  f.chirp = prec == MCI_F64 ? upload<double2>(c, e) : upload<float2>(c, e);
  if (!f.chirp || e != hipSuccess) return fail(MCI_E_DEVICE, "chirp upload");
  f.bhat = prec == MCI_F64 ? upload<double2>(b, e) : upload<float2>(b, e);
  if (!f.bhat || e != hipSuccess) return fail(MCI_E_DEVICE, "chirp spectrum upload");
  return MCI_OK;
}

// ----------------------------------------------------------------- validation
static mci_status validate(const mci_plan_desc* d) {
  if (!d) return fail(MCI_E_INVALID_ARG, "desc is NULL");
  if (d->M < 1 || d->M > MCI_MAX_CHANNELS) return fail(MCI_E_INVALID_ARG, "M must be in 1..4");
  if (d->n_ops < 1 || d->n_ops > MCI_MAX_OPS) return fail(MCI_E_INVALID_ARG, "n_ops must be in 1..4");
  if (d->N < 1 || d->N > (int64_t)1 << 26) return fail(MCI_E_INVALID_ARG, "N out of range");
  if (d->n_out < 1 || d->n_out > (int64_t)1 << 28) return fail(MCI_E_INVALID_ARG, "n_out out of range");
  if (d->precision != MCI_F32 && d->precision != MCI_F64) return fail(MCI_E_INVALID_ARG, "precision");
  if (d->storage != MCI_STORE_NATIVE && d->storage != MCI_STORE_F16) return fail(MCI_E_INVALID_ARG, "storage");
  if (d->storage == MCI_STORE_F16 && d->precision != MCI_F32)
    return fail(MCI_E_INVALID_ARG, "F16 storage needs an F32 plan");
  if (d->real_io != 0 && d->real_io != 1) return fail(MCI_E_INVALID_ARG, "real_io must be 0 or 1");
  if (d->flags & ~MCI_ALLOW_SINGULAR_ZERO) return fail(MCI_E_INVALID_ARG, "unknown flag");
  if (!(d->cond_max >= 0.0)) return fail(MCI_E_INVALID_ARG, "cond_max");
  for (int k = 0; k < d->M; ++k) {
    const mci_channel& c = d->ch[k];
    if (c.kind == MCI_MULT_DERIV) {
      if (c.order < 0 || c.order > 8) return fail(MCI_E_INVALID_ARG, "derivative order must be in 0..8");
    } else if (c.kind == MCI_MULT_TABLE) {
      if (!c.table) return fail(MCI_E_INVALID_ARG, "table channel without table");
    } else if (c.kind != MCI_MULT_HILBERT) {
      return fail(MCI_E_INVALID_ARG, "unknown multiplier kind");
    }
  }
  for (int o = 0; o < d->n_ops; ++o) {
    if (d->ops[o] < MCI_OUT_IDENTITY || d->ops[o] > MCI_OUT_DERIV) return fail(MCI_E_INVALID_ARG, "unknown output op");
    if (d->ops[o] == MCI_OUT_DERIV && (d->op_orders[o] < 0 || d->op_orders[o] > 8))
      return fail(MCI_E_INVALID_ARG, "output derivative order must be in 0..8");
  }
  return MCI_OK;
}

static void destroy_plan(mci_plan_s* p) {
  if (!p) return;
  for (int a = 0; a < 2; ++a) {
    if (p->lp_H[a]) (void)hipFree(p->lp_H[a]);
    if (p->lp_tw[a]) (void)hipFree(p->lp_tw[a]);
  }
  if (p->tab) (void)hipFree(p->tab);
  if (p->qdev) (void)hipFree(p->qdev);
  free_side(p->fwd);
  free_side(p->inv);
  free_side(p->rfwd);
  free_side(p->rinv);
  if (p->r_wN) (void)hipFree(p->r_wN);
  if (p->r_D) (void)hipFree(p->r_D);
  fused_release(p->fused);
  destroy_plan(p->rows);
  destroy_plan(p->cols);
  delete p;
}

struct DevBufs {
  std::vector<void*> v;
  ~DevBufs() {
    for (void* p : v)
      if (p) (void)hipFree(p);
  }
  void* alloc(size_t n, hipError_t& e) {
    void* p = nullptr;
    e = hipMalloc(&p, n);
    if (e == hipSuccess) v.push_back(p);
    return e == hipSuccess ? p : nullptr;
  }
};

// Tables of the real-mode multi-kernel path, when the plan qualifies (FP32 arithmetic, FP32 or
// FP16 storage, real mode, even n_out with n_out / 2 a one- or two-pass length).
static mci_status build_real_path(mci_plan_s* p) {
  const mci_plan_desc& d = p->d;
  int fa, fb;
  if (p->prec != MCI_F32 || (p->store != ST_F32 && p->store != ST_F16) || !d.real_io || d.n_out % 2 ||
      !two_pass_factors(d.n_out / 2, fa, fb))
    return MCI_OK;
  // even N: rows read as N/2 complex pairs; odd N: the length-N transform of the real row
  const bool half = d.N % 2 == 0;
  const int64_t N = d.N, H = half ? N / 2 : N, P = d.n_out / 2, mu = p->mu;
  mci_status st;
  if ((st = build_side(p->rfwd, H, -1, MCI_F32)) != MCI_OK) return st;
  if (!p->rfwd.fa) {   // the length neither factors nor needs Bluestein: take Bluestein at a length that factors
    free_side(p->rfwd);
    p->rfwd = FftSide();
    if ((st = build_side(p->rfwd, H, -1, MCI_F32, true)) != MCI_OK) return st;
  }
  if ((st = build_side(p->rinv, P, +1, MCI_F32)) != MCI_OK) return st;
  if (!p->rfwd.fa || !p->rinv.fa || p->rinv.blue) return MCI_OK;
  const int64_t K = std::max<int64_t>(std::llabs(d.n1), std::llabs(d.n1 + mu - 1));
  if (mu > ((int64_t)1 << 29) || K + P > ((int64_t)1 << 30)) return MCI_OK;   // the path's indices are 32-bit
  std::vector<std::complex<double>> wN(H);
  for (int64_t k = 0; k < H; ++k) wN[k] = root_of_unity(k, N);
  // D[op][m][k + K] = (T_k[m] + conj T_-k[m]) / 2 (1 + i e^{2 pi i k / n_out}), T_k[m] the apply
  // table's entry of channel m at band position k (0 outside the band), from the FP64 table:
  // the real part and the polyphase gather of the output folded into the apply's weights
  const int M = d.M;
  const int64_t W2 = 2 * K + 1;
  auto T = [&](int op, int m, int64_t k) -> std::complex<double> {
    const int64_t dd = k - d.n1;
    if (dd < 0 || dd >= mu) return 0.0;
    const int64_t j = dd / N, i = dd % N;
    return p->tab_host[(((size_t)op * M + m) * M + j) * N + i];
  };
  std::vector<std::complex<double>> D((size_t)d.n_ops * M * W2);
  for (int op = 0; op < d.n_ops; ++op)
    for (int m = 0; m < M; ++m)
      for (int64_t k = -K; k <= K; ++k) {
        const std::complex<double> wo = 1.0 + std::complex<double>(0.0, 1.0) * std::conj(root_of_unity(k, d.n_out));
        D[((size_t)op * M + m) * W2 + (k + K)] = 0.5 * (T(op, m, k) + std::conj(T(op, m, -k))) * wo;
      }
  hipError_t e;
  p->r_wN = upload<float2>(wN, e);
  if (!p->r_wN || e != hipSuccess) return fail(MCI_E_DEVICE, "real-path table upload");
  p->r_D = upload<float2>(D, e);
  if (!p->r_D || e != hipSuccess) return fail(MCI_E_DEVICE, "real-path table upload");
  RealPath& r = p->real;
  r.M = d.M; r.n_ops = d.n_ops; r.N = N; r.H = H; r.n1 = d.n1; r.n_out = d.n_out; r.P = P; r.K = K;
  r.half = half;
  r.f16 = p->store == ST_F16;
  r.fwd = &p->rfwd; r.inv = &p->rinv;
  r.wN = (const float2*)p->r_wN; r.D = (const float2*)p->r_D;
  r.ok = true;
  return MCI_OK;
}

mci_status mci::build_plan(const mci_plan_desc* desc, int device, mci_plan_s** out, const std::vector<double>* oscale) {
  mci_status st = validate(desc);
  if (st != MCI_OK) return st;
  int ndev = 0;
  HIP_TRY(hipGetDeviceCount(&ndev));
  if (device < 0 || device >= ndev) return fail(MCI_E_INVALID_ARG, "device index");
  HIP_TRY(hipSetDevice(device));
  mci_plan_s* p = new (std::nothrow) mci_plan_s();
  if (!p) return fail(MCI_E_OUT_OF_MEMORY, "plan");
  p->device = device;
  p->d = *desc;
  for (int k = 0; k < MCI_MAX_CHANNELS; ++k) p->d.ch[k].table = nullptr;
  p->mu = (int64_t)desc->M * desc->N;
  if (p->d.n1 == MCI_N1_DEFAULT) p->d.n1 = -((p->mu - 1) / 2);
  if (p->d.cond_max == 0.0) p->d.cond_max = 1e12;
  p->prec = desc->precision;
  p->store = desc->precision == MCI_F64 ? ST_F64 : (desc->storage == MCI_STORE_F16 ? ST_F16 : ST_F32);

  const int M = desc->M, n_ops = desc->n_ops;
  const int64_t N = desc->N, mu = p->mu;
  DevBufs tmp;
  hipError_t e;
  // channel tables (FP64) on the device
  double2* d_tables = nullptr;
  bool any_table = false;
  for (int k = 0; k < M; ++k) any_table |= desc->ch[k].kind == MCI_MULT_TABLE;
  if (any_table) {
    std::vector<double2> h((size_t)M * mu, make_double2(0.0, 0.0));
    for (int k = 0; k < M; ++k)
      if (desc->ch[k].kind == MCI_MULT_TABLE)
        for (int64_t i = 0; i < mu; ++i) h[(size_t)k * mu + i] = make_double2(desc->ch[k].table[2 * i], desc->ch[k].table[2 * i + 1]);
    d_tables = (double2*)tmp.alloc(h.size() * sizeof(double2), e);
    if (!d_tables) { destroy_plan(p); return fail(MCI_E_OUT_OF_MEMORY, "channel tables"); }
    if ((e = hipMemcpy(d_tables, h.data(), h.size() * sizeof(double2), hipMemcpyHostToDevice)) != hipSuccess) {
      destroy_plan(p);
      return fail(MCI_E_DEVICE, "channel table upload");
    }
  }
  const size_t ntab = (size_t)n_ops * M * M * N;
  double2* tab64 = (double2*)tmp.alloc(ntab * sizeof(double2), e);
  float2* tab32 = (float2*)tmp.alloc(ntab * sizeof(float2), e);
  double* cond = (double*)tmp.alloc((size_t)N * sizeof(double), e);
  int* sing = (int*)tmp.alloc((size_t)N * sizeof(int), e);
  if (!tab64 || !tab32 || !cond || !sing) { destroy_plan(p); return fail(MCI_E_OUT_OF_MEMORY, "plan scratch"); }
  if ((e = hipMalloc(&p->qdev, (size_t)N * M * M * sizeof(double2))) != hipSuccess) {
    p->qdev = nullptr;
    destroy_plan(p);
    return fail(MCI_E_OUT_OF_MEMORY, "inverse table");
  }

  PlanKernelArgs a{};
  a.M = M; a.n_ops = n_ops; a.N = N; a.n1 = p->d.n1;
  for (int k = 0; k < M; ++k) { a.kinds[k] = desc->ch[k].kind; a.orders[k] = desc->ch[k].order; }
  for (int o = 0; o < n_ops; ++o) { a.ops[o] = desc->ops[o]; a.op_orders[o] = desc->op_orders[o]; }
  a.tables = d_tables; a.tab64 = tab64; a.tab32 = tab32; a.cond = cond; a.sing = sing;
  a.qraw = (double2*)p->qdev;
  a.allow_zero = (desc->flags & MCI_ALLOW_SINGULAR_ZERO) ? 1 : 0;
  if (oscale) {
    if ((int64_t)oscale->size() != mu) { destroy_plan(p); return fail(MCI_E_INVALID_ARG, "output scale length"); }
    double* d_os = (double*)tmp.alloc((size_t)mu * sizeof(double), e);
    if (!d_os) { destroy_plan(p); return fail(MCI_E_OUT_OF_MEMORY, "output scale"); }
    if ((e = hipMemcpy(d_os, oscale->data(), (size_t)mu * sizeof(double), hipMemcpyHostToDevice)) != hipSuccess) {
      destroy_plan(p);
      return fail(MCI_E_DEVICE, "output scale upload");
    }
    a.oscale = d_os;
  }
  if ((e = launch_plan_tables(a, 0)) != hipSuccess) { destroy_plan(p); return fail(MCI_E_DEVICE, hipGetErrorString(e)); }
  std::vector<double> hc(N);
  std::vector<int> hs(N);
  if ((e = hipMemcpy(hc.data(), cond, N * sizeof(double), hipMemcpyDeviceToHost)) != hipSuccess ||
      (e = hipMemcpy(hs.data(), sing, N * sizeof(int), hipMemcpyDeviceToHost)) != hipSuccess) {
    destroy_plan(p);
    return fail(MCI_E_DEVICE, std::string("plan readback: ") + hipGetErrorString(e));
  }
  for (int64_t i = 0; i < N; ++i) {
    if (hs[i]) {
      if (!p->n_sing) p->first_sing = p->d.n1 + i;
      ++p->n_sing;
    } else {
      p->max_cond = std::max(p->max_cond, hc[i]);
    }
  }
  if (p->n_sing && !(desc->flags & MCI_ALLOW_SINGULAR_ZERO)) {
    const int64_t bad = p->first_sing;
    destroy_plan(p);
    return fail(MCI_E_SINGULAR, "H_n singular at n = " + std::to_string(bad));
  }
  if (p->max_cond > p->d.cond_max) {
    const double c = p->max_cond;
    destroy_plan(p);
    return fail(MCI_E_ILL_CONDITIONED, "max condition number " + std::to_string(c));
  }
  {
    std::vector<double2> h64(ntab);
    if ((e = hipMemcpy(h64.data(), tab64, ntab * sizeof(double2), hipMemcpyDeviceToHost)) != hipSuccess) {
      destroy_plan(p);
      return fail(MCI_E_DEVICE, "table readback");
    }
    p->tab_host.resize(ntab);
    for (size_t q = 0; q < ntab; ++q) p->tab_host[q] = {h64[q].x, h64[q].y};
  }
  // keep the table in plan precision
  if (p->prec == MCI_F64) {
    if ((e = hipMalloc(&p->tab, ntab * sizeof(double2))) != hipSuccess) { destroy_plan(p); return fail(MCI_E_OUT_OF_MEMORY, "tab"); }
    if ((e = hipMemcpy(p->tab, tab64, ntab * sizeof(double2), hipMemcpyDeviceToDevice)) != hipSuccess) { destroy_plan(p); return fail(MCI_E_DEVICE, "tab copy"); }
  } else {
    if ((e = hipMalloc(&p->tab, ntab * sizeof(float2))) != hipSuccess) { destroy_plan(p); return fail(MCI_E_OUT_OF_MEMORY, "tab"); }
    if ((e = hipMemcpy(p->tab, tab32, ntab * sizeof(float2), hipMemcpyDeviceToDevice)) != hipSuccess) { destroy_plan(p); return fail(MCI_E_DEVICE, "tab copy"); }
  }
  if ((st = build_side(p->fwd, N, -1, p->prec)) != MCI_OK) { destroy_plan(p); return st; }
  if ((st = build_side(p->inv, desc->n_out, +1, p->prec)) != MCI_OK) { destroy_plan(p); return st; }
  if ((st = fused_select(p->d, p->prec, p->store, p->tab, p->fused)) != MCI_OK) { destroy_plan(p); return st; }
  if ((st = build_real_path(p)) != MCI_OK) { destroy_plan(p); return st; }
  HIP_TRY(hipDeviceSynchronize());
  {
    const uint32_t m = plan_variant_mask(p);
    (void)plan_set_variant(p, p->fused.kind                               ? MCI_VARIANT_FUSED_T1
                              : (m >> MCI_VARIANT_REAL_TWO_PASS & 1u) ? MCI_VARIANT_REAL_TWO_PASS
                              : (m >> MCI_VARIANT_TWO_PASS & 1u)      ? MCI_VARIANT_TWO_PASS
                                                                        : MCI_VARIANT_MULTIPASS_R8);
  }
  *out = p;
  return MCI_OK;
}

// variant recorded for this plan's shape in $MCI_TUNE_CACHE, applied when available
static void apply_tune_cache(mci_plan_s* p) {
  const char* path = std::getenv("MCI_TUNE_CACHE");
  if (!path || !*path) return;
  const int v = tune_cache_lookup(path, plan_tune_key(p));
  if (v >= 0 && (plan_variant_mask(p) >> v & 1u)) (void)plan_set_variant(p, v);
}

static Generic1D generic_of(const mci_plan_s* p) {
  Generic1D g;
  g.M = p->d.M; g.n_ops = p->d.n_ops; g.real_io = p->d.real_io;
  g.N = p->d.N; g.n1 = p->d.n1; g.n_out = p->d.n_out;
  g.tab = p->tab; g.fwd = &p->fwd; g.inv = &p->inv;
  return g;
}

static size_t ws_1d(const mci_plan_s* p, int64_t batch) {
  if (batch <= 0) return 0;
  if (p->use_fused) return 0;
  if (p->use_real) return real_path_workspace(p->real, batch);
  return generic_1d_workspace(generic_of(p), p->prec, batch);
}


static size_t ws_2d(const mci_plan_s* p, int64_t batch) {
  if (batch <= 0) return 0;
  if (p->lp) return (size_t)batch * p->d2.scale * p->d2.h * p->d2.w * sizeof(float) + 256;
  const int64_t h = p->d2.h, w = p->d2.w, s = p->d2.scale, M = p->d2.channels;
  const size_t e = p->prec == MCI_F64 ? 8 : 4;
  auto al = [](size_t n) { return (n + 255) & ~(size_t)255; };
  // row channels, mid image, column channels, column result, and the larger 1-D workspace
  size_t rows_in = al((size_t)batch * h * M * w * e);
  size_t mid = al((size_t)batch * h * s * w * e);
  size_t cols_in = al((size_t)batch * s * w * M * h * e);
  size_t cols_out = al((size_t)batch * s * w * s * h * e);
  size_t w1 = std::max(ws_1d(p->rows, batch * h), ws_1d(p->cols, batch * s * w));
  return rows_in + mid + cols_in + cols_out + al(w1) + 256;
}

// ================================================================= internal entry points
namespace mci {

int store_bytes(int store) { return store == ST_F64 ? 8 : (store == ST_F16 ? 2 : 4); }

int64_t instance_in_elems(const mci_plan_s* p) {
  if (p->dims == 2) return (int64_t)p->d2.h * p->d2.w;
  return p->mu * (p->d.real_io ? 1 : 2);
}

int64_t instance_out_elems(const mci_plan_s* p) {
  if (p->dims == 2) return (int64_t)p->d2.scale * p->d2.h * p->d2.scale * p->d2.w;
  return (int64_t)p->d.n_ops * p->d.n_out * (p->d.real_io ? 1 : 2);
}

size_t plan_workspace(const mci_plan_s* p, int64_t batch) { return p->dims == 2 ? ws_2d(p, batch) : ws_1d(p, batch); }

static mci_status run_2d(const mci_plan_s* p, const void* lr, void* hr, int64_t batch, void* workspace,
                         const int64_t* offs, hipStream_t stream) {
  if (p->lp) {
    // columns first: lr [B][h][w] -> mid [B][s h][w]; then rows: mid -> hr [B][s h][s w].  (Images
    // in chunks small enough for mid to be read back from the memory-side cache measured slower:
    // x2 0.134 -> 0.144 ms at 64 MiB chunks, 0.27 ms at 16 MiB.)
    const int64_t h = p->d2.h, w = p->d2.w, sc = p->d2.scale;
    float* mid = (float*)(((uintptr_t)workspace + 255) & ~(uintptr_t)255);
    // with the sample rows passed through, mid holds only the rows s q + r, r >= 1
    const bool zr = p->lp_zr;
    const int64_t mid_rows = zr ? (sc - 1) * h : sc * h;
    const int64_t max_y = 65535;   // images per column-pass launch (grid y)
    for (int64_t b0 = 0; b0 < batch; b0 += max_y) {
      const int64_t nb = std::min(max_y, batch - b0);
      const char* x0 = offs ? (const char*)lr : (const char*)lr + b0 * h * w * store_bytes(p->store);
      LinePassArgs ac{x0, mid + b0 * mid_rows * w, 0, w, (const float2*)p->lp_H[0], (const float2*)p->lp_tw[0],
                      offs ? offs + 2 * b0 : nullptr, 1};
      hipError_t err = run_line_pass((int)h, (int)sc, true, zr, p->store, ST_F32, ac, nb, stream);
      if (err != hipSuccess) return fail(MCI_E_DEVICE, std::string("column pass: ") + hipGetErrorString(err));
    }
    LinePassArgs ar{mid, hr, batch * sc * h, 0, (const float2*)p->lp_H[1], (const float2*)p->lp_tw[1], offs, sc * h};
    if (zr) ar.x0 = lr;
    hipError_t err = run_line_pass((int)w, (int)sc, false, zr, ST_F32, p->store, ar, 0, stream);
    if (err != hipSuccess) return fail(MCI_E_DEVICE, std::string("row pass: ") + hipGetErrorString(err));
    return MCI_OK;
  }
  const int64_t h = p->d2.h, w = p->d2.w, s = p->d2.scale, H = s * h, W = s * w;
  const int M = p->d2.channels;
  const size_t e = p->prec == MCI_F64 ? 8 : 4;
  auto al = [](size_t n) { return (n + 255) & ~(size_t)255; };
  char* base = (char*)(((uintptr_t)workspace + 255) & ~(uintptr_t)255);
  char* rows_in = base;
  char* mid = rows_in + al((size_t)batch * h * M * w * e);
  char* cols_in = mid + al((size_t)batch * h * W * e);
  char* cols_out = cols_in + al((size_t)batch * W * M * h * e);
  char* w1 = cols_out + al((size_t)batch * W * H * e);
  hipError_t err;
  if ((err = launch_fd_channels(p->prec, p->store, lr, rows_in, batch, h, w, 0, offs, M, stream)) != hipSuccess)
    return fail(MCI_E_DEVICE, hipGetErrorString(err));
  mci_status st = plan_run(p->rows, rows_in, mid, batch * h, w1, nullptr, stream);
  if (st != MCI_OK) return st;
  if ((err = launch_fd_channels(p->prec, p->prec == MCI_F64 ? ST_F64 : ST_F32, mid, cols_in, batch, h, W, 1, nullptr, M,
                                stream)) != hipSuccess)
    return fail(MCI_E_DEVICE, hipGetErrorString(err));
  if ((st = plan_run(p->cols, cols_in, cols_out, batch * W, w1, nullptr, stream)) != MCI_OK) return st;
  if ((err = launch_transpose_out(p->prec, p->store, cols_out, hr, batch, W, H, offs, stream)) != hipSuccess)
    return fail(MCI_E_DEVICE, hipGetErrorString(err));
  return MCI_OK;
}

mci_status plan_run(const mci_plan_s* p, const void* in, void* out, int64_t batch, void* ws, const int64_t* offs,
                    hipStream_t s) {
  if (batch <= 0) return MCI_OK;
  if (p->dims == 2) return run_2d(p, in, out, batch, ws, offs, s);
  hipError_t e;
  if (p->use_fused) e = fused_run(p->fused, in, out, batch, offs, s);
  else if (p->use_real) e = run_real_1d(p->real, in, out, batch, ws, offs, s);
  else e = run_generic_1d(generic_of(p), p->prec, p->store, in, out, batch, ws, offs, s);
  if (e != hipSuccess) return fail(MCI_E_DEVICE, std::string("reconstruct: ") + hipGetErrorString(e));
  return MCI_OK;
}

uint32_t plan_variant_mask(const mci_plan_s* p) {
  uint32_t m = 1u << MCI_VARIANT_MULTIPASS_R8;
  if (p->dims == 2) {
    if (p->lp_avail) m |= 1u << MCI_VARIANT_LINE_PASS;
    return m;
  }
  m |= 1u << MCI_VARIANT_MULTIPASS_R4;
  if (p->fwd.fa || p->inv.fa) m |= 1u << MCI_VARIANT_TWO_PASS;
  if (p->real.ok) m |= 1u << MCI_VARIANT_REAL_TWO_PASS;
  if (p->fused.kind) {
    m |= 1u << MCI_VARIANT_FUSED_T1;
    if (p->fused.n_ti == 2) m |= 1u << MCI_VARIANT_FUSED_T2;
  }
  return m;
}

mci_status plan_set_variant(mci_plan_s* p, int v) {
  if (v < 0 || v >= MCI_NUM_VARIANTS || !(plan_variant_mask(p) >> v & 1u))
    return fail(MCI_E_UNSUPPORTED, "variant " + std::to_string(v) + " is not available for this plan");
  if (p->dims == 2) {
    p->lp = v == MCI_VARIANT_LINE_PASS;
  } else if (v == MCI_VARIANT_REAL_TWO_PASS) {
    p->use_fused = false;
    p->use_real = true;
  } else if (v == MCI_VARIANT_FUSED_T1 || v == MCI_VARIANT_FUSED_T2) {
    p->use_fused = true;
    p->use_real = false;
    fused_set_ti(p->fused, v == MCI_VARIANT_FUSED_T2 ? 2 : 1);
  } else {
    p->use_fused = false;
    p->use_real = false;
    const bool r4 = v == MCI_VARIANT_MULTIPASS_R4;
    p->fwd.radices = r4 ? p->fwd.radices4 : p->fwd.radices8;
    p->inv.radices = r4 ? p->inv.radices4 : p->inv.radices8;
    p->fwd.two_pass = v == MCI_VARIANT_TWO_PASS && p->fwd.fa;
    p->inv.two_pass = v == MCI_VARIANT_TWO_PASS && p->inv.fa;
  }
  p->variant = v;
  return MCI_OK;
}

}  // namespace mci

// ================================================================= C ABI
extern "C" {

const char* mci_status_string(mci_status s) {
  switch (s) {
    case MCI_OK: return "MCI_OK";
    case MCI_E_INVALID_ARG: return "MCI_E_INVALID_ARG";
    case MCI_E_SINGULAR: return "MCI_E_SINGULAR";
    case MCI_E_ILL_CONDITIONED: return "MCI_E_ILL_CONDITIONED";
    case MCI_E_UNSUPPORTED: return "MCI_E_UNSUPPORTED";
    case MCI_E_OUT_OF_MEMORY: return "MCI_E_OUT_OF_MEMORY";
    case MCI_E_DEVICE: return "MCI_E_DEVICE";
  }
  return "MCI_E_UNKNOWN";
}

const char* mci_last_error(void) { return g_last_error.c_str(); }

mci_status mci_plan(const mci_plan_desc* desc, int device, mci_plan_t* out) {
  if (!out) return fail(MCI_E_INVALID_ARG, "out is NULL");
  *out = nullptr;
  mci_plan_s* p = nullptr;
  mci_status st = build_plan(desc, device, &p);
  if (st != MCI_OK) return st;
  apply_tune_cache(p);
  *out = p;
  return MCI_OK;
}

mci_status mci_plan_destroy(mci_plan_t plan) {
  if (!plan) return MCI_OK;
  (void)hipSetDevice(plan->device);
  destroy_plan(plan);
  return MCI_OK;
}

mci_status mci_plan_info(mci_plan_t p, mci_plan_info_t* info) {
  if (!p || !info) return fail(MCI_E_INVALID_ARG, "NULL argument");
  const mci_plan_s* q = p->dims == 2 ? p->rows : p;
  info->max_cond = q->max_cond;
  info->n_singular = q->n_sing;
  info->first_singular = q->first_sing;
  info->n1 = q->d.n1;
  info->fft_len_fwd = q->fwd.lexec;
  info->fft_len_inv = q->inv.lexec;
  info->path = p->dims == 2 ? (p->lp ? 1 : 0) : (p->use_fused ? 1 : 0);
  info->variant = p->variant;
  return MCI_OK;
}

mci_status mci_plan_kernel_name(mci_plan_t p, char* name, size_t len) {
  if (!p || !name || len == 0) return fail(MCI_E_INVALID_ARG, "NULL argument or zero length");
  std::string s;
  auto side = [](const FftSide& f) {
    std::string t = f.fa > 1 ? std::to_string(f.fa) + " x " + std::to_string(f.fb) : std::to_string(f.lexec);
    if (f.blue) t += " (Bluestein for " + std::to_string(f.len) + ")";
    return t;
  };
  if (p->dims == 2) {
    if (p->lp)
      s = "k_line_pass: columns " + std::to_string(p->d2.h) + " -> rows " + std::to_string(p->d2.w) + ", scale " +
          std::to_string(p->d2.scale) + ", " + std::to_string(p->d2.channels) + " channels" +
          (p->lp_zr ? ", sample rows passed through" : "");
    else
      s = "2-D multi-pass: 1-D multi-pass rows and columns";
  } else if (p->use_fused) {
    s = p->fused.name;
    if (p->fused.ti == 2) s += ", output transforms side by side";
  } else if (p->use_real) {
    s = "real two-pass: k_fft_lines forward " + side(p->rfwd) + ", inverse " + side(p->rinv) +
        " with the apply in its first pass";
  } else {
    s = std::string("multi-pass ") + (p->variant == MCI_VARIANT_TWO_PASS ? "two-pass transforms"
                                      : p->variant == MCI_VARIANT_MULTIPASS_R4 ? "radix-4 passes" : "radix-8 passes") +
        ": forward " + std::to_string(p->fwd.lexec) + (p->fwd.blue ? " (Bluestein)" : "") + ", inverse " +
        std::to_string(p->inv.lexec) + (p->inv.blue ? " (Bluestein)" : "");
  }
  std::snprintf(name, len, "%s", s.c_str());
  return MCI_OK;
}

mci_status mci_workspace_size(mci_plan_t p, int64_t batch, size_t* bytes) {
  if (!p || !bytes || batch < 0) return fail(MCI_E_INVALID_ARG, "bad argument");
  *bytes = p->dims == 2 ? ws_2d(p, batch) : ws_1d(p, batch);
  return MCI_OK;
}

mci_status mci_reconstruct_1d(mci_plan_t p, const void* g, void* y, int64_t batch, void* workspace, size_t ws_bytes,
                              hipStream_t stream) {
  if (!p || p->dims != 1) return fail(MCI_E_INVALID_ARG, "not a 1-D plan");
  if (batch < 0) return fail(MCI_E_INVALID_ARG, "batch < 0");
  if (batch == 0) return MCI_OK;
  if (!g || !y) return fail(MCI_E_INVALID_ARG, "NULL data pointer");
  if (!aligned16(g) || !aligned16(y) || !aligned16(workspace))
    return fail(MCI_E_INVALID_ARG, "data pointers and workspace must be 16-byte aligned");
  if (batch > ((int64_t)1 << 40) / std::max<int64_t>(p->mu, p->d.n_out * p->d.n_ops))
    return fail(MCI_E_INVALID_ARG, "batch too large");
  const size_t need = ws_1d(p, batch);
  if (need && (!workspace || ws_bytes < need))
    return fail(MCI_E_INVALID_ARG, "workspace too small: need " + std::to_string(need) + " bytes");
  HIP_TRY(hipSetDevice(p->device));
  return plan_run(p, g, y, batch, workspace, nullptr, stream);
}

// offsets table of a strided call: signal b's samples at b ld_g, its outputs at b ld_y
__global__ void k_strided_offsets(int64_t* __restrict__ offs, int64_t batch, int64_t ld_g, int64_t ld_y) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b < batch) {
    offs[2 * b] = b * ld_g;
    offs[2 * b + 1] = b * ld_y;
  }
}

// the run's scratch first (256-byte aligned), then the offsets table
static size_t ws_1d_strided(const mci_plan_s* p, int64_t batch) {
  return ((ws_1d(p, batch) + 255) & ~(size_t)255) + (size_t)batch * 2 * sizeof(int64_t) + 256;
}

mci_status mci_workspace_size_strided(mci_plan_t p, int64_t batch, size_t* bytes) {
  if (!p || !bytes || batch < 0 || p->dims != 1) return fail(MCI_E_INVALID_ARG, "bad argument");
  *bytes = batch ? ws_1d_strided(p, batch) : 0;
  return MCI_OK;
}

mci_status mci_reconstruct_1d_strided(mci_plan_t p, const void* g, int64_t ld_g, void* y, int64_t ld_y, int64_t batch,
                                      void* workspace, size_t ws_bytes, hipStream_t stream) {
  if (!p || p->dims != 1) return fail(MCI_E_INVALID_ARG, "not a 1-D plan");
  if (batch < 0) return fail(MCI_E_INVALID_ARG, "batch < 0");
  if (batch == 0) return MCI_OK;
  if (!g || !y || !workspace) return fail(MCI_E_INVALID_ARG, "NULL data pointer or workspace");
  if (!aligned16(g) || !aligned16(y) || !aligned16(workspace))
    return fail(MCI_E_INVALID_ARG, "data pointers and workspace must be 16-byte aligned");
  const int64_t c = p->d.real_io ? 1 : 2;
  const int64_t in_elems = p->mu * c, out_elems = p->d.n_out * p->d.n_ops * c;
  if (ld_g < in_elems || ld_y < out_elems)
    return fail(MCI_E_INVALID_ARG, "stride smaller than one signal: ld_g >= " + std::to_string(in_elems) +
                                       ", ld_y >= " + std::to_string(out_elems) + " elements");
  if (ld_g % 4 || ld_y % 4) return fail(MCI_E_INVALID_ARG, "strides must be multiples of 4 elements");
  if (batch > ((int64_t)1 << 40) / std::max(ld_g, ld_y)) return fail(MCI_E_INVALID_ARG, "batch too large");
  const size_t need = ws_1d_strided(p, batch);
  if (ws_bytes < need) return fail(MCI_E_INVALID_ARG, "workspace too small: need " + std::to_string(need) + " bytes");
  HIP_TRY(hipSetDevice(p->device));
  char* base = (char*)workspace;   // 16-byte aligned (checked); the paths align their own scratch
  int64_t* offs = (int64_t*)(base + ((ws_1d(p, batch) + 255) & ~(size_t)255));
  hipLaunchKernelGGL(k_strided_offsets, dim3((unsigned)((batch + 255) / 256)), dim3(256), 0, stream, offs, batch,
                     ld_g, ld_y);
  HIP_TRY(hipGetLastError());
  return plan_run(p, g, y, batch, base, offs, stream);
}

mci_status mci_plan_2d(const mci_plan2d_desc* desc, int device, mci_plan_t* out) {
  if (!out) return fail(MCI_E_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!desc) return fail(MCI_E_INVALID_ARG, "desc is NULL");
  if (desc->h < 2 || desc->w < 2 || desc->scale < 1 || desc->h > (1 << 16) || desc->w > (1 << 16) || desc->scale > 16)
    return fail(MCI_E_INVALID_ARG, "image size or scale out of range");
  if (desc->precision != MCI_F32 && desc->precision != MCI_F64) return fail(MCI_E_INVALID_ARG, "precision");
  if (desc->storage != MCI_STORE_NATIVE && desc->storage != MCI_STORE_F16) return fail(MCI_E_INVALID_ARG, "storage");
  if (desc->storage == MCI_STORE_F16 && desc->precision != MCI_F32) return fail(MCI_E_INVALID_ARG, "F16 needs F32");
  if (desc->channels != 0 && desc->channels != 2 && desc->channels != 3)
    return fail(MCI_E_INVALID_ARG, "channels must be 2 or 3 (0 means 2)");
  mci_plan_s* p = new (std::nothrow) mci_plan_s();
  if (!p) return fail(MCI_E_OUT_OF_MEMORY, "plan");
  p->dims = 2;
  p->device = device;
  p->d2 = *desc;
  if (p->d2.channels == 0) p->d2.channels = 2;
  const int M2 = p->d2.channels;
  p->prec = desc->precision;
  p->store = desc->precision == MCI_F64 ? ST_F64 : (desc->storage == MCI_STORE_F16 ? ST_F16 : ST_F32);
  for (int axis = 0; axis < 2; ++axis) {
    const int64_t len = axis == 0 ? desc->w : desc->h;
    mci_plan_desc d{};
    d.M = M2; d.n_ops = 1; d.N = len; d.n1 = MCI_N1_DEFAULT; d.n_out = (int64_t)desc->scale * len;
    for (int m = 0; m < M2; ++m) { d.ch[m].kind = MCI_MULT_DERIV; d.ch[m].order = m; }
    d.ops[0] = MCI_OUT_IDENTITY;
    d.real_io = 1;
    d.precision = desc->precision;
    d.storage = MCI_STORE_NATIVE;
    mci_plan_s* q = nullptr;
    mci_status st = build_plan(&d, device, &q);
    if (st != MCI_OK) { destroy_plan(p); return st; }
    (axis == 0 ? p->rows : p->cols) = q;
  }
  if (desc->precision == MCI_F32 && line_pass_supported(desc->h, desc->scale) &&
      line_pass_supported(desc->w, desc->scale) && !std::getenv("MCI_DISABLE_FUSED")) {
    // axis 0: columns (length h), axis 1: rows (length w)
    double h0_dev = 0.0;   // max |len H_0 - 1| of the columns pass
    for (int axis = 0; axis < 2; ++axis) {
      const mci_plan_s* q = axis == 0 ? p->cols : p->rows;
      const int64_t len = q->d.N;
      std::vector<std::complex<double>> H = line_windows(q->tab_host, len, q->d.n1, desc->scale, M2);
      // the line passes' transforms are unnormalised: the identity window is 1 / len
      if (axis == 0)
        for (int64_t k = 0; k < len; ++k) h0_dev = std::max(h0_dev, std::abs(H[k] * (double)len - 1.0));
      std::vector<std::complex<double>> tw(len);
      for (int64_t k = 0; k < len; ++k) tw[k] = root_of_unity(k, len);
      hipError_t e;
      p->lp_H[axis] = upload<float2>(H, e);
      if (!p->lp_H[axis] || e != hipSuccess) { destroy_plan(p); return fail(MCI_E_DEVICE, "window upload"); }
      p->lp_tw[axis] = upload<float2>(tw, e);
      if (!p->lp_tw[axis] || e != hipSuccess) { destroy_plan(p); return fail(MCI_E_DEVICE, "twiddle upload"); }
    }
    // The columns pass's window H_0 is the identity when the grid's row s q is the sample row
    // q (interpolation consistency); then that row is the input row itself and the passes
    // move it straight from the input (FP32 storage).  Measured on one box at 100 steps: x2
    // 0.1278 -> 0.1226 ms; x3 0.0673 -> 0.0708 and x4 0.1009 -> 0.1024 ms, where the rows pass's
    // extra reads of the input cost more than the smaller intermediate saves.  So it is the
    // default at scale 2 only; MCI_LP_ZR=1 takes it at every scale, MCI_LP_FULL_COLUMNS=1 at none.
    const bool zr_env = std::getenv("MCI_LP_ZR") && std::getenv("MCI_LP_ZR")[0] == '1';
    p->lp_zr = p->store == ST_F32 && h0_dev <= 1e-9 && (desc->scale == 2 || zr_env) &&
               !std::getenv("MCI_LP_FULL_COLUMNS");
    if (prepare_line_pass(desc->h, desc->scale, true, p->lp_zr, p->store, ST_F32) != hipSuccess ||
        prepare_line_pass(desc->w, desc->scale, false, p->lp_zr, ST_F32, p->store) != hipSuccess) {
      destroy_plan(p);
      return fail(MCI_E_DEVICE, "line-pass LDS attribute");
    }
    p->lp_avail = true;
  }
  (void)plan_set_variant(p, p->lp_avail ? MCI_VARIANT_LINE_PASS : MCI_VARIANT_MULTIPASS_R8);
  apply_tune_cache(p);
  *out = p;
  return MCI_OK;
}

mci_status mci_upsample_2d(mci_plan_t p, const void* lr, void* hr, int64_t batch, void* workspace, size_t ws_bytes,
                           hipStream_t stream) {
  if (!p || p->dims != 2) return fail(MCI_E_INVALID_ARG, "not a 2-D plan");
  if (batch < 0) return fail(MCI_E_INVALID_ARG, "batch < 0");
  if (batch == 0) return MCI_OK;
  if (!lr || !hr) return fail(MCI_E_INVALID_ARG, "NULL data pointer");
  if (!aligned16(lr) || !aligned16(hr) || !aligned16(workspace))
    return fail(MCI_E_INVALID_ARG, "data pointers and workspace must be 16-byte aligned");
  if (batch > ((int64_t)1 << 40) / instance_out_elems(p)) return fail(MCI_E_INVALID_ARG, "batch too large");
  const size_t need = ws_2d(p, batch);
  if (!workspace || ws_bytes < need) return fail(MCI_E_INVALID_ARG, "workspace too small: need " + std::to_string(need));
  HIP_TRY(hipSetDevice(p->device));
  return plan_run(p, lr, hr, batch, workspace, nullptr, stream);
}

mci_status mci_plan_variants(mci_plan_t p, uint32_t* mask) {
  if (!p || !mask) return fail(MCI_E_INVALID_ARG, "NULL argument");
  *mask = plan_variant_mask(p);
  return MCI_OK;
}

mci_status mci_plan_set_variant(mci_plan_t p, int32_t v) {
  if (!p) return fail(MCI_E_INVALID_ARG, "NULL plan");
  if (v < 0 || v >= MCI_NUM_VARIANTS) return fail(MCI_E_INVALID_ARG, "unknown variant");
  return plan_set_variant(p, v);
}

}  // extern "C"
