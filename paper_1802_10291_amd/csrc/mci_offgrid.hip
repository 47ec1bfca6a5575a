// mci_offgrid.hip -- evaluation of the reconstruction at arbitrary real points t.
//
// Theorem 3.3 holds at every t, not only on a uniform grid: the recovered band
// coefficients a(n), n in [n1, n1 + M N), define f(t) = sum_n o(n) a(n) e^{i n t} (eq.
// DFTexpression with the output operator of the closing paragraph of Section 3).  A direct
// sum costs M N operations per point; this file evaluates it as a type-2 nonuniform FFT:
//
//   1. the regular reconstruction path (channel DFTs, per-residue apply, scatter, inverse
//      FFT) runs onto an oversampled grid of L points, L the power of two at or above
//      4 K + 2 with K = max |n| over the band (oversampling sigma = L / (2 K + 1) in [2, 4)),
//      its apply tables multiplied by d(n) = 1 / (L psi_hat(n));
//   2. each point t gathers the w grid values around it, weighted by the kernel
//      psi(t) = ES(t / alpha), alpha = pi w / L, with the "exponential of semicircle"
//      ES(x) = exp(beta (sqrt(1 - x^2) - 1)) on |x| <= 1 (Barnett, Magland and af
//      Klinteberg, SIAM J. Sci. Comput. 41 (2019)), beta = 0.97 pi w (1 - 1 / (2 sigma)).
//
// Why it is exact up to the kernel's aliasing: with u_j = (1/L) sum_n c(n) e^{i n t_j},
// t_j = 2 pi j / L, and Psi the 2 pi-periodisation of psi, whose Fourier coefficients are
// psi_hat(m) = (1/2 pi) int psi(t) e^{-i m t} dt,
//     sum_j u_j Psi(t - t_j) = sum_n c(n) sum_p psi_hat(n + p L) e^{i (n + p L) t}.
// With c(n) = o(n) a(n) / psi_hat(n) the p = 0 term is f(t); the p != 0 terms are the
// error, bounded by psi_hat(n + p L) / psi_hat(n) with |n + p L| >= L - K >= 3K: measured
// at 5 to 20 times exp(-pi w sqrt(1 - 1 / sigma)), which sets the default width.  psi_hat
// is an integral of ES against a cosine, evaluated in FP64 by Gauss-Legendre quadrature at
// plan time.
//
// Points shared by the whole batch (the common case: many signals resampled at the same
// instants) get their grid start and w weights computed once per call into a small table;
// one workgroup per output row then stages the row's grid in LDS and sums from it, so the
// gather reads the grid from HBM once and its only divergent accesses are LDS reads.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <new>
#include <string>
#include <vector>

#include "mci_fftlines.h"
#include "mci_plan.h"

struct mci_offgrid_s {
  mci_plan_s* grid = nullptr;   // reconstruction onto the oversampled grid, deconvolved tables
  int device = 0;
  int prec = MCI_F32;
  int real_io = 1;
  int n_ops = 1;
  int64_t L = 0;                // grid length
  int w = 8;                    // kernel width in grid points
  double beta = 0.0;
};

namespace mci {
namespace og {

constexpr int MAX_W = 16;
constexpr int NT = 256;

struct EvalArgs {
  const void* grid;   // [batch][n_ops][L] (real) or [batch][n_ops][L][2]
  const double* t;    // [n_t] (shared) or [batch][n_t]
  void* y;            // [batch][n_ops][n_t] (real) or [batch][n_ops][n_t][2]
  int* start;         // shared points: grid index of each point's first tap, [n_t]
  void* wt;           // shared points: weights [w][n_t] in plan precision
  int64_t L, n_t, batch, t_stride;
  int n_ops, w;
  double beta, L_over_2pi;
};

template <typename T>
__device__ __forceinline__ T es_weight(T x, T beta) {
  const T a = T(1) - x * x;
  return a > T(0) ? exp(beta * (sqrt(a) - T(1))) : T(0);
}

// Grid position of t in FP64, t L / (2 pi) reduced to [0, L); first tap i0 = ceil(pos - w/2)
// (may be negative: indices wrap modulo L, a power of two) and the offset of tap 0.
__device__ __forceinline__ int64_t first_tap(double t, const EvalArgs& a, double& x0) {
  double pos = t * a.L_over_2pi;
  pos -= floor(pos / (double)a.L) * (double)a.L;
  if (pos >= (double)a.L) pos -= (double)a.L;
  const double start = ceil(pos - 0.5 * a.w);
  x0 = (start - pos) * (2.0 / a.w);   // kernel argument of tap 0, in [-1, -1 + 2/w)
  return (int64_t)start;
}

// Shared points: the weight table, one thread per point.
template <typename T>
__global__ __launch_bounds__(NT) void k_weights(EvalArgs a) {
  const int64_t j = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (j >= a.n_t) return;
  double x0;
  const int64_t i0 = first_tap(a.t[j], a, x0);
  a.start[j] = (int)(i0 & (a.L - 1));
  const double step = 2.0 / a.w;
  for (int k = 0; k < a.w; ++k) ((T*)a.wt)[k * a.n_t + j] = es_weight<T>((T)(x0 + k * step), (T)a.beta);
}

// Shared points, rows that fit the LDS: one workgroup per RR output rows (signal b, operator op)
// copies the rows' grids into LDS with coalesced loads, then every thread evaluates points
// j = tid, tid + NG, ... from the table.  The table (start and W weights per point, shared by
// every row) is what the gather reads most; taking RR = 2 rows per workgroup reads it once for
// both (the two 64 KB FP32 rows of the 16384-point grids fit the LDS together).
constexpr int NG = 512;

template <int RR> constexpr int gather_threads() { return RR * NG; }   // one LDS-resident workgroup per CU at RR = 2

template <typename T, bool REAL, int W, int RR>
__global__ __launch_bounds__(gather_threads<RR>()) void k_gather_lds(EvalArgs a) {
  constexpr int NTG = gather_threads<RR>();
  extern __shared__ __align__(16) unsigned char lds_raw[];
  using V = typename std::conditional<REAL, T, typename std::conditional<sizeof(T) == 4, float2, double2>::type>::type;
  V* rows = (V*)lds_raw;
  const int64_t L = a.L;
  const int64_t r0 = (int64_t)blockIdx.x * RR;
  const int64_t n_rows = a.batch * a.n_ops;
  const int nr = (int)(n_rows - r0 < RR ? n_rows - r0 : RR);
  {
    // 16-byte copies: a row is L sizeof(V) bytes, a multiple of 16 (L is a power of two >= 32)
    // the rows are read once (non-temporal), leaving L2 to the shared weight table
    typedef unsigned u4_nt __attribute__((ext_vector_type(4)));
    const u4_nt* src = (const u4_nt*)((const V*)a.grid + r0 * L);
    u4_nt* dst = (u4_nt*)rows;
    const int64_t n16 = nr * L * (int64_t)sizeof(V) / 16;
    for (int64_t q = threadIdx.x; q < n16; q += NTG) dst[q] = __builtin_nontemporal_load(src + q);
  }
  __syncthreads();
  const T* wt = (const T*)a.wt;
  const int mask = (int)(L - 1);
  // the table loads of a point (start and W weights) are independent: with W fixed at
  // compile time they issue back to back and share one wait
  for (int64_t j = threadIdx.x; j < a.n_t; j += NTG) {
    const int s0 = a.start[j];
    T c[W];
#pragma unroll
    for (int k = 0; k < W; ++k) c[k] = wt[k * a.n_t + j];
#pragma unroll
    for (int rr = 0; rr < RR; ++rr) {
      if (rr >= nr) break;
      const V* row = rows + rr * L;
      const int64_t r = r0 + rr;
      if constexpr (REAL) {
        T acc = T(0);
#pragma unroll
        for (int k = 0; k < W; ++k) acc += c[k] * row[(s0 + k) & mask];
        __builtin_nontemporal_store(acc, (T*)a.y + r * a.n_t + j);
      } else {
        T re = T(0), im = T(0);
#pragma unroll
        for (int k = 0; k < W; ++k) {
          const V g = row[(s0 + k) & mask];
          re += c[k] * g.x;
          im += c[k] * g.y;
        }
        T* y = (T*)a.y + 2 * (r * a.n_t + j);
        __builtin_nontemporal_store(re, y);
        __builtin_nontemporal_store(im, y + 1);
      }
    }
  }
}

// Every other case: one thread per (row, point), grid read through L2.  Shared points take
// their tap start and weights from the table; per-signal points compute their own.
template <typename T, bool REAL, bool SHARED, int W>
__global__ __launch_bounds__(NT) void k_gather(EvalArgs a) {
  const int64_t j = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (j >= a.n_t) return;
  const int64_t mask = a.L - 1;
  for (int64_t b = blockIdx.y; b < a.batch; b += gridDim.y) {
    T wt[W];
    int64_t s0;
    if constexpr (SHARED) {
      s0 = a.start[j];
#pragma unroll
      for (int k = 0; k < W; ++k) wt[k] = ((const T*)a.wt)[k * a.n_t + j];
    } else {
      double x0;
      s0 = first_tap(a.t[b * a.t_stride + j], a, x0);
      const double step = 2.0 / W;
#pragma unroll
      for (int k = 0; k < W; ++k) wt[k] = es_weight<T>((T)(x0 + k * step), (T)a.beta);
    }
    for (int op = 0; op < a.n_ops; ++op) {
      const int64_t row = b * a.n_ops + op;
      if constexpr (REAL) {
        const T* g = (const T*)a.grid + row * a.L;
        T acc = T(0);
#pragma unroll
        for (int k = 0; k < W; ++k) acc += wt[k] * g[(s0 + k) & mask];
        ((T*)a.y)[row * a.n_t + j] = acc;
      } else {
        const T* g = (const T*)a.grid + 2 * row * a.L;
        T re = T(0), im = T(0);
#pragma unroll
        for (int k = 0; k < W; ++k) {
          const int64_t q = (s0 + k) & mask;
          re += wt[k] * g[2 * q];
          im += wt[k] * g[2 * q + 1];
        }
        T* y = (T*)a.y + 2 * (row * a.n_t + j);
        y[0] = re;
        y[1] = im;
      }
    }
  }
}

// dynamic LDS of the two-row gather (its limit is raised at plan time)
constexpr size_t kGatherLds2 = 128 * 1024;

template <typename T, bool REAL, int W>
static hipError_t prep_gather_w() {
  return hipFuncSetAttribute((const void*)k_gather_lds<T, REAL, W, 2>, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)kGatherLds2);
}
template <typename T, bool REAL>
static hipError_t prep_gather_t(int w) {
  switch (w) {
#define MCI_OG_W(W) \
  case W: return prep_gather_w<T, REAL, W>();
    MCI_OG_W(2) MCI_OG_W(3) MCI_OG_W(4) MCI_OG_W(5) MCI_OG_W(6) MCI_OG_W(7) MCI_OG_W(8) MCI_OG_W(9)
    MCI_OG_W(10) MCI_OG_W(11) MCI_OG_W(12) MCI_OG_W(13) MCI_OG_W(14) MCI_OG_W(15) MCI_OG_W(16)
#undef MCI_OG_W
    default: return hipErrorInvalidValue;
  }
}
static hipError_t prep_gather(int prec, bool real, int w) {
  if (prec == MCI_F64) return real ? prep_gather_t<double, true>(w) : prep_gather_t<double, false>(w);
  return real ? prep_gather_t<float, true>(w) : prep_gather_t<float, false>(w);
}

template <typename T, bool REAL, int W>
static hipError_t launch_eval_w(const EvalArgs& a, bool shared, hipStream_t s) {
  const int64_t gx = (a.n_t + NT - 1) / NT;
  const dim3 g2((unsigned)gx, (unsigned)std::min<int64_t>(a.batch, 65535));
  if (!shared) {
    hipLaunchKernelGGL((k_gather<T, REAL, false, W>), g2, dim3(NT), 0, s, a);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_weights<T>, dim3((unsigned)gx), dim3(NT), 0, s, a);
  const size_t row_bytes = (size_t)a.L * sizeof(T) * (REAL ? 1 : 2);
  const int64_t rows = a.batch * a.n_ops;
  // (MCI_GATHER_ONE_ROW=1 keeps one row per workgroup, the form measured against)
  static const bool one_row = std::getenv("MCI_GATHER_ONE_ROW") && std::getenv("MCI_GATHER_ONE_ROW")[0] == '1';
  if (!one_row && 2 * row_bytes <= kGatherLds2 && rows >= 2 && rows <= 0x7fffffff)
    hipLaunchKernelGGL((k_gather_lds<T, REAL, W, 2>), dim3((unsigned)((rows + 1) / 2)), dim3(gather_threads<2>()),
                       2 * row_bytes, s, a);
  else if (row_bytes <= 64 * 1024 && rows <= 0x7fffffff)
    hipLaunchKernelGGL((k_gather_lds<T, REAL, W, 1>), dim3((unsigned)rows), dim3(gather_threads<1>()), row_bytes, s, a);
  else
    hipLaunchKernelGGL((k_gather<T, REAL, true, W>), g2, dim3(NT), 0, s, a);
  return hipGetLastError();
}

template <typename T, bool REAL>
static hipError_t launch_eval(const EvalArgs& a, bool shared, hipStream_t s) {
  switch (a.w) {
#define MCI_OG_W(W) \
  case W: return launch_eval_w<T, REAL, W>(a, shared, s);
    MCI_OG_W(2) MCI_OG_W(3) MCI_OG_W(4) MCI_OG_W(5) MCI_OG_W(6) MCI_OG_W(7) MCI_OG_W(8) MCI_OG_W(9)
    MCI_OG_W(10) MCI_OG_W(11) MCI_OG_W(12) MCI_OG_W(13) MCI_OG_W(14) MCI_OG_W(15) MCI_OG_W(16)
#undef MCI_OG_W
    default: return hipErrorInvalidValue;
  }
}

// Gauss-Legendre nodes and weights on [-1, 1] (Newton iteration on P_q from the
// three-term recurrence, starting at the Chebyshev-like guesses cos(pi (i - 1/4) / (q + 1/2))).
static void gauss_legendre(int q, std::vector<double>& x, std::vector<double>& wq) {
  x.assign(q, 0.0);
  wq.assign(q, 0.0);
  for (int i = 0; i < (q + 1) / 2; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (q + 0.5)), dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 1; k < q; ++k) {
        const double p2 = ((2.0 * k + 1.0) * z * p1 - k * p0) / (k + 1.0);
        p0 = p1;
        p1 = p2;
      }
      dp = q * (z * p1 - p0) / (z * z - 1.0);
      const double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    x[i] = -z;
    x[q - 1 - i] = z;
    wq[i] = wq[q - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

// grid length: the power of two at or above lmin (every variant of the reconstruction runs
// it, and the gather wraps indices with a mask)
static int64_t choose_grid_length(int64_t lmin) {
  int64_t L = 2;
  while (L < lmin) L <<= 1;
  return L;
}

// default width: the smallest w whose estimated error 20 exp(-pi w sqrt(1 - 1 / sigma))
// stays below eps (4e-7 for FP32 plans, near their rounding; 1e-12 for FP64 plans)
static int default_width(double sigma, int prec) {
  const double eps = prec == MCI_F64 ? 1e-12 : 4e-7;
  const double w = std::log(20.0 / eps) / (M_PI * std::sqrt(1.0 - 1.0 / sigma));
  return std::min(MAX_W, std::max(2, (int)std::ceil(w - 1e-9)));
}

}  // namespace og
}  // namespace mci

using namespace mci;
using namespace mci::og;

extern "C" {

mci_status mci_offgrid_plan(const mci_plan_desc* desc, int32_t width, int device, mci_offgrid_t* out) {
  if (!out) return fail(MCI_E_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!desc) return fail(MCI_E_INVALID_ARG, "desc is NULL");
  if (desc->storage != MCI_STORE_NATIVE) return fail(MCI_E_UNSUPPORTED, "off-grid evaluation needs native storage");
  if (desc->precision != MCI_F32 && desc->precision != MCI_F64) return fail(MCI_E_INVALID_ARG, "precision");
  if (width != 0 && (width < 2 || width > MAX_W)) return fail(MCI_E_INVALID_ARG, "width must be 0 or in 2..16");
  if (desc->M < 1 || desc->M > MCI_MAX_CHANNELS || desc->N < 1) return fail(MCI_E_INVALID_ARG, "M or N");
  const int64_t mu = (int64_t)desc->M * desc->N;
  if (mu > (int64_t)1 << 26) return fail(MCI_E_INVALID_ARG, "band too long for off-grid evaluation");
  const int64_t n1 = desc->n1 == MCI_N1_DEFAULT ? -((mu - 1) / 2) : desc->n1;
  const int64_t K = std::max<int64_t>(std::llabs(n1), std::llabs(n1 + mu - 1));
  const int64_t L = choose_grid_length(std::max<int64_t>(4 * K + 2, 2 * MAX_W));
  const double sigma = (double)L / (double)(2 * K + 1);
  const int w = width ? width : default_width(sigma, desc->precision);
  const double beta = 0.97 * M_PI * w * (1.0 - 0.5 / sigma), alpha = M_PI * w / (double)L;
  // d(n) = 1 / (L psi_hat(n)), psi_hat(n) = (alpha / 2 pi) int_{-1}^{1} ES(x) cos(n alpha x) dx
  std::vector<double> xq, wq, ew;
  gauss_legendre(96, xq, wq);
  ew.resize(xq.size());
  for (size_t q = 0; q < xq.size(); ++q) ew[q] = wq[q] * std::exp(beta * (std::sqrt(1.0 - xq[q] * xq[q]) - 1.0));
  std::vector<double> d((size_t)mu);
  for (int64_t i = 0; i < mu; ++i) {
    const double n = (double)(n1 + i);
    double s = 0.0;
    for (size_t q = 0; q < xq.size(); ++q) s += ew[q] * std::cos(n * alpha * xq[q]);
    d[(size_t)i] = 1.0 / ((double)L * alpha / (2.0 * M_PI) * s);
  }
  mci_plan_desc g = *desc;
  g.n1 = n1;
  g.n_out = L;
  mci_plan_s* gp = nullptr;
  mci_status st = build_plan(&g, device, &gp, &d);
  if (st != MCI_OK) return st;
  mci_offgrid_s* p = new (std::nothrow) mci_offgrid_s();
  if (!p) {
    (void)mci_plan_destroy(gp);
    return fail(MCI_E_OUT_OF_MEMORY, "off-grid plan");
  }
  p->grid = gp;
  p->device = device;
  p->prec = desc->precision;
  p->real_io = desc->real_io ? 1 : 0;
  if (prep_gather(p->prec, p->real_io != 0, w) != hipSuccess) {
    (void)mci_plan_destroy(gp);
    delete p;
    return fail(MCI_E_DEVICE, "gather LDS attribute");
  }
  p->n_ops = desc->n_ops;
  p->L = L;
  p->w = w;
  p->beta = beta;
  *out = p;
  return MCI_OK;
}

mci_status mci_offgrid_destroy(mci_offgrid_t p) {
  if (!p) return MCI_OK;
  (void)mci_plan_destroy(p->grid);
  delete p;
  return MCI_OK;
}

mci_status mci_offgrid_info(mci_offgrid_t p, int64_t* grid_len, int32_t* width, double* beta, mci_plan_t* grid_plan) {
  if (!p) return fail(MCI_E_INVALID_ARG, "plan is NULL");
  if (grid_len) *grid_len = p->L;
  if (width) *width = p->w;
  if (beta) *beta = p->beta;
  if (grid_plan) *grid_plan = p->grid;
  return MCI_OK;
}

static size_t al256(size_t n) { return (n + 255) & ~(size_t)255; }

static size_t grid_bytes(const mci_offgrid_s* p, int64_t batch) {
  const size_t el = (p->prec == MCI_F64 ? 8 : 4) * (p->real_io ? 1 : 2);
  return al256((size_t)batch * p->n_ops * p->L * el);
}

// weight table of shared points: tap starts (int) and w weights per point
static size_t table_bytes(const mci_offgrid_s* p, int64_t n_t) {
  return al256((size_t)n_t * sizeof(int)) + al256((size_t)n_t * p->w * (p->prec == MCI_F64 ? 8 : 4));
}

mci_status mci_offgrid_workspace_size(mci_offgrid_t p, int64_t batch, int64_t n_t, size_t* bytes) {
  if (!p || !bytes || batch < 0 || n_t < 0) return fail(MCI_E_INVALID_ARG, "plan, bytes, batch or n_t");
  *bytes = grid_bytes(p, batch) + table_bytes(p, n_t) + plan_workspace(p->grid, batch);
  return MCI_OK;
}

mci_status mci_evaluate_1d(mci_offgrid_t p, const void* g, const double* t, int64_t n_t, int32_t t_shared, void* y,
                           int64_t batch, void* workspace, size_t ws_bytes, hipStream_t stream) {
  if (!p) return fail(MCI_E_INVALID_ARG, "plan is NULL");
  if (batch < 0 || n_t < 0) return fail(MCI_E_INVALID_ARG, "batch and n_t must be >= 0");
  if (batch == 0 || n_t == 0) return MCI_OK;
  if (!g || !t || !y) return fail(MCI_E_INVALID_ARG, "NULL array");
  if (!aligned16(g) || !aligned16(y) || !aligned16(workspace) || ((uintptr_t)t & 7))
    return fail(MCI_E_INVALID_ARG, "g, y and workspace must be 16-byte aligned, t 8-byte aligned");
  const size_t gb = grid_bytes(p, batch), tb = table_bytes(p, n_t), need = gb + tb + plan_workspace(p->grid, batch);
  if (!workspace || ws_bytes < need) return fail(MCI_E_INVALID_ARG, "workspace too small");
  if (n_t > 0x7fffffffLL * NT) return fail(MCI_E_INVALID_ARG, "too many points");
  if (hipSetDevice(p->device) != hipSuccess) return fail(MCI_E_DEVICE, "hipSetDevice");
  char* base = (char*)workspace;
  void* grid = base;
  EvalArgs a{};
  a.start = (int*)(base + gb);
  a.wt = base + gb + al256((size_t)n_t * sizeof(int));
  void* inner = need > gb + tb ? (void*)(base + gb + tb) : nullptr;
  mci_status st = plan_run(p->grid, g, grid, batch, inner, nullptr, stream);
  if (st != MCI_OK) return st;
  a.grid = grid;
  a.t = t;
  a.y = y;
  a.L = p->L;
  a.n_t = n_t;
  a.batch = batch;
  a.t_stride = t_shared ? 0 : n_t;
  a.n_ops = p->n_ops;
  a.w = p->w;
  a.beta = p->beta;
  a.L_over_2pi = (double)p->L / (2.0 * M_PI);
  const bool sh = t_shared != 0;
  hipError_t e;
  if (p->prec == MCI_F64) e = p->real_io ? launch_eval<double, true>(a, sh, stream) : launch_eval<double, false>(a, sh, stream);
  else e = p->real_io ? launch_eval<float, true>(a, sh, stream) : launch_eval<float, false>(a, sh, stream);
  if (e != hipSuccess) return fail(MCI_E_DEVICE, std::string("off-grid evaluation: ") + hipGetErrorString(e));
  return MCI_OK;
}

}  // extern "C"
