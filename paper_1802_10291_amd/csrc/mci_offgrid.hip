// mci_offgrid.hip -- evaluation of the reconstruction at arbitrary real points t.
//
// Theorem 3.3 holds at every t, not only on a uniform grid: the recovered band
// coefficients a(n), n in [n1, n1 + M N), define f(t) = sum_n o(n) a(n) e^{i n t} (eq.
// DFTexpression with the output operator of the closing paragraph of Section 3).  A direct
// sum costs M N operations per point; this file evaluates it as a type-2 nonuniform FFT:
//
//   1. the regular reconstruction path (channel DFTs, per-residue apply, scatter, inverse
//      FFT) runs onto an oversampled grid of L points, L >= 4 K + 2 with K = max |n| over
//      the band, its apply tables multiplied by d(n) = 1 / (L psi_hat(n));
//   2. each point t gathers the w grid values around it, weighted by the kernel
//      psi(t) = ES(t / alpha), alpha = pi w / L, with the "exponential of semicircle"
//      ES(x) = exp(beta (sqrt(1 - x^2) - 1)) on |x| <= 1 (Barnett, Magland and af
//      Klinteberg, SIAM J. Sci. Comput. 41 (2019); beta = 2.30 w for oversampling 2).
//
// Why it is exact up to the kernel's aliasing: with u_j = (1/L) sum_n c(n) e^{i n t_j},
// t_j = 2 pi j / L, and Psi the 2 pi-periodisation of psi, whose Fourier coefficients are
// psi_hat(m) = (1/2 pi) int psi(t) e^{-i m t} dt,
//     sum_j u_j Psi(t - t_j) = sum_n c(n) sum_p psi_hat(n + p L) e^{i (n + p L) t}.
// With c(n) = o(n) a(n) / psi_hat(n) the p = 0 term is f(t); the p != 0 terms are the
// error, bounded by psi_hat(n + p L) / psi_hat(n) with |n + p L| >= L - K >= 3K: about
// 10^(1-w) for this kernel.  psi_hat is an integral of ES against a cosine, evaluated in
// FP64 by Gauss-Legendre quadrature at plan time.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
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
  int64_t L, n_t, batch, t_stride;
  int n_ops, w;
  double beta, L_over_2pi;
};

template <typename T>
__device__ __forceinline__ T es_weight(T x, T beta) {
  const T a = T(1) - x * x;
  return a > T(0) ? exp(beta * (sqrt(a) - T(1))) : T(0);
}

// One thread per (signal, point): the w kernel weights are computed once and applied to
// every output operator's grid.  Grid values of a signal (L elements per operator) are
// re-read by neighbouring points, so they are served from L2.
template <typename T, bool REAL>
__global__ __launch_bounds__(NT) void k_eval(EvalArgs a) {
  const int64_t j = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (j >= a.n_t) return;
  for (int64_t b = blockIdx.y; b < a.batch; b += gridDim.y) {
    // position on the grid in FP64: t L / (2 pi) reduced to [0, L)
    double pos = a.t[b * a.t_stride + j] * a.L_over_2pi;
    pos -= floor(pos / (double)a.L) * (double)a.L;
    if (pos >= (double)a.L) pos -= (double)a.L;
    const double start = ceil(pos - 0.5 * a.w);
    const int64_t i0 = (int64_t)start;
    const double step = 2.0 / a.w;
    T wt[MAX_W];
    int64_t idx[MAX_W];
#pragma unroll
    for (int k = 0; k < MAX_W; ++k) {
      if (k < a.w) {
        const T x = (T)((start + k - pos) * step);
        wt[k] = es_weight<T>(x, (T)a.beta);
        int64_t q = i0 + k;
        q += q < 0 ? a.L : 0;
        q -= q >= a.L ? a.L : 0;
        idx[k] = q;
      }
    }
    for (int op = 0; op < a.n_ops; ++op) {
      const int64_t row = b * a.n_ops + op;
      if constexpr (REAL) {
        const T* g = (const T*)a.grid + row * a.L;
        T acc = T(0);
#pragma unroll
        for (int k = 0; k < MAX_W; ++k)
          if (k < a.w) acc += wt[k] * g[idx[k]];
        ((T*)a.y)[row * a.n_t + j] = acc;
      } else {
        const T* g = (const T*)a.grid + 2 * row * a.L;
        T re = T(0), im = T(0);
#pragma unroll
        for (int k = 0; k < MAX_W; ++k)
          if (k < a.w) {
            re += wt[k] * g[2 * idx[k]];
            im += wt[k] * g[2 * idx[k] + 1];
          }
        T* y = (T*)a.y + 2 * (row * a.n_t + j);
        y[0] = re;
        y[1] = im;
      }
    }
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

// smallest grid length >= lmin that the reconstruction runs on a fast path: 2 A B with A B
// a two-pass transform length, a power of two, else the next 7-smooth length
static int64_t choose_grid_length(int64_t lmin) {
  int64_t best = 2 * next_smooth_length((lmin + 1) / 2);
  for (int64_t c = 2; c < 2 * best; c *= 2)
    if (c >= lmin && c < best) best = c;
  for (int a : {1, 32, 48, 64, 96, 128, 192, 256, 384, 512})
    for (int b : {32, 48, 64, 96, 128, 192, 256, 384, 512}) {
      const int64_t c = 2LL * a * b;
      if (c >= lmin && c < best) best = c;
    }
  return best;
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
  const int w = width ? width : (desc->precision == MCI_F64 ? 16 : 8);
  if (w < 2 || w > MAX_W) return fail(MCI_E_INVALID_ARG, "width must be 0 or in 2..16");
  if (desc->M < 1 || desc->M > MCI_MAX_CHANNELS || desc->N < 1) return fail(MCI_E_INVALID_ARG, "M or N");
  const int64_t mu = (int64_t)desc->M * desc->N;
  if (mu > (int64_t)1 << 26) return fail(MCI_E_INVALID_ARG, "band too long for off-grid evaluation");
  const int64_t n1 = desc->n1 == MCI_N1_DEFAULT ? -((mu - 1) / 2) : desc->n1;
  const int64_t K = std::max<int64_t>(std::llabs(n1), std::llabs(n1 + mu - 1));
  const int64_t L = choose_grid_length(std::max<int64_t>(4 * K + 2, 2 * w));
  const double beta = 2.30 * w, alpha = M_PI * w / (double)L;
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

static size_t grid_bytes(const mci_offgrid_s* p, int64_t batch) {
  const size_t el = (p->prec == MCI_F64 ? 8 : 4) * (p->real_io ? 1 : 2);
  return ((size_t)batch * p->n_ops * p->L * el + 255) & ~(size_t)255;
}

mci_status mci_offgrid_workspace_size(mci_offgrid_t p, int64_t batch, size_t* bytes) {
  if (!p || !bytes || batch < 0) return fail(MCI_E_INVALID_ARG, "plan, bytes or batch");
  *bytes = grid_bytes(p, batch) + plan_workspace(p->grid, batch);
  return MCI_OK;
}

mci_status mci_evaluate_1d(mci_offgrid_t p, const void* g, const double* t, int64_t n_t, int32_t t_shared, void* y,
                           int64_t batch, void* workspace, size_t ws_bytes, hipStream_t stream) {
  if (!p) return fail(MCI_E_INVALID_ARG, "plan is NULL");
  if (batch < 0 || n_t < 0) return fail(MCI_E_INVALID_ARG, "batch and n_t must be >= 0");
  if (batch == 0 || n_t == 0) return MCI_OK;
  if (!g || !t || !y) return fail(MCI_E_INVALID_ARG, "NULL array");
  const size_t gb = grid_bytes(p, batch), need = gb + plan_workspace(p->grid, batch);
  if (!workspace || ws_bytes < need) return fail(MCI_E_INVALID_ARG, "workspace too small");
  if (hipSetDevice(p->device) != hipSuccess) return fail(MCI_E_DEVICE, "hipSetDevice");
  void* grid = workspace;
  void* inner = need > gb ? (void*)((char*)workspace + gb) : nullptr;
  mci_status st = plan_run(p->grid, g, grid, batch, inner, nullptr, stream);
  if (st != MCI_OK) return st;
  EvalArgs a{};
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
  const int64_t gx = (n_t + NT - 1) / NT;
  if (gx > 0x7fffffff) return fail(MCI_E_INVALID_ARG, "too many points");
  const dim3 grd((unsigned)gx, (unsigned)std::min<int64_t>(batch, 65535));
  if (p->prec == MCI_F64) {
    if (p->real_io) hipLaunchKernelGGL((k_eval<double, true>), grd, dim3(NT), 0, stream, a);
    else hipLaunchKernelGGL((k_eval<double, false>), grd, dim3(NT), 0, stream, a);
  } else {
    if (p->real_io) hipLaunchKernelGGL((k_eval<float, true>), grd, dim3(NT), 0, stream, a);
    else hipLaunchKernelGGL((k_eval<float, false>), grd, dim3(NT), 0, stream, a);
  }
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(MCI_E_DEVICE, std::string("off-grid evaluation: ") + hipGetErrorString(e));
  return MCI_OK;
}

}  // extern "C"
