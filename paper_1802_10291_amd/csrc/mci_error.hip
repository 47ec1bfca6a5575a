// mci_error.hip -- the averaged approximation error of Theorem 4.4 for batches of signals
// under several candidate plans, and the plan of least error per signal.
//
// For a signal with Fourier coefficients a(n) (not necessarily in the band), the error of
// the approximation operator averaged over the sampling phase is (eq. averageerror)
//   eps^2 = sum_{n outside the band} |a(n)|^2 (1 + sum_{l=1..M} |sum_m r_m(n + (l - k) N) b_m(n)|^2),
// n in block I_k = [n1 + (k-1) N, n1 + k N).  The shifted index n + (l - k) N lies in block
// I_l at the residue of n, where r_m equals the inverse entry q_{m,l}, so the bracket is a
// weight w_c(n) of the plan c alone (w_c = 0 inside the band).  Over a batch of signals and
// a set of plans the error is then a product E[s][c] = sum_n |a_s(n)|^2 w_c(n): the weights
// are built once per call, and one streaming pass over the spectra accumulates every plan's
// sum.  The pass reads each coefficient once (8 bytes in FP32) for about 2 C + 3 flops, far
// below the ratio where arithmetic would bound it, so it is written for HBM bandwidth:
// coalesced row loads, several signals per workgroup sharing each weight load.
//
// The bound of eq. errorestimate has the same form with another weight: Cauchy-Schwarz on
// each |sum_m r_m b_m|^2 gives
//   eps^2 <= sum_{n outside the band} |a(n)|^2 (1 + M (sum_k Omega_k) sum_m |b_m(n)|^2),
// Omega_k = sup over the band of |r_k|^2 = the largest |q_{k,l}(n)|^2 over residues and
// blocks (the definition after Theorem 4.4 with eq. defrm).  A small kernel reduces each
// plan's sum_k Omega_k from the inverse table; the weight and reduction kernels then run as
// for the error itself.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "mci_plan.h"

namespace mci {
namespace err {

constexpr int MAX_PLANS = 16;
constexpr int NT = 256;

struct PlanRef {
  const double2* q;   // [N][M][M]: q_mj(n1 + i)
  int64_t N, n1;
  int M;
  int kinds[MCI_MAX_CHANNELS], orders[MCI_MAX_CHANNELS];
};

enum { Q_AVERAGED = 0, Q_BOUND = 1 };

struct ErrArgs {
  PlanRef plans[MAX_PLANS];
  int n_plans, cp;      // plans, and the padded count the weight table holds
  int quantity;         // Q_AVERAGED: eq. averageerror; Q_BOUND: eq. errorestimate
  int64_t n_lo, n_span, n_sig;
  const void* a;        // [n_sig][n_span] complex
  void* w;              // [cp][n_span] weights
  double* omsum;        // [MAX_PLANS] sum_k Omega_k per plan (Q_BOUND)
  double* eps;          // [n_sig][n_plans]
  int* best;            // [n_sig] or null
};

// sum_k Omega_k of plan blockIdx.x: per channel k the largest |q_{k,l}(n)|^2 over the
// residues n and blocks l, then the sum over k
__global__ __launch_bounds__(NT) void k_omega(ErrArgs a) {
  const PlanRef& p = a.plans[blockIdx.x];
  double mx[MCI_MAX_CHANNELS];
  for (int m = 0; m < MCI_MAX_CHANNELS; ++m) mx[m] = 0.0;
  const int64_t cnt = p.N * p.M * p.M;
  for (int64_t e = threadIdx.x; e < cnt; e += NT) {
    const int m = (int)((e / p.M) % p.M);   // [N][M][M]: row m, column l
    const double2 q = p.q[e];
    mx[m] = fmax(mx[m], q.x * q.x + q.y * q.y);
  }
  __shared__ double red[NT / 64][MCI_MAX_CHANNELS];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int m = 0; m < p.M; ++m) {
    double v = mx[m];
    for (int d = 32; d > 0; d >>= 1) v = fmax(v, __shfl_xor(v, d));
    if (lane == 0) red[wave][m] = v;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double sum = 0.0;
    for (int m = 0; m < p.M; ++m) {
      double v = red[0][m];
      for (int k = 1; k < NT / 64; ++k) v = fmax(v, red[k][m]);
      sum += v;
    }
    a.omsum[blockIdx.x] = sum;
  }
}

__device__ inline double2 mult_b(int kind, int order, int64_t n) {
  if (kind == MCI_MULT_HILBERT) return make_double2(0.0, n > 0 ? -1.0 : (n < 0 ? 1.0 : 0.0));
  double mag = 1.0;
  for (int r = 0; r < order; ++r) mag *= (double)n;
  switch (order & 3) {
    case 0: return make_double2(mag, 0.0);
    case 1: return make_double2(0.0, mag);
    case 2: return make_double2(-mag, 0.0);
    default: return make_double2(0.0, -mag);
  }
}

// w_c(n) in FP64, stored in the call's precision; rows c >= n_plans are zero
template <typename T>
__global__ __launch_bounds__(NT) void k_weights(ErrArgs a) {
  const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
  const int c = blockIdx.y;
  if (i >= a.n_span) return;
  T* w = (T*)a.w + (int64_t)c * a.n_span;
  if (c >= a.n_plans) {
    w[i] = T(0);
    return;
  }
  const PlanRef& p = a.plans[c];
  const int64_t n = a.n_lo + i;
  const int64_t off = n - p.n1;
  if (off >= 0 && off < p.M * p.N) {
    w[i] = T(0);
    return;
  }
  const int64_t res = ((off % p.N) + p.N) % p.N;
  double2 b[MCI_MAX_CHANNELS];
  for (int m = 0; m < p.M; ++m) b[m] = mult_b(p.kinds[m], p.orders[m], n);
  if (a.quantity == Q_BOUND) {
    double b2 = 0.0;
    for (int m = 0; m < p.M; ++m) b2 += b[m].x * b[m].x + b[m].y * b[m].y;
    w[i] = (T)(1.0 + p.M * a.omsum[c] * b2);
    return;
  }
  double acc = 1.0;
  for (int l = 0; l < p.M; ++l) {
    double sx = 0.0, sy = 0.0;
    for (int m = 0; m < p.M; ++m) {
      const double2 q = p.q[(res * p.M + m) * p.M + l];
      sx += q.x * b[m].x - q.y * b[m].y;
      sy += q.x * b[m].y + q.y * b[m].x;
    }
    acc += sx * sx + sy * sy;
  }
  w[i] = (T)acc;
}

// SB signals per workgroup, C weight rows (C >= n_plans, a power of two): every thread
// strides over n, keeps the C weights of its n in registers and accumulates |a_s(n)|^2 w_c(n)
// for the SB signals; the block then reduces the SB C partial sums.
template <typename T, int C, int SB>
__global__ __launch_bounds__(NT) void k_reduce(ErrArgs a) {
  using V = typename std::conditional<sizeof(T) == 4, float2, double2>::type;
  const int64_t s0 = (int64_t)blockIdx.x * SB;
  const int ns = (int)std::min<int64_t>(SB, a.n_sig - s0);
  const V* av = (const V*)a.a + s0 * a.n_span;
  const T* wt = (const T*)a.w;
  T acc[SB][C];
#pragma unroll
  for (int s = 0; s < SB; ++s)
#pragma unroll
    for (int c = 0; c < C; ++c) acc[s][c] = T(0);
  for (int64_t i = threadIdx.x; i < a.n_span; i += NT) {
    T w[C];
#pragma unroll
    for (int c = 0; c < C; ++c) w[c] = wt[c * a.n_span + i];
    V v[SB];
#pragma unroll
    for (int s = 0; s < SB; ++s) v[s] = s < ns ? av[s * a.n_span + i] : V{T(0), T(0)};
#pragma unroll
    for (int s = 0; s < SB; ++s) {
      const T p = v[s].x * v[s].x + v[s].y * v[s].y;
#pragma unroll
      for (int c = 0; c < C; ++c) acc[s][c] += p * w[c];
    }
  }
  __shared__ T red[NT / 64][SB * C];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int s = 0; s < SB; ++s)
#pragma unroll
    for (int c = 0; c < C; ++c) {
      T v = acc[s][c];
#pragma unroll
      for (int d = 32; d > 0; d >>= 1) v += __shfl_xor(v, d);
      if (lane == 0) red[wave][s * C + c] = v;
    }
  __syncthreads();
  const int t = threadIdx.x;
  if (t < SB * C) {
    const int s = t / C, c = t % C;
    if (s < ns && c < a.n_plans) {
      double sum = 0.0;
      for (int k = 0; k < NT / 64; ++k) sum += (double)red[k][t];
      a.eps[(s0 + s) * a.n_plans + c] = sqrt(sum);
    }
  }
  if (a.best) {
    __syncthreads();
    if (t < ns) {
      int bi = 0;
      double bv = 0.0;
      for (int c = 0; c < a.n_plans; ++c) {
        double sum = 0.0;
        for (int k = 0; k < NT / 64; ++k) sum += (double)red[k][t * C + c];
        if (c == 0 || sum < bv) { bv = sum; bi = c; }
      }
      a.best[s0 + t] = bi;
    }
  }
}

template <typename T>
static hipError_t launch(const ErrArgs& a, hipStream_t s) {
  if (a.quantity == Q_BOUND) hipLaunchKernelGGL(k_omega, dim3((unsigned)a.n_plans), dim3(NT), 0, s, a);
  hipLaunchKernelGGL(k_weights<T>, dim3((unsigned)((a.n_span + NT - 1) / NT), (unsigned)a.cp), dim3(NT), 0, s, a);
  const int64_t sb = a.cp <= 4 ? 8 : 4;
  const dim3 grid((unsigned)((a.n_sig + sb - 1) / sb));
  switch (a.cp) {
    case 1: hipLaunchKernelGGL((k_reduce<T, 1, 8>), grid, dim3(NT), 0, s, a); break;
    case 2: hipLaunchKernelGGL((k_reduce<T, 2, 8>), grid, dim3(NT), 0, s, a); break;
    case 4: hipLaunchKernelGGL((k_reduce<T, 4, 8>), grid, dim3(NT), 0, s, a); break;
    case 8: hipLaunchKernelGGL((k_reduce<T, 8, 4>), grid, dim3(NT), 0, s, a); break;
    default: hipLaunchKernelGGL((k_reduce<T, 16, 4>), grid, dim3(NT), 0, s, a); break;
  }
  return hipGetLastError();
}

static int padded(int n) {
  int c = 1;
  while (c < n) c <<= 1;
  return c;
}

// Workspace of mci_averaged_error_noalloc: a file-scope device array, one copy per GPU.  In
// host code its name is only a stand-in; the device address comes from hipGetSymbolAddress
// (once per device, with that device current) and only that address is passed on.
constexpr size_t kScratchBytes = (size_t)4 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 256;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices];

static mci_status scratch_address(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(MCI_E_INVALID_ARG, "device index");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    if (hipSetDevice(dev) != hipSuccess) return fail(MCI_E_DEVICE, "hipSetDevice");
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(MCI_E_DEVICE, std::string("scratch address: ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return MCI_OK;
}

}  // namespace err
}  // namespace mci

using namespace mci;
using namespace mci::err;

extern "C" {

mci_status mci_averaged_error_workspace_size(int32_t n_plans, int64_t n_span, int32_t precision, size_t* bytes) {
  if (!bytes || n_plans < 1 || n_plans > MAX_PLANS || n_span < 0) return fail(MCI_E_INVALID_ARG, "n_plans, n_span or bytes");
  if (precision != MCI_F32 && precision != MCI_F64) return fail(MCI_E_INVALID_ARG, "precision");
  // the weight table, then 256 bytes for the per-plan Omega sums of the bound
  *bytes = ((((size_t)padded(n_plans) * n_span * (precision == MCI_F64 ? 8 : 4)) + 255) & ~(size_t)255) + 256;
  return MCI_OK;
}

static mci_status error_call(int quantity, const mci_plan_t* plans, int32_t n_plans, const void* a, int64_t n_lo,
                             int64_t n_span, int64_t n_sig, int32_t precision, double* eps, int32_t* best,
                             void* workspace, size_t ws_bytes, hipStream_t stream) {
  if (!plans || n_plans < 1 || n_plans > MAX_PLANS) return fail(MCI_E_INVALID_ARG, "plans / n_plans (1..16)");
  if (precision != MCI_F32 && precision != MCI_F64) return fail(MCI_E_INVALID_ARG, "precision");
  if (n_span < 0 || n_sig < 0) return fail(MCI_E_INVALID_ARG, "n_span and n_sig must be >= 0");
  if (n_lo < -((int64_t)1 << 40) || n_lo > ((int64_t)1 << 40) || n_span > ((int64_t)1 << 40))
    return fail(MCI_E_INVALID_ARG, "coefficient range");
  ErrArgs ea{};
  int dev = -1;
  for (int c = 0; c < n_plans; ++c) {
    const mci_plan_s* p = plans[c];
    if (!p) return fail(MCI_E_INVALID_ARG, "NULL plan");
    if (p->dims != 1) return fail(MCI_E_INVALID_ARG, "averaged error takes 1-D plans");
    if (dev >= 0 && p->device != dev) return fail(MCI_E_INVALID_ARG, "plans on different devices");
    dev = p->device;
    if (p->n_sing) return fail(MCI_E_SINGULAR, "a plan has singular residues: eq. averageerror needs every H_n invertible");
    PlanRef& r = ea.plans[c];
    r.q = (const double2*)p->qdev;
    r.N = p->d.N;
    r.n1 = p->d.n1;
    r.M = p->d.M;
    for (int m = 0; m < r.M; ++m) {
      if (p->d.ch[m].kind == MCI_MULT_TABLE)
        return fail(MCI_E_UNSUPPORTED, "table channels give no multiplier outside the band");
      r.kinds[m] = p->d.ch[m].kind;
      r.orders[m] = p->d.ch[m].order;
    }
  }
  if (n_sig == 0 || n_span == 0) {
    if (n_sig > 0) return fail(MCI_E_INVALID_ARG, "n_span = 0 with signals: nothing defines their error");
    return MCI_OK;
  }
  if (!a || !eps || !workspace) return fail(MCI_E_INVALID_ARG, "NULL array");
  if (!aligned16(a) || !aligned16(workspace) || ((uintptr_t)eps & 7) || ((uintptr_t)best & 3))
    return fail(MCI_E_INVALID_ARG, "a and workspace must be 16-byte aligned");
  size_t need = 0;
  mci_status st = mci_averaged_error_workspace_size(n_plans, n_span, precision, &need);
  if (st != MCI_OK) return st;
  if (ws_bytes < need) return fail(MCI_E_INVALID_ARG, "workspace too small");
  if ((n_span + NT - 1) / NT > 0x7fffffff || (n_sig + 3) / 4 > 0x7fffffff) return fail(MCI_E_INVALID_ARG, "too large");
  if (hipSetDevice(dev) != hipSuccess) return fail(MCI_E_DEVICE, "hipSetDevice");
  ea.n_plans = n_plans;
  ea.cp = padded(n_plans);
  ea.n_lo = n_lo;
  ea.n_span = n_span;
  ea.n_sig = n_sig;
  ea.a = a;
  ea.w = workspace;
  ea.omsum = (double*)((char*)workspace + need - 256);
  ea.quantity = quantity;
  ea.eps = eps;
  ea.best = best;
  const hipError_t e = precision == MCI_F64 ? launch<double>(ea, stream) : launch<float>(ea, stream);
  if (e != hipSuccess) return fail(MCI_E_DEVICE, std::string("averaged error: ") + hipGetErrorString(e));
  return MCI_OK;
}

mci_status mci_averaged_error(const mci_plan_t* plans, int32_t n_plans, const void* a, int64_t n_lo, int64_t n_span,
                              int64_t n_sig, int32_t precision, double* eps, int32_t* best, void* workspace,
                              size_t ws_bytes, hipStream_t stream) {
  return error_call(Q_AVERAGED, plans, n_plans, a, n_lo, n_span, n_sig, precision, eps, best, workspace, ws_bytes,
                    stream);
}

mci_status mci_averaged_error_noalloc(const mci_plan_t* plans, int32_t n_plans, const void* a, int64_t n_lo,
                                      int64_t n_span, int64_t n_sig, int32_t precision, double* eps, int32_t* best,
                                      hipStream_t stream) {
  size_t need = 0;
  mci_status st = mci_averaged_error_workspace_size(n_plans, n_span, precision, &need);
  if (st != MCI_OK) return st;
  if (need > kScratchBytes)
    return fail(MCI_E_INVALID_ARG, "weight table of " + std::to_string(need) + " bytes exceeds the " +
                                       std::to_string(kScratchBytes) + "-byte static workspace (use mci_averaged_error)");
  if (!plans || !plans[0]) return fail(MCI_E_INVALID_ARG, "NULL plan");
  void* ws = nullptr;
  if ((st = scratch_address(plans[0]->device, &ws)) != MCI_OK) return st;
  return error_call(Q_AVERAGED, plans, n_plans, a, n_lo, n_span, n_sig, precision, eps, best, ws, kScratchBytes,
                    stream);
}

mci_status mci_error_bound(const mci_plan_t* plans, int32_t n_plans, const void* a, int64_t n_lo, int64_t n_span,
                           int64_t n_sig, int32_t precision, double* bound, void* workspace, size_t ws_bytes,
                           hipStream_t stream) {
  return error_call(Q_BOUND, plans, n_plans, a, n_lo, n_span, n_sig, precision, bound, nullptr, workspace, ws_bytes,
                    stream);
}

mci_status mci_plan_omega(mci_plan_t plan, double* omega, int32_t len) {
  if (!plan || !omega) return fail(MCI_E_INVALID_ARG, "NULL argument");
  if (plan->dims != 1 || !plan->qdev) return fail(MCI_E_INVALID_ARG, "Omega is defined for 1-D plans");
  const int M = plan->d.M;
  if (len < M) return fail(MCI_E_INVALID_ARG, "omega needs M entries");
  if (plan->n_sing) return fail(MCI_E_SINGULAR, "a plan with singular residues has no inverse everywhere");
  const int64_t cnt = plan->d.N * M * M;
  std::vector<double2> q((size_t)cnt);
  if (hipSetDevice(plan->device) != hipSuccess ||
      hipMemcpy(q.data(), plan->qdev, (size_t)cnt * sizeof(double2), hipMemcpyDeviceToHost) != hipSuccess)
    return fail(MCI_E_DEVICE, "inverse table readback");
  for (int m = 0; m < M; ++m) omega[m] = 0.0;
  for (int64_t e = 0; e < cnt; ++e) {
    const int m = (int)((e / M) % M);
    omega[m] = std::max(omega[m], q[e].x * q[e].x + q[e].y * q[e].y);
  }
  return MCI_OK;
}

}  // extern "C"
