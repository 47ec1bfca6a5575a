// mci_kernels.hip -- plan-building kernel (FP64) and the multi-pass 1-D path of libmci.
//
// The multi-pass path runs every step of the method as its own kernel over a workspace
// in HBM: (1) load + optional Bluestein pre-chirp, (2) Stockham FFT passes of each
// channel, (3) the per-residue M x M apply gathered straight into the output spectrum,
// (4) Stockham inverse passes of length n_out, (5) store (real part in real mode).  It
// handles every size the plan accepts; the fused single-pass kernels cover the large
// batched workloads.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "mci_device.h"
#include "mci_fftlines.h"
#include "mci_internal.h"

namespace mci {

// ================================================================= plan tables (FP64)
// For residue n = n1 + i of I_1 (Section 3): H_n[j][k] = b_k(n + j N) (eq. defH).  The
// system A_n H_n = D_n (eq. matrixeqn1) is solved through G = H_n^T, whose rows
// (channels) are first divided by their largest entry -- derivative channels grow like
// (M N)^k -- then inverted by Gauss-Jordan elimination with partial pivoting.  The
// kernel writes Tab[op][m][j][i] = q_mj(n) o_op(n + j N) / N, where q_mj(n) are the
// entries of H_n^{-1}, o_op is the output operator and 1/N is the factor of Lemma 3.1,
// so the apply step is a plain product with the raw channel DFTs.
__device__ inline double2 ipow_d(int64_t n, int q) {
  double mag = 1.0;
  for (int r = 0; r < q; ++r) mag *= (double)n;
  switch (q & 3) {
    case 0: return make_double2(mag, 0.0);
    case 1: return make_double2(0.0, mag);
    case 2: return make_double2(-mag, 0.0);
    default: return make_double2(0.0, -mag);
  }
}

__device__ inline double2 mult_d(const PlanKernelArgs& a, int k, int64_t n) {
  switch (a.kinds[k]) {
    case MCI_MULT_DERIV: return ipow_d(n, a.orders[k]);
    case MCI_MULT_HILBERT: return make_double2(0.0, n > 0 ? -1.0 : (n < 0 ? 1.0 : 0.0));
    default: {
      const int64_t mu = (int64_t)a.M * a.N;
      const int64_t off = n - a.n1;
      if (off < 0 || off >= mu) return make_double2(0.0, 0.0);
      return a.tables[(int64_t)k * mu + off];
    }
  }
}

__device__ inline double2 outop_d(int op, int order, int64_t n) {
  switch (op) {
    case MCI_OUT_IDENTITY: return make_double2(1.0, 0.0);
    case MCI_OUT_HILBERT: return make_double2(0.0, n > 0 ? -1.0 : (n < 0 ? 1.0 : 0.0));
    default: return ipow_d(n, order);
  }
}

__device__ inline double cabs_d(double2 z) { return sqrt(z.x * z.x + z.y * z.y); }
__device__ inline double2 cdiv_d(double2 a, double2 b) {
  const double den = b.x * b.x + b.y * b.y;
  return make_double2((a.x * b.x + a.y * b.y) / den, (a.y * b.x - a.x * b.y) / den);
}

__global__ void k_plan_tables(PlanKernelArgs a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.N) return;
  const int M = a.M;
  const int64_t n = a.n1 + i;
  double2 G[MCI_MAX_CHANNELS][MCI_MAX_CHANNELS], V[MCI_MAX_CHANNELS][MCI_MAX_CHANNELS];
  double rs[MCI_MAX_CHANNELS];
  bool singular = false;
  for (int k = 0; k < M; ++k) {
    double s = 0.0;
    for (int j = 0; j < M; ++j) {
      G[k][j] = mult_d(a, k, n + (int64_t)j * a.N);
      s = fmax(s, cabs_d(G[k][j]));
    }
    rs[k] = s;
    if (s == 0.0) singular = true;
  }
  double norm_g = 0.0, norm_v = 0.0;
  if (!singular) {
    for (int k = 0; k < M; ++k)
      for (int j = 0; j < M; ++j) {
        G[k][j].x /= rs[k];
        G[k][j].y /= rs[k];
        V[k][j] = make_double2(k == j ? 1.0 : 0.0, 0.0);
      }
    for (int j = 0; j < M; ++j) {
      double c = 0.0;
      for (int k = 0; k < M; ++k) c += cabs_d(G[k][j]);
      norm_g = fmax(norm_g, c);
    }
    // Gauss-Jordan: [G | I] -> [I | G^{-1}]
    for (int c = 0; c < M && !singular; ++c) {
      int piv = c;
      double best = cabs_d(G[c][c]);
      for (int r = c + 1; r < M; ++r) {
        const double v = cabs_d(G[r][c]);
        if (v > best) { best = v; piv = r; }
      }
      if (best <= 1e-13) { singular = true; break; }
      if (piv != c)
        for (int j = 0; j < M; ++j) {
          double2 t = G[c][j]; G[c][j] = G[piv][j]; G[piv][j] = t;
          t = V[c][j]; V[c][j] = V[piv][j]; V[piv][j] = t;
        }
      const double2 p = G[c][c];
      for (int j = 0; j < M; ++j) {
        G[c][j] = cdiv_d(G[c][j], p);
        V[c][j] = cdiv_d(V[c][j], p);
      }
      for (int r = 0; r < M; ++r) {
        if (r == c) continue;
        const double2 f = G[r][c];
        for (int j = 0; j < M; ++j) {
          G[r][j].x -= f.x * G[c][j].x - f.y * G[c][j].y;
          G[r][j].y -= f.x * G[c][j].y + f.y * G[c][j].x;
          V[r][j].x -= f.x * V[c][j].x - f.y * V[c][j].y;
          V[r][j].y -= f.x * V[c][j].y + f.y * V[c][j].x;
        }
      }
    }
    if (!singular)
      for (int j = 0; j < M; ++j) {
        double c = 0.0;
        for (int k = 0; k < M; ++k) c += cabs_d(V[k][j]);
        norm_v = fmax(norm_v, c);
      }
  }
  a.sing[i] = singular ? 1 : 0;
  a.cond[i] = singular ? 0.0 : norm_g * norm_v;
  const double invN = 1.0 / (double)a.N;
  for (int op = 0; op < a.n_ops; ++op)
    for (int m = 0; m < M; ++m)
      for (int j = 0; j < M; ++j) {
        double2 t = make_double2(0.0, 0.0);
        if (!singular) {
          // (G^{-1})[j][m] with the row scaling undone; q_mj(n) = (H_n^{-1})[m][j] = (G^{-1})[j][m]
          double2 q = V[j][m];
          q.x /= rs[m];
          q.y /= rs[m];
          const double2 o = outop_d(a.ops[op], a.op_orders[op], n + (int64_t)j * a.N);
          const double sc = a.oscale ? a.oscale[i + (int64_t)j * a.N] * invN : invN;
          t = make_double2((q.x * o.x - q.y * o.y) * sc, (q.x * o.y + q.y * o.x) * sc);
        }
        const int64_t idx = (((int64_t)op * M + m) * M + j) * a.N + i;
        a.tab64[idx] = t;
        a.tab32[idx] = make_float2((float)t.x, (float)t.y);
      }
  if (a.qraw)
    for (int m = 0; m < M; ++m)
      for (int j = 0; j < M; ++j) {
        double2 q = make_double2(0.0, 0.0);
        if (!singular) {
          q = V[j][m];
          q.x /= rs[m];
          q.y /= rs[m];
        }
        a.qraw[(i * M + m) * M + j] = q;
      }
}

hipError_t launch_plan_tables(const PlanKernelArgs& a, hipStream_t s) {
  const int bs = 128;
  const int64_t nb = (a.N + bs - 1) / bs;
  hipLaunchKernelGGL(k_plan_tables, dim3((unsigned)nb), dim3(bs), 0, s, a);
  return hipGetLastError();
}

// ================================================================= multi-pass 1-D path
static inline unsigned grid_for(int64_t total, int bs) {
  int64_t b = (total + bs - 1) / bs;
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(b, 1 << 20));
}

// (1) samples -> complex buffer of length L per channel (zero padded, pre-chirped)
//     Row t is channel t % rows of signal t / rows; with offs, signal b's samples start at
//     element offs[2 b] of g, otherwise the rows are dense.
template <typename T, typename St>
__global__ void k_load(const St* __restrict__ g, cx<T>* __restrict__ x, int64_t count, int64_t len, int64_t L,
                       int real_io, const cx<T>* __restrict__ chirp, const int64_t* __restrict__ offs, int rows) {
  const int64_t total = count * L;
  const int64_t cw = real_io ? 1 : 2;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t t = e / L, k = e - t * L;
    cx<T> v = cmake<cx<T>>((T)0, (T)0);
    if (k < len) {
      const int64_t row = offs ? offs[2 * (t / rows)] + (t % rows) * len * cw : t * len * cw;
      const int64_t src = row + k * cw;
      if (real_io) v.x = ld_as<T>(g, src);
      else { v.x = ld_as<T>(g, src); v.y = ld_as<T>(g, src + 1); }
      if (chirp) v = cmul(v, chirp[k]);
    }
    x[e] = v;
  }
}

// (2) one Stockham pass of radix R over `count` transforms of length len
template <typename T, int R, int S>
__global__ void k_fft_pass(const cx<T>* __restrict__ src, cx<T>* __restrict__ dst, int64_t len, int64_t Ns,
                           int64_t count, const cx<T>* __restrict__ tw) {
  const int64_t nb = len / R;
  const int64_t total = nb * count;
  const int64_t step = len / (Ns * R);
  for (int64_t gi = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; gi < total;
       gi += (int64_t)gridDim.x * blockDim.x) {
    const int64_t t = gi / nb, j = gi - t * nb;
    const cx<T>* s = src + t * len;
    cx<T>* d = dst + t * len;
    const int64_t k = j % Ns;
    cx<T> v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = s[j + r * nb];
    if (Ns > 1) {
#pragma unroll
      for (int r = 1; r < R; ++r) v[r] = cmul(v[r], twid<S>(tw, k * r * step));
    }
    dft_small<R, S>(v, tw, len);
    const int64_t base = (j / Ns) * Ns * R + k;
#pragma unroll
    for (int r = 0; r < R; ++r) d[base + r * Ns] = v[r];
  }
}

// Bluestein: multiply every transform by a fixed spectrum
template <typename T>
__global__ void k_pointwise(cx<T>* __restrict__ x, int64_t count, int64_t L, const cx<T>* __restrict__ h) {
  const int64_t total = count * L;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x)
    x[e] = cmul(x[e], h[e % L]);
}

// (3) apply + output operator + placement on the output grid, one thread per output bin.
// Band index k = n1 + i + j N (residue i, alias j) lands on bin k mod n_out; its value is
// sum_m d_m(n1 + i) Tab[op][m][j][i], with d_m read from the channel DFT at (n1 + i) mod N.
template <typename T>
__global__ void k_apply(const cx<T>* __restrict__ X, int64_t Lx, const cx<T>* __restrict__ post, const cx<T>* __restrict__ tab,
                        cx<T>* __restrict__ F, int64_t Lf, const cx<T>* __restrict__ pre_out, int M, int n_ops, int64_t N,
                        int64_t n1, int64_t n_out, int64_t batch) {
  const int64_t mu = (int64_t)M * N;
  const int64_t total = batch * n_ops * Lf;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t bin = e % Lf;
    const int64_t bo = e / Lf;
    const int op = (int)(bo % n_ops);
    const int64_t b = bo / n_ops;
    cx<T> acc = cmake<cx<T>>((T)0, (T)0);
    if (bin < n_out) {
      int64_t k = n1 + (((bin - n1) % n_out) + n_out) % n_out;
      for (; k < n1 + mu; k += n_out) {
        const int64_t off = k - n1;
        const int64_t j = off / N, i = off - j * N;
        const int64_t xi = (((n1 + i) % N) + N) % N;
        for (int m = 0; m < M; ++m) {
          cx<T> d = X[(b * M + m) * Lx + xi];
          if (post) d = cmul(d, post[xi]);
          acc = cadd(acc, cmul(d, tab[(((int64_t)op * M + m) * M + j) * N + i]));
        }
      }
      if (pre_out) acc = cmul(acc, pre_out[bin]);
    }
    F[e] = acc;
  }
}

// (5) output: real part (real mode) or complex, optional Bluestein post-chirp
//     Row t is output op t % rows of signal t / rows (signal b's outputs start at element
//     offs[2 b + 1] of y with offs, otherwise dense).
template <typename T, typename St>
__global__ void k_store(const cx<T>* __restrict__ F, int64_t Lf, St* __restrict__ y, int64_t count, int64_t n_out,
                        int real_io, const cx<T>* __restrict__ post, const int64_t* __restrict__ offs, int rows) {
  const int64_t total = count * n_out;
  const int64_t cw = real_io ? 1 : 2;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t t = e / n_out, j = e - t * n_out;
    cx<T> v = F[t * Lf + j];
    if (post) v = cmul(v, post[j]);
    const int64_t dst = (offs ? offs[2 * (t / rows) + 1] + (t % rows) * n_out * cw : t * n_out * cw) + j * cw;
    if (real_io) st_as<T>(y, dst, v.x);
    else { st_as<T>(y, dst, v.x); st_as<T>(y, dst + 1, v.y); }
  }
}

template <typename T, int S>
static hipError_t launch_pass(int R, const cx<T>* src, cx<T>* dst, int64_t len, int64_t Ns, int64_t count,
                              const cx<T>* tw, hipStream_t s) {
  const int bs = 256;
  const unsigned gr = grid_for(count * (len / R), bs);
  switch (R) {
    case 2: hipLaunchKernelGGL((k_fft_pass<T, 2, S>), dim3(gr), dim3(bs), 0, s, src, dst, len, Ns, count, tw); break;
    case 3: hipLaunchKernelGGL((k_fft_pass<T, 3, S>), dim3(gr), dim3(bs), 0, s, src, dst, len, Ns, count, tw); break;
    case 4: hipLaunchKernelGGL((k_fft_pass<T, 4, S>), dim3(gr), dim3(bs), 0, s, src, dst, len, Ns, count, tw); break;
    case 5: hipLaunchKernelGGL((k_fft_pass<T, 5, S>), dim3(gr), dim3(bs), 0, s, src, dst, len, Ns, count, tw); break;
    case 7: hipLaunchKernelGGL((k_fft_pass<T, 7, S>), dim3(gr), dim3(bs), 0, s, src, dst, len, Ns, count, tw); break;
    case 8: hipLaunchKernelGGL((k_fft_pass<T, 8, S>), dim3(gr), dim3(bs), 0, s, src, dst, len, Ns, count, tw); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Run all Stockham passes of one direction over buf[cur] (ping-pong with buf[1-cur]).
template <typename T, int S>
static hipError_t run_passes(cx<T>* buf[2], int& cur, int64_t count, int64_t len, const std::vector<int>& radices,
                             const cx<T>* tw, hipStream_t s) {
  int64_t Ns = 1;
  for (int R : radices) {
    hipError_t e = launch_pass<T, S>(R, buf[cur], buf[1 - cur], len, Ns, count, tw, s);
    if (e != hipSuccess) return e;
    cur = 1 - cur;
    Ns *= R;
  }
  return hipSuccess;
}

// One direction of a transform over buf[cur]: radix passes, or (FP32, two_pass) the one- or
// two-pass LDS transform, which leaves its result in buf[cur] with buf[1 - cur] as scratch.
template <typename T>
static hipError_t direction(const FftSide& f, int sign, cx<T>* buf[2], int& cur, int64_t count, hipStream_t s) {
  const cx<T>* tw = (const cx<T>*)f.tw;
  if constexpr (std::is_same<T, float>::value) {
    if (f.two_pass)
      return fft_two_pass(buf[cur], buf[cur], buf[1 - cur], count, f.fa, f.fb, sign, (const float2*)f.twA,
                          (const float2*)f.twB, (const float2*)f.twL, s);
  }
  if (sign < 0) return run_passes<T, -1>(buf, cur, count, f.lexec, f.radices, tw, s);
  return run_passes<T, +1>(buf, cur, count, f.lexec, f.radices, tw, s);
}

// A full DFT of one FftSide over buf[cur]; the input must already be loaded (and
// pre-chirped and zero padded for Bluestein).  Leaves the result in buf[cur] (before the
// Bluestein post-chirp, which the consumer applies).
template <typename T>
static hipError_t run_side(const FftSide& f, cx<T>* buf[2], int& cur, int64_t count, hipStream_t s) {
  hipError_t e;
  if (!f.blue) return direction<T>(f, f.sign, buf, cur, count, s);
  if ((e = direction<T>(f, -1, buf, cur, count, s)) != hipSuccess) return e;
  hipLaunchKernelGGL((k_pointwise<T>), dim3(grid_for(count * f.lexec, 256)), dim3(256), 0, s, buf[cur], count,
                     f.lexec, (const cx<T>*)f.bhat);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  return direction<T>(f, +1, buf, cur, count, s);
}

size_t generic_1d_workspace(const Generic1D& g, int prec, int64_t batch) {
  const size_t esz = prec == MCI_F64 ? sizeof(double2) : sizeof(float2);
  const size_t nx = (size_t)batch * g.M * g.fwd->lexec;
  const size_t nf = (size_t)batch * g.n_ops * g.inv->lexec;
  return (2 * nx + 2 * nf) * esz + 256;
}

template <typename T, typename St>
static hipError_t generic_1d_t(const Generic1D& g, const void* in, void* out, int64_t batch, void* ws,
                               const int64_t* offs, hipStream_t s) {
  const FftSide& fw = *g.fwd;
  const FftSide& iv = *g.inv;
  cx<T>* base = (cx<T>*)(((uintptr_t)ws + 255) & ~(uintptr_t)255);
  const int64_t nx = batch * g.M * fw.lexec;
  const int64_t nf = batch * g.n_ops * iv.lexec;
  cx<T>* X[2] = {base, base + nx};
  cx<T>* F[2] = {base + 2 * nx, base + 2 * nx + nf};
  const int bs = 256;
  hipError_t e;
  // (1) load
  hipLaunchKernelGGL((k_load<T, St>), dim3(grid_for(batch * g.M * fw.lexec, bs)), dim3(bs), 0, s, (const St*)in,
                     X[0], batch * g.M, g.N, fw.lexec, g.real_io, fw.blue ? (const cx<T>*)fw.chirp : nullptr, offs, g.M);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // (2) channel DFTs
  int cx_ = 0;
  if ((e = run_side<T>(fw, X, cx_, batch * g.M, s)) != hipSuccess) return e;
  // (3) apply + placement (+ pre-chirp of the output transform)
  hipLaunchKernelGGL((k_apply<T>), dim3(grid_for(nf, bs)), dim3(bs), 0, s, X[cx_], fw.lexec,
                     fw.blue ? (const cx<T>*)fw.chirp : nullptr, (const cx<T>*)g.tab, F[0], iv.lexec,
                     iv.blue ? (const cx<T>*)iv.chirp : nullptr, g.M, g.n_ops, g.N, g.n1, g.n_out, batch);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // (4) output transform
  int cf = 0;
  if ((e = run_side<T>(iv, F, cf, batch * g.n_ops, s)) != hipSuccess) return e;
  // (5) store
  hipLaunchKernelGGL((k_store<T, St>), dim3(grid_for(batch * g.n_ops * g.n_out, bs)), dim3(bs), 0, s, F[cf],
                     iv.lexec, (St*)out, batch * g.n_ops, g.n_out, g.real_io,
                     iv.blue ? (const cx<T>*)iv.chirp : nullptr, offs, g.n_ops);
  return hipGetLastError();
}

hipError_t run_generic_1d(const Generic1D& g, int prec, int store, const void* in, void* out, int64_t batch,
                          void* ws, const int64_t* offs, hipStream_t s) {
  if (prec == MCI_F64) return generic_1d_t<double, double>(g, in, out, batch, ws, offs, s);
  if (store == ST_F16) return generic_1d_t<float, __half>(g, in, out, batch, ws, offs, s);
  return generic_1d_t<float, float>(g, in, out, batch, ws, offs, s);
}

// ================================================================= 2-D helpers
// Channels of each line: the line itself, its centred difference (x[p+1] - x[p-1]) / (2h) and,
// with M = 3, its second difference (x[p+1] - 2 x[p] + x[p-1]) / h^2; h = 2 pi / len, circular.
// Output G[line][M][len] in the compute type.
template <typename T, typename St>
__global__ void k_fd_channels(const St* __restrict__ x, T* __restrict__ G, int64_t B, int64_t h, int64_t w,
                              int along_cols, const int64_t* __restrict__ offs, int M) {
  const int64_t len = along_cols ? h : w;
  const int64_t lines_per_img = along_cols ? w : h;
  const int64_t total = B * lines_per_img * len;
  const T sc = (T)((double)len / (4.0 * 3.14159265358979323846));
  const T sc2 = (T)(((double)len / (2.0 * 3.14159265358979323846)) * ((double)len / (2.0 * 3.14159265358979323846)));
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t p = e % len;
    const int64_t line = e / len;
    const int64_t b = line / lines_per_img, l = line - b * lines_per_img;
    const int64_t pn = (p + 1 == len) ? 0 : p + 1, pp = (p == 0) ? len - 1 : p - 1;
    T v, vn, vp;
    if (!along_cols) {
      const int64_t r0 = (offs ? offs[2 * b] : b * h * w) + l * w;
      v = ld_as<T>(x, r0 + p); vn = ld_as<T>(x, r0 + pn); vp = ld_as<T>(x, r0 + pp);
    } else {
      const int64_t c0 = (offs ? offs[2 * b] : b * h * w) + l;
      v = ld_as<T>(x, c0 + p * w); vn = ld_as<T>(x, c0 + pn * w); vp = ld_as<T>(x, c0 + pp * w);
    }
    G[(line * M) * len + p] = v;
    G[(line * M + 1) * len + p] = (vn - vp) * sc;
    if (M == 3) G[(line * M + 2) * len + p] = (vn - (T)2 * v + vp) * sc2;
  }
}

hipError_t launch_fd_channels(int prec, int store_in, const void* x, void* G, int64_t B, int64_t h, int64_t w,
                              int along_cols, const int64_t* offs, int M, hipStream_t s) {
  const int64_t total = B * h * w;
  const int bs = 256;
  if (prec == MCI_F64)
    hipLaunchKernelGGL((k_fd_channels<double, double>), dim3(grid_for(total, bs)), dim3(bs), 0, s,
                       (const double*)x, (double*)G, B, h, w, along_cols, offs, M);
  else if (store_in == ST_F16)
    hipLaunchKernelGGL((k_fd_channels<float, __half>), dim3(grid_for(total, bs)), dim3(bs), 0, s,
                       (const __half*)x, (float*)G, B, h, w, along_cols, offs, M);
  else
    hipLaunchKernelGGL((k_fd_channels<float, float>), dim3(grid_for(total, bs)), dim3(bs), 0, s,
                       (const float*)x, (float*)G, B, h, w, along_cols, offs, M);
  return hipGetLastError();
}

template <typename T, typename St>
__global__ void k_transpose_out(const T* __restrict__ src, St* __restrict__ dst, int64_t B, int64_t W, int64_t H,
                                const int64_t* __restrict__ offs) {
  const int64_t total = B * W * H;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = e % W;
    const int64_t r = (e / W) % H;
    const int64_t b = e / (W * H);
    st_as<T>(dst, (offs ? offs[2 * b + 1] : b * W * H) + r * W + c, src[(b * W + c) * H + r]);
  }
}

hipError_t launch_transpose_out(int prec, int store_out, const void* src, void* dst, int64_t B, int64_t W,
                                int64_t H, const int64_t* offs, hipStream_t s) {
  const int64_t total = B * W * H;
  const int bs = 256;
  if (prec == MCI_F64)
    hipLaunchKernelGGL((k_transpose_out<double, double>), dim3(grid_for(total, bs)), dim3(bs), 0, s,
                       (const double*)src, (double*)dst, B, W, H, offs);
  else if (store_out == ST_F16)
    hipLaunchKernelGGL((k_transpose_out<float, __half>), dim3(grid_for(total, bs)), dim3(bs), 0, s,
                       (const float*)src, (__half*)dst, B, W, H, offs);
  else
    hipLaunchKernelGGL((k_transpose_out<float, float>), dim3(grid_for(total, bs)), dim3(bs), 0, s,
                       (const float*)src, (float*)dst, B, W, H, offs);
  return hipGetLastError();
}

}  // namespace mci
