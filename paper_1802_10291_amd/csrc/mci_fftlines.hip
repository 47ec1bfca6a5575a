// mci_fftlines.hip -- long FP32 transforms of the multi-pass path in one or two LDS passes.
//
// A length L = A B transform runs as the four-step factorisation: with n = a + A b and
// k = k_b + B k_a,
//   X[k_b + B k_a] = sum_a w_A^{a k_a} w_L^{a k_b} sum_b x[a + A b] w_B^{b k_b},
// so pass 1 takes the A lines {x[a + A b]}_b (length B), transforms them, multiplies by
// w_L^{a k_b} and writes Y[k_b A + a]; pass 2 takes the B contiguous lines {Y[k_b A + a]}_a
// (length A), transforms them and writes X[k_b + B k_a].  A workgroup transforms 16 lines
// with the register-staged line FFT; where the 16 lines are interleaved in memory (element
// stride > 1, line stride 1) they go through an LDS tile, so every global access is a run
// of 16 consecutive complex values.  A length that is itself a line length takes one pass.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "mci_fftlines.h"
#include "mci_linefft.h"

namespace mci {

namespace fl {

using namespace lfft;

constexpr int FL = 16;   // lines per workgroup

template <int N> constexpr int threads() { return FL * (N / LineFFT<N>::E); }

struct LinesArgs {
  const float2* in;
  float2* out;
  int64_t n_lines;          // count * U
  int64_t U;                // lines per transform
  int64_t sig_in, u_in, e_in;     // complex strides: transform, line, element
  int64_t sig_out, u_out, e_out;
  const float2* tw;         // N entries e^{-2 pi i k / N}
  const float2* twL;        // L entries e^{-2 pi i m / L} (pass 1 of two), or null
};

// IN_T / OUT_T: the 16 lines of the workgroup are interleaved (line stride 1, element stride
// e); they then share one transform and U is a multiple of 16.  Otherwise lines are rows
// (element stride 1).
template <int N, int S, bool IN_T, bool OUT_T>
__global__ __launch_bounds__(threads<N>()) void k_fft_lines(LinesArgs a) {
  constexpr int E = LineFFT<N>::E, G = N / E, NT = threads<N>();
  constexpr int TS = N + 1;
  extern __shared__ float2 sml[];
  const int tid = threadIdx.x;
  const int g = tid / G, l = tid % G;
  const int64_t t0 = (int64_t)blockIdx.x * FL;
  if constexpr (IN_T) {
    const int64_t sig = t0 / a.U, u0 = t0 - sig * a.U;
    const float2* base = a.in + sig * a.sig_in + u0;
    for (int e = tid; e < N * FL; e += NT) {
      const int n = e / FL, c = e % FL;
      sml[c * TS + n] = base[c + n * a.e_in];
    }
  } else {
    for (int e = tid; e < N * FL; e += NT) {
      const int c = e / N, n = e % N;
      const int64_t t = t0 + c;
      float2 v = make_float2(0.f, 0.f);
      if (t < a.n_lines) {
        const int64_t sig = t / a.U, u = t - sig * a.U;
        v = a.in[sig * a.sig_in + u * a.u_in + n];
      }
      sml[c * TS + n] = v;
    }
  }
  __syncthreads();
  float2 v[E];
#pragma unroll
  for (int c = 0; c < E; ++c) v[c] = sml[g * TS + l + G * c];
  // the tile and the scratch share LDS: the line FFT's first store waits on a barrier
  gfft<N, S>(sml + g * padded(N), l, v, a.tw);
  const int64_t t = t0 + g;
  const int64_t sig = t / a.U, u = t - sig * a.U;
  if (a.twL) {
#pragma unroll
    for (int c = 0; c < E; ++c) {
      float2 w = a.twL[u * (l + G * c)];
      if constexpr (S > 0) w.y = -w.y;
      v[c] = cmul(v[c], w);
    }
  }
  if constexpr (OUT_T) {
    constexpr int OS = FL + 1;
    __syncthreads();
#pragma unroll
    for (int c = 0; c < E; ++c) sml[(l + G * c) * OS + g] = v[c];
    __syncthreads();
    const int64_t sig0 = t0 / a.U, u0 = t0 - sig0 * a.U;
    float2* base = a.out + sig0 * a.sig_out + u0;
    for (int e = tid; e < N * FL; e += NT) {
      const int k = e / FL, c = e % FL;
      base[c + k * a.e_out] = sml[k * OS + c];
    }
  } else {
    if (t < a.n_lines) {
      float2* o = a.out + sig * a.sig_out + u * a.u_out;
#pragma unroll
      for (int c = 0; c < E; ++c) o[l + G * c] = v[c];
    }
  }
}

template <int N, bool IN_T, bool OUT_T>
constexpr size_t lds_bytes() {
  const size_t tile = (size_t)FL * (N + 1) * sizeof(float2);
  const size_t scratch = (size_t)FL * padded(N) * sizeof(float2);
  const size_t otile = OUT_T ? (size_t)N * (FL + 1) * sizeof(float2) : 0;
  return std::max(tile, std::max(scratch, otile));
}

template <int N, int S, bool IN_T, bool OUT_T>
static hipError_t launch(const LinesArgs& a, hipStream_t s, bool prep) {
  const size_t lds = lds_bytes<N, IN_T, OUT_T>();
  if (prep)
    return lds > 64 * 1024 ? hipFuncSetAttribute((const void*)k_fft_lines<N, S, IN_T, OUT_T>,
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds)
                           : hipSuccess;
  const dim3 grid((unsigned)((a.n_lines + FL - 1) / FL)), block(threads<N>());
  hipLaunchKernelGGL((k_fft_lines<N, S, IN_T, OUT_T>), grid, block, lds, s, a);
  return hipGetLastError();
}

// mode 0: rows in, rows out (one pass); 1: interleaved in and out (pass 1); 2: rows in,
// interleaved out (pass 2)
template <int S>
static hipError_t dispatch(int N, int mode, const LinesArgs& a, hipStream_t s, bool prep) {
#define MCI_FL(NN)                                                  \
  if (N == NN) {                                                    \
    if (mode == 0) return launch<NN, S, false, false>(a, s, prep);  \
    if (mode == 1) return launch<NN, S, true, true>(a, s, prep);    \
    return launch<NN, S, false, true>(a, s, prep);                  \
  }
  MCI_FL(32) MCI_FL(48) MCI_FL(64) MCI_FL(96) MCI_FL(128) MCI_FL(192) MCI_FL(256) MCI_FL(384) MCI_FL(512)
#undef MCI_FL
  return hipErrorInvalidValue;
}

static hipError_t run(int N, int S, int mode, const LinesArgs& a, hipStream_t s, bool prep) {
  return S < 0 ? dispatch<-1>(N, mode, a, s, prep) : dispatch<+1>(N, mode, a, s, prep);
}

}  // namespace fl

bool line_length_ok(int64_t n) {
  return n == 32 || n == 48 || n == 64 || n == 96 || n == 128 || n == 192 || n == 256 || n == 384 || n == 512;
}

bool two_pass_factors(int64_t L, int& A, int& B) {
  if (line_length_ok(L)) {
    A = 1;
    B = (int)L;
    return true;
  }
  A = B = 0;
  double best = 1e30;
  for (int a : {32, 48, 64, 96, 128, 192, 256, 384, 512}) {
    if (L % a || !line_length_ok(L / a)) continue;
    const double bal = std::fabs(std::log((double)a) - std::log((double)(L / a)));
    if (bal < best) {
      best = bal;
      A = a;
      B = (int)(L / a);
    }
  }
  return A > 0;
}

int64_t next_two_pass_length(int64_t n) {
  int64_t best = -1;
  for (int a : {1, 32, 48, 64, 96, 128, 192, 256, 384, 512})
    for (int b : {32, 48, 64, 96, 128, 192, 256, 384, 512}) {
      const int64_t m = (int64_t)a * b;
      if (m >= n && (best < 0 || m < best)) best = m;
    }
  return best;
}

hipError_t prepare_two_pass(int A, int B) {
  hipError_t e = hipSuccess;
  for (int S : {-1, +1}) {
    if (A == 1) {
      e = fl::run(B, S, 0, fl::LinesArgs{}, nullptr, true);
    } else {
      if ((e = fl::run(B, S, 1, fl::LinesArgs{}, nullptr, true)) != hipSuccess) return e;
      e = fl::run(A, S, 2, fl::LinesArgs{}, nullptr, true);
    }
    if (e != hipSuccess) return e;
  }
  return e;
}

hipError_t fft_two_pass(const float2* in, float2* out, float2* tmp, int64_t count, int A, int B, int sign,
                        const float2* twA, const float2* twB, const float2* twL, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  if (A == 1) {
    fl::LinesArgs a{in, out, count, 1, B, 0, 1, B, 0, 1, twB, nullptr};
    return fl::run(B, sign, 0, a, s, false);
  }
  const int64_t L = (int64_t)A * B;
  fl::LinesArgs p1{in, tmp, count * A, A, L, 1, A, L, 1, A, twB, twL};
  hipError_t e = fl::run(B, sign, 1, p1, s, false);
  if (e != hipSuccess) return e;
  fl::LinesArgs p2{tmp, out, count * B, B, L, A, 1, L, 1, B, twA, nullptr};
  return fl::run(A, sign, 2, p2, s, false);
}

}  // namespace mci
