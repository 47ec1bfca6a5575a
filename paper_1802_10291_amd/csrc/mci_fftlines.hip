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
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cmath>

#include "mci_fftlines.h"
#include "mci_jobs.h"
#include "mci_linefft.h"

namespace mci {

namespace fl {

using namespace lfft;

constexpr int FL = 16;   // lines per workgroup

template <int N> constexpr int threads() { return FL * (N / LinesFFT<N>::E); }

// Where transform t of a side (input or output) starts, in complex elements: with a table,
// offs[2 (t / per) + side] / 2 + (t % per) tr (offs in real elements, even); else
// (t / per) sig + (t % per) tr.
struct Side {
  const int64_t* offs = nullptr;
  int side = 0;        // 0: input offsets, 1: output offsets
  int div = 2;         // real elements per addressed element: 2 complex, 1 real input
  int64_t per = 1, sig = 0, tr = 0;
  __device__ __forceinline__ int64_t base(int64_t t) const {
    const int64_t q = t / per, r = t - q * per;
    return offs ? offs[2 * q + side] / div + r * tr : q * sig + r * tr;
  }
};

struct LinesArgs {
  const float2* in;
  float2* out;
  int64_t n_lines;          // count * U
  int64_t U;                // lines per transform
  Side si, so;              // transform bases
  int64_t u_in, e_in;       // complex strides of a line and of its elements (input)
  int64_t u_out, e_out;     // (output)
  const float2* tw;         // N entries e^{-2 pi i k / N}
  const float2* twL;        // pass 1 of two: the two-level table of e^{-2 pi i m / L} (mci_fftlines.h), or null
  const float2* pre;        // input position p: p < len_in ? in * pre[p] : 0 (if pre), else in
  int64_t len_in;           // with pre or real input: positions at or beyond it read as zero
  const float2* post;       // output position k multiplied by post[k], or null
  int real_in;              // input holds real values: position p reads (in[p], 0)
  int in_half, out_half;    // input / output stored as FP16 (half2 pairs, or halves for real input)
  BandGen gen;              // GEN kernels: input position p of transform t is band_bin(gen, t, p)
  const float2* mid;        // MID kernels: the filter multiplying the spectrum between the two transforms
};

// input position p of the transform whose first element is element `base` of the input
__device__ __forceinline__ float2 load_in(const LinesArgs& a, int64_t base, int64_t p) {
  const int64_t q = base + p;
  if (a.real_in) {
    if (p >= a.len_in) return make_float2(0.f, 0.f);
    const float x = a.in_half ? __half2float(((const __half*)a.in)[q]) : ((const float*)a.in)[q];
    return a.pre ? make_float2(x * a.pre[p].x, x * a.pre[p].y) : make_float2(x, 0.f);
  }
  if (a.pre && p >= a.len_in) return make_float2(0.f, 0.f);
  const float2 v = a.in_half ? __half22float2(((const __half2*)a.in)[q]) : a.in[q];
  return a.pre ? cmul(v, a.pre[p]) : v;
}

__device__ __forceinline__ void store_out(const LinesArgs& a, int64_t q, float2 w) {
  if (a.out_half) ((__half2*)a.out)[q] = __float22half2_rn(w);
  else a.out[q] = w;
}

// IN_T / OUT_T: the 16 lines of the workgroup are interleaved (line stride 1, element stride
// e); they then share one transform and U is a multiple of 16.  Otherwise lines are rows
// (element stride 1).  Positions inside a transform: input u u_in + n e_in, output
// u u_out + k e_out.
template <int N, int S, bool IN_T, bool OUT_T, bool GEN, bool MID>
__device__ __forceinline__ void lines_body(const LinesArgs& a, int64_t bx) {
  constexpr int E = LinesFFT<N>::E, G = N / E, NT = threads<N>();
  constexpr int TS = N + 1;
  extern __shared__ float2 sml[];
  const int tid = threadIdx.x;
  const int g = tid / G, l = tid % G;
  const int64_t t0 = bx * FL;
  // plain complex input (no chirp, no real or FP16 storage): a bare load per element
  const bool plain = !a.real_in && !a.pre && !a.in_half;
  if constexpr (IN_T && GEN) {
    // the tile's 16 lines belong to one transform: positions u0 + c + n e_in
    const int64_t tr = t0 / a.U, u0 = t0 - tr * a.U;
#pragma unroll
    for (int e = tid; e < N * FL; e += NT) {
      const int n = e / FL, c = e % FL;
      sml[c * TS + n] = band_bin(a.gen, tr, (int)(u0 + c + n * a.e_in));
    }
  } else if constexpr (IN_T) {
    const int64_t tr = t0 / a.U, u0 = t0 - tr * a.U;
    const int64_t base = a.si.base(tr);
    if (plain && ((base + u0) & 1) == 0 && (a.e_in & 1) == 0 && ((uintptr_t)a.in & 15) == 0) {
      // two neighbouring lines' elements per float4 (u0 is a multiple of 16, so every pair
      // starts at an even element)
      for (int e2 = tid; e2 < N * FL / 2; e2 += NT) {
        const int n = e2 / (FL / 2), c = 2 * (e2 % (FL / 2));
        const float4 v = *(const float4*)(a.in + base + u0 + c + n * a.e_in);
        sml[c * TS + n] = make_float2(v.x, v.y);
        sml[(c + 1) * TS + n] = make_float2(v.z, v.w);
      }
    } else if (plain) {
      for (int e = tid; e < N * FL; e += NT) {
        const int n = e / FL, c = e % FL;
        sml[c * TS + n] = a.in[base + u0 + c + n * a.e_in];
      }
    } else {
      for (int e = tid; e < N * FL; e += NT) {
        const int n = e / FL, c = e % FL;
        sml[c * TS + n] = load_in(a, base, u0 + c + n * a.e_in);
      }
    }
  } else {
    // the 16 lines' transform bases and in-transform offsets, once per workgroup (the
    // divisions by U and by the side's lines per signal stay out of the element loop)
    __shared__ int64_t lbase[FL], lpos[FL];
    if (tid < FL) {
      const int64_t t = t0 + tid;
      int64_t b = -1, pos = 0;
      if (t < a.n_lines) {
        const int64_t tr = t / a.U, u = t - tr * a.U;
        b = GEN ? tr : a.si.base(tr);    // GEN: the transform index
        pos = u * a.u_in;
      }
      lbase[tid] = b;
      lpos[tid] = pos;
    }
    __syncthreads();
    for (int e = tid; e < N * FL; e += NT) {
      const int c = e / N, n = e % N;
      const int64_t b = lbase[c];
      float2 v = make_float2(0.f, 0.f);
      if constexpr (GEN) {
        if (b >= 0) v = band_bin(a.gen, b, (int)(lpos[c] + n));
      } else {
        if (b >= 0) v = plain ? a.in[b + lpos[c] + n] : load_in(a, b, lpos[c] + n);
      }
      sml[c * TS + n] = v;
    }
  }
  __syncthreads();
  float2 v[E];
#pragma unroll
  for (int c = 0; c < E; ++c) v[c] = sml[g * TS + l + G * c];
  // the tile and the scratch share LDS: the line FFT's first store waits on a barrier
  gfft<N, S, LinesFFT<N>>(sml + g * padded(N), l, v, a.tw);
  const int64_t t = t0 + g;
  const int64_t tr = t / a.U, u = t - tr * a.U;
  // MID: this is the last pass of a forward transform (factors A x B, line u = k_b, element
  // k = k_a); the spectrum is multiplied by the filter at its natural position k_b + B k_a and
  // the inverse transform (factors B x A) takes its first pass on the same line
  constexpr int ST = MID ? +1 : S;   // direction of the twiddles below
  if constexpr (MID) {
#pragma unroll
    for (int c = 0; c < E; ++c) v[c] = cmul(v[c], a.mid[u + a.U * (int64_t)(l + G * c)]);
    gfft<N, +1, LinesFFT<N>>(sml + g * padded(N), l, v, a.tw);
  }
  if (a.twL) {
#pragma unroll
    for (int c = 0; c < E; ++c) {
      const int m = (int)(u * (l + G * c));   // < L
      float2 w = cmul(a.twL[m & (int)(kTwLo - 1)], a.twL[kTwLo + (m >> kTwLoBits)]);
      if constexpr (ST > 0) w.y = -w.y;
      v[c] = cmul(v[c], w);
    }
  }
  if constexpr (OUT_T) {
    constexpr int OS = FL + 1;
    __syncthreads();
#pragma unroll
    for (int c = 0; c < E; ++c) sml[(l + G * c) * OS + g] = v[c];
    __syncthreads();
    const int64_t tr0 = t0 / a.U, u0 = t0 - tr0 * a.U;
    const int64_t base = a.so.base(tr0);
    if (!a.post && !a.out_half && ((base + u0) & 1) == 0 && (a.e_out & 1) == 0 && ((uintptr_t)a.out & 15) == 0) {
      // two neighbouring lines' outputs per float4 store
      for (int e2 = tid; e2 < N * FL / 2; e2 += NT) {
        const int k = e2 / (FL / 2), c = 2 * (e2 % (FL / 2));
        const float2 w0 = sml[k * OS + c], w1 = sml[k * OS + c + 1];
        *(float4*)(a.out + base + u0 + c + k * a.e_out) = make_float4(w0.x, w0.y, w1.x, w1.y);
      }
    } else {
      for (int e = tid; e < N * FL; e += NT) {
        const int k = e / FL, c = e % FL;
        const int64_t q = u0 + c + k * a.e_out;
        float2 w = sml[k * OS + c];
        if (a.post) w = cmul(w, a.post[q]);
        store_out(a, base + q, w);
      }
    }
  } else {
    if (t < a.n_lines) {
      const int64_t base = a.so.base(tr);
#pragma unroll
      for (int c = 0; c < E; ++c) {
        const int64_t q = u * a.u_out + l + G * c;
        store_out(a, base + q, a.post ? cmul(v[c], a.post[q]) : v[c]);
      }
    }
  }
}

template <int N, int S, bool IN_T, bool OUT_T, bool GEN, bool MID>
__global__ __launch_bounds__(threads<N>()) void k_fft_lines(LinesArgs a) {
  // the generating first pass: the blocks of one transform all read that signal's channel
  // spectra, so they go to one XCD, whose L2 then serves the re-reads
  lines_body<N, S, IN_T, OUT_T, GEN, MID>(a, GEN && IN_T ? xcd_block(blockIdx.x, gridDim.x) : (int64_t)blockIdx.x);
}

// merged form: one persistent launch over the jobs of an uneven batch
template <int N, int S, bool IN_T, bool OUT_T, bool GEN, bool MID>
__global__ __launch_bounds__(threads<N>()) void k_fft_lines_jobs(const LinesArgs* jobs, const JobGrid* grids,
                                                                 const int64_t* first, int n_jobs, int64_t total,
                                                                 JobBases b) {
  run_jobs(jobs, grids, first, n_jobs, total, [&](const LinesArgs& j, int64_t bx, int, int) {
    LinesArgs a = j;
    a.in = rebase(a.in, b);
    a.out = rebase(a.out, b);
    if constexpr (GEN) a.gen.Z = rebase(a.gen.Z, b);
    lines_body<N, S, IN_T, OUT_T, GEN, MID>(a, bx);
  });
}

template <int N, bool IN_T, bool OUT_T>
constexpr size_t lds_bytes() {
  const size_t tile = (size_t)FL * (N + 1) * sizeof(float2);
  const size_t scratch = (size_t)FL * padded(N) * sizeof(float2);
  const size_t otile = OUT_T ? (size_t)N * (FL + 1) * sizeof(float2) : 0;
  return std::max(tile, std::max(scratch, otile));
}

template <int N, int S, bool IN_T, bool OUT_T, bool GEN, bool MID>
static hipError_t launch_jobs(const MergedLaunch& m, const JobBases& b, hipStream_t s) {
  return merged_launch<LinesArgs>((const void*)k_fft_lines_jobs<N, S, IN_T, OUT_T, GEN, MID>, threads<N>(), m, b, s);
}
template <int N, int S, bool IN_T, bool OUT_T, bool GEN, bool MID>
static int occupancy_jobs(size_t lds) {
  return occupancy_of((const void*)k_fft_lines_jobs<N, S, IN_T, OUT_T, GEN, MID>, threads<N>(), lds);
}

template <int N, int S, bool IN_T, bool OUT_T, bool GEN, bool MID>
static hipError_t launch(const LinesArgs& a, hipStream_t s, bool prep) {
  const size_t lds = lds_bytes<N, IN_T, OUT_T>();
  if (prep) {
    if (lds <= 64 * 1024) return hipSuccess;
    hipError_t e = hipFuncSetAttribute((const void*)k_fft_lines<N, S, IN_T, OUT_T, GEN, MID>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute((const void*)k_fft_lines_jobs<N, S, IN_T, OUT_T, GEN, MID>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  }
  const int64_t blocks = (a.n_lines + FL - 1) / FL;
  if (job_recorder()) {
    record_job(launch_jobs<N, S, IN_T, OUT_T, GEN, MID>, occupancy_jobs<N, S, IN_T, OUT_T, GEN, MID>, a, blocks, 1, lds);
    return hipSuccess;
  }
  const dim3 grid((unsigned)blocks), block(threads<N>());
  hipLaunchKernelGGL((k_fft_lines<N, S, IN_T, OUT_T, GEN, MID>), grid, block, lds, s, a);
  return hipGetLastError();
}

// mode 0: rows in, rows out (one pass); 1: interleaved in and out (pass 1); 2: rows in,
// interleaved out (pass 2); 3: as 2, then the filter product and the inverse transform's first
// pass (forward direction only; the chirp convolution's middle).  gen: the input is computed by
// the band generator (inverse transforms of the real-mode path, modes 0 and 1).
template <int S>
static hipError_t dispatch(int N, int mode, bool gen, const LinesArgs& a, hipStream_t s, bool prep) {
#define MCI_FL(NN)                                                                                  \
  if (N == NN) {                                                                                    \
    if (gen && S > 0 && mode == 0) return launch<NN, S, false, false, (S > 0), false>(a, s, prep);  \
    if (gen && S > 0 && mode == 1) return launch<NN, S, true, true, (S > 0), false>(a, s, prep);    \
    if (gen) return hipErrorInvalidValue;                                                           \
    if (mode == 0) return launch<NN, S, false, false, false, false>(a, s, prep);                    \
    if (mode == 1) return launch<NN, S, true, true, false, false>(a, s, prep);                      \
    if (mode == 3) return S < 0 ? launch<NN, S, false, true, false, (S < 0)>(a, s, prep)            \
                                : hipErrorInvalidValue;                                             \
    return launch<NN, S, false, true, false, false>(a, s, prep);                                    \
  }
  MCI_FL(32) MCI_FL(48) MCI_FL(64) MCI_FL(96) MCI_FL(128) MCI_FL(192) MCI_FL(256) MCI_FL(384) MCI_FL(512)
#undef MCI_FL
  return hipErrorInvalidValue;
}

static hipError_t run(int N, int S, int mode, const LinesArgs& a, hipStream_t s, bool prep, bool gen = false) {
  return S < 0 ? dispatch<-1>(N, mode, gen, a, s, prep) : dispatch<+1>(N, mode, gen, a, s, prep);
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
  // between equally balanced factorisations the longer second pass (shorter first-pass lines)
  // wins: the first pass carries the twiddles and, in the real-mode path, the band generation,
  // and its smaller workgroups hide their latency better (an output transform of 131072 points
  // as 512 x 256 instead of 256 x 512: 0.204 -> 0.190 ms for its class, 65536 samples and M = 3)
  for (int a : {32, 48, 64, 96, 128, 192, 256, 384, 512}) {
    if (L % a || !line_length_ok(L / a)) continue;
    const double bal = std::fabs(std::log((double)a) - std::log((double)(L / a)));
    if (bal < best + 1e-9) {
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
      if (e == hipSuccess && S > 0) e = fl::run(B, S, 0, fl::LinesArgs{}, nullptr, true, true);
    } else {
      if ((e = fl::run(B, S, 1, fl::LinesArgs{}, nullptr, true)) != hipSuccess) return e;
      if (S > 0 && (e = fl::run(B, S, 1, fl::LinesArgs{}, nullptr, true, true)) != hipSuccess) return e;
      e = fl::run(A, S, 2, fl::LinesArgs{}, nullptr, true);
      if (e == hipSuccess && S < 0) e = fl::run(A, S, 3, fl::LinesArgs{}, nullptr, true);
    }
    if (e != hipSuccess) return e;
  }
  return e;
}

hipError_t fft_lines(const LineXform& x, hipStream_t s) {
  if (x.count <= 0) return hipSuccess;
  const int A = x.A, B = x.B;
  fl::Side si, so;
  si.offs = x.in_offs; si.side = 0; si.div = x.real_in ? 1 : 2; si.per = x.in_per; si.sig = x.in_sig; si.tr = x.in_tr;
  so.offs = x.out_offs; so.side = 1; so.per = x.out_per; so.sig = x.out_sig; so.tr = x.out_tr;
  const BandGen gen = x.gen ? *x.gen : BandGen{};
  if (A == 1) {
    fl::LinesArgs a{x.in, x.out, x.count, 1, si, so, 0, 1, 0, 1, x.twB, nullptr, x.pre, x.len_in, x.post, x.real_in,
                    x.in_half, x.out_half, gen};
    return fl::run(B, x.sign, 0, a, s, false, x.gen != nullptr);
  }
  const int64_t L = (int64_t)A * B;
  fl::Side dense;
  dense.per = 1; dense.sig = L;
  // pass 1: A lines x[a + A b] of length B, twiddled, to tmp[k_b A + a]
  fl::LinesArgs p1{x.in, x.tmp, x.count * A, A, si, dense, 1, A, 1, A, x.twB, x.twL, x.pre, x.len_in, nullptr,
                   x.real_in, x.in_half, 0, gen};
  hipError_t e = fl::run(B, x.sign, 1, p1, s, false, x.gen != nullptr);
  if (e != hipSuccess) return e;
  // pass 2: B contiguous lines tmp[k_b A + a] of length A, to out[k_b + B k_a]
  fl::LinesArgs p2{x.tmp, x.out, x.count * B, B, dense, so, A, 1, 1, B, x.twA, nullptr, nullptr, 0, x.post, 0, 0,
                   x.out_half, BandGen{}};
  return fl::run(A, x.sign, 2, p2, s, false);
}

hipError_t fft_chirp_conv(const LineXform& x, const float2* filt, float2* mid, hipStream_t s) {
  if (x.count <= 0) return hipSuccess;
  const int A = x.A, B = x.B;
  if (A == 1 || x.sign > 0 || x.gen || x.out_half) return hipErrorInvalidValue;
  fl::Side si, so;
  si.offs = x.in_offs; si.side = 0; si.div = x.real_in ? 1 : 2; si.per = x.in_per; si.sig = x.in_sig; si.tr = x.in_tr;
  so.offs = x.out_offs; so.side = 1; so.per = x.out_per; so.sig = x.out_sig; so.tr = x.out_tr;
  const int64_t L = (int64_t)A * B;
  fl::Side dense;
  dense.per = 1; dense.sig = L;
  // forward pass 1: A lines x[a + A b] of length B (x.pre applied as they load), twiddled, to tmp[k_b A + a]
  fl::LinesArgs p1{x.in, x.tmp, x.count * A, A, si, dense, 1, A, 1, A, x.twB, x.twL, x.pre, x.len_in, nullptr,
                   x.real_in, x.in_half, 0, BandGen{}};
  hipError_t e = fl::run(B, -1, 1, p1, s, false);
  if (e != hipSuccess) return e;
  // the middle: B contiguous lines tmp[k_b A + a] of length A, transformed (the forward
  // spectrum at k_b + B k_a), times filt there, inverse-transformed along the same line (the
  // inverse's first pass, factors B x A), twiddled by w_L^{+k_b k'}, to mid[k' B + k_b]
  fl::LinesArgs pm{x.tmp, mid, x.count * B, B, dense, dense, A, 1, 1, B, x.twA, x.twL, nullptr, 0, nullptr, 0, 0, 0,
                   BandGen{}, filt};
  if ((e = fl::run(A, -1, 3, pm, s, false)) != hipSuccess) return e;
  // inverse pass 2: A contiguous lines mid[k' B + a'] of length B, to out[k' + A k_a'] (x.post
  // applied as they store)
  fl::LinesArgs p2{mid, x.out, x.count * A, A, dense, so, B, 1, 1, A, x.twB, nullptr, nullptr, 0, x.post, 0, 0, 0,
                   BandGen{}};
  return fl::run(B, +1, 2, p2, s, false);
}

hipError_t fft_two_pass(const float2* in, float2* out, float2* tmp, int64_t count, int A, int B, int sign,
                        const float2* twA, const float2* twB, const float2* twL, hipStream_t s) {
  LineXform x;
  x.in = in; x.out = out; x.tmp = tmp; x.count = count; x.A = A; x.B = B; x.sign = sign;
  x.twA = twA; x.twB = twB; x.twL = twL;
  x.in_sig = x.out_sig = (int64_t)A * B;
  return fft_lines(x, s);
}

}  // namespace mci
