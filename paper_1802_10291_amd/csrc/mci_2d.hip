// mci_2d.hip -- fused line-pass kernels for separable 2-D upsampling (Section 5.2).
//
// One pass reconstructs every line of length N (rows or columns) from the channels {x, Dx},
// Dx the circular centred difference (x[p+1] - x[p-1]) N / (4 pi) whose Fourier multiplier is
// fd(n) = i N sin(2 pi n / N) / (2 pi), with multipliers {1, i n} on the band [n1, n1 + 2N),
// and keeps the real part on the grid s times finer.  Composed, these steps are a real
// linear map that commutes with shifting the line by one sample (and the output by s):
//   a(k) = X(k mod N) G(k),  G(n + jN) = Tab[0][j][i] + fd(n) Tab[1][j][i]   (eq. matrixeqn1),
//   S(k) = (a(k) + conj a(-k)) / 2 = X(k mod N) Wr(k),  Wr(k) = (G(k) + conj G(-k)) / 2,
// with X the DFT of the line.  Splitting the output into its s polyphase components,
//   y[s q + r] = sum_k S(k) e^{2 pi i k (s q + r) / (s N)} = IDFT_N(X H_r)[q],
//   H_r[k'] = sum_{k = k' mod N} Wr(k) e^{2 pi i k r / (s N)},
// so a pass is one length-N DFT, s products with fixed windows H_r and s inverse DFTs.  The
// windows are built at plan time in FP64 from the FP64 per-residue inverses.  The map is
// complex-linear, so two real lines a, b go through it together as z = a + i b: Re of the
// result is line a upsampled, Im is line b.
//
// A workgroup takes 32 lines (16 pairs); lanes are grouped G = N / 16 per pair and hold 16
// elements each (element l + G c in lane l).  Both transforms are two Stockham passes.
// Columns run first (input and output go through LDS tiles so global accesses stay
// row-contiguous), rows last (the output rows leave straight from registers as s-float
// vectors, G lanes covering 128 contiguous bytes).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <type_traits>
#include <complex>
#include <vector>

#include "mci_2d.h"
#include "mci_device.h"
#include "mci_host_util.h"
#include "mci_jobs.h"
#include "mci_linefft.h"

namespace mci {

namespace l2d {

constexpr int LINES = 32;   // lines per workgroup
constexpr int PAIRS = 16;

using namespace lfft;

// the images are read once and the upsampled rows written once: non-temporal accesses
// (the column-to-row intermediate keeps ordinary ones, the row pass reads it back)
typedef float f2_nt __attribute__((ext_vector_type(2)));
typedef float f4_nt __attribute__((ext_vector_type(4)));

template <int N> constexpr int line_threads() { return PAIRS * (N / LineFFT<N>::E); }
// output row blocks that go through the LDS tile in the columns pass
template <int N, int SC> constexpr int out_parts() { return SC * N > 1024 ? 4 : 2; }

template <int N, int SC, bool COLS, bool ZR, typename TI, typename TO>
__device__ __forceinline__ void line_pass_body(const LinePassArgs& a, int64_t bx, int by) {
  constexpr int E = LineFFT<N>::E, G = N / E, NT = line_threads<N>();
  // ZR: the columns pass leaves out polyphase row 0 (it equals the input), the rows pass
  // takes those lines from the input image
  constexpr int R0 = ZR && COLS ? 1 : 0;   // first polyphase component computed
  constexpr int SR = SC - R0;              // output rows written per q (columns pass)
  extern __shared__ float2 sm2[];
  float* tile = (float*)sm2;                   // input [32][N + 1] floats
  float* otile = (float*)sm2;                  // output block [SC N / OP][32 + 1] floats (columns)
  const int tid = threadIdx.x;
  const int g = tid / G, l = tid % G;          // pair g = lines 2g, 2g + 1
  float2* buf = sm2 + g * padded(N);           // FFT scratch of pair g
  constexpr int TS = N + 1;
  const TI* x = (const TI*)a.x;
  TO* y = (TO*)a.y;
  int64_t line0;
  int64_t img = 0, col0 = 0;
  if constexpr (COLS) {
    col0 = bx * LINES;
    img = by;
  } else {
    line0 = bx * LINES;
  }
  // ---- load 32 lines into the tile (line-major)
  const int64_t xoff = COLS ? (a.offs ? a.offs[2 * img] : img * N * (int64_t)a.W) : 0;
  // FP32 inputs are read as float4 where the rows allow it (N is a multiple of 16, so four
  // consecutive values of a row segment never straddle a line or the image's last column
  // when W is a multiple of 4)
  if constexpr (COLS) {
    // row n of image img, columns col0 .. col0 + 31: 32 contiguous values per row
    // (FP16 inputs likewise as four halves in 8 bytes)
    bool vec = false;
    if constexpr (std::is_same<TI, float>::value) vec = ((xoff | a.W) & 3) == 0 && ((uintptr_t)x & 15) == 0;
    else vec = ((xoff | a.W) & 3) == 0 && ((uintptr_t)x & 7) == 0;
    if (vec) {
      for (int e4 = tid; e4 < N * LINES / 4; e4 += NT) {
        const int n = e4 / (LINES / 4), c = 4 * (e4 % (LINES / 4));
        const int64_t col = col0 + c;
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (col < a.W) {
          if constexpr (std::is_same<TI, float>::value) {
            // read once (non-temporal), or kept for the rows pass, which reads the sample rows again
            const f4_nt* src = (const f4_nt*)((const float*)x + xoff + n * (int64_t)a.W + col);
            const f4_nt t = ZR ? *src : __builtin_nontemporal_load(src);
            v = make_float4(t.x, t.y, t.z, t.w);
          } else {
            const uint2 raw = *(const uint2*)((const TI*)x + xoff + n * (int64_t)a.W + col);
            const float2 lo = __half22float2(*(const __half2*)&raw.x), hi = __half22float2(*(const __half2*)&raw.y);
            v = make_float4(lo.x, lo.y, hi.x, hi.y);
          }
        }
        tile[c * TS + n] = v.x;
        tile[(c + 1) * TS + n] = v.y;
        tile[(c + 2) * TS + n] = v.z;
        tile[(c + 3) * TS + n] = v.w;
      }
    } else {
      for (int e = tid; e < N * LINES; e += NT) {
        const int n = e / LINES, c = e % LINES;
        const int64_t col = col0 + c;
        float v = 0.f;
        if (col < a.W) v = ld_as<float>(x, xoff + n * (int64_t)a.W + col);
        tile[c * TS + n] = v;
      }
    }
  } else if constexpr (ZR) {
    // line s q + r of image b: row q of the input image for r = 0, else row (s - 1) q + r - 1
    // of image b's packed intermediate.  The block's lines span at most two images
    // (lines_per_img = s h >= 64 > 32): their bases are block-uniform, and the per-line
    // choice is a select between them, so the loads stay branch-free and pipelined.
    const int lpi = (int)a.lines_per_img, hh = lpi / SC;
    const int64_t b0 = line0 / lpi;
    const int R0l = (int)(line0 - b0 * lpi);
    const float* in_b[2];
    const float* mid_b[2];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int64_t b = b0 + j;
      const int64_t bc = b < a.lines / lpi ? b : a.lines / lpi - 1;   // the block may end in image b0
      in_b[j] = (const float*)a.x0 + (a.offs ? a.offs[2 * bc] : bc * hh * N);
      mid_b[j] = (const float*)x + b * hh * (SC - 1) * (int64_t)N;
    }
    const bool vec = (((uintptr_t)in_b[0] | (uintptr_t)in_b[1] | (uintptr_t)x) & 15) == 0;
    auto src = [&](int c) -> const float* {
      int R = R0l + c;
      const int j = R >= lpi ? 1 : 0;
      R -= j * lpi;
      const int q = R / SC, r = R - q * SC;
      return r == 0 ? in_b[j] + q * N : mid_b[j] + (q * (SC - 1) + r - 1) * N;
    };
    if (vec) {
      for (int e4 = tid; e4 < N * LINES / 4; e4 += NT) {
        const int c = (4 * e4) / N, n = (4 * e4) % N;
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (line0 + c < a.lines) v = *(const float4*)(src(c) + n);
        tile[c * TS + n] = v.x;
        tile[c * TS + n + 1] = v.y;
        tile[c * TS + n + 2] = v.z;
        tile[c * TS + n + 3] = v.w;
      }
    } else {
      for (int e = tid; e < N * LINES; e += NT) {
        const int c = e / N, n = e % N;
        float v = 0.f;
        if (line0 + c < a.lines) v = src(c)[n];
        tile[c * TS + n] = v;
      }
    }
  } else if constexpr (std::is_same<TI, float>::value) {
    // 32 consecutive lines of the intermediate are one contiguous block
    const float4* x4 = (const float4*)((const float*)x + line0 * N);
    for (int e4 = tid; e4 < N * LINES / 4; e4 += NT) {
      const int c = (4 * e4) / N, n = (4 * e4) % N;
      float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
      if (line0 + c < a.lines) v = x4[e4];
      tile[c * TS + n] = v.x;
      tile[c * TS + n + 1] = v.y;
      tile[c * TS + n + 2] = v.z;
      tile[c * TS + n + 3] = v.w;
    }
  } else {
    for (int e = tid; e < N * LINES; e += NT) {
      const int c = e / N, n = e % N;
      const int64_t line = line0 + c;
      float v = 0.f;
      if (line < a.lines) v = ld_as<float>(x, line * N + n);
      tile[c * TS + n] = v;
    }
  }
  __syncthreads();
  float2 z[E];
#pragma unroll
  for (int c = 0; c < E; ++c) {
    const int n = l + G * c;
    z[c] = make_float2(tile[(2 * g) * TS + n], tile[(2 * g + 1) * TS + n]);
  }
  // the tile and the scratch share LDS: gfft's first store waits on a barrier
  gfft<N, -1>(buf, l, z, a.tw);
  float2 out[SC][E];
#pragma unroll
  for (int r = R0; r < SC; ++r) {
    float2 v[E];
#pragma unroll
    for (int c = 0; c < E; ++c) v[c] = cmul(z[c], a.H[r * N + l + G * c]);
    gfft<N, +1>(buf, l, v, a.tw);
#pragma unroll
    for (int c = 0; c < E; ++c) out[r][c] = v[c];
  }
  if constexpr (!COLS) {
    // rows: line 2g gets Re, line 2g + 1 gets Im; SC consecutive outputs per q
#pragma unroll
    for (int h2 = 0; h2 < 2; ++h2) {
      const int64_t line = line0 + 2 * g + h2;
      if (line >= a.lines) continue;
      TO* yl = y + (a.offs ? a.offs[2 * (line / a.lines_per_img) + 1] + (line % a.lines_per_img) * (int64_t)(SC * N)
                           : line * (int64_t)(SC * N));
#pragma unroll
      for (int c = 0; c < E; ++c) {
        const int q = l + G * c;
        float o[SC];
#pragma unroll
        for (int r = 0; r < SC; ++r) o[r] = h2 ? out[r][c].y : out[r][c].x;
        if constexpr (std::is_same<TO, float>::value && SC == 4) {
          const f4_nt t = {o[0], o[1], o[2], o[3]};
          __builtin_nontemporal_store(t, (f4_nt*)(yl + 4 * q));
        } else if constexpr (std::is_same<TO, float>::value && SC == 2) {
          const f2_nt t = {o[0], o[1]};
          __builtin_nontemporal_store(t, (f2_nt*)(yl + 2 * q));
        } else if constexpr (std::is_same<TO, __half>::value && SC == 4) {
          // FP16 rows: the s outputs of a position as one 8-byte (s = 4) or 4-byte (s = 2) store
          const __half2 h0 = __floats2half2_rn(o[0], o[1]), h1 = __floats2half2_rn(o[2], o[3]);
          uint2 raw;
          __builtin_memcpy(&raw.x, &h0, 4);
          __builtin_memcpy(&raw.y, &h1, 4);
          *(uint2*)(yl + 4 * q) = raw;
        } else if constexpr (std::is_same<TO, __half>::value && SC == 2) {
          *(__half2*)(yl + 2 * q) = __floats2half2_rn(o[0], o[1]);
        } else {
#pragma unroll
          for (int r = 0; r < SC; ++r) st_as<float>(yl, (int64_t)SC * q + r, o[r]);
        }
      }
    }
  } else {
    // columns: output rows SC q + r; OP blocks of q (element c of a lane is q = l + G c, so
    // block p holds c in [p E / OP, (p + 1) E / OP)) through an LDS tile
    constexpr int OT = LINES + 1;
    constexpr int OP = out_parts<N, SC>();
    static_assert(E % OP == 0, "output blocks must split the elements per lane");
#pragma unroll
    for (int part = 0; part < OP; ++part) {
      __syncthreads();
#pragma unroll
      for (int c = part * (E / OP); c < (part + 1) * (E / OP); ++c) {
        const int q = l + G * c;
#pragma unroll
        for (int r = R0; r < SC; ++r) {
          const int row = SR * q + (r - R0) - part * (SR * N / OP);
          otile[row * OT + 2 * g] = out[r][c].x;
          otile[row * OT + 2 * g + 1] = out[r][c].y;
        }
      }
      __syncthreads();
      if ((a.W & 3) == 0 && ((uintptr_t)y & 15) == 0) {
        // four consecutive columns of an output row per float4 store
        for (int e4 = tid; e4 < (SR * N / OP) * LINES / 4; e4 += NT) {
          const int row = e4 / (LINES / 4), c = 4 * (e4 % (LINES / 4));
          const int64_t col = col0 + c;
          if (col < a.W)
            *(float4*)((float*)y + (img * (SR * N) + part * (SR * N / OP) + row) * (int64_t)a.W + col) =
                make_float4(otile[row * OT + c], otile[row * OT + c + 1], otile[row * OT + c + 2],
                            otile[row * OT + c + 3]);
        }
      } else {
        for (int e = tid; e < (SR * N / OP) * LINES; e += NT) {
          const int row = e / LINES, c = e % LINES;
          const int64_t col = col0 + c;
          if (col < a.W)
            st_as<float>(y, (img * (SR * N) + part * (SR * N / OP) + row) * (int64_t)a.W + col, otile[row * OT + c]);
        }
      }
    }
  }
}

template <int N, int SC, bool COLS, bool ZR, typename TI, typename TO>
__global__ __launch_bounds__(line_threads<N>()) void k_line_pass(LinePassArgs a) {
  line_pass_body<N, SC, COLS, ZR, TI, TO>(a, blockIdx.x, blockIdx.y);
}

// merged form: one persistent launch over the jobs of an uneven batch
template <int N, int SC, bool COLS, bool ZR, typename TI, typename TO>
__global__ __launch_bounds__(line_threads<N>()) void k_line_pass_jobs(const LinePassArgs* jobs, const JobGrid* grids,
                                                                      const int64_t* first, int n_jobs, int64_t total,
                                                                      JobBases b) {
  run_jobs(jobs, grids, first, n_jobs, total, [&](const LinePassArgs& j, int64_t bx, int by, int) {
    LinePassArgs a = j;
    a.x = rebase(a.x, b);
    a.y = rebase(a.y, b);
    a.x0 = rebase(a.x0, b);
    line_pass_body<N, SC, COLS, ZR, TI, TO>(a, bx, by);
  });
}

template <int N, int SC, bool COLS, bool ZR, typename TI, typename TO>
static hipError_t launch_jobs(const MergedLaunch& m, const JobBases& b, hipStream_t s) {
  return merged_launch<LinePassArgs>((const void*)k_line_pass_jobs<N, SC, COLS, ZR, TI, TO>, line_threads<N>(), m, b, s);
}
template <int N, int SC, bool COLS, bool ZR, typename TI, typename TO>
static int occupancy_jobs(size_t lds) {
  return occupancy_of((const void*)k_line_pass_jobs<N, SC, COLS, ZR, TI, TO>, line_threads<N>(), lds);
}

template <int N, int SC, bool COLS>
static size_t lds_bytes() {
  const size_t tile = (size_t)LINES * (N + 1) * sizeof(float);
  const size_t scratch = (size_t)PAIRS * padded(N) * sizeof(float2);
  const size_t otile = COLS ? (size_t)(SC * N / out_parts<N, SC>()) * (LINES + 1) * sizeof(float) : 0;
  return std::max(tile, std::max(scratch, otile));
}

template <int N, int SC, bool COLS, bool ZR, typename TI, typename TO>
static hipError_t launch(const LinePassArgs& a, int64_t images, hipStream_t s) {
  dim3 grid;
  if constexpr (COLS) grid = dim3((unsigned)((a.W + LINES - 1) / LINES), (unsigned)images);
  else grid = dim3((unsigned)((a.lines + LINES - 1) / LINES));
  const size_t lds = lds_bytes<N, SC, COLS>();
  if (job_recorder()) {
    record_job(launch_jobs<N, SC, COLS, ZR, TI, TO>, occupancy_jobs<N, SC, COLS, ZR, TI, TO>, a, grid.x, (int)grid.y, lds);
    return hipSuccess;
  }
  const dim3 block(line_threads<N>());
  hipLaunchKernelGGL((k_line_pass<N, SC, COLS, ZR, TI, TO>), grid, block, lds, s, a);
  return hipGetLastError();
}

// raise the dynamic-LDS limit of a kernel that needs more than 64 KB (at plan time)
template <int N, int SC, bool COLS, bool ZR, typename TI, typename TO>
static hipError_t prepare(const LinePassArgs&, int64_t, hipStream_t) {
  const size_t lds = lds_bytes<N, SC, COLS>();
  if (lds <= 64 * 1024) return hipSuccess;
  hipError_t e = hipFuncSetAttribute((const void*)k_line_pass<N, SC, COLS, ZR, TI, TO>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void*)k_line_pass_jobs<N, SC, COLS, ZR, TI, TO>,
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

template <bool COLS, bool ZR, typename TI, typename TO>
static hipError_t dispatch(int N, int SC, const LinePassArgs& a, int64_t images, hipStream_t s, bool prep) {
#define MCI_LP(NN, SS)                                                                  \
  if (N == NN && SC == SS)                                                              \
    return prep ? prepare<NN, SS, COLS, ZR, TI, TO>(a, images, s) : launch<NN, SS, COLS, ZR, TI, TO>(a, images, s);
  MCI_LP(32, 2) MCI_LP(32, 3) MCI_LP(32, 4) MCI_LP(48, 2) MCI_LP(48, 3) MCI_LP(48, 4) MCI_LP(64, 2) MCI_LP(64, 3)
  MCI_LP(64, 4) MCI_LP(96, 2) MCI_LP(96, 3) MCI_LP(96, 4) MCI_LP(128, 2) MCI_LP(128, 3) MCI_LP(128, 4)
  MCI_LP(192, 2) MCI_LP(192, 3) MCI_LP(192, 4) MCI_LP(256, 2) MCI_LP(256, 3) MCI_LP(256, 4) MCI_LP(384, 2)
  MCI_LP(384, 3) MCI_LP(384, 4) MCI_LP(512, 2) MCI_LP(512, 3) MCI_LP(512, 4)
#undef MCI_LP
  return hipErrorInvalidValue;
}

}  // namespace l2d

bool line_pass_supported(int N, int SC) {
  const bool n_ok = N == 32 || N == 48 || N == 64 || N == 96 || N == 128 || N == 192 || N == 256 || N == 384 || N == 512;
  return n_ok && (SC == 2 || SC == 3 || SC == 4);
}

// Polyphase windows of one axis from the FP64 apply table Tab[M][M][N] (identity output,
// channels {x, Dx} or {x, Dx, D2x}, multipliers {1, i n, (i n)^2}).  Channel m of a line is
// the line filtered by its difference operator, whose Fourier multiplier at n (theta =
// 2 pi n / N) is 1, fd(n) = i N sin(theta) / (2 pi) or fd2(n) = (2 cos(theta) - 2) (N / 2 pi)^2,
// so a(n + jN) = X(n) G(n + jN) with G(n + jN) = sum_m mult_m(n) Tab[m][j][i].  Returns
// H[SC][N] (FP64).
std::vector<std::complex<double>> line_windows(const std::vector<std::complex<double>>& tab, int64_t N, int64_t n1,
                                               int SC, int M) {
  using C = std::complex<double>;
  const int64_t mu = (int64_t)M * N;
  const int64_t K = std::max<int64_t>(std::llabs(n1), std::llabs(n1 + mu - 1));
  std::vector<C> G(2 * K + 1, 0.0);  // G(k), k = -K..K, zero outside the band
  const double sN = (double)N / (2.0 * M_PI);
  for (int64_t i = 0; i < N; ++i) {
    const int64_t n = n1 + i;
    const double th = 2.0 * M_PI * (double)(((n % N) + N) % N) / (double)N;
    const C mult[3] = {C(1.0, 0.0), C(0.0, sN * std::sin(th)), C((2.0 * std::cos(th) - 2.0) * sN * sN, 0.0)};
    for (int j = 0; j < M; ++j) {
      const int64_t k = n + j * N;
      C g = 0.0;
      for (int m = 0; m < M; ++m) g += mult[m] * tab[((size_t)m * M + j) * N + i];
      G[k + K] = g;
    }
  }
  std::vector<C> H((size_t)SC * N, 0.0);
  for (int64_t k = -K; k <= K; ++k) {
    const C wr = 0.5 * (G[k + K] + std::conj(G[-k + K]));
    if (wr == 0.0) continue;
    const int64_t kp = ((k % N) + N) % N;
    for (int r = 0; r < SC; ++r) H[(size_t)r * N + kp] += wr * std::conj(root_of_unity(k * r, SC * N));
  }
  return H;
}

static hipError_t line_pass(int N, int SC, bool cols, bool zr, int store_in, int store_out, const LinePassArgs& a,
                            int64_t images, hipStream_t s, bool prep) {
  if (zr) {
    if (store_in != ST_F32 || store_out != ST_F32) return hipErrorInvalidValue;
    return cols ? l2d::dispatch<true, true, float, float>(N, SC, a, images, s, prep)
                : l2d::dispatch<false, true, float, float>(N, SC, a, images, s, prep);
  }
  if (cols) {
    if (store_in == ST_F16) return l2d::dispatch<true, false, __half, float>(N, SC, a, images, s, prep);
    return l2d::dispatch<true, false, float, float>(N, SC, a, images, s, prep);
  }
  if (store_out == ST_F16) return l2d::dispatch<false, false, float, __half>(N, SC, a, images, s, prep);
  return l2d::dispatch<false, false, float, float>(N, SC, a, images, s, prep);
}

hipError_t run_line_pass(int N, int SC, bool cols, bool zr, int store_in, int store_out, const LinePassArgs& a,
                         int64_t images, hipStream_t s) {
  return line_pass(N, SC, cols, zr, store_in, store_out, a, images, s, false);
}

hipError_t prepare_line_pass(int N, int SC, bool cols, bool zr, int store_in, int store_out) {
  return line_pass(N, SC, cols, zr, store_in, store_out, LinePassArgs{}, 0, nullptr, true);
}

}  // namespace mci
