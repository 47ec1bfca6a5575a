// mci_refiner.hip -- learned residual refiner for the MCI upsample: y = u + CNN(u), u the MCI
// upsample of an RGB image, CNN = conv3x3(3->32) ReLU conv3x3(32->32) ReLU conv3x3(32->32) ReLU
// conv3x3(32->3), zero padding.  Forward and backward run on BF16 MFMA with FP32 accumulation;
// master weights and the Adam state are FP32.
//
// Layouts: RGB images (MCI output, target, refined output) FP32 [B][3][H][W]; hidden
// activations BF16 NHWC [B][H][W][32].  A workgroup (256 threads, 4 waves) owns a 16 x 16
// pixel tile.  Convolutions are implicit GEMMs on v_mfma_f32_16x16x32_bf16:
//   lane l supplies A[l % 16][8 (l / 16) + j], B[8 (l / 16) + j][l % 16], j < 8, and receives
//   D[4 (l / 16) + i][l % 16], i < 4.
// With 32 input channels a tap's 32 channels are one K step (A rows = 16 pixels of one tile row,
// B = weights [co][tap][ci]); with 3 input channels the 27 (tap, channel) products of a pixel
// form one K step padded to 32.  Backward-data is the same kernel with flipped, transposed
// weights and a ReLU-mask epilogue; weight gradients contract over pixels (K = 32 pixels, two
// tile rows) from LDS tiles stored channel-major.
#include <hip/hip_bf16.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <random>
#include <string>
#include <vector>

#include "../../include/mci.h"

namespace mci {
namespace ref {

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int C = 32;   // hidden channels
constexpr int T = 16;   // tile side
constexpr int HT = 18;  // tile side with the 1-pixel halo
constexpr int NT = 256;

// parameter block offsets (FP32 master, 20259 values)
constexpr int W1 = 0, B1 = W1 + 32 * 27, W2 = B1 + 32, B2 = W2 + 32 * 9 * 32, W3 = B2 + 32, B3 = W3 + 32 * 9 * 32,
              W4 = B3 + 32, B4 = W4 + 3 * 9 * 32, NPARAM = B4 + 3;
// master layouts: W1[co][tap][ci<3], W2/W3[co][tap][ci<32], W4[co<3][tap][ci<32]

// BF16 kernel-layout weights: forward Wf1[32][32] (k = tap*3+ci, padded), Wf2/Wf3[32][9][32],
// Wf4[16][9][32] (co padded); backward-data Wb4[32][32] (co' = ci, k = tap'*3 + co),
// Wb3/Wb2[32][9][32] (co' = ci, tap' = 8 - tap, ci' = co).
constexpr int OF1 = 0, OF2 = OF1 + 32 * 32, OF3 = OF2 + 32 * 9 * 32, OF4 = OF3 + 32 * 9 * 32, OB4 = OF4 + 16 * 9 * 32,
              OB3 = OB4 + 32 * 32, OB2 = OB3 + 32 * 9 * 32, NBF = OB2 + 32 * 9 * 32;

__device__ __forceinline__ bf16 tobf(float x) { return (bf16)x; }
__device__ __forceinline__ float tof(bf16 x) { return (float)x; }

// ---------------------------------------------------------------- weight layouts
__global__ void k_weights_bf16(const float* __restrict__ p, bf16* __restrict__ w) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= NBF) return;
  float v = 0.f;
  if (e < OF2) {                       // Wf1[co][k]
    const int co = e / 32, k = e % 32;
    if (k < 27) v = p[W1 + co * 27 + k];
  } else if (e < OF3) {                // Wf2[co][tap][ci]
    v = p[W2 + (e - OF2)];
  } else if (e < OF4) {
    v = p[W3 + (e - OF3)];
  } else if (e < OB4) {                // Wf4[co<16][tap][ci]
    const int q = e - OF4, co = q / 288, r = q % 288;
    if (co < 3) v = p[W4 + co * 288 + r];
  } else if (e < OB3) {                // Wb4[ci][k = tap'*3 + co] = W4[co][8 - tap'][ci]
    const int q = e - OB4, ci = q / 32, k = q % 32;
    if (k < 27) {
      const int tp = k / 3, co = k % 3;
      v = p[W4 + (co * 9 + (8 - tp)) * 32 + ci];
    }
  } else {                             // Wb3 / Wb2 [ci][tap'][co] = W[co][8 - tap'][ci]
    const bool l3 = e < OB2;
    const int q = e - (l3 ? OB3 : OB2), ci = q / 288, r = q % 288, tp = r / 32, co = r % 32;
    v = p[(l3 ? W3 : W2) + (co * 9 + (8 - tp)) * 32 + ci];
  }
  w[e] = tobf(v);
}

// ---------------------------------------------------------------- convolution (implicit GEMM)
enum { IN3 = 0, IN32 = 1 };                    // input: 3-channel FP32 NCHW or 32-channel BF16 NHWC
enum { EPI_RELU = 0, EPI_RESID = 1, EPI_MASK = 2 };

struct ConvArgs {
  const void* in;        // IN3: float [B][3][H][W]; IN32: bf16 [B][H][W][32]
  const bf16* w;         // IN3: [COUT][32] (k = tap*3 + ci); IN32: [COUT][9][32]
  const float* bias;     // [cout] or null
  const float* base;     // EPI_RESID: float [B][3][H][W] added to the result
  const bf16* mask;      // EPI_MASK: bf16 [B][H][W][32]; output *= (mask > 0)
  void* out;             // EPI_RELU / EPI_MASK: bf16 [B][H][W][32]; EPI_RESID: float [B][3][H][W]
  float* rpart;          // EPI_RESID, optional: per-tile sums (residual^2, base^2), [B][tiles][2]
  int H, W;
};

template <int INM, int COUT, int EPI>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4))) void k_conv(ConvArgs a) {
  constexpr int NB = COUT / 16;                 // 16-wide output-channel blocks
  __shared__ __attribute__((aligned(16))) bf16 tin[INM == IN32 ? HT * HT * C : HT * HT * 4];
  __shared__ __attribute__((aligned(16))) float tout[T * T * (EPI == EPI_RESID ? 4 : 16)];   // reused per epilogue
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int tx0 = blockIdx.x * T, ty0 = blockIdx.y * T, b = blockIdx.z;
  const int H = a.H, W = a.W;
  const int px = lane & 15, kb = lane >> 4;
  // ---- weights: the first NPRE taps load before the tile (their loads overlap the tile's);
  // tap t + NPRE loads as tap t's MFMAs start, so at most NPRE + 1 taps are live and the
  // registers stay within the budget of 4 waves per SIMD
  constexpr int NTAP = INM == IN32 ? 9 : 1;
  constexpr int NPRE = INM == IN32 ? 4 : 1;
  bf16x8 bw[NTAP][NB];
#pragma unroll
  for (int tap = 0; tap < NPRE; ++tap)
#pragma unroll
    for (int n = 0; n < NB; ++n)
      bw[tap][n] = INM == IN32 ? *(const bf16x8*)(a.w + ((16 * n + px) * 9 + tap) * C + 8 * kb)
                               : *(const bf16x8*)(a.w + (16 * n + px) * 32 + 8 * kb);
  // ---- halo tile (zero outside the image): every load issued before the first LDS write
  constexpr int CH = HT * HT * 4, IT = (CH + NT - 1) / NT;
  if constexpr (INM == IN32) {
    const bf16* in = (const bf16*)a.in + (size_t)b * H * W * C;
    uint4 v[IT];
#pragma unroll
    for (int it = 0; it < IT; ++it) {            // 16-byte chunks: 4 per pixel
      const int e = tid + NT * it;
      const int pix = e >> 2, part = e & 3;
      const int y = ty0 - 1 + pix / HT, x = tx0 - 1 + pix % HT;
      v[it] = make_uint4(0, 0, 0, 0);
      if (e < CH && y >= 0 && y < H && x >= 0 && x < W) v[it] = *(const uint4*)(in + ((size_t)y * W + x) * C + part * 8);
    }
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int e = tid + NT * it;
      if (e < CH) *(uint4*)(tin + (e >> 2) * C + (e & 3) * 8) = v[it];
    }
  } else {
    const float* in = (const float*)a.in + (size_t)b * 3 * H * W;
    float v[IT];
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int e = tid + NT * it;
      const int pix = e >> 2, ci = e & 3;
      const int y = ty0 - 1 + pix / HT, x = tx0 - 1 + pix % HT;
      v[it] = 0.f;
      if (e < CH && ci < 3 && y >= 0 && y < H && x >= 0 && x < W) v[it] = in[((size_t)ci * H + y) * W + x];
    }
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int e = tid + NT * it;
      if (e < CH) tin[e] = tobf(v[it]);
    }
  }
  __syncthreads();
  // ---- MFMA: wave handles tile rows 4 wave .. 4 wave + 3
  f4 acc[4][NB];
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int n = 0; n < NB; ++n) acc[m][n] = f4{0.f, 0.f, 0.f, 0.f};
  if constexpr (INM == IN32) {
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) {
      if (tap + NPRE < NTAP)
#pragma unroll
        for (int n = 0; n < NB; ++n)
          bw[tap + NPRE][n] = *(const bf16x8*)(a.w + ((16 * n + px) * 9 + tap + NPRE) * C + 8 * kb);
      const int dy = tap / 3, dx = tap % 3;
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const int row = 4 * wave + m;
        const bf16x8 av = *(const bf16x8*)(tin + ((row + dy) * HT + (px + dx)) * C + 8 * kb);
#pragma unroll
        for (int n = 0; n < NB; ++n)
          acc[m][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bw[tap][n], acc[m][n], 0, 0, 0);
      }
    }
  } else {
    // this lane's 8 (tap, channel) slots k = 8 kb + j
    int off[8], chn[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int k = 8 * kb + j, tap = k / 3;
      off[j] = k < 27 ? (tap / 3) * HT + (tap % 3) : -1;
      chn[j] = k % 3;
    }
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const int row = 4 * wave + m;
      bf16x8 av;
#pragma unroll
      for (int j = 0; j < 8; ++j) av[j] = off[j] >= 0 ? tin[(row * HT + px + off[j]) * 4 + chn[j]] : tobf(0.f);
#pragma unroll
      for (int n = 0; n < NB; ++n) acc[m][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bw[0][n], acc[m][n], 0, 0, 0);
    }
  }
  // ---- epilogue: D[pixel = 4 kb + i][co = px + 16 n] of tile row 4 wave + m
  if constexpr (EPI == EPI_RESID) {
    // 3 output channels: stage [3][16][16] floats, then add the base image and store
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
      for (int i = 0; i < 4; ++i)
        if (px < 3) tout[(px * T + 4 * wave + m) * T + 4 * kb + i] = acc[m][0][i];
    __syncthreads();
    float* out = (float*)a.out + (size_t)b * 3 * H * W;
    const float* base = a.base ? a.base + (size_t)b * 3 * H * W : nullptr;
    float sr = 0.f, su = 0.f;   // this thread's share of ||residual||^2 and ||base||^2
    for (int e = tid; e < 3 * T * T; e += NT) {
      const int co = e / (T * T), r = (e / T) % T, c = e % T;
      const int y = ty0 + r, x = tx0 + c;
      if (y < H && x < W) {
        const size_t o = ((size_t)co * H + y) * W + x;
        const float res = tout[e] + (a.bias ? a.bias[co] : 0.f), u0 = base ? base[o] : 0.f;
        sr += res * res;
        su += u0 * u0;
        out[o] = res + u0;
      }
    }
    if (a.rpart) {
      // per-tile partial sums for the residual ratio: wave sums, then the 4 waves in LDS
      __shared__ float red[2][NT / 64];
#pragma unroll
      for (int d = 32; d > 0; d >>= 1) {
        sr += __shfl_xor(sr, d);
        su += __shfl_xor(su, d);
      }
      if (lane == 0) { red[0][wave] = sr; red[1][wave] = su; }
      __syncthreads();
      if (tid == 0) {
        float r2 = 0.f, u2 = 0.f;
        for (int w = 0; w < NT / 64; ++w) { r2 += red[0][w]; u2 += red[1][w]; }
        const size_t t = ((size_t)b * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
        a.rpart[2 * t] = r2;
        a.rpart[2 * t + 1] = u2;
      }
    }
  } else {
    // 32 output channels: two passes of 16 channels through LDS, 16-byte stores
    bf16* out = (bf16*)a.out + (size_t)b * H * W * C;
    const bf16* mask = EPI == EPI_MASK ? a.mask + (size_t)b * H * W * C : nullptr;
#pragma unroll
    for (int n = 0; n < NB; ++n) {
      __syncthreads();
#pragma unroll
      for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          float v = acc[m][n][i];
          if constexpr (EPI == EPI_RELU) v = fmaxf(v + a.bias[16 * n + px], 0.f);
          tout[((4 * wave + m) * T + 4 * kb + i) * 16 + px] = v;
        }
      __syncthreads();
      for (int e = tid; e < T * T * 2; e += NT) {          // 8 channels per chunk
        const int pix = e >> 1, part = e & 1;
        const int y = ty0 + pix / T, x = tx0 + pix % T;
        if (y >= H || x >= W) continue;
        const size_t o = ((size_t)y * W + x) * C + 16 * n + 8 * part;
        bf16x8 v;
        if constexpr (EPI == EPI_MASK) {
          const bf16x8 mk = *(const bf16x8*)(mask + o);
#pragma unroll
          for (int j = 0; j < 8; ++j) v[j] = tobf(tof(mk[j]) > 0.f ? tout[pix * 16 + 8 * part + j] : 0.f);
        } else {
#pragma unroll
          for (int j = 0; j < 8; ++j) v[j] = tobf(tout[pix * 16 + 8 * part + j]);
        }
        *(bf16x8*)(out + o) = v;
      }
    }
  }
}

// ---------------------------------------------------------------- two hidden layers in one pass
// Inference form of layers 2 and 3 (conv 32 -> 32, ReLU, twice) on one 16 x 16 tile: layer 2
// runs on the 18 x 18 region that layer 3's halo needs (324 pixels, flattened into 21 MFMA
// row blocks of 16), its BF16 result stays in LDS (zero outside the image: layer 3's padding),
// and only layer 3's output goes to memory.  Each output is accumulated in the same order as
// by k_conv, and the intermediate is rounded to BF16 as k_conv stores it.
constexpr int HT2 = T + 4;               // input tile side: the two layers' two-pixel halo
constexpr int NP2 = HT * HT;             // layer-2 pixels
constexpr int MB2 = (NP2 + 15) / 16;     // their 16-pixel row blocks
constexpr int MW2 = (MB2 + 3) / 4;       // row blocks per wave (block m goes to wave m % 4)

struct Conv23Args {
  const bf16* in;                        // layer-1 activations [B][H][W][32]
  const bf16* w2;                        // [32][9][32]
  const float* b2;
  const bf16* w3;
  const float* b3;
  bf16* out;                             // layer-3 activations [B][H][W][32]
  int H, W;
};

__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4))) void k_conv23(Conv23Args a) {
  // the input tile [20 x 20][32]; layer 2's result [18 x 18][32] and the output staging reuse
  // it once every wave is past the MFMAs that read it
  __shared__ __attribute__((aligned(16))) bf16 tl[HT2 * HT2 * C];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int tx0 = blockIdx.x * T, ty0 = blockIdx.y * T, b = blockIdx.z;
  const int H = a.H, W = a.W;
  const int px = lane & 15, kb = lane >> 4;
  constexpr int NPRE = 4;   // weight taps loaded ahead, as in k_conv
  bf16x8 bw[9][2];
#pragma unroll
  for (int tap = 0; tap < NPRE; ++tap)
#pragma unroll
    for (int n = 0; n < 2; ++n) bw[tap][n] = *(const bf16x8*)(a.w2 + ((16 * n + px) * 9 + tap) * C + 8 * kb);
  {
    constexpr int CH = HT2 * HT2 * 4, IT = (CH + NT - 1) / NT;
    const bf16* in = a.in + (size_t)b * H * W * C;
    uint4 v[IT];
#pragma unroll
    for (int it = 0; it < IT; ++it) {            // 16-byte chunks: 4 per pixel
      const int e = tid + NT * it;
      const int pix = e >> 2, part = e & 3;
      const int y = ty0 - 2 + pix / HT2, x = tx0 - 2 + pix % HT2;
      v[it] = make_uint4(0, 0, 0, 0);
      if (e < CH && y >= 0 && y < H && x >= 0 && x < W) v[it] = *(const uint4*)(in + ((size_t)y * W + x) * C + part * 8);
    }
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int e = tid + NT * it;
      if (e < CH) *(uint4*)(tl + (e >> 2) * C + (e & 3) * 8) = v[it];
    }
  }
  __syncthreads();
  // ---- layer 2 on the 18 x 18 region (region pixel p at (p / 18, p % 18), tile pixel (p / 18 - 1, p % 18 - 1))
  f4 acc[MW2][2];
  int abase[MW2];
#pragma unroll
  for (int j = 0; j < MW2; ++j) {
    const int p = min(16 * (wave + 4 * j) + px, NP2 - 1);   // rows past the region compute a copy, unused
    abase[j] = ((p / HT) * HT2 + p % HT) * C + 8 * kb;
#pragma unroll
    for (int n = 0; n < 2; ++n) acc[j][n] = f4{0.f, 0.f, 0.f, 0.f};
  }
#pragma unroll
  for (int tap = 0; tap < 9; ++tap) {
    if (tap + NPRE < 9)
#pragma unroll
      for (int n = 0; n < 2; ++n)
        bw[tap + NPRE][n] = *(const bf16x8*)(a.w2 + ((16 * n + px) * 9 + tap + NPRE) * C + 8 * kb);
    const int off = ((tap / 3) * HT2 + tap % 3) * C;
#pragma unroll
    for (int j = 0; j < MW2; ++j) {
      if (wave + 4 * j < MB2) {   // uniform per wave
        const bf16x8 av = *(const bf16x8*)(tl + abase[j] + off);
#pragma unroll
        for (int n = 0; n < 2; ++n) acc[j][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bw[tap][n], acc[j][n], 0, 0, 0);
      }
    }
  }
#pragma unroll
  for (int tap = 0; tap < NPRE; ++tap)
#pragma unroll
    for (int n = 0; n < 2; ++n) bw[tap][n] = *(const bf16x8*)(a.w3 + ((16 * n + px) * 9 + tap) * C + 8 * kb);
  __syncthreads();   // every wave is done reading the input tile
  // bias, ReLU, zero outside the image; D[pixel 4 kb + i of the block][channel px + 16 n]
#pragma unroll
  for (int j = 0; j < MW2; ++j) {
    const int m = wave + 4 * j;
    if (m >= MB2) continue;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int p = 16 * m + 4 * kb + i;
      if (p >= NP2) continue;
      const int y = ty0 - 1 + p / HT, x = tx0 - 1 + p % HT;
      const bool inside = y >= 0 && y < H && x >= 0 && x < W;
#pragma unroll
      for (int n = 0; n < 2; ++n)
        tl[p * C + 16 * n + px] = tobf(inside ? fmaxf(acc[j][n][i] + a.b2[16 * n + px], 0.f) : 0.f);
    }
  }
  __syncthreads();
  // ---- layer 3: tile rows 4 wave .. 4 wave + 3, as k_conv's 32-channel path
  f4 acc3[4][2];
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int n = 0; n < 2; ++n) acc3[m][n] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int tap = 0; tap < 9; ++tap) {
    if (tap + NPRE < 9)
#pragma unroll
      for (int n = 0; n < 2; ++n)
        bw[tap + NPRE][n] = *(const bf16x8*)(a.w3 + ((16 * n + px) * 9 + tap + NPRE) * C + 8 * kb);
    const int dy = tap / 3, dx = tap % 3;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const int row = 4 * wave + m;
      const bf16x8 av = *(const bf16x8*)(tl + ((row + dy) * HT + (px + dx)) * C + 8 * kb);
#pragma unroll
      for (int n = 0; n < 2; ++n) acc3[m][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bw[tap][n], acc3[m][n], 0, 0, 0);
    }
  }
  // ---- epilogue: two passes of 16 channels through the staging area, 16-byte stores
  float* tout = (float*)tl;
  bf16* out = a.out + (size_t)b * H * W * C;
#pragma unroll
  for (int n = 0; n < 2; ++n) {
    __syncthreads();
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
      for (int i = 0; i < 4; ++i)
        tout[((4 * wave + m) * T + 4 * kb + i) * 16 + px] = fmaxf(acc3[m][n][i] + a.b3[16 * n + px], 0.f);
    __syncthreads();
    for (int e = tid; e < T * T * 2; e += NT) {          // 8 channels per chunk
      const int pix = e >> 1, part = e & 1;
      const int y = ty0 + pix / T, x = tx0 + pix % T;
      if (y >= H || x >= W) continue;
      bf16x8 v;
#pragma unroll
      for (int j = 0; j < 8; ++j) v[j] = tobf(tout[pix * 16 + 8 * part + j]);
      *(bf16x8*)(out + ((size_t)y * W + x) * C + 16 * n + 8 * part) = v;
    }
  }
}

// ---------------------------------------------------------------- weight gradients
// dW[co][tap][ci] = sum_p G[p][co] X[p + off(tap)][ci] over this tile's 256 pixels, written as a
// per-tile partial; db[co] = sum_p G[p][co] likewise.  A = G^T (rows co, K = pixels), B = shifted
// X (K = pixels, cols ci); a K step is 32 pixels = two tile rows, 8 consecutive pixels per lane.
// Both tiles are stored channel-major in LDS; X is kept twice (shifted by one column) so every
// 8-pixel fragment starts on a 4-byte boundary.
struct WgradArgs {
  const void* g;        // G: GIN3: float [B][3][H][W]; else bf16 [B][H][W][32]
  const void* x;        // X: XIN3: float [B][3][H][W]; else bf16 [B][H][W][32]
  float* part;          // [tiles][NOUT] partial dW (layout of the master weights) followed by db
  int H, W;
};

template <bool GIN3, bool XIN3>
__global__ __launch_bounds__(NT) void k_wgrad(WgradArgs a) {
  constexpr int CO = GIN3 ? 3 : 32, CI = XIN3 ? 3 : 32;
  constexpr int MB = GIN3 ? 1 : 2;                       // 16-wide co blocks
  constexpr int NCOL = XIN3 ? 32 : 9 * 32;               // (tap, ci) columns, padded for XIN3
  constexpr int NBLK = NCOL / 16;
  constexpr int HW2 = 20;                                // halo row pitch (even)
  __shared__ __attribute__((aligned(16))) bf16 gt[CO < 16 ? 16 * T * T : CO * T * T];   // [co][256]
  __shared__ __attribute__((aligned(16))) bf16 xt[2][CI * HT * HW2];                    // [copy][ci][18][20]
  __shared__ float bsum[4][32];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int tx0 = blockIdx.x * T, ty0 = blockIdx.y * T, b = blockIdx.z;
  const int H = a.H, W = a.W;
  // ---- G tile, channel-major (co rows beyond CO are zero)
  for (int e = tid; e < (CO < 16 ? 16 : CO) * T * T; e += NT) {
    const int co = e / (T * T), pix = e % (T * T);
    const int y = ty0 + pix / T, x = tx0 + pix % T;
    float v = 0.f;
    if (co < CO && y < H && x < W) {
      if constexpr (GIN3) v = ((const float*)a.g)[(((size_t)b * 3 + co) * H + y) * W + x];
      else v = tof(((const bf16*)a.g)[(((size_t)b * H + y) * W + x) * C + co]);
    }
    gt[e] = tobf(v);
  }
  // ---- X halo tile, channel-major, two copies (copy 1 shifted left by one column)
  for (int e = tid; e < CI * HT * HW2; e += NT) {
    const int ci = e / (HT * HW2), r = (e / HW2) % HT, c = e % HW2;
    const int y = ty0 - 1 + r;
#pragma unroll
    for (int cp = 0; cp < 2; ++cp) {
      const int x = tx0 - 1 + c + cp;
      float v = 0.f;
      if (c + cp < HT && y >= 0 && y < H && x >= 0 && x < W) {
        if constexpr (XIN3) v = ((const float*)a.x)[(((size_t)b * 3 + ci) * H + y) * W + x];
        else v = tof(((const bf16*)a.x)[(((size_t)b * H + y) * W + x) * C + ci]);
      }
      xt[cp][e] = tobf(v);
    }
  }
  __syncthreads();
  // ---- bias partial: sum over pixels of G[.][co]
  if (tid < 128) {
    const int co = tid & 31, q = tid >> 5;
    float s = 0.f;
    if (co < CO)
      for (int p = q * 64; p < q * 64 + 64; ++p) s += tof(gt[co * T * T + p]);
    bsum[q][co] = s;
  }
  // ---- MFMA over the (co block, column block) pairs, round-robin across waves
  const int ln = lane & 15, kb = lane >> 4;
  float* part = a.part + ((size_t)b * gridDim.y * gridDim.x + blockIdx.y * gridDim.x + blockIdx.x) * (CO * 9 * CI + CO);
  for (int blk = wave; blk < MB * NBLK; blk += 4) {
    const int mb = blk / NBLK, nb = blk % NBLK;
    // this lane's B column: (tap, ci)
    int tap, ci;
    if constexpr (XIN3) { const int k = 16 * nb + ln; tap = k / 3; ci = k % 3; if (k >= 27) tap = -1; }
    else { tap = (16 * nb) / 32; ci = (16 * nb) % 32 + ln; }
    const int dy = tap >= 0 ? tap / 3 : 0, dx = tap >= 0 ? tap % 3 : 0;
    const int cp = dx & 1, dxe = dx - cp;                 // copy and even column shift
    f4 acc = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < 8; ++ks) {                      // 32 pixels: rows 2ks, 2ks+1
      const int row = 2 * ks + (kb >> 1), col = 8 * (kb & 1);
      const bf16x8 av = *(const bf16x8*)(gt + (16 * mb + ln) * T * T + row * T + col);
      bf16x8 bv;
      if (tap >= 0) {
        const bf16* src = xt[cp] + (ci * HT + row + dy) * HW2 + col + dxe;
#pragma unroll
        for (int j = 0; j < 8; j += 2) {
          const uint32_t w2 = *(const uint32_t*)(src + j);
          bf16 lo, hi;
          __builtin_memcpy(&lo, &w2, 2);
          __builtin_memcpy(&hi, (const char*)&w2 + 2, 2);
          bv[j] = lo;
          bv[j + 1] = hi;
        }
      } else {
#pragma unroll
        for (int j = 0; j < 8; ++j) bv[j] = tobf(0.f);
      }
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc, 0, 0, 0);
    }
    // D[co = 4 kb + i][col = ln] of this block -> partial dW[co][tap][ci]
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int co = 16 * mb + 4 * kb + i;
      if (co < CO && tap >= 0) part[(co * 9 + tap) * CI + ci] = acc[i];
    }
  }
  __syncthreads();
  if (tid < CO) part[CO * 9 * CI + tid] = bsum[0][tid] + bsum[1][tid] + bsum[2][tid] + bsum[3][tid];
}

// sum the per-tile partials into the gradient slice (deterministic)
// Sum the per-tile partials in two deterministic stages: stage 1 gives RS slices of the tiles
// (t = s, s + RS, ...) to separate threads, 64 consecutive parameters per wave (256 contiguous
// bytes of a partials row); stage 2 adds the RS slice sums of a parameter in order.
constexpr int RS = 32;

__global__ void k_reduce_parts1(const float* __restrict__ part, int tiles, int n, float* __restrict__ part2) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const int sl = blockIdx.y;
  if (e >= n) return;
  float s = 0.f;
  for (int t = sl; t < tiles; t += RS) s += part[(size_t)t * n + e];
  part2[(size_t)sl * n + e] = s;
}

__global__ void k_reduce_parts2(const float* __restrict__ part2, int n, float* __restrict__ grad_w,
                                float* __restrict__ grad_b, int nw) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  float s = 0.f;
#pragma unroll 8
  for (int sl = 0; sl < RS; ++sl) s += part2[(size_t)sl * n + e];
  if (e < nw) grad_w[e] = s;
  else grad_b[e - nw] = s;
}

// ---------------------------------------------------------------- loss, Adam, fallback
// dr = 2 (out - hr) / count; per-block partial sums of the squared error
__global__ void k_loss(const float* __restrict__ out, const float* __restrict__ hr, float* __restrict__ dr,
                       int64_t count, float* __restrict__ lpart) {
  __shared__ float red[NT];
  float s = 0.f;
  for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < count; e += (int64_t)gridDim.x * NT) {
    const float d = out[e] - hr[e];
    dr[e] = 2.f * d / (float)count;
    s += d * d;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = NT / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) lpart[blockIdx.x] = red[0];
}

__global__ void k_adam(float* __restrict__ p, float* __restrict__ m, float* __restrict__ v, const float* __restrict__ g,
                       int n, float lr, float b1, float b2, float eps, float c1, float c2) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const float gr = g[e];
  const float mm = b1 * m[e] + (1.f - b1) * gr;
  const float vv = b2 * v[e] + (1.f - b2) * gr * gr;
  m[e] = mm;
  v[e] = vv;
  p[e] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
}

// per-image ratio ||r||_2 / ||u||_2 of the CNN residual r = y - u to the MCI image u
// ratio[b] = ||residual_b|| / ||u_b|| from the last layer's per-tile partial sums
__global__ void k_ratio(const float* __restrict__ rpart, int tiles, float* __restrict__ ratio) {
  __shared__ float rn[NT], un[NT];
  const int b = blockIdx.x;
  float sr = 0.f, su = 0.f;
  for (int t = threadIdx.x; t < tiles; t += NT) {
    sr += rpart[2 * ((size_t)b * tiles + t)];
    su += rpart[2 * ((size_t)b * tiles + t) + 1];
  }
  rn[threadIdx.x] = sr;
  un[threadIdx.x] = su;
  __syncthreads();
  for (int w = NT / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) { rn[threadIdx.x] += rn[threadIdx.x + w]; un[threadIdx.x] += un[threadIdx.x + w]; }
    __syncthreads();
  }
  if (threadIdx.x == 0) ratio[b] = sqrtf(rn[0]) / fmaxf(sqrtf(un[0]), 1e-30f);
}

// images whose residual ratio exceeds tau fall back to the plain MCI upsample
__global__ void k_fallback(float* __restrict__ y, const float* __restrict__ u, int64_t per_img, const float* __restrict__ ratio,
                           float tau, int* __restrict__ used) {
  const int b = blockIdx.y;
  const bool fb = !(ratio[b] <= tau);      // NaN ratios fall back too
  if (threadIdx.x == 0 && blockIdx.x == 0) used[b] = fb ? 0 : 1;
  if (!fb) return;
  for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < per_img; e += (int64_t)gridDim.x * NT)
    y[b * per_img + e] = u[b * per_img + e];
}

}  // namespace ref
}  // namespace mci

// ================================================================== host side / C ABI
using namespace mci::ref;

struct mci_refiner_s {
  int device = 0;
  float* p = nullptr;     // FP32 master [NPARAM]
  float* m = nullptr;     // Adam moments
  float* v = nullptr;
  float* g = nullptr;     // gradient [NPARAM]
  bf16* w = nullptr;      // BF16 kernel layouts [NBF]
  int64_t step = 0;
  float tau = 0.f;        // fallback bound on ||CNN(u)|| / ||u||
};

static thread_local std::string r_err;
static mci_status rfail(mci_status s, const std::string& m) {
  r_err = m;
  return s;
}
#define RHIP(expr)                                                                                  \
  do {                                                                                              \
    hipError_t _e = (expr);                                                                         \
    if (_e != hipSuccess) return rfail(MCI_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(_e)); \
  } while (0)

static size_t al256(size_t n) { return (n + 255) & ~(size_t)255; }

// workspace layout for a batch of B images of H x W
struct RefWs {
  bf16 *a1, *a2, *a3, *d0, *d1;
  float *out, *dr, *part, *part2, *lpart;
  size_t bytes;
};
static RefWs ref_ws(void* base, int64_t B, int H, int W) {
  RefWs w{};
  char* p = (char*)(((uintptr_t)base + 255) & ~(uintptr_t)255);
  const size_t act = al256((size_t)B * H * W * C * sizeof(bf16));
  const size_t img = al256((size_t)B * 3 * H * W * sizeof(float));
  const int64_t tiles = B * ((H + T - 1) / T) * ((W + T - 1) / T);
  const size_t part = al256((size_t)tiles * (32 * 9 * 32 + 32) * sizeof(float));
  const size_t lp = al256(4096 * sizeof(float));
  char* q = p;
  w.a1 = (bf16*)q; q += act;
  w.a2 = (bf16*)q; q += act;
  w.a3 = (bf16*)q; q += act;
  w.d0 = (bf16*)q; q += act;
  w.d1 = (bf16*)q; q += act;
  w.out = (float*)q; q += img;
  w.dr = (float*)q; q += img;
  w.part = (float*)q; q += part;
  w.part2 = (float*)q; q += al256((size_t)RS * (32 * 9 * 32 + 32) * sizeof(float));
  w.lpart = (float*)q; q += lp;
  w.bytes = (size_t)(q - (char*)base) + 256;
  return w;
}

static hipError_t conv(int inm, int cout, int epi, const ConvArgs& a, int64_t B, hipStream_t s) {
  dim3 grid((a.W + T - 1) / T, (a.H + T - 1) / T, (unsigned)B);
  if (inm == IN3 && cout == 32 && epi == EPI_RELU) hipLaunchKernelGGL((k_conv<IN3, 32, EPI_RELU>), grid, dim3(NT), 0, s, a);
  else if (inm == IN32 && cout == 32 && epi == EPI_RELU) hipLaunchKernelGGL((k_conv<IN32, 32, EPI_RELU>), grid, dim3(NT), 0, s, a);
  else if (inm == IN32 && cout == 16 && epi == EPI_RESID) hipLaunchKernelGGL((k_conv<IN32, 16, EPI_RESID>), grid, dim3(NT), 0, s, a);
  else if (inm == IN3 && cout == 32 && epi == EPI_MASK) hipLaunchKernelGGL((k_conv<IN3, 32, EPI_MASK>), grid, dim3(NT), 0, s, a);
  else if (inm == IN32 && cout == 32 && epi == EPI_MASK) hipLaunchKernelGGL((k_conv<IN32, 32, EPI_MASK>), grid, dim3(NT), 0, s, a);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

// forward through the four layers; out = u + CNN(u).  fused23: layers 2 and 3 in one pass
// (inference: the layer-2 activations, which training reads back, are not stored)
static hipError_t ref_forward(mci_refiner_s* r, const float* u, float* out, int64_t B, int H, int W, const RefWs& ws,
                              hipStream_t s, float* rpart = nullptr, bool fused23 = false) {
  hipError_t e;
  ConvArgs a{};
  a.H = H; a.W = W;
  a.in = u; a.w = r->w + OF1; a.bias = r->p + B1; a.out = ws.a1;
  if ((e = conv(IN3, 32, EPI_RELU, a, B, s)) != hipSuccess) return e;
  if (fused23) {
    const Conv23Args c{ws.a1, r->w + OF2, r->p + B2, r->w + OF3, r->p + B3, ws.a3, H, W};
    hipLaunchKernelGGL(k_conv23, dim3((W + T - 1) / T, (H + T - 1) / T, (unsigned)B), dim3(NT), 0, s, c);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  } else {
    a.in = ws.a1; a.w = r->w + OF2; a.bias = r->p + B2; a.out = ws.a2;
    if ((e = conv(IN32, 32, EPI_RELU, a, B, s)) != hipSuccess) return e;
    a.in = ws.a2; a.w = r->w + OF3; a.bias = r->p + B3; a.out = ws.a3;
    if ((e = conv(IN32, 32, EPI_RELU, a, B, s)) != hipSuccess) return e;
  }
  a.in = ws.a3; a.w = r->w + OF4; a.bias = r->p + B4; a.base = u; a.out = out; a.rpart = rpart;
  return conv(IN32, 16, EPI_RESID, a, B, s);
}

static hipError_t wgrad(bool gin3, bool xin3, const void* g, const void* x, float* part, float* part2, float* gw,
                        float* gb, int nw, int nb, int64_t B, int H, int W, hipStream_t s) {
  WgradArgs a{g, x, part, H, W};
  dim3 grid((W + T - 1) / T, (H + T - 1) / T, (unsigned)B);
  if (!gin3 && xin3) hipLaunchKernelGGL((k_wgrad<false, true>), grid, dim3(NT), 0, s, a);
  else if (!gin3 && !xin3) hipLaunchKernelGGL((k_wgrad<false, false>), grid, dim3(NT), 0, s, a);
  else if (gin3 && !xin3) hipLaunchKernelGGL((k_wgrad<true, false>), grid, dim3(NT), 0, s, a);
  else return hipErrorInvalidValue;
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int tiles = (int)(B * grid.x * grid.y), n = nw + nb;
  hipLaunchKernelGGL(k_reduce_parts1, dim3((n + 255) / 256, RS), dim3(256), 0, s, part, tiles, n, part2);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_reduce_parts2, dim3((n + 255) / 256), dim3(256), 0, s, part2, n, gw, gb, nw);
  return hipGetLastError();
}

// forward + loss + backward: r->g holds dL/dtheta, lpart the per-block squared-error sums
static hipError_t ref_backward(mci_refiner_s* r, const float* u, const float* hr, int64_t B, int H, int W,
                               const RefWs& ws, int* nlpart, hipStream_t s) {
  hipError_t e;
  if ((e = ref_forward(r, u, ws.out, B, H, W, ws, s)) != hipSuccess) return e;
  const int64_t count = B * 3 * (int64_t)H * W;
  const int lb = (int)std::min<int64_t>(1024, (count + NT - 1) / NT);
  hipLaunchKernelGGL(k_loss, dim3(lb), dim3(NT), 0, s, ws.out, hr, ws.dr, count, ws.lpart);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  *nlpart = lb;
  // layer 4: dW4, db4 from (dr, a3); da3 masked by a3 > 0
  if ((e = wgrad(true, false, ws.dr, ws.a3, ws.part, ws.part2, r->g + W4, r->g + B4, 3 * 9 * 32, 3, B, H, W, s)) != hipSuccess) return e;
  ConvArgs a{};
  a.H = H; a.W = W;
  a.in = ws.dr; a.w = r->w + OB4; a.mask = ws.a3; a.out = ws.d0;
  if ((e = conv(IN3, 32, EPI_MASK, a, B, s)) != hipSuccess) return e;
  // layer 3
  if ((e = wgrad(false, false, ws.d0, ws.a2, ws.part, ws.part2, r->g + W3, r->g + B3, 32 * 9 * 32, 32, B, H, W, s)) != hipSuccess) return e;
  a.in = ws.d0; a.w = r->w + OB3; a.mask = ws.a2; a.out = ws.d1;
  if ((e = conv(IN32, 32, EPI_MASK, a, B, s)) != hipSuccess) return e;
  // layer 2
  if ((e = wgrad(false, false, ws.d1, ws.a1, ws.part, ws.part2, r->g + W2, r->g + B2, 32 * 9 * 32, 32, B, H, W, s)) != hipSuccess) return e;
  a.in = ws.d1; a.w = r->w + OB2; a.mask = ws.a1; a.out = ws.d0;
  if ((e = conv(IN32, 32, EPI_MASK, a, B, s)) != hipSuccess) return e;
  // layer 1: dW1, db1 from (dz1, u)
  return wgrad(false, true, ws.d0, u, ws.part, ws.part2, r->g + W1, r->g + B1, 32 * 27, 32, B, H, W, s);
}

static hipError_t refresh_bf16(mci_refiner_s* r, hipStream_t s) {
  hipLaunchKernelGGL(k_weights_bf16, dim3((NBF + 255) / 256), dim3(256), 0, s, r->p, r->w);
  return hipGetLastError();
}

static mci_status check_img(int64_t B, int H, int W) {
  if (B < 0 || H < 1 || W < 1 || H > (1 << 15) || W > (1 << 15)) return rfail(MCI_E_INVALID_ARG, "bad image batch shape");
  return MCI_OK;
}

extern "C" {

mci_status mci_refiner_create(int device, uint64_t seed, mci_refiner_t* out) {
  if (!out) return rfail(MCI_E_INVALID_ARG, "out is NULL");
  *out = nullptr;
  int ndev = 0;
  RHIP(hipGetDeviceCount(&ndev));
  if (device < 0 || device >= ndev) return rfail(MCI_E_INVALID_ARG, "device");
  RHIP(hipSetDevice(device));
  mci_refiner_s* r = new mci_refiner_s();
  r->device = device;
  // He-normal initial weights for the hidden layers, a small last layer: the refiner starts
  // close to the identity map on the MCI upsample
  std::vector<float> h(NPARAM, 0.f);
  std::mt19937_64 rng(seed);
  std::normal_distribution<double> nd(0.0, 1.0);
  auto fill = [&](int off, int n, double sd) { for (int i = 0; i < n; ++i) h[off + i] = (float)(nd(rng) * sd); };
  fill(W1, 32 * 27, std::sqrt(2.0 / 27));
  fill(W2, 32 * 288, std::sqrt(2.0 / 288));
  fill(W3, 32 * 288, std::sqrt(2.0 / 288));
  fill(W4, 3 * 288, 1e-3);
  bool ok = hipMalloc(&r->p, NPARAM * 4) == hipSuccess && hipMalloc(&r->m, NPARAM * 4) == hipSuccess &&
            hipMalloc(&r->v, NPARAM * 4) == hipSuccess && hipMalloc(&r->g, NPARAM * 4) == hipSuccess &&
            hipMalloc(&r->w, NBF * sizeof(bf16)) == hipSuccess;
  if (!ok) { mci_refiner_destroy(r); return rfail(MCI_E_OUT_OF_MEMORY, "refiner parameters"); }
  std::vector<float> z(NPARAM, 0.f);
  if (hipMemcpy(r->p, h.data(), NPARAM * 4, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(r->m, z.data(), NPARAM * 4, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(r->v, z.data(), NPARAM * 4, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(r->g, z.data(), NPARAM * 4, hipMemcpyHostToDevice) != hipSuccess ||
      refresh_bf16(r, 0) != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
    mci_refiner_destroy(r);
    return rfail(MCI_E_DEVICE, "refiner init");
  }
  *out = r;
  return MCI_OK;
}

mci_status mci_refiner_destroy(mci_refiner_t r) {
  if (!r) return MCI_OK;
  (void)hipSetDevice(r->device);
  for (void* q : {(void*)r->p, (void*)r->m, (void*)r->v, (void*)r->g, (void*)r->w})
    if (q) (void)hipFree(q);
  delete r;
  return MCI_OK;
}

int64_t mci_refiner_num_params(void) { return NPARAM; }

mci_status mci_refiner_get_params(mci_refiner_t r, float* host, float* tau) {
  if (!r || !host) return rfail(MCI_E_INVALID_ARG, "NULL argument");
  RHIP(hipSetDevice(r->device));
  RHIP(hipDeviceSynchronize());
  RHIP(hipMemcpy(host, r->p, NPARAM * 4, hipMemcpyDeviceToHost));
  if (tau) *tau = r->tau;
  return MCI_OK;
}

mci_status mci_refiner_set_params(mci_refiner_t r, const float* host, float tau) {
  if (!r || !host) return rfail(MCI_E_INVALID_ARG, "NULL argument");
  if (!(tau >= 0.f)) return rfail(MCI_E_INVALID_ARG, "tau must be >= 0");
  RHIP(hipSetDevice(r->device));
  RHIP(hipDeviceSynchronize());
  RHIP(hipMemcpy(r->p, host, NPARAM * 4, hipMemcpyHostToDevice));
  RHIP(refresh_bf16(r, 0));
  RHIP(hipDeviceSynchronize());
  r->tau = tau;
  return MCI_OK;
}

// Checkpoint layout (little-endian, host memory): header {magic "MCIRFN01", int64 n_params,
// int64 step, float tau, uint32 reserved}, then the FP32 master parameters, the Adam first
// and second moments, n_params values each.
namespace {
struct CkptHeader {
  char magic[8];
  int64_t n_params;
  int64_t step;
  float tau;
  uint32_t reserved;
};
constexpr char kCkptMagic[8] = {'M', 'C', 'I', 'R', 'F', 'N', '0', '1'};
}  // namespace

size_t mci_refiner_state_size(void) { return sizeof(CkptHeader) + (size_t)3 * NPARAM * sizeof(float); }

mci_status mci_refiner_save_state(mci_refiner_t r, void* host, size_t len) {
  if (!r || !host) return rfail(MCI_E_INVALID_ARG, "NULL argument");
  if (len < mci_refiner_state_size()) return rfail(MCI_E_INVALID_ARG, "buffer smaller than mci_refiner_state_size()");
  RHIP(hipSetDevice(r->device));
  RHIP(hipDeviceSynchronize());
  CkptHeader h{};
  std::memcpy(h.magic, kCkptMagic, 8);
  h.n_params = NPARAM;
  h.step = r->step;
  h.tau = r->tau;
  char* out = (char*)host;
  std::memcpy(out, &h, sizeof h);
  float* body = (float*)(out + sizeof h);
  RHIP(hipMemcpy(body, r->p, NPARAM * 4, hipMemcpyDeviceToHost));
  RHIP(hipMemcpy(body + NPARAM, r->m, NPARAM * 4, hipMemcpyDeviceToHost));
  RHIP(hipMemcpy(body + 2 * NPARAM, r->v, NPARAM * 4, hipMemcpyDeviceToHost));
  return MCI_OK;
}

mci_status mci_refiner_load_state(mci_refiner_t r, const void* host, size_t len) {
  if (!r || !host) return rfail(MCI_E_INVALID_ARG, "NULL argument");
  if (len < mci_refiner_state_size()) return rfail(MCI_E_INVALID_ARG, "buffer smaller than mci_refiner_state_size()");
  CkptHeader h;
  std::memcpy(&h, host, sizeof h);
  if (std::memcmp(h.magic, kCkptMagic, 8) != 0 || h.n_params != NPARAM || h.step < 0 || !(h.tau >= 0.f))
    return rfail(MCI_E_INVALID_ARG, "not a refiner checkpoint of this network");
  const float* body = (const float*)((const char*)host + sizeof h);
  RHIP(hipSetDevice(r->device));
  RHIP(hipDeviceSynchronize());
  RHIP(hipMemcpy(r->p, body, NPARAM * 4, hipMemcpyHostToDevice));
  RHIP(hipMemcpy(r->m, body + NPARAM, NPARAM * 4, hipMemcpyHostToDevice));
  RHIP(hipMemcpy(r->v, body + 2 * NPARAM, NPARAM * 4, hipMemcpyHostToDevice));
  RHIP(refresh_bf16(r, 0));
  RHIP(hipDeviceSynchronize());
  r->step = h.step;
  r->tau = h.tau;
  return MCI_OK;
}

mci_status mci_refiner_get_grads(mci_refiner_t r, float* host) {
  if (!r || !host) return rfail(MCI_E_INVALID_ARG, "NULL argument");
  RHIP(hipSetDevice(r->device));
  RHIP(hipDeviceSynchronize());
  RHIP(hipMemcpy(host, r->g, NPARAM * 4, hipMemcpyDeviceToHost));
  return MCI_OK;
}

mci_status mci_refiner_workspace_size(int64_t batch, int h, int w, size_t* bytes) {
  if (!bytes) return rfail(MCI_E_INVALID_ARG, "NULL argument");
  mci_status st = check_img(batch, h, w);
  if (st != MCI_OK) return st;
  *bytes = ref_ws(nullptr, batch, h, w).bytes + 256;
  return MCI_OK;
}

mci_status mci_refiner_forward(mci_refiner_t r, const float* u, float* y, int64_t batch, int h, int w,
                               int apply_fallback, float* ratio, int* used, void* workspace, size_t ws_bytes,
                               hipStream_t stream) {
  if (!r || !u || !y) return rfail(MCI_E_INVALID_ARG, "NULL argument");
  mci_status st = check_img(batch, h, w);
  if (st != MCI_OK) return st;
  if (batch == 0) return MCI_OK;
  RefWs ws = ref_ws(workspace, batch, h, w);
  if (!workspace || ws_bytes < ws.bytes) return rfail(MCI_E_INVALID_ARG, "workspace too small");
  if (apply_fallback && (!ratio || !used)) return rfail(MCI_E_INVALID_ARG, "fallback needs ratio and used arrays");
  RHIP(hipSetDevice(r->device));
  // the weight-gradient partials buffer (unused by a forward call) takes the ratio's
  // per-tile sums
  RHIP(ref_forward(r, u, y, batch, h, w, ws, stream, ratio ? ws.part : nullptr, !std::getenv("MCI_REFINER_LAYERED")));
  if (ratio) {
    const int64_t per = 3 * (int64_t)h * w;
    const int tiles = ((h + T - 1) / T) * ((w + T - 1) / T);
    hipLaunchKernelGGL(k_ratio, dim3((unsigned)batch), dim3(NT), 0, stream, ws.part, tiles, ratio);
    RHIP(hipGetLastError());
    if (apply_fallback) {
      hipLaunchKernelGGL(k_fallback, dim3(64, (unsigned)batch), dim3(NT), 0, stream, y, u, per, ratio, r->tau, used);
      RHIP(hipGetLastError());
    }
  }
  return MCI_OK;
}

mci_status mci_refiner_backward(mci_refiner_t r, const float* u, const float* hr, int64_t batch, int h, int w,
                                float* loss_parts, int* n_parts, void* workspace, size_t ws_bytes, hipStream_t stream) {
  if (!r || !u || !hr) return rfail(MCI_E_INVALID_ARG, "NULL argument");
  mci_status st = check_img(batch, h, w);
  if (st != MCI_OK) return st;
  if (batch == 0) return rfail(MCI_E_INVALID_ARG, "empty batch");
  RefWs ws = ref_ws(workspace, batch, h, w);
  if (!workspace || ws_bytes < ws.bytes) return rfail(MCI_E_INVALID_ARG, "workspace too small");
  RHIP(hipSetDevice(r->device));
  int nl = 0;
  RHIP(ref_backward(r, u, hr, batch, h, w, ws, &nl, stream));
  if (loss_parts) RHIP(hipMemcpyAsync(loss_parts, ws.lpart, nl * sizeof(float), hipMemcpyDeviceToDevice, stream));
  if (n_parts) *n_parts = nl;
  return MCI_OK;
}

mci_status mci_refiner_train_step(mci_refiner_t r, const float* u, const float* hr, int64_t batch, int h, int w,
                                  float lr, float* loss_parts, int* n_parts, void* workspace, size_t ws_bytes,
                                  hipStream_t stream) {
  if (!(lr > 0.f)) return rfail(MCI_E_INVALID_ARG, "lr must be > 0");
  mci_status st = mci_refiner_backward(r, u, hr, batch, h, w, loss_parts, n_parts, workspace, ws_bytes, stream);
  if (st != MCI_OK) return st;
  r->step += 1;
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.f - std::pow(b1, (float)r->step), c2 = 1.f - std::pow(b2, (float)r->step);
  hipLaunchKernelGGL(k_adam, dim3((NPARAM + 255) / 256), dim3(256), 0, stream, r->p, r->m, r->v, r->g, NPARAM, lr, b1, b2,
                     1e-8f, c1, c2);
  RHIP(hipGetLastError());
  RHIP(refresh_bf16(r, stream));
  return MCI_OK;
}

const char* mci_refiner_last_error(void) { return r_err.c_str(); }

}  // extern "C"
