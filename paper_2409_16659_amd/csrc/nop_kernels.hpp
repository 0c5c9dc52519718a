// nop_kernels.hpp -- kernels of the convolutional neural-operator surrogate
// (gfx950): BF16 MFMA implicit-GEMM 3x3 periodic convolutions (forward,
// input gradient through the same kernel with flipped transposed weights,
// weight gradient), and the FP32 VALU kernels around them (patch encoder,
// pixel-shuffle decoder, GELU, residual sums, bias sums, MSE, Adam).
//
// Latent tensors are NHWC: [batch][gy][gx][C], C a multiple of 32, x
// fastest after the channels; the grid is periodic in both directions.
// Conv weights for the MFMA kernels are BF16 [9][C_out][C_in] (offset
// o = 3 (dy + 1) + (dx + 1)), C_in contiguous, so that one lane's 8
// consecutive k values are one 16-byte load.
//
// MFMA v_mfma_f32_16x16x32_bf16 lane layout (wave64): A (16 x 32): lane l
// holds row l % 16, k = 8 (l / 16) .. +7; B (32 x 16): lane l holds column
// l % 16 for the same k; D (16 x 16): lane l holds rows 4 (l / 16) + i,
// i = 0..3, column l % 16.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nop {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4v __attribute__((ext_vector_type(4)));

__device__ inline int pwrap(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

__device__ inline bf16x8 ld8(const __bf16* p) {
  const u32x4v w = *reinterpret_cast<const u32x4v*>(p);
  return __builtin_bit_cast(bf16x8, w);
}

// ---- 3x3 periodic convolution, forward (also used for the input gradient)
// out[b, y, x, co] = bias[co] + sum_{o, ci} W[o][co][ci] in[b, y+dy, x+dx, ci]
// One workgroup = 4 waves = 4 rows of 64 pixels of one image; each wave
// computes 64 pixels x C output channels (C / 16 column tiles).  Requires
// gx == 64 * XT (XT >= 1 tiles of 64 pixels per row handled by the grid),
// C % 32 == 0, C <= 256.
template <int C>
__global__ void __launch_bounds__(256) conv3x3_fwd(const __bf16* __restrict__ in, const __bf16* __restrict__ w,
                                                    const float* __restrict__ bias, float* __restrict__ out, int gy,
                                                    int gx) {
  constexpr int NT = C / 16;  // column (output channel) tiles per wave
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int xtiles = gx / 64;
  const int blk = blockIdx.x;
  const int xt = blk % xtiles;
  const int rowblk = blk / xtiles;  // (b, 4-row group)
  const int rows_per_img = gy / 4;
  const int b = rowblk / rows_per_img;
  const int y = (rowblk % rows_per_img) * 4 + wave;
  const int r = lane & 15, g = lane >> 4;
  f32x4 acc[4][NT];
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int n = 0; n < NT; ++n) acc[m][n] = f32x4{0.f, 0.f, 0.f, 0.f};
  const __bf16* img = in + (long long)b * gy * gx * C;
  for (int o = 0; o < 9; ++o) {
    const int dy = o / 3 - 1, dx = o % 3 - 1;
    const int yy = pwrap(y + dy, gy);
    const __bf16* rowp = img + (long long)yy * gx * C;
    const __bf16* wo = w + (long long)o * C * C;
#pragma unroll 1
    for (int c0 = 0; c0 < C; c0 += 32) {
      bf16x8 a[4], bb[NT];
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const int xx = pwrap(xt * 64 + 16 * m + r + dx, gx);
        a[m] = ld8(rowp + (long long)xx * C + c0 + 8 * g);
      }
#pragma unroll
      for (int n = 0; n < NT; ++n) bb[n] = ld8(wo + (long long)(16 * n + r) * C + c0 + 8 * g);
#pragma unroll
      for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int n = 0; n < NT; ++n) acc[m][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[m], bb[n], acc[m][n], 0, 0, 0);
    }
  }
  float* orow = out + (((long long)b * gy + y) * gx + xt * 64) * C;
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int n = 0; n < NT; ++n) {
      const int co = 16 * n + r;
      const float bv = bias ? bias[co] : 0.f;
#pragma unroll
      for (int i = 0; i < 4; ++i) orow[(long long)(16 * m + 4 * g + i) * C + co] = acc[m][n][i] + bv;
    }
}

// ---- 3x3 periodic convolution, weight gradient ----------------------------
// part[b][o][co][ci] = sum_{y, x} dy[b, y, x, co] in[b, y+dy_o, x+dx_o, ci]
// One workgroup per (image b, offset o); it marches the image in chunks of
// 32 pixels of one row, staging dY and the shifted input transposed in LDS
// ([channel][pixel]) so that 8 consecutive pixels are one 16-byte read.
// The C x C result is split over 4 waves by output-channel row tiles.
template <int C>
__global__ void __launch_bounds__(256) conv3x3_wgrad(const __bf16* __restrict__ in, const __bf16* __restrict__ dout,
                                                      float* __restrict__ part, int gy, int gx) {
  constexpr int NT = C / 16;          // tiles per dimension
  constexpr int RT = NT / 4;          // row tiles per wave (C / 64)
  constexpr int KP = 32 + 8;          // padded pixel stride of an LDS row (bf16)
  __shared__ __bf16 sd[C * KP];       // dY chunk, [co][px]
  __shared__ __bf16 sx[C * KP];       // input chunk, [ci][px]
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int b = blockIdx.x / 9, o = blockIdx.x % 9;
  const int dy = o / 3 - 1, dx = o % 3 - 1;
  const int r = lane & 15, g = lane >> 4;
  f32x4 acc[RT][NT];
#pragma unroll
  for (int m = 0; m < RT; ++m)
#pragma unroll
    for (int n = 0; n < NT; ++n) acc[m][n] = f32x4{0.f, 0.f, 0.f, 0.f};
  const __bf16* dimg = dout + (long long)b * gy * gx * C;
  const __bf16* ximg = in + (long long)b * gy * gx * C;
  const int chunks_per_row = gx / 32;
  for (int ch = 0; ch < gy * chunks_per_row; ++ch) {
    const int y = ch / chunks_per_row, x0 = (ch % chunks_per_row) * 32;
    const int ys = pwrap(y + dy, gy);
    // stage: 32 pixels x C channels of each tensor, 8 channels per thread-load
    for (int t = threadIdx.x; t < 32 * (C / 8); t += 256) {
      const int px = t / (C / 8), c8 = (t % (C / 8)) * 8;
      const bf16x8 vd = ld8(dimg + ((long long)y * gx + x0 + px) * C + c8);
      const int xs = pwrap(x0 + px + dx, gx);
      const bf16x8 vx = ld8(ximg + ((long long)ys * gx + xs) * C + c8);
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        sd[(c8 + j) * KP + px] = vd[j];
        sx[(c8 + j) * KP + px] = vx[j];
      }
    }
    __syncthreads();
    bf16x8 a[RT], bb[NT];
#pragma unroll
    for (int m = 0; m < RT; ++m) a[m] = ld8(sd + (16 * (wave * RT + m) + r) * KP + 8 * g);
#pragma unroll
    for (int n = 0; n < NT; ++n) bb[n] = ld8(sx + (16 * n + r) * KP + 8 * g);
#pragma unroll
    for (int m = 0; m < RT; ++m)
#pragma unroll
      for (int n = 0; n < NT; ++n) acc[m][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[m], bb[n], acc[m][n], 0, 0, 0);
    __syncthreads();
  }
  float* pb = part + ((long long)b * 9 + o) * C * C;
#pragma unroll
  for (int m = 0; m < RT; ++m)
#pragma unroll
    for (int n = 0; n < NT; ++n) {
      const int ci = 16 * n + r;
#pragma unroll
      for (int i = 0; i < 4; ++i) pb[(long long)(16 * (wave * RT + m) + 4 * g + i) * C + ci] = acc[m][n][i];
    }
}

}  // namespace nop
