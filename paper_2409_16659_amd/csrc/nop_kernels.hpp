// nop_kernels.hpp -- matrix-core kernels of the convolutional
// neural-operator surrogate (gfx950): BF16 MFMA implicit-GEMM 3x3 periodic
// convolutions (forward with its GELU / residual epilogues, the input
// gradient through the same kernel with flipped transposed weights, and
// the weight gradient).  The FP32 VALU kernels around them (patch encoder,
// pixel-shuffle decoder, GELU gradient, reductions, MSE, Adam) are in
// surrogate.hip.
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

// tanh-form GELU and, if dg is given, its derivative
__device__ inline float gelu_f(float a, float* dg) {
  const float k0 = 0.7978845608028654f, k1 = 0.044715f;
  const float u = k0 * (a + k1 * a * a * a);
  const float th = tanhf(u);
  if (dg) *dg = 0.5f * (1.f + th) + 0.5f * a * (1.f - th * th) * k0 * (1.f + 3.f * k1 * a * a);
  return 0.5f * a * (1.f + th);
}

// Epilogues of the forward convolution: v = products + bias, then
//  kEpiPlain: out = v;
//  kEpiGelu:  out = v (pre-activation, FP32), outb = bf16(gelu(v));
//  kEpiResid: out = res + v, outb = bf16(out)  (residual block output).
enum { kEpiPlain = 0, kEpiGelu = 1, kEpiResid = 2 };

__device__ inline bf16x8 ld8(const __bf16* p) {
  const u32x4v w = *reinterpret_cast<const u32x4v*>(p);
  return __builtin_bit_cast(bf16x8, w);
}

// ---- 3x3 periodic convolution, forward (also used for the input gradient)
// out[b, y, x, co] = bias[co] + sum_{o, ci} W[o][co][ci] in[b, y+dy, x+dx, ci]
// A workgroup of WAVES waves covers WAVES rows of 64 pixels of one image and
// CO of the C output channels (channel group blockIdx.y); each wave computes
// 64 pixels x CO channels (CO / 16 column tiles).  The input channels are
// taken in slabs of 32 (one MFMA k-step): per slab the workgroup stages in
// LDS its WAVES + 2 input rows with one halo pixel on each side
// ([row][66][40] bf16) and the slab's weights of all nine offsets for its
// output channels ([9][CO][40] bf16; the stride of 40 spreads the 16 rows a
// wave reads over the banks), then every product of the slab reads LDS
// only.  Accumulation order per output: slabs, then offsets.  Dynamic LDS
// conv3x3_fwd_lds() bytes (up to ~142 KiB).  Requires gx % 64 == 0,
// gy % WAVES == 0, C % 32 == 0, CO | C.
constexpr int kConvPS = 40;  // LDS stride of a pixel / weight row (bf16)

__host__ __device__ constexpr size_t conv3x3_fwd_lds(int CO, int waves) {
  return (size_t)((waves + 2) * 66 + 9 * CO) * kConvPS * 2;
}

template <int C, int CO, int WAVES, int EPI>
__global__ void __launch_bounds__(64 * WAVES) conv3x3_fwd(const __bf16* __restrict__ in,
                                                           const __bf16* __restrict__ w,
                                                           const float* __restrict__ bias, float* __restrict__ out,
                                                           const float* __restrict__ res, __bf16* __restrict__ outb,
                                                           int gy, int gx) {
  constexpr int NT = CO / 16, NTH = 64 * WAVES, PS = kConvPS, ROWS = WAVES + 2, PX = 66;
  constexpr int NXP = ROWS * PX * 4, NWP = 9 * CO * 4;  // 16-byte pieces of a slab
  constexpr int XPER = (NXP + NTH - 1) / NTH, WPER = (NWP + NTH - 1) / NTH, NP = XPER + WPER;
  // Prefetch the next slab into registers during this slab's products when
  // the staging registers fit beside the accumulators; otherwise stage each
  // slab after the barrier that frees LDS, in groups of loads issued together.
  constexpr bool kPrefetch = 16 * NT + 4 * NP <= 160;
  constexpr int G = kPrefetch ? NP : 4;
  extern __shared__ __bf16 conv_smem[];
  __bf16* sx = conv_smem;                 // [ROWS][PX][PS]
  __bf16* sw = conv_smem + ROWS * PX * PS; // [9][CO][PS]
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int xtiles = gx / 64;
  const int xt = blockIdx.x % xtiles;
  const int rowblk = blockIdx.x / xtiles;  // (b, group of WAVES rows)
  const int rows_per_img = gy / WAVES;
  const int b = rowblk / rows_per_img;
  const int y0 = (rowblk % rows_per_img) * WAVES;
  const int cg = blockIdx.y;
  const int r = lane & 15, g = lane >> 4;
  f32x4 acc[4][NT];
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int n = 0; n < NT; ++n) acc[m][n] = f32x4{0.f, 0.f, 0.f, 0.f};
  const __bf16* img = in + (long long)b * gy * gx * C;
  // 16-byte piece j of this thread (input pieces first, then weights):
  // its source at slab c0 and its place in LDS; false past the slab's end
  auto piece = [&](int j, int c0, const u32x4v*& src, u32x4v*& dst) -> bool {
    const int t = threadIdx.x + (j < XPER ? j : j - XPER) * NTH;
    const int q = t & 3;
    if (j < XPER) {
      if (t >= NXP) return false;
      const int px = (t >> 2) % PX, row = (t >> 2) / PX;
      const int yy = pwrap(y0 - 1 + row, gy), xx = pwrap(xt * 64 - 1 + px, gx);
      src = reinterpret_cast<const u32x4v*>(img + (yy * gx + xx) * C + c0 + 8 * q);
      dst = reinterpret_cast<u32x4v*>(sx + (row * PX + px) * PS + 8 * q);
    } else {
      if (t >= NWP) return false;
      const int co = (t >> 2) % CO, o = (t >> 2) / CO;
      src = reinterpret_cast<const u32x4v*>(w + (o * C + cg * CO + co) * C + c0 + 8 * q);
      dst = reinterpret_cast<u32x4v*>(sw + (o * CO + co) * PS + 8 * q);
    }
    return true;
  };
  u32x4v st[G];
  auto fetch = [&](int j0, int c0) {
#pragma unroll
    for (int j = 0; j < G; ++j) {
      const u32x4v* src;
      u32x4v* dst;
      if (j0 + j < NP && piece(j0 + j, c0, src, dst)) st[j] = *src;
    }
  };
  auto put = [&](int j0) {
#pragma unroll
    for (int j = 0; j < G; ++j) {
      const u32x4v* src;
      u32x4v* dst;
      if (j0 + j < NP && piece(j0 + j, 0, src, dst)) *dst = st[j];
    }
  };
  auto products = [&]() {
#pragma unroll
    for (int o = 0; o < 9; ++o) {
      const int dy = o / 3 - 1, dx = o % 3 - 1;
      const __bf16* xrow = sx + (wave + 1 + dy) * PX * PS;
      bf16x8 a[4], bb[NT];
#pragma unroll
      for (int m = 0; m < 4; ++m) a[m] = ld8(xrow + (16 * m + r + 1 + dx) * PS + 8 * g);
#pragma unroll
      for (int n = 0; n < NT; ++n) bb[n] = ld8(sw + (o * CO + 16 * n + r) * PS + 8 * g);
#pragma unroll
      for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int n = 0; n < NT; ++n) acc[m][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[m], bb[n], acc[m][n], 0, 0, 0);
    }
  };
  if constexpr (kPrefetch) {
    fetch(0, 0);
#pragma unroll
    for (int c0 = 0; c0 < C; c0 += 32) {
      if (c0) __syncthreads();  // the previous slab's products are done with LDS
      put(0);
      __syncthreads();
      if (c0 + 32 < C) fetch(0, c0 + 32);
      products();
    }
  } else {
#pragma unroll 1
    for (int c0 = 0; c0 < C; c0 += 32) {
      if (c0) __syncthreads();
#pragma unroll
      for (int j0 = 0; j0 < NP; j0 += G) {
        fetch(j0, c0);
        put(j0);
      }
      __syncthreads();
      products();
    }
  }
  const int y = y0 + wave;
  const long long base = (((long long)b * gy + y) * gx + xt * 64) * C;
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int n = 0; n < NT; ++n) {
      const int co = cg * CO + 16 * n + r;
      const float bv = bias ? bias[co] : 0.f;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const long long e = base + (long long)(16 * m + 4 * g + i) * C + co;
        const float v = acc[m][n][i] + bv;
        if constexpr (EPI == kEpiPlain) {
          out[e] = v;
        } else if constexpr (EPI == kEpiGelu) {
          out[e] = v;
          outb[e] = (__bf16)gelu_f(v, nullptr);
        } else {
          const float s = res[e] + v;
          out[e] = s;
          outb[e] = (__bf16)s;
        }
      }
    }
}

// ---- 3x3 periodic convolution, weight gradient ----------------------------
// part[b][o][co][ci] = sum_{y, x} dy[b, y, x, co] in[b, y+dy_o, x+dx_o, ci]
// One workgroup per (image b, row offset dy, block of COB output channels):
// it marches the image in chunks of 64 pixels of one row and accumulates
// the three offsets (dy, -1), (dy, 0), (dy, +1) together.  Per chunk the
// workgroup stages dY (its COB channels) and the input row y + dy
// transposed in LDS ([channel][pixel], stride 72 so that 8 consecutive
// pixels are one 16-byte read), the input three times, shifted by
// dx = -1, 0, 1: a thread loads 8 channels of 4 consecutive pixels of dY
// and of 6 consecutive pixels of the input (one halo pixel each side) and
// writes 8-byte runs of 4 pixels of one channel.  Consecutive lanes take
// consecutive pixel groups, so the 16 lanes that write one channel row
// write 128 contiguous bytes (no bank conflicts; channel-fast lanes wrote
// 16 rows 8 apart into two bank groups, half the kernel's time).  The next
// chunk's loads are issued before the current products.  The 2 x 2 waves
// split the COB x C block; pixels are accumulated in order (32 per MFMA
// step), so every launch shape gives the same bits.  Dynamic LDS
// conv3x3_wgrad_lds() bytes.  Requires gx % 64 == 0, COB % 32 == 0, COB | C.
__host__ __device__ constexpr size_t conv3x3_wgrad_lds(int C, int COB) {
  return (size_t)(COB + 3 * C) * (64 + 8) * 2;
}

template <int C, int COB>
__global__ void __launch_bounds__(256) conv3x3_wgrad(const __bf16* __restrict__ in, const __bf16* __restrict__ dout,
                                                      float* __restrict__ part, int gy, int gx) {
  constexpr int CH = 64;                      // pixels per chunk
  constexpr int KP = CH + 8;                  // padded pixel stride of an LDS row (bf16)
  constexpr int RT = COB / 32, NT = C / 32;   // tiles per wave (2 x 2 waves over COB x C)
  constexpr int HB = C / COB;                 // output-channel blocks
  constexpr int DP = (CH / 4) * (COB / 8);    // dY pieces (4 pixels x 8 channels)
  constexpr int XP = (CH / 4) * (C / 8);      // input pieces (6 pixels x 8 channels)
  static_assert(DP <= 256 && XP <= 256, "one piece of each tensor per thread");
  typedef unsigned int u32x2v __attribute__((ext_vector_type(2)));
  extern __shared__ __bf16 wg_smem[];
  __bf16* sd = wg_smem;             // [COB][KP]  dY chunk
  __bf16* sx = wg_smem + COB * KP;  // [3][C][KP] input chunk shifted by dx = -1, 0, 1
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int h = blockIdx.x % HB, dyi = (blockIdx.x / HB) % 3, b = blockIdx.x / (3 * HB);
  const int r = lane & 15, g = lane >> 4;
  const int co0 = (wave >> 1) * (COB / 2), ci0 = (wave & 1) * (C / 2);
  f32x4 acc[3][RT][NT];
#pragma unroll
  for (int s = 0; s < 3; ++s)
#pragma unroll
    for (int m = 0; m < RT; ++m)
#pragma unroll
      for (int n = 0; n < NT; ++n) acc[s][m][n] = f32x4{0.f, 0.f, 0.f, 0.f};
  const __bf16* dimg = dout + (long long)b * gy * gx * C + h * COB;
  const __bf16* ximg = in + (long long)b * gy * gx * C;
  const int chunks_per_row = gx / CH, nch = gy * chunks_per_row;
  const int t = threadIdx.x;
  const int p4 = (t % (CH / 4)) * 4, c8 = (t / (CH / 4)) * 8;  // this thread's pieces
  bf16x8 vd[4], vx[6];
  auto fetch = [&](int ch) {
    const int y = ch / chunks_per_row, x0 = (ch % chunks_per_row) * CH;
    const int ys = pwrap(y + dyi - 1, gy);
    if (t < DP) {
#pragma unroll
      for (int q = 0; q < 4; ++q) vd[q] = ld8(dimg + (y * gx + x0 + p4 + q) * C + c8);
    }
    if (t < XP) {
#pragma unroll
      for (int q = 0; q < 6; ++q) vx[q] = ld8(ximg + (ys * gx + pwrap(x0 + p4 + q - 1, gx)) * C + c8);
    }
  };
  auto put = [&]() {
    if (t < DP) {
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        __bf16 a4[4] = {vd[0][e], vd[1][e], vd[2][e], vd[3][e]};
        *reinterpret_cast<u32x2v*>(sd + (c8 + e) * KP + p4) = __builtin_bit_cast(u32x2v, a4);
      }
    }
    if (t < XP) {
#pragma unroll
      for (int s = 0; s < 3; ++s)
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          __bf16 b4[4] = {vx[s][e], vx[s + 1][e], vx[s + 2][e], vx[s + 3][e]};
          *reinterpret_cast<u32x2v*>(sx + (s * C + c8 + e) * KP + p4) = __builtin_bit_cast(u32x2v, b4);
        }
    }
  };
  fetch(0);
  for (int ch = 0; ch < nch; ++ch) {
    put();
    __syncthreads();
    if (ch + 1 < nch) fetch(ch + 1);
#pragma unroll
    for (int k0 = 0; k0 < CH; k0 += 32) {
      bf16x8 a[RT];
#pragma unroll
      for (int m = 0; m < RT; ++m) a[m] = ld8(sd + (co0 + 16 * m + r) * KP + k0 + 8 * g);
#pragma unroll
      for (int s = 0; s < 3; ++s) {
        bf16x8 bb[NT];
#pragma unroll
        for (int n = 0; n < NT; ++n) bb[n] = ld8(sx + (s * C + ci0 + 16 * n + r) * KP + k0 + 8 * g);
#pragma unroll
        for (int m = 0; m < RT; ++m)
#pragma unroll
          for (int n = 0; n < NT; ++n)
            acc[s][m][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[m], bb[n], acc[s][m][n], 0, 0, 0);
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int s = 0; s < 3; ++s) {
    float* pb = part + ((long long)b * 9 + dyi * 3 + s) * C * C;
#pragma unroll
    for (int m = 0; m < RT; ++m)
#pragma unroll
      for (int n = 0; n < NT; ++n) {
        const int ci = ci0 + 16 * n + r;
#pragma unroll
        for (int i = 0; i < 4; ++i) pb[(long long)(h * COB + co0 + 16 * m + 4 * g + i) * C + ci] = acc[s][m][n][i];
      }
  }
}

}  // namespace nop
