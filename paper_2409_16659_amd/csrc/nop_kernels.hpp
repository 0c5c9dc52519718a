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

// tanh-form GELU, 0.5 a (1 + tanh(u)) with u = k0 (a + k1 a^3), and, if dg
// is given, its derivative.  Evaluated through the identity
// 0.5 (1 + tanh(u)) = 1 / (1 + exp(-2u)) = s with the hardware exp2 and
// reciprocal (each within about an ulp): gelu = a s and
// gelu' = s + 2 a s (1 - s) u'.  For large |a| the exponential saturates to
// 0 or infinity and s to 1 or 0 exactly.
__device__ inline float gelu_f(float a, float* dg) {
  const float k0 = 0.7978845608028654f, k1 = 0.044715f;
  const float u = k0 * (a + k1 * a * a * a);
  const float e = __builtin_amdgcn_exp2f(-2.8853900817779268f * u);  // exp(-2u), 2 log2(e) = 2.885...
  const float s = __builtin_amdgcn_rcpf(1.f + e);
  if (dg) *dg = s + 2.f * a * s * (1.f - s) * k0 * (1.f + 3.f * k1 * a * a);
  return a * s;
}

// Epilogues of the forward convolution: v = products + bias, then
//  kEpiPlain: out = v;
//  kEpiGelu:  out = v (pre-activation, FP32), outb = bf16(gelu(v));
//  kEpiResid: out = res + v, outb = bf16(out)  (residual block output; res
//             joins the accumulators partway through the products, in an
//             order fixed per output channel).
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
// taken in slabs of 32 (one MFMA k-step).  Per slab the workgroup stages in
// LDS its WAVES + 2 input rows with one halo pixel on each side
// ([row][66 pixels][32 channels] bf16), and the weights one row offset dy
// at a time ([3 dx][CO][32] bf16, three stages per slab, two buffers: the
// next stage's weights load during this stage's products), so that the
// LDS of a 4-wave workgroup (73 KiB at CO = 128) lets two workgroups share
// a CU: one's staging and epilogue overlap the other's products.  LDS rows
// are 64 bytes with their four 16-byte chunks permuted by XOR with
// (row / 2) % 4: the eight consecutive rows that eight lanes of a fragment
// read fall in distinct banks without padding.  Accumulation order per
// output: slabs, then offsets.  Dynamic LDS conv3x3_fwd_lds() bytes.
// Requires gx % 64 == 0, gy % WAVES == 0, C % 32 == 0, CO | C.
// Column tiles per epilogue pass (two: 32 channels, one 128-byte FP32 line
// per pixel) and the LDS of the products and of the epilogue.
__host__ __device__ constexpr int conv_epi_group(int CO) { return CO / 16 < 2 ? CO / 16 : 2; }
__host__ __device__ constexpr size_t conv3x3_fwd_lds(int CO, int waves) {
  const size_t prod = (size_t)((waves + 2) * 66 + 2 * 3 * CO) * 64;
  const size_t epi = (size_t)waves * 64 * (16 * conv_epi_group(CO) + 4) * 4;
  return prod > epi ? prod : epi;
}

// byte offset of 16-byte chunk q of 64-byte LDS row `row`
__device__ inline int swz(int row, int q) { return row * 64 + ((q ^ (row >> 1)) & 3) * 16; }

template <int C, int CO, int WAVES, int EPI>
__global__ void __launch_bounds__(64 * WAVES, 2) conv3x3_fwd(const __bf16* __restrict__ in,
                                                              const __bf16* __restrict__ w,
                                                              const float* __restrict__ bias, float* __restrict__ out,
                                                              const float* __restrict__ res, __bf16* __restrict__ outb,
                                                              int gy, int gx) {
  constexpr int NT = CO / 16, ROWS = WAVES + 2, PX = 66;
  constexpr int NXP = ROWS * PX * 4, NWP = 3 * CO * 4;  // 16-byte pieces: input rows, one offset row of weights
  constexpr int NXI = (NXP + 63) / 64, NWI = (NWP + 63) / 64;  // LDS-direct wave loads of 64 pieces
  constexpr int NST = (C / 32) * 3;                            // stages: slab x row offset
  extern __shared__ __attribute__((aligned(16))) unsigned char conv_lds[];
  unsigned char* sx = conv_lds;              // [ROWS * PX] rows of 64 bytes
  unsigned char* sw0 = conv_lds + NXP * 16;  // [2][3 * CO] rows of 64 bytes
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
  // Staging with LDS-direct loads (global_load_lds_dwordx4): lane l of a
  // wave's load i writes 16 bytes at base + 1024 i + 16 l, so piece
  // t = 64 i + l fills position t & 3 of LDS row t / 4; the swizzle is
  // applied on the source side (that position holds chunk
  // (t & 3) ^ ((row / 2) % 4)).  No staging registers; the loads are waited
  // for (vmcnt) before the barrier that publishes them.
  auto issue_x = [&](int c0) {  // the slab's input rows: row = (tile row, pixel)
#pragma unroll
    for (int i = wave; i < NXI; i += WAVES) {
      const int t = 64 * i + lane;
      if (t < NXP) {
        const int R = t >> 2, q = (t & 3) ^ ((R >> 1) & 3);
        const int yy = pwrap(y0 - 1 + R / PX, gy), xx = pwrap(xt * 64 - 1 + R % PX, gx);
        __builtin_amdgcn_global_load_lds(img + ((long long)yy * gx + xx) * C + c0 + 8 * q, sx + 1024 * i, 16, 0, 0);
      }
    }
  };
  auto issue_w = [&](int c0, int d, int buf) {  // the slab's weights of row offset d: row = (dx, co)
    unsigned char* sw = sw0 + buf * NWP * 16;
#pragma unroll
    for (int i = wave; i < NWI; i += WAVES) {
      const int t = 64 * i + lane;
      if (t < NWP) {
        const int R = t >> 2, q = (t & 3) ^ ((R >> 1) & 3);
        const int o = 3 * d + R / CO, co = R % CO;
        __builtin_amdgcn_global_load_lds(w + ((long long)o * C + cg * CO + co) * C + c0 + 8 * q, sw + 1024 * i, 16,
                                         0, 0);
      }
    }
  };
  // Residual epilogue: the residual input of global column tile t
  // (channels 16 t ..) is added to its accumulators after stage 3 t / 2,
  // loaded before that stage's products, so that its traffic spreads over
  // the products instead of adding to the epilogue's burst.  The stage of each
  // output channel depends on the channel only: every launch shape
  // accumulates in the same order.
  const long long pbase = (((long long)b * gy + y0 + wave) * gx + xt * 64) * C;
  float rv[4][4];
  // Stage s (slab s / 3, row offset d = s % 3) reads the input rows and
  // weight buffer s % 2; the next stage's weights load into the other
  // buffer during its products; a new slab's input rows load after the
  // barrier that ends the previous slab.
  issue_x(0);
  issue_w(0, 0, 0);
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
#pragma unroll 1
  for (int st = 0; st < NST; ++st) {
    const int c0 = (st / 3) * 32, d = st % 3;
    if (st + 1 < NST) issue_w(((st + 1) / 3) * 32, (st + 1) % 3, (st + 1) & 1);
    // global tile t joins after stage 3 t / 2: C / 16 tiles spread over the
    // 3 C / 32 stages (stages 0, 1, 3, 4, 6, ...)
    const int tres = (2 * st + 2) / 3;
    const int nres = ((3 * tres) / 2 == st ? tres : -1 - NT * (C / CO)) - cg * NT;
    if constexpr (EPI == kEpiResid) {
      if (nres >= 0 && nres < NT) {
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
          for (int i = 0; i < 4; ++i)
            rv[m][i] = res[pbase + (long long)(16 * m + 4 * g + i) * C + cg * CO + 16 * nres + r];
      }
    }
    const unsigned char* sw = sw0 + (st & 1) * NWP * 16;
    const int xrow = (wave + d) * PX;  // input row y + dy, dy = d - 1
#pragma unroll
    for (int dx = 0; dx < 3; ++dx) {
      bf16x8 a[4];
#pragma unroll
      for (int m = 0; m < 4; ++m)
        a[m] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u32x4v*>(sx + swz(xrow + 16 * m + r + dx, g)));
      // each weight fragment is read just before its four products: holding
      // all NT of them would take the residual variant past 256 VGPRs
#pragma unroll
      for (int n = 0; n < NT; ++n) {
        const bf16x8 bn =
            __builtin_bit_cast(bf16x8, *reinterpret_cast<const u32x4v*>(sw + swz(dx * CO + 16 * n + r, g)));
#pragma unroll
        for (int m = 0; m < 4; ++m)
          acc[m][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[m], bn, acc[m][n], 0, 0, 0);
      }
    }
    if constexpr (EPI == kEpiResid) {
#pragma unroll
      for (int n = 0; n < NT; ++n)
        if (n == nres) {
#pragma unroll
          for (int m = 0; m < 4; ++m)
#pragma unroll
            for (int i = 0; i < 4; ++i) acc[m][n][i] += rv[m][i];
        }
    }
    __builtin_amdgcn_s_waitcnt(0);  // the next stage's weights are in LDS
    __syncthreads();                // and every wave is done with this stage's
    if (st + 1 < NST && d == 2) {   // a new slab: its input rows
      issue_x(c0 + 32);
      __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
    }
  }
  // Epilogue through LDS: the accumulators (+ bias) of two column tiles at
  // a time go to a per-wave [64 pixels][36] FP32 tile (row stride 4 banks
  // off a multiple of 32: the two pixel rows a b32 write spans fall in
  // different bank halves) and come back as 4 consecutive channels per
  // lane, 8 lanes per pixel, so that every global store of the epilogue
  // (FP32 output, its BF16 copy) is a 16- or 8-byte access of whole
  // 128-byte lines.  Same arithmetic per element as a direct store.
  constexpr int TG = conv_epi_group(CO), ES = 16 * TG + 4;
  constexpr int Q = 4 * TG, P = 64 / Q, IT = 64 / P;  // lanes per pixel, pixels per pass, passes per tile group
  static_assert((size_t)WAVES * 64 * ES * 4 <= conv3x3_fwd_lds(CO, WAVES) && NT % TG == 0, "epilogue tile fits");
  float* se = reinterpret_cast<float*>(conv_lds) + wave * 64 * ES;
  const long long base = pbase + cg * CO;
  const int c4 = 4 * (lane % Q), p0 = lane / Q;
#pragma unroll
  for (int n0 = 0; n0 < NT; n0 += TG) {
    if (n0) __syncthreads();  // the previous group has been read back
#pragma unroll
    for (int nn = 0; nn < TG; ++nn) {
      const float bv = bias ? bias[cg * CO + 16 * (n0 + nn) + r] : 0.f;
#pragma unroll
      for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int i = 0; i < 4; ++i) se[(16 * m + 4 * g + i) * ES + 16 * nn + r] = acc[m][n0 + nn][i] + bv;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < IT; ++k) {
      const f32x4 o = *reinterpret_cast<const f32x4*>(se + (p0 + P * k) * ES + c4);
      const long long e = base + (long long)(p0 + P * k) * C + 16 * n0 + c4;
      *reinterpret_cast<f32x4*>(out + e) = o;
      if constexpr (EPI != kEpiPlain) {
        __bf16 q4[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) q4[j] = (__bf16)(EPI == kEpiGelu ? gelu_f(o[j], nullptr) : o[j]);
        typedef unsigned int u32x2e __attribute__((ext_vector_type(2)));
        *reinterpret_cast<u32x2e*>(outb + e) = __builtin_bit_cast(u32x2e, q4);
      }
    }
  }
}

// ---- 3x3 periodic convolution, weight gradient ----------------------------
// part[s][o][co][ci] = sum over the pixels (b, y, x) of slice s of
//                      dy[b, y, x, co] in[b, y+dy_o, x+dx_o, ci]
// The batch's pixels, in chunks of 64 of one row in (image, row, column)
// order, are cut into nslice slices of consecutive chunks (a slice may span
// images; the row offset wraps within each image).  One workgroup per
// (slice, row offset dy) computes the three offsets (dy, -1), (dy, 0),
// (dy, +1) for all C x C channel pairs: waves WM x WN split the (co, ci)
// block, each holding 3 x (C/WM) x (C/WN) accumulators; with 3 nslice no
// larger than the CU count every CU holds one workgroup, whatever the
// batch.  The slice is marched chunk by chunk.  Per chunk the
// workgroup stages dY and the input row y + dy transposed in LDS, the input
// once: [k-half][channel] rows of 64 bytes (32 pixels, one MFMA k-step)
// whose four 16-byte chunks are permuted by XOR with (row / 2) % 4, the
// layout whose fragment reads (16 consecutive rows x 4 chunks) run without
// bank conflicts on gfx950 (rows padded to 72 or 88 bf16 cost twice as
// much); the input's two halo pixels sit in two dword arrays.  The
// fragments shifted by one pixel (dx = -1, +1) are formed in registers
// from the unshifted one and the dwords on either side (v_alignbit), so
// LDS holds and serves each input value once.  A thread stages pieces of
// 8 channels x 4 consecutive pixels (four 16-byte global loads, eight
// 8-byte LDS writes); consecutive lanes take consecutive pixel groups.
// Two LDS buffers: the next chunk's loads are issued before the current
// chunk's products and written after them, one barrier per chunk.  Pixels
// are accumulated in order (32 per MFMA step), so every launch with the
// same nslice gives the same bits.  On the device's eight XCDs (each with
// its own L2) the three workgroups of one slice are given to one XCD when
// the grid divides by 8.
// Dynamic LDS conv3x3_wgrad_lds(C) bytes.  Requires gx % 64 == 0,
// C % (16 WM) == 0, C % (16 WN) == 0.
constexpr int kWgChunk = 64;  // pixels per chunk (two k-halves of 32)
__host__ __device__ constexpr size_t conv3x3_wgrad_lds(int C) {
  return (size_t)2 * (2 * 2 * C * 64 + 2 * C * 4);  // per buffer: dY and input half-rows, halo dwords
}

template <int C, int WM, int WN>
__global__ void __launch_bounds__(64 * WM * WN) conv3x3_wgrad(const __bf16* __restrict__ in,
                                                               const __bf16* __restrict__ dout,
                                                               float* __restrict__ part, int batch, int gy, int gx,
                                                               int nslice) {
  constexpr int NTH = 64 * WM * WN, CH = kWgChunk;
  constexpr int MT = C / WM / 16, NT = C / WN / 16;  // 16 x 16 tiles per wave (co, ci)
  constexpr int PC = (CH / 4) * (C / 8);             // pieces of one tensor per chunk
  constexpr int HALO = 2 * (C / 8);                  // halo pieces: 1 pixel x 8 channels
  constexpr int NPC = 2 * PC + HALO, NSP = (NPC + NTH - 1) / NTH;
  constexpr int BUFB = 2 * 2 * C * 64 + 2 * C * 4;   // bytes per buffer
  static_assert(C % (16 * WM) == 0 && C % (16 * WN) == 0, "wave tiles of whole 16 x 16 blocks");
  typedef unsigned int u32x2v __attribute__((ext_vector_type(2)));
  extern __shared__ __attribute__((aligned(16))) unsigned char wg_lds[];
  // buffer layout: dY rows [2][C], input rows [2][C] (64 bytes each), then
  // halo dwords [2][C]: (0, in[-1]) and (in[64], 0) as bf16 pairs
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, t = threadIdx.x;
  // (slice, row offset) of this workgroup; the three row offsets of a
  // slice share an XCD when the grid divides by 8 (padding workgroups
  // beyond 3 nslice exit)
  const int nwg = gridDim.x;
  const int item = nwg % 8 == 0 ? (blockIdx.x % 8) * (nwg / 8) + blockIdx.x / 8 : blockIdx.x;
  if (item >= 3 * nslice) return;
  const int sl = item / 3, dyi = item % 3;
  const int r = lane & 15, g = lane >> 4;
  const int co0 = (wave / WN) * (C / WM), ci0 = (wave % WN) * (C / WN);
  f32x4 acc[3][MT][NT];
#pragma unroll
  for (int s = 0; s < 3; ++s)
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
      for (int n = 0; n < NT; ++n) acc[s][m][n] = f32x4{0.f, 0.f, 0.f, 0.f};
  // chunks of CH pixels in (image, row, column) order; slice sl takes
  // [c0, c1) of the batch's chunks
  const int cpr = gx / CH, cpi = gy * cpr;
  const long long total = (long long)batch * cpi;
  const int c0 = (int)(total * sl / nslice), c1 = (int)(total * (sl + 1) / nslice);
  typedef u32x4v Stage[NSP][4];
  Stage sa;
  // piece j: [0, PC) dY, [PC, 2 PC) input (pixel group j % 16, channels
  // 8 (j / 16) ..), then the halo pixels
  auto fetch = [&](int ch, Stage& st) {
    const int b = ch / cpi, cc = ch - b * cpi;
    const int y = cc / cpr, x0 = (cc % cpr) * CH;
    const int ys = pwrap(y + dyi - 1, gy);
    const __bf16* dimg = dout + (long long)b * gy * gx * C;
    const __bf16* ximg = in + (long long)b * gy * gx * C;
#pragma unroll
    for (int jj = 0; jj < NSP; ++jj) {
      const int j = t + jj * NTH;
      if (j < 2 * PC) {
        const int jp = j < PC ? j : j - PC;
        const int pg = jp % (CH / 4), c8 = (jp / (CH / 4)) * 8;
        const __bf16* src = j < PC ? dimg + ((long long)y * gx + x0 + 4 * pg) * C + c8
                                   : ximg + ((long long)ys * gx + x0 + 4 * pg) * C + c8;
#pragma unroll
        for (int q = 0; q < 4; ++q) st[jj][q] = *reinterpret_cast<const u32x4v*>(src + q * C);
      } else if (j < NPC) {
        const int jh = j - 2 * PC, side = jh / (C / 8), c8 = (jh % (C / 8)) * 8;
        const int xs = side ? pwrap(x0 + CH, gx) : pwrap(x0 - 1, gx);
        st[jj][0] = *reinterpret_cast<const u32x4v*>(ximg + ((long long)ys * gx + xs) * C + c8);
      }
    }
  };
  auto put = [&](int buf, const Stage& st) {
    unsigned char* base = wg_lds + buf * BUFB;
#pragma unroll
    for (int jj = 0; jj < NSP; ++jj) {
      const int j = t + jj * NTH;
      if (j < 2 * PC) {
        const bool isd = j < PC;
        const int jp = isd ? j : j - PC;
        const int pg = jp % (CH / 4), c8 = (jp / (CH / 4)) * 8;
        const int kh = pg / 8, q = (pg % 8) / 2;
        const int row0 = (isd ? 0 : 2 * C) + kh * C + c8;
        bf16x8 v[4];
#pragma unroll
        for (int qq = 0; qq < 4; ++qq) v[qq] = __builtin_bit_cast(bf16x8, st[jj][qq]);
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          __bf16 a4[4] = {v[0][e], v[1][e], v[2][e], v[3][e]};
          *reinterpret_cast<u32x2v*>(base + swz(row0 + e, q) + 8 * (pg % 2)) = __builtin_bit_cast(u32x2v, a4);
        }
      } else if (j < NPC) {
        const int jh = j - 2 * PC, side = jh / (C / 8), c8 = (jh % (C / 8)) * 8;
        // channels c8 .. c8 + 7, two per dword (low half first); taken apart
        // with shifts: a bit cast of a vector element compiled to element 0
        // for every e here
        const u32x4v w = st[jj][0];
        unsigned* hx = reinterpret_cast<unsigned*>(base + 4 * C * 64) + side * C + c8;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const unsigned bits = (e & 1) ? w[e / 2] >> 16 : w[e / 2] & 0xffffu;
          hx[e] = side ? bits : bits << 16;
        }
      }
    }
  };
  auto compute = [&](int buf) {
    const unsigned char* base = wg_lds + buf * BUFB;
    const unsigned* hx = reinterpret_cast<const unsigned*>(base + 4 * C * 64);
#pragma unroll
    for (int kh = 0; kh < 2; ++kh) {
      bf16x8 a[MT];
#pragma unroll
      for (int m = 0; m < MT; ++m)
        a[m] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u32x4v*>(base + swz(kh * C + co0 + 16 * m + r, g)));
#pragma unroll
      for (int n = 0; n < NT; ++n) {
        const int ci = ci0 + 16 * n + r, xr = 2 * C + ci;  // input row of k-half 0
        // pixels p = 32 kh + 8 g .. + 7 of channel ci; the dword holding
        // pixel p - 1 (high half) and the one holding p + 8 (low half)
        const u32x4v d = *reinterpret_cast<const u32x4v*>(base + swz(xr + kh * C, g));
        const unsigned* pp = (kh == 0 && g == 0)
                                 ? hx + ci
                                 : reinterpret_cast<const unsigned*>(
                                       base + swz(xr + (g == 0 ? kh - 1 : kh) * C, (g + 3) & 3) + 12);
        const unsigned* pn = (kh == 1 && g == 3)
                                 ? hx + C + ci
                                 : reinterpret_cast<const unsigned*>(base + swz(xr + (g == 3 ? kh + 1 : kh) * C,
                                                                                (g + 1) & 3));
        const unsigned prev = *pp, next = *pn;
        const unsigned t0 = __builtin_amdgcn_alignbit(d.x, prev, 16), t1 = __builtin_amdgcn_alignbit(d.y, d.x, 16);
        const unsigned t2 = __builtin_amdgcn_alignbit(d.z, d.y, 16), t3 = __builtin_amdgcn_alignbit(d.w, d.z, 16);
        const unsigned t4 = __builtin_amdgcn_alignbit(next, d.w, 16);
        const bf16x8 bm = __builtin_bit_cast(bf16x8, u32x4v{t0, t1, t2, t3});  // in[p - 1]
        const bf16x8 b0 = __builtin_bit_cast(bf16x8, d);                      // in[p]
        const bf16x8 bp = __builtin_bit_cast(bf16x8, u32x4v{t1, t2, t3, t4});  // in[p + 1]
#pragma unroll
        for (int m = 0; m < MT; ++m) {
          acc[0][m][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[m], bm, acc[0][m][n], 0, 0, 0);
          acc[1][m][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[m], b0, acc[1][m][n], 0, 0, 0);
          acc[2][m][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[m], bp, acc[2][m][n], 0, 0, 0);
        }
      }
    }
  };
  // chunk ch lives in LDS buffer ch % 2; the next chunk's loads are in
  // flight during its products
  fetch(c0, sa);
  put(0, sa);
  __syncthreads();
  for (int ch = c0; ch < c1; ++ch) {
    if (ch + 1 < c1) fetch(ch + 1, sa);
    compute((ch - c0) & 1);
    if (ch + 1 < c1) put((ch + 1 - c0) & 1, sa);
    __syncthreads();
  }
#pragma unroll
  for (int s = 0; s < 3; ++s) {
    float* pb = part + ((long long)sl * 9 + dyi * 3 + s) * C * C;
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
      for (int n = 0; n < NT; ++n) {
        const int ci = ci0 + 16 * n + r;
#pragma unroll
        for (int i = 0; i < 4; ++i) pb[(long long)(co0 + 16 * m + 4 * g + i) * C + ci] = acc[s][m][n][i];
      }
  }
}

}  // namespace nop
