// step_kernel.hpp -- fused N-layer thin-film lattice Boltzmann step for
// gfx950 (one launch per time step).
//
// What one step computes (Sec. III with the pressure and friction of Sec. II
// of Richter, Malgaretti & Harting, arXiv 2409.16659), per node and layer:
//   moments   h_i = sum_k f_ki, q_i = sum_k c_k f_ki
//   z_i = z_{i-1} + h_i; grad z_i, lap z_i (isotropic 9-point stencils)
//   phi_lk = S_lk phi_k(z_{l+k} - z_l), phi'_lk  (Eq. wetting_potential)
//   Delta_i = -(gamma_i + sum_k phi_ik) lap z_i
//             - sum_k phi'_ik (1 + |grad z_i|^2/2)
//             + sum_{l<i} phi'_{l,i-l} (1 + |grad z_l|^2/2)
//             (Eqs. Laplace_pressure, disjoining_pressure)
//   p_i = sum_{j>=i} Delta_j; F_i = -h_i grad p_i + friction_i (Eq. force)
//   f*_ki = f_ki - (f_ki - f^eq_ki)/tau + 3 w_k c_k.F_i   (Eq. BGK)
//   f_ki(x + c_k, t+1) = f*_ki(x), periodic
//
// Layout and schedule (gfx950, wave64):
//  * Populations are stored per direction k: plane k = ny rows of `pitch`
//    nodes, x fastest, and each node holds the populations of all N layers
//    next to each other.  One 4N- (FP32), 8N- (FP64) or 2N-byte (16-bit)
//    vector access then moves a direction's populations of every layer,
//    N times fewer memory instructions than one access per layer; the step
//    is otherwise bound by the rate of vector-memory instructions.
//  * Streaming is split by axis: the y-shift is applied when a population is
//    written (push) and the x-shift when it is read (pull).  Plane k stores
//    at column x the population that belongs to node x + c_kx:
//      f_k(x, y) = S_k(x - c_kx, y),   S_k(x, y + c_ky) <- f*_k(x, y).
//    Every store of a wavefront is thus a column-aligned run (no partial
//    cache lines written twice); only loads carry the +-1 column offsets,
//    which the caches absorb.
//  * The rest population is stored as its deviation from the per-layer
//    reference height hbar_i (moving populations as they are), so that FP32
//    (and 16-bit) storage keeps the small height perturbations exact to
//    storage precision; heights are hbar_i + dh_i and interface heights are
//    handled as deviations dz_i from the reference stack.
//  * The rest plane may have its own storage type R (FP32 rest with 16-bit
//    moving populations): the rest population carries the height, whose
//    per-step change is far below a 16-bit ulp of its deviation, while the
//    moving ones are rebuilt from the moments every step.  The buffer is the
//    rest plane followed by the eight moving planes, addressed in bytes.
//  * A workgroup owns a strip of columns and marches along a segment of rows
//    (a sliding window).  Its lanes cover the strip plus two halo columns on
//    each side (overlapped tiling): every lane loads and reduces one column,
//    the inner lanes form pressures and the innermost ones collide and
//    stream.  Segments alternate their marching direction, so the two
//    workgroups that share halo rows read them at about the same time, and
//    tiles are numbered so that neighbours run on the same XCD (shared L2).
//  * LDS holds a ring of 5 rows of dz (two stencil levels behind a written
//    row) and a ring of 3 rows of p.  The moments of the last three rows
//    stay in registers, and the next row's populations are prefetched into
//    registers while the current row is processed.
//  * Friction: the Poiseuille profiles of Sec. II.A.2 are fixed by the
//    interface velocities v_i (v_0 = 0).  Flux, bottom/top velocities and
//    stress continuity give a symmetric diagonally dominant tridiagonal
//    system in v, solved by Thomas elimination without pivoting:
//      g_i v_{i-1} + 2 (g_i + g_{i+1}) v_i + g_{i+1} v_{i+1}
//          = 3 (g_i U_i + g_{i+1} U_{i+1}),   g_i = mu_i / h_i, g_{N+1} = 0,
//    and friction_i = 2 mu_i h_i a_i = 6 g_i (v_{i-1} + v_i - 2 U_i).
//    With slip lengths the profile's bottom velocity w_i replaces v_{i-1}
//    (see the slip branch below); the system stays tridiagonal.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace mlf {

constexpr int kMaxLayers = 4;
constexpr int kQ = 9;
constexpr int kXcds = 8;  // MI355X: workgroup b runs on XCD b % 8

// D2Q9 ordering: rest, then counter-clockwise from east.
//   k:  0  1  2  3  4  5  6  7  8
//  cx:  0  1  1  0 -1 -1 -1  0  1
//  cy:  0  0  1  1  1  0 -1 -1 -1

template <typename C>
struct StepConsts {
  int nx, ny, pitch;
  int nstrip, wout, seg_h, nseg;
  long long plane;                 // elements per (layer, direction) plane
  C hbar[kMaxLayers];              // reference heights
  C dbar[kMaxLayers][kMaxLayers];  // reference gaps z_{l+k} - z_l, [l][k-1]
  C gamma[kMaxLayers];             // gamma_{i,i+1}
  C mu[kMaxLayers];
  C sa[kMaxLayers][kMaxLayers];   // S_lk a/(a-b), [l][k-1]
  C sb[kMaxLayers][kMaxLayers];   // S_lk b/(a-b)
  C sab[kMaxLayers][kMaxLayers];  // S_lk a b/(a-b)
  C khs[kMaxLayers];              // k h*, [k-1]
  C omega;                           // 1/tau
  C scale[kMaxLayers], iscale[kMaxLayers];  // storage scale per layer (16-bit formats)
  int ea, eb;                        // runtime exponents (generic path)
  unsigned pairs;                    // bit l*4 + k-1 set: S_lk != 0
  int slip_on;                       // any slip length != 0
  C slip[kMaxLayers];                // slip lengths beta_i
  int* flag;                         // guard flag (0 ok, 1 h<=0, 2 non-finite)
  int sr_on;                         // stochastic rounding of a 16-bit rest plane
  unsigned sr_step;                  // step count of this launch (its random draws)
};

// Storage access through raw buffer descriptors: one descriptor per group of
// three direction planes (base address and byte size in scalar registers),
// the plane's offset inside its group as the scalar offset, and per-lane
// 32-bit byte offsets shared by the planes of one type.  Accesses beyond the
// descriptor's size read zero and drop the write instead of faulting.
constexpr int kRsrcWord3 = 0x00020000;  // gfx9-family raw buffer, 32-bit format
// Per-lane offset of a masked access: at least the descriptor size (a group
// of three planes is limited to 2 GiB) and, with any plane offset added,
// still below 2^32, so the access is out of range whether or not the range
// check includes the scalar offset.
constexpr uint32_t kMasked = 0x80000000u;

__device__ inline __amdgpu_buffer_rsrc_t make_rsrc(const void* p, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, kRsrcWord3);
}

// Element formats.  16-bit formats hold the deviations of the populations
// scaled by a per-layer power of two (IEEE half: keeps the small populations
// out of the subnormal range; bfloat16: scale 1) and are converted to and
// from FP32 with round-to-nearest-even.
template <typename T>
struct Elem {
  static constexpr bool kScaled = sizeof(T) == 2;
};

template <int NW>
struct Words {
  uint32_t w[NW];
};
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x3 __attribute__((ext_vector_type(3)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// NW consecutive 32-bit words at byte offset voff + soff (+ j) through the
// widest raw buffer accesses (16, 12, 8, 4 bytes).
template <int NW>
__device__ inline void load_words(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff, uint32_t (&w)[NW]) {
  int j = 0;
#pragma unroll
  for (; j + 4 <= NW; j += 4) {
    const u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(r, (int)(voff + 4 * j), (int)soff, 0);
    w[j] = v.x, w[j + 1] = v.y, w[j + 2] = v.z, w[j + 3] = v.w;
  }
  if constexpr (NW % 4 == 3) {
    const u32x3 v = __builtin_amdgcn_raw_buffer_load_b96(r, (int)(voff + 4 * (NW - 3)), (int)soff, 0);
    w[NW - 3] = v.x, w[NW - 2] = v.y, w[NW - 1] = v.z;
  } else if constexpr (NW % 4 == 2) {
    const u32x2 v = __builtin_amdgcn_raw_buffer_load_b64(r, (int)(voff + 4 * (NW - 2)), (int)soff, 0);
    w[NW - 2] = v.x, w[NW - 1] = v.y;
  } else if constexpr (NW % 4 == 1) {
    w[NW - 1] = __builtin_amdgcn_raw_buffer_load_b32(r, (int)(voff + 4 * (NW - 1)), (int)soff, 0);
  }
}
template <int NW>
__device__ inline void store_words(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff, const uint32_t (&w)[NW]) {
  int j = 0;
#pragma unroll
  for (; j + 4 <= NW; j += 4)
    __builtin_amdgcn_raw_buffer_store_b128(u32x4{w[j], w[j + 1], w[j + 2], w[j + 3]}, r, (int)(voff + 4 * j),
                                           (int)soff, 0);
  if constexpr (NW % 4 == 3)
    __builtin_amdgcn_raw_buffer_store_b96(u32x3{w[NW - 3], w[NW - 2], w[NW - 1]}, r,
                                          (int)(voff + 4 * (NW - 3)), (int)soff, 0);
  else if constexpr (NW % 4 == 2)
    __builtin_amdgcn_raw_buffer_store_b64(u32x2{w[NW - 2], w[NW - 1]}, r, (int)(voff + 4 * (NW - 2)), (int)soff, 0);
  else if constexpr (NW % 4 == 1)
    __builtin_amdgcn_raw_buffer_store_b32(w[NW - 1], r, (int)(voff + 4 * (NW - 1)), (int)soff, 0);
}

__device__ inline float half_bits_to_f32(uint32_t b) {
  return (float)__builtin_bit_cast(_Float16, (unsigned short)(b & 0xffffu));
}
__device__ inline uint32_t f32_to_half_bits(float v) { return __builtin_bit_cast(unsigned short, (_Float16)v); }
__device__ inline float bf16_bits_to_f32(uint32_t b) { return __builtin_bit_cast(float, b << 16); }
__device__ inline uint32_t f32_to_bf16_bits(float v) { return __builtin_bit_cast(unsigned short, (__bf16)v); }

// 32-bit integer mixer (C. Wellons' "lowbias32": xorshift-multiply rounds).
__host__ __device__ inline uint32_t mix32(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  return x;
}

// Random bits of pair `pair` of layers (2 pair and 2 pair + 1 take the low
// and high 16 bits) of node `node` at the step whose key is `step_key`
// (mix32 of the step count, the same for the whole launch): a counter-based
// hash, so the draws depend on where and when they are taken, not on the
// launch shape.
__device__ inline uint32_t sr_bits(uint32_t node, int pair, uint32_t step_key) {
  return mix32((node * 2u + (uint32_t)pair) ^ step_key);
}

// Stochastic rounding of v to the 16-bit type T with the 16-bit uniform
// k16: the representable value just below or just above v, the upper one
// with probability equal to v's distance from the lower one over their gap
// (to 2^-16), so the rounding error has zero mean.  The gap is a power of
// two, so (k16 2^-16) gap and v - lo are exact in FP32 (away from the
// 16-bit type's smallest subnormals) and the comparison needs no division.
// Values T holds exactly are returned unchanged.
template <typename T>
__device__ inline float sr_round(float v, uint32_t k16) {
  constexpr bool kHalf = std::is_same_v<T, _Float16>;
  const uint32_t b = kHalf ? f32_to_half_bits(v) : f32_to_bf16_bits(v);  // nearest
  const float n = kHalf ? half_bits_to_f32(b) : bf16_bits_to_f32(b);
  if (!(n != v) || !(v - v == 0.f)) return n;  // exact, or not finite
  // the neighbour of n on v's side (sign-magnitude bit patterns)
  const bool neg = (b & 0x8000u) != 0;
  uint32_t o;
  if (n < v)
    o = neg ? (b == 0x8000u ? 0x0001u : b - 1) : b + 1;
  else
    o = neg ? b + 1 : (b == 0u ? 0x8001u : b - 1);
  const float m = kHalf ? half_bits_to_f32(o) : bf16_bits_to_f32(o);
  const float lo = n < m ? n : m, hi = n < m ? m : n;
  return (float)k16 * 0x1p-16f * (hi - lo) < v - lo ? hi : lo;
}

// The NL populations of one direction at one node (layers next to each
// other), converted to the arithmetic type C.
template <typename T, int NL, typename C>
__device__ inline void load_node(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff, C (&v)[NL]) {
  if constexpr (sizeof(T) == 4) {
    uint32_t w[NL];
    load_words<NL>(r, voff, soff, w);
#pragma unroll
    for (int i = 0; i < NL; ++i) v[i] = C(__builtin_bit_cast(float, w[i]));
  } else if constexpr (sizeof(T) == 8) {
    uint32_t w[2 * NL];
    load_words<2 * NL>(r, voff, soff, w);
#pragma unroll
    for (int i = 0; i < NL; ++i)
      v[i] = C(__builtin_bit_cast(double, (unsigned long long)w[2 * i] | ((unsigned long long)w[2 * i + 1] << 32)));
  } else if constexpr (NL % 2 == 0) {  // 16-bit, whole words
    uint32_t w[NL / 2];
    load_words<NL / 2>(r, voff, soff, w);
#pragma unroll
    for (int i = 0; i < NL; ++i) {
      const uint32_t b = (i & 1) ? (w[i / 2] >> 16) : (w[i / 2] & 0xffffu);
      v[i] = C(std::is_same_v<T, _Float16> ? half_bits_to_f32(b) : bf16_bits_to_f32(b));
    }
  } else {  // 16-bit, odd layer count: one 2-byte access per layer
#pragma unroll
    for (int i = 0; i < NL; ++i) {
      const uint32_t b = __builtin_amdgcn_raw_buffer_load_b16(r, (int)(voff + 2 * i), (int)soff, 0);
      v[i] = C(std::is_same_v<T, _Float16> ? half_bits_to_f32(b) : bf16_bits_to_f32(b));
    }
  }
}
template <typename T, int NL, typename C>
__device__ inline void store_node(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff, const C (&v)[NL]) {
  if constexpr (sizeof(T) == 4) {
    uint32_t w[NL];
#pragma unroll
    for (int i = 0; i < NL; ++i) w[i] = __builtin_bit_cast(uint32_t, (float)v[i]);
    store_words<NL>(r, voff, soff, w);
  } else if constexpr (sizeof(T) == 8) {
    uint32_t w[2 * NL];
#pragma unroll
    for (int i = 0; i < NL; ++i) {
      const unsigned long long b = __builtin_bit_cast(unsigned long long, (double)v[i]);
      w[2 * i] = (uint32_t)b;
      w[2 * i + 1] = (uint32_t)(b >> 32);
    }
    store_words<2 * NL>(r, voff, soff, w);
  } else {
    uint32_t b[NL];
#pragma unroll
    for (int i = 0; i < NL; ++i)
      b[i] = std::is_same_v<T, _Float16> ? f32_to_half_bits((float)v[i]) : f32_to_bf16_bits((float)v[i]);
    if constexpr (NL % 2 == 0) {
      uint32_t w[NL / 2];
#pragma unroll
      for (int j = 0; j < NL / 2; ++j) w[j] = b[2 * j] | (b[2 * j + 1] << 16);
      store_words<NL / 2>(r, voff, soff, w);
    } else {
#pragma unroll
      for (int i = 0; i < NL; ++i)
        __builtin_amdgcn_raw_buffer_store_b16((unsigned short)b[i], r, (int)(voff + 2 * i), (int)soff, 0);
    }
  }
}

// Reciprocal: the hardware approximation (1 ulp) in FP32, a correctly
// rounded division in FP64.
__device__ inline float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ inline double rcp(double x) { return 1.0 / x; }

template <int E, typename C>
__device__ inline C ipow_c(C r) {
  if constexpr (E == 1) {
    return r;
  } else if constexpr (E % 2 == 0) {
    C h = ipow_c<E / 2>(r);
    return h * h;
  } else {
    return r * ipow_c<E - 1>(r);
  }
}

template <typename C>
__device__ inline C ipow_rt(C r, int e) {
  C v = C(1), b = r;
  while (e > 0) {
    if (e & 1) v *= b;
    b *= b;
    e >>= 1;
  }
  return v;
}

// r^a and r^b; EA == 0 selects the runtime exponents.
template <int EA, int EB, typename C>
__device__ inline void pow_ab(C r, const StepConsts<C>& k, C& ra, C& rb) {
  if constexpr (EA == 9 && EB == 3) {
    C r3 = r * r * r;
    rb = r3;
    ra = r3 * r3 * r3;
  } else if constexpr (EA > 0) {
    ra = ipow_c<EA>(r);
    rb = ipow_c<EB>(r);
  } else {
    ra = ipow_rt(r, k.ea);
    rb = ipow_rt(r, k.eb);
  }
}

// phi = S_lk phi_k(d) = S (a r^b - b r^a)/(a - b) and
// phi' = S a b (r^a - r^b)/((a - b) d) of pair (l, k) from r^a, r^b, 1/d.
// With compile-time exponents only S a/(a - b) is read from the constants
// (b/a and b are literals): fewer live scalar registers in the row loop.
template <int EA, int EB, typename C>
__device__ inline void wetting(const StepConsts<C>& k, int l, int kk, C ra, C rb, C rd, C& phi, C& dphi) {
  const C s = k.sa[l][kk - 1];
  if constexpr (EA > 0) {
    phi = s * (rb - C(double(EB) / double(EA)) * ra);
    dphi = (s * C(EB)) * (ra - rb) * rd;
  } else {
    phi = s * rb - k.sb[l][kk - 1] * ra;
    dphi = k.sab[l][kk - 1] * (ra - rb) * rd;
  }
}

__host__ __device__ inline int wrap(int v, int n) {
  v = v < 0 ? v + n : v;
  v = v >= n ? v - n : v;
  if (v < 0 || v >= n) v = ((v % n) + n) % n;  // only for n < 3
  return v;
}

// Strips of equal width wout <= W - 4 (the lanes cover two halo columns on
// each side); recomputing the count from wout guarantees no empty strip.
__host__ __device__ inline int strip_width(int nx, int W) {
  const int n = (nx + (W - 4) - 1) / (W - 4);
  return (nx + n - 1) / n;
}
__host__ __device__ inline int strip_count(int nx, int W) {
  const int wo = strip_width(nx, W);
  return (nx + wo - 1) / wo;
}

// Tile of workgroup b in a grid of gridDim.x (a multiple of kXcds)
// workgroups: consecutive tiles go to the same XCD.
__device__ inline int tile_of_block(int b, int nblocks) {
  const int per = nblocks / kXcds;
  return (b % kXcds) * per + b / kXcds;
}

// Pressures p_i = sum_{j>=i} Delta_j of one node (Eqs. Laplace_pressure,
// disjoining_pressure, wetting_potential) from the interface deviations of
// its 3x3 neighbourhood: z(i, r, c) for interface i + 1, rows r = 0, 1, 2 at
// y - 1, y, y + 1 and columns c at x - 1, x, x + 1 (read where used, so
// that they are not all live at once).
template <typename C, int NL, int EA, int EB, typename Z>
__device__ inline void node_pressure(const StepConsts<C>& kc, Z&& z, C (&p)[NL]) {
  C dzv[NL + 1], lap[NL + 1], qq[NL + 1];
  dzv[0] = C(0);
  qq[0] = C(0);
  lap[0] = C(0);
#pragma unroll
  for (int i = 0; i < NL; ++i) {
    const C sw = z(i, 0, 0), s = z(i, 0, 1), se = z(i, 0, 2);
    const C wv = z(i, 1, 0), cc = z(i, 1, 1), e = z(i, 1, 2);
    const C nw = z(i, 2, 0), nn = z(i, 2, 1), ne = z(i, 2, 2);
    const C gx = (e - wv) * C(1.0 / 3.0) + ((ne + se) - (nw + sw)) * C(1.0 / 12.0);
    const C gy = (nn - s) * C(1.0 / 3.0) + ((ne + nw) - (se + sw)) * C(1.0 / 12.0);
    lap[i + 1] = (C(4) * ((e + wv) + (nn + s)) + ((ne + nw) + (se + sw)) - C(20) * cc) * C(1.0 / 6.0);
    qq[i + 1] = gx * gx + gy * gy;
    dzv[i + 1] = cc;
  }
  C sphi[NL + 1], dup[NL + 1], ddn[NL + 1];
#pragma unroll
  for (int i = 0; i <= NL; ++i) sphi[i] = dup[i] = ddn[i] = C(0);
#pragma unroll
  for (int l = 0; l < NL; ++l) {
#pragma unroll
    for (int kk = 1; kk <= NL - l; ++kk) {
      // pairs with S_lk = 0 contribute exactly zero (uniform branch)
      if (!(kc.pairs >> (l * 4 + kk - 1) & 1u)) continue;
      const C d = kc.dbar[l][kk - 1] + (dzv[l + kk] - dzv[l]);
      const C rd = rcp(d);
      const C rr = kc.khs[kk - 1] * rd;
      C ra, rb;
      pow_ab<EA, EB>(rr, kc, ra, rb);
      C phi, dphi;
      wetting<EA, EB>(kc, l, kk, ra, rb, rd, phi, dphi);
      sphi[l] += phi;
      dup[l] += dphi;
      ddn[l + kk] += dphi * (C(1) + C(0.5) * qq[l]);
    }
  }
  C acc = C(0);
#pragma unroll
  for (int i = NL; i >= 1; --i) {
    const C delta = -(kc.gamma[i - 1] + sphi[i]) * lap[i] - dup[i] * (C(1) + C(0.5) * qq[i]) + ddn[i];
    acc += delta;
    p[i - 1] = acc;
  }
}

// Force (pressure gradient from the 3x3 pressure neighbourhood pz(i, r, c),
// laid out as z above and read where used, plus friction), and the BGK
// collision with forcing of one node from its moments dh (rest-height
// deviation), qx, qy.  With tau = 1 fo is the post-collision state
// f^eq + 3 w_k c_k.F; otherwise it is omega (f^eq) + forcing and the caller
// adds (1 - omega) f.
template <typename C, int NL, bool TAU1, typename P>
__device__ inline void node_collide(const StepConsts<C>& kc, const C (&dh2)[NL], const C (&qx2)[NL],
                                    const C (&qy2)[NL], P&& pz, C (&fo)[NL][kQ]) {
  C h[NL], ux[NL], uy[NL], g[NL + 1], rh[NL];
#pragma unroll
  for (int i = 0; i < NL; ++i) {
    h[i] = kc.hbar[i] + dh2[i];
    rh[i] = rcp(h[i]);
    ux[i] = qx2[i] * rh[i];
    uy[i] = qy2[i] * rh[i];
    g[i] = kc.mu[i] * rh[i];
  }
  g[NL] = C(0);
  // Thomas elimination for the interface velocities v (x and y share
  // pivots) and the bottom velocities w of the layers' profiles
  C cpr[NL], vx[NL], vy[NL], wx[NL], wy[NL];
  if (!kc.slip_on) {
    // no slip: w_i = v_{i-1}
#pragma unroll
    for (int i = 0; i < NL; ++i) {
      const C diag = C(2) * (g[i] + g[i + 1]);
      const C rx = C(3) * (g[i] * ux[i] + (i + 1 < NL ? g[i + 1] * ux[i + 1] : C(0)));
      const C ry = C(3) * (g[i] * uy[i] + (i + 1 < NL ? g[i + 1] * uy[i + 1] : C(0)));
      if (i == 0) {
        const C im = rcp(diag);
        cpr[i] = g[i + 1] * im;
        vx[i] = rx * im;
        vy[i] = ry * im;
      } else {
        const C im = rcp(diag - g[i] * cpr[i - 1]);
        cpr[i] = g[i + 1] * im;
        vx[i] = (rx - g[i] * vx[i - 1]) * im;
        vy[i] = (ry - g[i] * vy[i - 1]) * im;
      }
    }
#pragma unroll
    for (int i = NL - 2; i >= 0; --i) {
      vx[i] -= cpr[i] * vx[i + 1];
      vy[i] -= cpr[i] * vy[i + 1];
    }
#pragma unroll
    for (int i = 0; i < NL; ++i) {
      wx[i] = i > 0 ? vx[i - 1] : C(0);
      wy[i] = i > 0 ? vy[i - 1] : C(0);
    }
  } else {
    // slip lengths beta_i, rho = beta_i / h_i:
    //   w_i = A_i v_{i-1} + B_i v_i + E_i U_i,  A = 1 / ((1 + rho)(1 + 3 rho)),
    //   B = -rho (3 rho + 2) A,  E = 6 rho (rho + 1) A;
    // stress continuity g_i (4 v_i + 2 w_i - 6 U_i) + g_{i+1} (4 w_{i+1} + 2 v_{i+1} - 6 U_{i+1}) = 0
    C sa[NL + 1], sb[NL + 1], se[NL + 1];
#pragma unroll
    for (int i = 0; i < NL; ++i) {
      const C r = kc.slip[i] * rh[i];
      sa[i] = rcp((C(1) + r) * (C(1) + C(3) * r));
      sb[i] = -r * (C(3) * r + C(2)) * sa[i];
      se[i] = C(6) * r * (r + C(1)) * sa[i];
    }
    sa[NL] = sb[NL] = se[NL] = C(0);
#pragma unroll
    for (int i = 0; i < NL; ++i) {
      const C sub = C(2) * g[i] * sa[i];
      const C diag = g[i] * (C(4) + C(2) * sb[i]) + C(4) * g[i + 1] * sa[i + 1];
      const C sup = g[i + 1] * (C(4) * sb[i + 1] + C(2));
      const C k0 = g[i] * (C(6) - C(2) * se[i]), k1 = g[i + 1] * (C(6) - C(4) * se[i + 1]);
      const C rx = k0 * ux[i] + (i + 1 < NL ? k1 * ux[i + 1] : C(0));
      const C ry = k0 * uy[i] + (i + 1 < NL ? k1 * uy[i + 1] : C(0));
      if (i == 0) {
        const C im = rcp(diag);
        cpr[i] = sup * im;
        vx[i] = rx * im;
        vy[i] = ry * im;
      } else {
        const C im = rcp(diag - sub * cpr[i - 1]);
        cpr[i] = sup * im;
        vx[i] = (rx - sub * vx[i - 1]) * im;
        vy[i] = (ry - sub * vy[i - 1]) * im;
      }
    }
#pragma unroll
    for (int i = NL - 2; i >= 0; --i) {
      vx[i] -= cpr[i] * vx[i + 1];
      vy[i] -= cpr[i] * vy[i + 1];
    }
#pragma unroll
    for (int i = 0; i < NL; ++i) {
      wx[i] = sa[i] * (i > 0 ? vx[i - 1] : C(0)) + sb[i] * vx[i] + se[i] * ux[i];
      wy[i] = sa[i] * (i > 0 ? vy[i - 1] : C(0)) + sb[i] * vy[i] + se[i] * uy[i];
    }
  }
#pragma unroll
  for (int i = 0; i < NL; ++i) {
    const C sw = pz(i, 0, 0), s = pz(i, 0, 1), se = pz(i, 0, 2);
    const C wv = pz(i, 1, 0), e = pz(i, 1, 2);
    const C nw = pz(i, 2, 0), nn = pz(i, 2, 1), ne = pz(i, 2, 2);
    const C gpx = (e - wv) * C(1.0 / 3.0) + ((ne + se) - (nw + sw)) * C(1.0 / 12.0);
    const C gpy = (nn - s) * C(1.0 / 3.0) + ((ne + nw) - (se + sw)) * C(1.0 / 12.0);
    const C frx = C(6) * g[i] * ((wx[i] + vx[i]) - C(2) * ux[i]);
    const C fry = C(6) * g[i] * ((wy[i] + vy[i]) - C(2) * uy[i]);
    const C Fx = -h[i] * gpx + frx;
    const C Fy = -h[i] * gpy + fry;
    const C qx = qx2[i], qy = qy2[i];
    const C qu = qx * ux[i] + qy * uy[i];
    const C t15 = C(1.5) * qu;
    // Shallow-water equilibrium with the rest population as deviation
    // from hbar, split into its even part (quadratic in U, shared by
    // opposite directions) and odd part c.q/c_s^2 w_k; the forcing
    // 3 w_k c_k.F is odd too.  With q_k = c_k.q and u_k = c_k.U:
    //   f^eq_k = w_k (3 q_k + 4.5 q_k u_k - 1.5 q.U),  k >= 1.
    const C ex = C(1.0 / 9.0) * (C(4.5) * qx * ux[i] - t15);  // axial x, even
    const C ey = C(1.0 / 9.0) * (C(4.5) * qy * uy[i] - t15);  // axial y, even
    const C spq = qx + qy, smq = qy - qx, spu = ux[i] + uy[i], smu = uy[i] - ux[i];
    const C ep = C(1.0 / 36.0) * (C(4.5) * spq * spu - t15);  // diagonal (1,1), even
    const C em = C(1.0 / 36.0) * (C(4.5) * smq * smu - t15);  // diagonal (-1,1), even
    C ox, oy;                                                  // axial odd parts
    if constexpr (TAU1) {
      ox = C(1.0 / 3.0) * (qx + Fx);
      oy = C(1.0 / 3.0) * (qy + Fy);
      fo[i][0] = dh2[i] - C(2.0 / 3.0) * qu;
    } else {
      const C w = kc.omega;
      ox = C(1.0 / 3.0) * (w * qx + Fx);
      oy = C(1.0 / 3.0) * (w * qy + Fy);
      fo[i][0] = w * (dh2[i] - C(2.0 / 3.0) * qu);
    }
    const C op = C(0.25) * (ox + oy), om = C(0.25) * (oy - ox);  // diagonal odd parts
    C gx = ex, gy = ey, gp = ep, gm = em;
    if constexpr (!TAU1) {
      gx = kc.omega * ex;
      gy = kc.omega * ey;
      gp = kc.omega * ep;
      gm = kc.omega * em;
    }
    fo[i][1] = gx + ox;
    fo[i][5] = gx - ox;
    fo[i][3] = gy + oy;
    fo[i][7] = gy - oy;
    fo[i][2] = gp + op;
    fo[i][6] = gp - op;
    fo[i][4] = gm + om;
    fo[i][8] = gm - om;
  }
}

// One tile (strip x segment) of one step: the whole workgroup marches the
// segment's rows.  `tile` is uniform and < kc.nstrip * kc.nseg.  AHEAD rows
// of populations are in flight while a row is processed (2 only with
// tau = 1); the arithmetic, and so every result, is the same for both.
// `sr_step` is the film's step count, the counter of its stochastic-rounding
// draws (read only when kc.sr_on).
template <typename R, typename S, typename C, int NL, bool TAU1, int EA, int EB, int AHEAD = 1>
__device__ inline void step_tile(const unsigned char* __restrict__ src, unsigned char* __restrict__ dst,
                                 const StepConsts<C>& kc, int tile, uint32_t sr_step) {
  static_assert(AHEAD == 1 || (AHEAD == 2 && TAU1), "two rows ahead needs tau = 1");
  const int W = blockDim.x;
  const int tid = threadIdx.x;
  const int strip = tile % kc.nstrip;
  const int seg = tile / kc.nstrip;
  const int x0 = strip * kc.wout;
  const int w = min(kc.wout, kc.nx - x0);
  const int y0 = seg * kc.seg_h;
  const int y1 = min(y0 + kc.seg_h, kc.ny);
  const int dir = (seg & 1) ? -1 : 1;  // marching direction in y
  constexpr uint32_t nodeb = NL * sizeof(S), nodebr = NL * sizeof(R);  // bytes per node
  const uint32_t rowb = (uint32_t)kc.pitch * nodeb;    // bytes per row, moving planes
  const uint32_t rowbr = (uint32_t)kc.pitch * nodebr;  // bytes per row, rest plane
  const uint32_t planeb = (uint32_t)(kc.plane * (long long)nodeb);
  const uint32_t planebr = (uint32_t)(kc.plane * (long long)nodebr);
  if (w <= 0 || y1 <= y0) return;  // uniform per workgroup; never taken with host geometry
  // descriptors of the plane groups {0, 1, 2}, {3, 4, 5}, {6, 7, 8}
  const uint32_t g0b = planebr + 2u * planeb, g1b = 3u * planeb;
  __amdgpu_buffer_rsrc_t rs[3], rd[3];
  rs[0] = make_rsrc(src, g0b);
  rs[1] = make_rsrc(src + g0b, g1b);
  rs[2] = make_rsrc(src + (long long)g0b + g1b, g1b);
  rd[0] = make_rsrc(dst, g0b);
  rd[1] = make_rsrc(dst + g0b, g1b);
  rd[2] = make_rsrc(dst + (long long)g0b + g1b, g1b);

  extern __shared__ unsigned char smem_raw[];
  C* zr = reinterpret_cast<C*>(smem_raw);  // [5][NL][W]
  C* pr = zr + 5 * NL * W;                 // [3][NL][W]

  const int lc = tid - 2;                      // local column of this lane
  const bool act1 = tid < w + 4;               // loads / dz
  const bool act2 = tid >= 1 && tid <= w + 2;  // pressure
  const bool act3 = tid >= 2 && tid < w + 2;   // collide + stream
  const int x = wrap(x0 + lc, kc.nx);
  const uint32_t bx = (uint32_t)x * nodeb;
  const uint32_t bxm = (uint32_t)wrap(x - 1, kc.nx) * nodeb;
  const uint32_t bxp = (uint32_t)wrap(x + 1, kc.nx) * nodeb;
  const uint32_t bxr = (uint32_t)x * nodebr;

  // register pipeline of moments: row of iteration it (0), it-1 (1), it-2 (2)
  C dh0[NL], qx0[NL], qy0[NL];
  C dh1[NL], qx1[NL], qy1[NL];
  C dh2[NL], qx2[NL], qy2[NL];
  // populations of the current row and of the AHEAD prefetched rows
  // (ping-pong for one; three buffers rotated for two)
  C fa[NL][kQ], fb[NL][kQ], fe[NL][kQ];
#pragma unroll
  for (int i = 0; i < NL; ++i) {
#pragma unroll
    for (int k = 0; k < kQ; ++k) fa[i][k] = fb[i][k] = fe[i][k] = C(0);
    dh0[i] = dh1[i] = dh2[i] = C(0);
    qx0[i] = qx1[i] = qx2[i] = C(0);
    qy0[i] = qy1[i] = qy2[i] = C(0);
  }

  // Every path through the row loop issues the same vector-memory sequence
  // (9 node loads, then 9 node stores), inactive lanes using masked offsets:
  // the compiler's wait for a row's loads then never covers the stores
  // issued after them, and the prefetched row stays in flight across P2 and
  // P3.  Pre-collision f_k(x, y) = S_k(x - c_kx, y): directions 1, 2, 8 read
  // column x - 1, directions 4, 5, 6 column x + 1.
  auto load_row = [&](int r, bool valid, C (&fn)[NL][kQ]) {
    const bool ok = act1 && valid;
    const uint32_t yr = (uint32_t)wrap(r, kc.ny);
    const uint32_t row = yr * rowb;
    const uint32_t om = ok ? row + bxm : kMasked, o0 = ok ? row + bx : kMasked,
                   op = ok ? row + bxp : kMasked, orr = ok ? yr * rowbr + bxr : kMasked;
    C v[kQ][NL];
    load_node<R, NL>(rs[0], orr, 0u, v[0]);
    load_node<S, NL>(rs[0], om, planebr, v[1]);
    load_node<S, NL>(rs[0], om, planebr + planeb, v[2]);
    load_node<S, NL>(rs[1], o0, 0u, v[3]);
    load_node<S, NL>(rs[1], op, planeb, v[4]);
    load_node<S, NL>(rs[1], op, 2u * planeb, v[5]);
    load_node<S, NL>(rs[2], op, 0u, v[6]);
    load_node<S, NL>(rs[2], o0, planeb, v[7]);
    load_node<S, NL>(rs[2], om, 2u * planeb, v[8]);
#pragma unroll
    for (int i = 0; i < NL; ++i) {
#pragma unroll
      for (int k = 0; k < kQ; ++k) fn[i][k] = v[k][i];
      if constexpr (Elem<R>::kScaled) fn[i][0] *= kc.iscale[i];
      if constexpr (Elem<S>::kScaled) {
#pragma unroll
        for (int k = 1; k < kQ; ++k) fn[i][k] *= kc.iscale[i];
      }
    }
  };
  // Post-collision f*_k(x, y) goes to S_k(x, y + c_ky): row offsets oS, oC, oN
  // are for rows y - 1, y, y + 1 at this lane's column (moving planes), oR
  // for row y of the rest plane.
  auto store_row = [&](bool ok, uint32_t oS, uint32_t oC, uint32_t oN, uint32_t oR, const C (&fo)[NL][kQ]) {
    const uint32_t mS = ok ? oS : kMasked, mC = ok ? oC : kMasked, mN = ok ? oN : kMasked,
                   mR = ok ? oR : kMasked;
    C v[kQ][NL];
#pragma unroll
    for (int i = 0; i < NL; ++i) {
      v[0][i] = Elem<R>::kScaled ? fo[i][0] * kc.scale[i] : fo[i][0];
#pragma unroll
      for (int k = 1; k < kQ; ++k) v[k][i] = Elem<S>::kScaled ? fo[i][k] * kc.scale[i] : fo[i][k];
    }
    store_node<R, NL>(rd[0], mR, 0u, v[0]);
    store_node<S, NL>(rd[0], mC, planebr, v[1]);
    store_node<S, NL>(rd[0], mN, planebr + planeb, v[2]);
    store_node<S, NL>(rd[1], mN, 0u, v[3]);
    store_node<S, NL>(rd[1], mN, planeb, v[4]);
    store_node<S, NL>(rd[1], mC, 2u * planeb, v[5]);
    store_node<S, NL>(rd[2], mS, 0u, v[6]);
    store_node<S, NL>(rd[2], mS, planeb, v[7]);
    store_node<S, NL>(rd[2], mS, 2u * planeb, v[8]);
  };

  const int niter = (y1 - y0) + 4;
  const int rstart = dir > 0 ? y0 - 2 : y1 + 1;  // row of iteration 0

  // store_tag: std::true_type for rows that collide and stream, false_type
  // for the four warm-up rows of a segment (no output row yet: no P3, no
  // stores).
  auto body = [&](auto store_tag, int it, C (&fc)[NL][kQ], C (&fn)[NL][kQ]) {
    constexpr bool kStore = decltype(store_tag)::value;
    const int r = rstart + dir * it;
    // ---- P1: moments and interface deviations of row r ------------------
    {
      const int zs = it % 5;
      C dz = C(0);
      int bad = 0;
#pragma unroll
      for (int i = 0; i < NL; ++i) {
        const C* f = fc[i];
        C dh = f[0] + f[1] + f[2] + f[3] + f[4] + f[5] + f[6] + f[7] + f[8];
        C qx = (f[1] + f[2] + f[8]) - (f[4] + f[5] + f[6]);
        C qy = (f[2] + f[3] + f[4]) - (f[6] + f[7] + f[8]);
        dh0[i] = dh;
        qx0[i] = qx;
        qy0[i] = qy;
        dz += dh;
        zr[(zs * NL + i) * W + tid] = dz;
        const C h = kc.hbar[i] + dh;
        const C chk = h + qx + qy;  // NaN if any of them is NaN or infinite
        if (!(h > C(0))) bad = 1;
        if (!(chk - chk == C(0))) bad = 2;
      }
      if (act1 && bad) kc.flag[0] = bad;
    }
    // Prefetch row it + AHEAD only after this row's registers are consumed:
    // the loads then stay in flight across both barriers and the stores of
    // P3, and the wait at P1 covers the loads of its own row only.
    load_row(r + AHEAD * dir, it + AHEAD < niter, fn);
    __syncthreads();
    // ---- P2: pressures of row r - dir ---------------------------------------
    if (it >= 2 && act2) {
      const int sA = (it - 2) % 5, sC = (it - 1) % 5, sB = it % 5;
      const int sS = dir > 0 ? sA : sB, sN = dir > 0 ? sB : sA;  // rows y-1, y+1
      C dzv[NL + 1], lap[NL + 1], qq[NL + 1];
      dzv[0] = C(0);
      qq[0] = C(0);
      lap[0] = C(0);
#pragma unroll
      for (int i = 0; i < NL; ++i) {
        const C* a = zr + (sS * NL + i) * W + tid;
        const C* c = zr + (sC * NL + i) * W + tid;
        const C* n = zr + (sN * NL + i) * W + tid;
        const C sw = a[-1], s = a[0], se = a[1];
        const C wv = c[-1], cc = c[0], e = c[1];
        const C nw = n[-1], nn = n[0], ne = n[1];
        const C gx = (e - wv) * C(1.0 / 3.0) + ((ne + se) - (nw + sw)) * C(1.0 / 12.0);
        const C gy = (nn - s) * C(1.0 / 3.0) + ((ne + nw) - (se + sw)) * C(1.0 / 12.0);
        lap[i + 1] = (C(4) * ((e + wv) + (nn + s)) + ((ne + nw) + (se + sw)) - C(20) * cc) *
                     C(1.0 / 6.0);
        qq[i + 1] = gx * gx + gy * gy;
        dzv[i + 1] = cc;
      }
      C sphi[NL + 1], dup[NL + 1], ddn[NL + 1];
#pragma unroll
      for (int i = 0; i <= NL; ++i) sphi[i] = dup[i] = ddn[i] = C(0);
#pragma unroll
      for (int l = 0; l < NL; ++l) {
#pragma unroll
        for (int kk = 1; kk <= NL - l; ++kk) {
          // pairs with S_lk = 0 contribute exactly zero (uniform branch)
          if (!(kc.pairs >> (l * 4 + kk - 1) & 1u)) continue;
          const C d = kc.dbar[l][kk - 1] + (dzv[l + kk] - dzv[l]);
          const C rd = rcp(d);
          const C rr = kc.khs[kk - 1] * rd;
          C ra, rb;
          pow_ab<EA, EB>(rr, kc, ra, rb);
          C phi, dphi;
          wetting<EA, EB>(kc, l, kk, ra, rb, rd, phi, dphi);
          sphi[l] += phi;
          dup[l] += dphi;
          ddn[l + kk] += dphi * (C(1) + C(0.5) * qq[l]);
        }
      }
      const int ps = (it - 2) % 3;
      C acc = C(0);
#pragma unroll
      for (int i = NL; i >= 1; --i) {
        const C delta = -(kc.gamma[i - 1] + sphi[i]) * lap[i] - dup[i] * (C(1) + C(0.5) * qq[i]) + ddn[i];
        acc += delta;
        pr[(ps * NL + (i - 1)) * W + tid] = acc;
      }
    }
    __syncthreads();
    // ---- P3: force, collision and streaming of row y = r - 2 dir ------------
    if constexpr (kStore) {
      const bool st_ok = it >= 4 && act3;
      const int y = wrap(r - 2 * dir, kc.ny);
      const uint32_t oC = (uint32_t)y * rowb + bx;
      const uint32_t oS = (uint32_t)wrap(y - 1, kc.ny) * rowb + bx;
      const uint32_t oN = (uint32_t)wrap(y + 1, kc.ny) * rowb + bx;
      const uint32_t oR = (uint32_t)y * rowbr + bxr;
      C fo[NL][kQ];
      if (st_ok) {
        const int pA = (it - 4) % 3, pC = (it - 3) % 3, pB = (it - 2) % 3;
        const int pS = dir > 0 ? pA : pB, pN = dir > 0 ? pB : pA;  // rows y-1, y+1
        const int ps3[3] = {pS, pC, pN};
        auto pz = [&](int i, int rr, int cc) { return pr[(ps3[rr] * NL + i) * W + tid + cc - 1]; };
        node_collide<C, NL, TAU1>(kc, dh2, qx2, qy2, pz, fo);
      } else {
#pragma unroll
        for (int i = 0; i < NL; ++i)
#pragma unroll
          for (int k = 0; k < kQ; ++k) fo[i][k] = C(0);
      }
      if constexpr (!TAU1) {
        // f* = (1 - omega) f + [omega f^eq + forcing]; the pre-collision
        // populations of row y are re-read (cache hits: loaded two rows ago)
        C fy[NL][kQ];
        load_row(y, st_ok, fy);
#pragma unroll
        for (int i = 0; i < NL; ++i)
#pragma unroll
          for (int k = 0; k < kQ; ++k) fo[i][k] += (C(1) - kc.omega) * fy[i][k];
      }
      if constexpr (Elem<R>::kScaled) {
        // stochastic rounding of the stored rest population: rounded here
        // in the scaled form the store writes, so that store_row's own
        // conversion is exact (the scales are powers of two)
        if (kc.sr_on) {
          const uint32_t node = (uint32_t)y * (uint32_t)kc.nx + (uint32_t)x;
          const uint32_t key = mix32(sr_step + 0x9e3779b9u);
          uint32_t bits[(NL + 1) / 2];
#pragma unroll
          for (int j = 0; j < (NL + 1) / 2; ++j) bits[j] = sr_bits(node, j, key);
#pragma unroll
          for (int i = 0; i < NL; ++i)
            fo[i][0] = sr_round<R>(fo[i][0] * kc.scale[i], (bits[i / 2] >> (16 * (i % 2))) & 0xffffu) *
                       kc.iscale[i];
        }
      }
      store_row(st_ok, oS, oC, oN, oR, fo);
    } else if constexpr (AHEAD == 2) {
      // warm-up rows issue dropped stores where later rows store, so the
      // row loop is entered with the pending sequence of every later
      // iteration (loads of rows it and it + 1, each followed by a row's
      // stores)
      C zero[NL][kQ];
#pragma unroll
      for (int i = 0; i < NL; ++i)
#pragma unroll
        for (int k = 0; k < kQ; ++k) zero[i][k] = C(0);
      store_row(false, 0, 0, 0, 0, zero);
    }
    // rotate the moment pipeline
#pragma unroll
    for (int i = 0; i < NL; ++i) {
      dh2[i] = dh1[i];
      qx2[i] = qx1[i];
      qy2[i] = qy1[i];
      dh1[i] = dh0[i];
      qx1[i] = qx0[i];
      qy1[i] = qy0[i];
    }
  };

  load_row(rstart, true, fa);
  if constexpr (AHEAD == 2) {
    // rows 0 and 1 in flight; iteration k reads buffer k % 3 (fa, fb, fe)
    // and loads row k + 2 into buffer (k + 2) % 3, the one read at k - 1
    load_row(rstart + dir, 1 < niter, fb);
    body(std::false_type{}, 0, fa, fe);
    body(std::false_type{}, 1, fb, fa);
    body(std::false_type{}, 2, fe, fb);
    body(std::false_type{}, 3, fa, fe);
    int it = 4;
    for (; it + 2 < niter; it += 3) {
      body(std::true_type{}, it, fb, fa);
      body(std::true_type{}, it + 1, fe, fb);
      body(std::true_type{}, it + 2, fa, fe);
    }
    if (it < niter) body(std::true_type{}, it, fb, fa);
    if (it + 1 < niter) body(std::true_type{}, it + 1, fe, fb);
    return;
  }
  int it = 0;
  if constexpr (TAU1) {
    // warm-up rows (niter >= 5 always): P1 and P2 only
    body(std::false_type{}, 0, fa, fb);
    body(std::false_type{}, 1, fb, fa);
    body(std::false_type{}, 2, fa, fb);
    body(std::false_type{}, 3, fb, fa);
    it = 4;
  }
  {
    // dropped stores: the loop is entered with the same pending sequence
    // (loads, then stores) as every later iteration
    C zero[NL][kQ];
#pragma unroll
    for (int i = 0; i < NL; ++i)
#pragma unroll
      for (int k = 0; k < kQ; ++k) zero[i][k] = C(0);
    store_row(false, 0, 0, 0, 0, zero);
  }
  for (; it + 1 < niter; it += 2) {
    body(std::true_type{}, it, fa, fb);
    body(std::true_type{}, it + 1, fb, fa);
  }
  if (it < niter) body(std::true_type{}, it, fa, fb);
}

// Largest workgroup the step kernel is compiled for: 512 lanes (two waves
// per SIMD, at most 256 VGPRs each), except FP64 arithmetic on four layers,
// whose working set needs more registers than that and keeps one wave per
// SIMD (256 lanes).
template <typename C, int NL>
constexpr int step_max_lanes() {
  return (sizeof(C) == 8 && NL == 4) ? 256 : 512;
}

template <typename R, typename S, typename C, int NL, bool TAU1, int EA, int EB, int AHEAD>
__global__ void __launch_bounds__((step_max_lanes<C, NL>()))
step_kernel(const unsigned char* __restrict__ src, unsigned char* __restrict__ dst, const StepConsts<C> kc) {
  const int tile = tile_of_block(blockIdx.x, gridDim.x);
  if (tile >= kc.nstrip * kc.nseg) return;  // padding workgroup (uniform)
  step_tile<R, S, C, NL, TAU1, EA, EB, AHEAD>(src, dst, kc, tile, kc.sr_step);
}

// ---- batches of independent films -----------------------------------------
// Per-film entry of the device table: step constants (launch geometry
// included), byte offset of the film's populations in both buffers, and
// its layer count.
template <typename C>
struct BatchFilm {
  StepConsts<C> kc;
  long long offset;
  int nl;
  int pad;
};

// One launch advances every film of a batch by one step.  Work item w
// (film, tile) is items[w]; items are ordered largest film first.  With
// gridDim.x < n_items the workgroups are persistent and take items
// w = r * gridDim.x + tile_of_block(blockIdx.x, gridDim.x), r = 0, 1, ...;
// either way consecutive items run on one XCD.  `flip` selects the source
// buffer (0: a -> b, 1: b -> a); AHEAD rows in flight as in step_tile;
// `step` is the batch's step count (every film's stochastic-rounding
// counter, so that a film draws as it would stepped alone).
template <typename R, typename S, typename C, bool TAU1, int EA, int EB, int AHEAD>
__global__ void __launch_bounds__(256)
batch_kernel(const BatchFilm<C>* __restrict__ films, const int2* __restrict__ items, int n_items,
             unsigned char* __restrict__ buf_a, unsigned char* __restrict__ buf_b, int flip, uint32_t step) {
  const int slot = tile_of_block(blockIdx.x, gridDim.x);
  for (int w = slot; w < n_items; w += gridDim.x) {
    const int2 item = items[w];
    const BatchFilm<C>& bf = films[item.x];
    const unsigned char* src = (flip ? buf_b : buf_a) + bf.offset;
    unsigned char* dst = (flip ? buf_a : buf_b) + bf.offset;
    switch (bf.nl) {
      case 1: step_tile<R, S, C, 1, TAU1, EA, EB, AHEAD>(src, dst, bf.kc, item.y, step); break;
      case 2: step_tile<R, S, C, 2, TAU1, EA, EB, AHEAD>(src, dst, bf.kc, item.y, step); break;
      case 3: step_tile<R, S, C, 3, TAU1, EA, EB, AHEAD>(src, dst, bf.kc, item.y, step); break;
      default: step_tile<R, S, C, 4, TAU1, EA, EB, AHEAD>(src, dst, bf.kc, item.y, step); break;
    }
    __syncthreads();  // LDS rings are reused by the next item
  }
}

}  // namespace mlf
