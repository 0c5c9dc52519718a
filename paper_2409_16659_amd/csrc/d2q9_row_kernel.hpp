// d2q9_row_kernel.hpp -- the D2Q9 step of a film one row high (ny == 1,
// the pseudo-1D form of the paper's 2D scheme, Sec. IV.A) with the whole
// film held in LDS for many steps per launch.
//
// On one periodic row the populations moving north or south stream back
// into the same row, and the stencils' north and south neighbours are the
// node's own row; the arithmetic per node is that of the strip kernel
// (same moment sums, the same pressure expressions, the shared
// node_collide), so results are bit-identical to stepping the film with
// step_kernel.  One workgroup of up to 128 lanes, one node each (wider rows
// take d2q9_row_tiled below); LDS holds the nine population planes, the
// interface deviations and the pressures (11 N nx values).  Three barriers per step: every read
// of a step's populations happens before the first one, every write after
// the second, so one LDS copy of the populations suffices.  A one-row film
// of a few hundred nodes does about a microsecond of work per step, less
// than a kernel launch costs.
#pragma once

#include "step_kernel.hpp"

namespace mlf {

constexpr int kRowThreads = 128;
constexpr int kRowMaxPerThread = 1;        // nodes per lane: nx <= 128
constexpr size_t kRowMaxLds = 160 * 1024;  // LDS of one workgroup on gfx950

// Bytes of LDS the resident one-row kernel needs for nx nodes of nl layers.
template <typename C>
__host__ __device__ constexpr size_t row_resident_lds(int nx, int nl) {
  return (size_t)11 * nl * nx * sizeof(C);
}

// Pressures of one node from the interface deviations around it; the same
// expressions as the strip kernel's pressure stage (z(i, r, c): interface
// i + 1, row r, column c of the 3x3 neighbourhood).
template <typename C, int NL, int EA, int EB, typename Z>
__device__ inline void row_pressure(const StepConsts<C>& kc, Z&& z, C (&p)[NL]) {
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

// `steps` steps of one D2Q9 film with ny == 1, src -> (LDS) -> dst, FP64 or
// FP32 storage (the arithmetic type; the rest plane holds deviations from
// hbar).  Global layout as for the strip kernel: plane k (0..8) of `plane`
// nodes, each node holding the N layers' values; plane k keeps at column x
// the population of node x + c_kx.  Lane t owns node t (and t + j blockDim
// for j < kRowMaxPerThread).
template <typename C, int NL, bool TAU1, int EA, int EB>
__global__ void __launch_bounds__(kRowThreads)
d2q9_row_resident(const C* __restrict__ src, C* __restrict__ dst, const StepConsts<C> kc, int steps) {
  extern __shared__ unsigned char smem_raw[];
  constexpr int kCxRow[kQ] = {0, 1, 1, 0, -1, -1, -1, 0, 1};
  const int nx = kc.nx;
  C* sf = reinterpret_cast<C*>(smem_raw);  // [9][nx][NL]
  C* sz = sf + kQ * nx * NL;               // [nx][NL]
  C* sp = sz + nx * NL;                    // [nx][NL]
  const long long plane = kc.plane;
  const int t = threadIdx.x, nt = blockDim.x;
  for (int e = t; e < nx * NL; e += nt)
#pragma unroll
    for (int k = 0; k < kQ; ++k) sf[k * nx * NL + e] = src[k * plane * NL + e];
  __syncthreads();
  int bad = 0;
  C f[kRowMaxPerThread][NL][kQ];
  C dh[kRowMaxPerThread][NL], qx[kRowMaxPerThread][NL], qy[kRowMaxPerThread][NL];
  for (int s = 0; s < steps; ++s) {
    // moments and interface deviations of the owned nodes (every read of
    // this step's populations happens here)
#pragma unroll
    for (int j = 0; j < kRowMaxPerThread; ++j) {
      const int x = t + j * nt;
      if (x < nx) {
#pragma unroll
        for (int k = 0; k < kQ; ++k) {
          const int col = wrap(x - kCxRow[k], nx);
#pragma unroll
          for (int i = 0; i < NL; ++i) f[j][i][k] = sf[(k * nx + col) * NL + i];
        }
        C dz = C(0);
#pragma unroll
        for (int i = 0; i < NL; ++i) {
          const C* ff = f[j][i];
          dh[j][i] = ff[0] + ff[1] + ff[2] + ff[3] + ff[4] + ff[5] + ff[6] + ff[7] + ff[8];
          qx[j][i] = (ff[1] + ff[2] + ff[8]) - (ff[4] + ff[5] + ff[6]);
          qy[j][i] = (ff[2] + ff[3] + ff[4]) - (ff[6] + ff[7] + ff[8]);
          dz += dh[j][i];
          sz[x * NL + i] = dz;
          const C h = kc.hbar[i] + dh[j][i];
          const C chk = h + qx[j][i] + qy[j][i];
          if (!(h > C(0))) bad = bad > 1 ? bad : 1;
          if (!(chk - chk == C(0))) bad = 2;
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kRowMaxPerThread; ++j) {
      const int x = t + j * nt;
      if (x < nx) {
        // north and south neighbours are the node's own row
        const int cm = wrap(x - 1, nx), cp = wrap(x + 1, nx);
        auto z = [&](int i, int, int c) { return sz[(c == 0 ? cm : (c == 1 ? x : cp)) * NL + i]; };
        C p[NL];
        row_pressure<C, NL, EA, EB>(kc, z, p);
#pragma unroll
        for (int i = 0; i < NL; ++i) sp[x * NL + i] = p[i];
      }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kRowMaxPerThread; ++j) {
      const int x = t + j * nt;
      if (x < nx) {
        const int cm = wrap(x - 1, nx), cp = wrap(x + 1, nx);
        auto pz = [&](int i, int, int c) { return sp[(c == 0 ? cm : (c == 1 ? x : cp)) * NL + i]; };
        C fo[NL][kQ];
        node_collide<C, NL, TAU1>(kc, dh[j], qx[j], qy[j], pz, fo);
#pragma unroll
        for (int i = 0; i < NL; ++i)
#pragma unroll
          for (int k = 0; k < kQ; ++k) {
            C v = fo[i][k];
            if constexpr (!TAU1) v += (C(1) - kc.omega) * f[j][i][k];
            // streamed to node x + c_k, kept at column x of plane k; the
            // y-shift stays in the row
            sf[(k * nx + x) * NL + i] = v;
          }
      }
    }
    __syncthreads();
  }
  for (int e = t; e < nx * NL; e += nt)
#pragma unroll
    for (int k = 0; k < kQ; ++k) dst[k * plane * NL + e] = sf[k * nx * NL + e];
  if (bad) kc.flag[0] = bad;
}

// ---- the same step on a row split over several workgroups ----------------
//
// A node's populations after a step depend on the populations of the nodes
// up to kRowReach columns away before it (moments read the neighbours'
// streamed values, the pressure reads the neighbours' interface deviations,
// the force the neighbours' pressures).  A workgroup that holds its `core`
// columns plus kRowReach * s columns on each side can therefore run s steps
// alone: errors from the cut edges of its tile move inwards by at most
// kRowReach columns a step and never reach the core.  Each workgroup runs
// on its own CU with one column per lane, so a step costs one wave's
// instruction stream instead of the whole row's share of one CU; the halo
// columns are computed redundantly.  Per-node arithmetic is that of
// d2q9_row_resident (and of the strip kernel): results are bit-identical.
constexpr int kRowReach = 3;
constexpr int kRowTileThreads = 128;  // lanes = tile columns
constexpr int kRowTileSteps = 16;     // steps per launch
constexpr int kRowTileCore = kRowTileThreads - 2 * kRowReach * kRowTileSteps;
static_assert(kRowTileCore > 0, "tile too narrow for its halo");

template <typename C>
__host__ __device__ constexpr size_t row_tile_lds(int nl) {
  return (size_t)11 * nl * kRowTileThreads * sizeof(C);
}

// `steps` (1..kRowTileSteps) steps of a one-row film whose columns are
// split into tiles of `core` columns (the last one may hold fewer), one
// workgroup of kRowTileThreads lanes each; src -> dst in the global layout
// of d2q9_row_resident.  The guard checks each node in the tile that owns
// it.
template <typename C, int NL, bool TAU1, int EA, int EB>
__global__ void __launch_bounds__(kRowTileThreads)
d2q9_row_tiled(const C* __restrict__ src, C* __restrict__ dst, const StepConsts<C> kc, int steps, int core) {
  extern __shared__ unsigned char smem_raw[];
  constexpr int kCxRow[kQ] = {0, 1, 1, 0, -1, -1, -1, 0, 1};
  const int nx = kc.nx;
  const int halo = kRowReach * steps;
  const int w = core + 2 * halo;  // tile columns, <= kRowTileThreads (host-checked)
  const int x0 = blockIdx.x * core;
  const int ncore = min(core, nx - x0);
  C* sf = reinterpret_cast<C*>(smem_raw);  // [9][w][NL]
  C* sz = sf + kQ * w * NL;                // [w][NL]
  C* sp = sz + w * NL;                     // [w][NL]
  const long long plane = kc.plane;
  const int l = threadIdx.x;  // the lane's tile column
  const bool live = l < w;
  const bool owned = l >= halo && l < halo + ncore;
  for (int e = l; e < w * NL; e += kRowTileThreads) {
    const int c = e / NL, i = e - c * NL;
    int g = (x0 - halo + c) % nx;  // periodic; x0 - halo + c >= -halo
    if (g < 0) g += nx;
#pragma unroll
    for (int k = 0; k < kQ; ++k) sf[(k * w + c) * NL + i] = src[k * plane * NL + (long long)g * NL + i];
  }
  __syncthreads();
  const int cm = max(l - 1, 0), cp = min(l + 1, w - 1);  // clamped at the cut edges
  int bad = 0;
  C f[NL][kQ];
  C dh[NL], qx[NL], qy[NL];
  for (int s = 0; s < steps; ++s) {
    if (live) {
#pragma unroll
      for (int k = 0; k < kQ; ++k) {
        const int col = min(max(l - kCxRow[k], 0), w - 1);
#pragma unroll
        for (int i = 0; i < NL; ++i) f[i][k] = sf[(k * w + col) * NL + i];
      }
      C dz = C(0);
#pragma unroll
      for (int i = 0; i < NL; ++i) {
        const C* ff = f[i];
        dh[i] = ff[0] + ff[1] + ff[2] + ff[3] + ff[4] + ff[5] + ff[6] + ff[7] + ff[8];
        qx[i] = (ff[1] + ff[2] + ff[8]) - (ff[4] + ff[5] + ff[6]);
        qy[i] = (ff[2] + ff[3] + ff[4]) - (ff[6] + ff[7] + ff[8]);
        dz += dh[i];
        sz[l * NL + i] = dz;
        if (owned) {
          const C h = kc.hbar[i] + dh[i];
          const C chk = h + qx[i] + qy[i];
          if (!(h > C(0))) bad = bad > 1 ? bad : 1;
          if (!(chk - chk == C(0))) bad = 2;
        }
      }
    }
    __syncthreads();
    if (live) {
      auto z = [&](int i, int, int c) { return sz[(c == 0 ? cm : (c == 1 ? l : cp)) * NL + i]; };
      C p[NL];
      row_pressure<C, NL, EA, EB>(kc, z, p);
#pragma unroll
      for (int i = 0; i < NL; ++i) sp[l * NL + i] = p[i];
    }
    __syncthreads();
    if (live) {
      auto pz = [&](int i, int, int c) { return sp[(c == 0 ? cm : (c == 1 ? l : cp)) * NL + i]; };
      C fo[NL][kQ];
      node_collide<C, NL, TAU1>(kc, dh, qx, qy, pz, fo);
#pragma unroll
      for (int i = 0; i < NL; ++i)
#pragma unroll
        for (int k = 0; k < kQ; ++k) {
          C v = fo[i][k];
          if constexpr (!TAU1) v += (C(1) - kc.omega) * f[i][k];
          sf[(k * w + l) * NL + i] = v;
        }
    }
    __syncthreads();
  }
  for (int e = l; e < ncore * NL; e += kRowTileThreads) {
    const int c = e / NL, i = e - c * NL;
    const long long g = x0 + c;
#pragma unroll
    for (int k = 0; k < kQ; ++k) dst[k * plane * NL + g * NL + i] = sf[(k * w + halo + c) * NL + i];
  }
  if (bad) kc.flag[0] = bad;
}

}  // namespace mlf
