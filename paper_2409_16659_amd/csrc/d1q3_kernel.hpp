// d1q3_kernel.hpp -- the N-layer thin-film lattice Boltzmann step on the
// D1Q3 lattice (pseudo-1D films, ny == 1) for gfx950.
//
// Same physics as the D2Q9 step (Sec. III with the pressures and friction of
// Sec. II), with three velocities c = (0, +1, -1), weights (2/3, 1/6, 1/6)
// and the 3-point stencils grad f = (f(x+1) - f(x-1))/2,
// lap f = f(x+1) + f(x-1) - 2 f(x).  Equilibrium (c_s^2 = 1/3, Eq.
// equilibrium_distribution reduced to one dimension): f_0 = h (1 - U^2),
// f_+- = h (U^2 +- U) / 2; forcing 3 w_k c_k F = +-F/2.  In exact
// arithmetic this is the D2Q9 step of a film one row high, each D1Q3
// population being the sum of the D2Q9 populations with the same c_x.
//
// Storage: three planes (rest, +x, -x) of `plane` nodes, each node holding
// the N layers' values next to each other; the rest population is stored as
// its deviation from hbar_i.  As for D2Q9, plane k keeps at column x the
// population that belongs to node x + c_k (the streaming shift is applied
// when a population is read), so a post-collision value is written back to
// its own column.
//
// Kernels:
//  * d1q3_resident: one workgroup per film runs many steps per launch with
//    the whole film in LDS (populations, interface deviations, pressures):
//    three barriers per step and no global traffic between the first load
//    and the last store.  Pseudo-1D films are tiny (10^2..10^3 nodes), so a
//    launch per step would cost far more than the step.
//  * d1q3_resident_batch: the same for many films at once, one workgroup
//    per film (the droplet sweeps of the paper's Sec. IV.B are batches of
//    such strips).
//  * d1q3_tiled: a film longer than one tile split over several
//    workgroups, each holding its tile plus the halo that its steps per
//    launch need, so that each wave has a SIMD to itself.
#pragma once

#include "step_kernel.hpp"

namespace mlf {

// Moments of the three populations of layer i: dh = f0 + f+ + f-, q = f+ - f-.
template <typename C, int NL>
__device__ inline void d1_moments(const C (&f)[NL][3], C (&dh)[NL], C (&q)[NL]) {
#pragma unroll
  for (int i = 0; i < NL; ++i) {
    dh[i] = f[i][0] + f[i][1] + f[i][2];
    q[i] = f[i][1] - f[i][2];
  }
}

// Interface deviations dz_i = sum_{j <= i} dh_j (z_0 = 0 is fixed).
template <typename C, int NL>
__device__ inline void d1_interfaces(const C (&dh)[NL], C (&dz)[NL]) {
  C acc = C(0);
#pragma unroll
  for (int i = 0; i < NL; ++i) {
    acc += dh[i];
    dz[i] = acc;
  }
}

// Pressures p_i = sum_{j >= i} Delta_j at a node from the interface
// deviations at x - 1, x, x + 1.
template <typename C, int NL, int EA, int EB>
__device__ inline void d1_pressure(const StepConsts<C>& kc, const C (&zm)[NL], const C (&zc)[NL], const C (&zp)[NL],
                                   C (&p)[NL]) {
  C dzv[NL + 1], lap[NL + 1], qq[NL + 1];
  dzv[0] = lap[0] = qq[0] = C(0);
#pragma unroll
  for (int i = 0; i < NL; ++i) {
    const C g = (zp[i] - zm[i]) * C(0.5);
    lap[i + 1] = (zp[i] + zm[i]) - C(2) * zc[i];
    qq[i + 1] = g * g;
    dzv[i + 1] = zc[i];
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
    acc += -(kc.gamma[i - 1] + sphi[i]) * lap[i] - dup[i] * (C(1) + C(0.5) * qq[i]) + ddn[i];
    p[i - 1] = acc;
  }
}

// Friction of every layer from the mean velocities (one flux component):
// interface velocities v by Thomas elimination, bottom velocities w of the
// profiles (w_i = v_{i-1} without slip), friction_i = 6 g_i (w_i + v_i - 2 U_i).
template <typename C, int NL>
__device__ inline void d1_friction(const StepConsts<C>& kc, const C (&u)[NL], const C (&rh)[NL], const C (&g)[NL],
                                   C (&fr)[NL]) {
  C sa[NL + 1], sb[NL + 1], se[NL + 1];
#pragma unroll
  for (int i = 0; i < NL; ++i) {
    if (kc.slip_on) {
      const C r = kc.slip[i] * rh[i];
      sa[i] = rcp((C(1) + r) * (C(1) + C(3) * r));
      sb[i] = -r * (C(3) * r + C(2)) * sa[i];
      se[i] = C(6) * r * (r + C(1)) * sa[i];
    } else {
      sa[i] = C(1);
      sb[i] = se[i] = C(0);
    }
  }
  sa[NL] = sb[NL] = se[NL] = C(0);
  C cpr[NL], v[NL];
#pragma unroll
  for (int i = 0; i < NL; ++i) {
    const C gn = i + 1 < NL ? g[i + 1] : C(0);
    const C sub = C(2) * g[i] * sa[i];
    const C diag = g[i] * (C(4) + C(2) * sb[i]) + C(4) * gn * sa[i + 1];
    const C sup = gn * (C(4) * sb[i + 1] + C(2));
    const C rhs = g[i] * (C(6) - C(2) * se[i]) * u[i] + (i + 1 < NL ? gn * (C(6) - C(4) * se[i + 1]) * u[i + 1] : C(0));
    if (i == 0) {
      const C im = rcp(diag);
      cpr[i] = sup * im;
      v[i] = rhs * im;
    } else {
      const C im = rcp(diag - sub * cpr[i - 1]);
      cpr[i] = sup * im;
      v[i] = (rhs - sub * v[i - 1]) * im;
    }
  }
#pragma unroll
  for (int i = NL - 2; i >= 0; --i) v[i] -= cpr[i] * v[i + 1];
#pragma unroll
  for (int i = 0; i < NL; ++i) {
    const C w = sa[i] * (i > 0 ? v[i - 1] : C(0)) + sb[i] * v[i] + se[i] * u[i];
    fr[i] = C(6) * g[i] * ((w + v[i]) - C(2) * u[i]);
  }
}

// Force, BGK collision and forcing at a node; returns the guard code (0 ok,
// 1 height <= 0, 2 non-finite).  f: pre-collision populations (rest as
// deviation), pm / pp: pressures at x - 1 / x + 1; fo: post-collision.
template <typename C, int NL, bool TAU1>
__device__ inline int d1_collide(const StepConsts<C>& kc, const C (&f)[NL][3], const C (&pm)[NL], const C (&pp)[NL],
                                 C (&fo)[NL][3]) {
  C dh[NL], q[NL], h[NL], rh[NL], u[NL], g[NL], fr[NL];
  d1_moments<C, NL>(f, dh, q);
  int bad = 0;
#pragma unroll
  for (int i = 0; i < NL; ++i) {
    h[i] = kc.hbar[i] + dh[i];
    rh[i] = rcp(h[i]);
    u[i] = q[i] * rh[i];
    g[i] = kc.mu[i] * rh[i];
    const C chk = h[i] + q[i];
    if (!(h[i] > C(0))) bad = 1;
    if (!(chk - chk == C(0))) bad = 2;
  }
  d1_friction<C, NL>(kc, u, rh, g, fr);
#pragma unroll
  for (int i = 0; i < NL; ++i) {
    const C F = -h[i] * ((pp[i] - pm[i]) * C(0.5)) + fr[i];
    const C qu = q[i] * u[i];
    if constexpr (TAU1) {
      fo[i][0] = dh[i] - qu;
      fo[i][1] = C(0.5) * (qu + (q[i] + F));
      fo[i][2] = C(0.5) * (qu - (q[i] + F));
    } else {
      const C w = kc.omega, r = C(1) - w;
      fo[i][0] = r * f[i][0] + w * (dh[i] - qu);
      fo[i][1] = r * f[i][1] + C(0.5) * (w * (qu + q[i]) + F);
      fo[i][2] = r * f[i][2] + C(0.5) * (w * (qu - q[i]) - F);
    }
  }
  return bad;
}

// Pre-collision populations of node x from planes stored as
// [3][plane][NL] (element index (k * plane + column) * NL + i).
template <typename C, int NL>
__device__ inline void d1_gather(const C* s, long long plane, int x, int nx, C (&f)[NL][3]) {
  const long long c0 = (long long)x * NL, cm = (long long)wrap(x - 1, nx) * NL,
                  cp = (long long)wrap(x + 1, nx) * NL;
#pragma unroll
  for (int i = 0; i < NL; ++i) {
    f[i][0] = s[c0 + i];
    f[i][1] = s[plane * NL + cm + i];
    f[i][2] = s[2 * plane * NL + cp + i];
  }
}

template <typename C, int NL>
__device__ inline void d1_scatter(C* d, long long plane, int x, const C (&fo)[NL][3]) {
  const long long c0 = (long long)x * NL;
#pragma unroll
  for (int i = 0; i < NL; ++i) {
    d[c0 + i] = fo[i][0];
    d[plane * NL + c0 + i] = fo[i][1];
    d[2 * plane * NL + c0 + i] = fo[i][2];
  }
}

constexpr int kD1Threads = 512;      // largest resident workgroup (256 VGPRs a lane)
constexpr int kD1MaxPerThread = 2;   // nodes per lane: nx <= 1024

// Bytes of LDS the resident kernel needs for a film of nx nodes.
template <typename C>
__host__ __device__ constexpr size_t d1_resident_lds(int nx, int nl) {
  return (size_t)5 * nl * nx * sizeof(C);
}

// `steps` steps of one film held in LDS: src -> (LDS) -> dst.  Lane t owns
// nodes t and t + blockDim (nx <= 2 blockDim; blockDim a multiple of 64).
template <typename C, int NL, bool TAU1, int EA, int EB>
__device__ void d1_resident_run(const C* __restrict__ src, C* __restrict__ dst, const StepConsts<C>& kc, int steps) {
  extern __shared__ unsigned char smem_raw[];
  const int nx = kc.nx;
  C* sf = reinterpret_cast<C*>(smem_raw);  // [3][nx][NL]
  C* sz = sf + 3 * nx * NL;                // [nx][NL]
  C* sp = sz + nx * NL;                    // [nx][NL]
  const long long plane = kc.plane;
  const int t = threadIdx.x, nt = blockDim.x;
  for (int e = t; e < nx * NL; e += nt)
#pragma unroll
    for (int k = 0; k < 3; ++k) sf[k * nx * NL + e] = src[k * plane * NL + e];
  __syncthreads();
  int bad = 0;
  C f[kD1MaxPerThread][NL][3];
  for (int s = 0; s < steps; ++s) {
    // moments and interface deviations of the owned nodes
#pragma unroll
    for (int j = 0; j < kD1MaxPerThread; ++j) {
      const int x = t + j * nt;
      if (x < nx) {
        d1_gather<C, NL>(sf, nx, x, nx, f[j]);
        C dh[NL], q[NL], dz[NL];
        d1_moments<C, NL>(f[j], dh, q);
        d1_interfaces<C, NL>(dh, dz);
#pragma unroll
        for (int i = 0; i < NL; ++i) sz[x * NL + i] = dz[i];
      }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kD1MaxPerThread; ++j) {
      const int x = t + j * nt;
      if (x < nx) {
        C zm[NL], zc[NL], zp[NL], p[NL];
        const int xm = wrap(x - 1, nx), xp = wrap(x + 1, nx);
#pragma unroll
        for (int i = 0; i < NL; ++i) {
          zm[i] = sz[xm * NL + i];
          zc[i] = sz[x * NL + i];
          zp[i] = sz[xp * NL + i];
        }
        d1_pressure<C, NL, EA, EB>(kc, zm, zc, zp, p);
#pragma unroll
        for (int i = 0; i < NL; ++i) sp[x * NL + i] = p[i];
      }
    }
    __syncthreads();
    // every read of sf for this step happened before the first barrier
#pragma unroll
    for (int j = 0; j < kD1MaxPerThread; ++j) {
      const int x = t + j * nt;
      if (x < nx) {
        C pm[NL], pp[NL], fo[NL][3];
        const int xm = wrap(x - 1, nx), xp = wrap(x + 1, nx);
#pragma unroll
        for (int i = 0; i < NL; ++i) {
          pm[i] = sp[xm * NL + i];
          pp[i] = sp[xp * NL + i];
        }
        const int b = d1_collide<C, NL, TAU1>(kc, f[j], pm, pp, fo);
        bad = b > bad ? b : bad;
        d1_scatter<C, NL>(sf, nx, x, fo);
      }
    }
    __syncthreads();
  }
  for (int e = t; e < nx * NL; e += nt)
#pragma unroll
    for (int k = 0; k < 3; ++k) dst[k * plane * NL + e] = sf[k * nx * NL + e];
  if (bad) kc.flag[0] = bad;
}

template <typename C, int NL, bool TAU1, int EA, int EB>
__global__ void __launch_bounds__(kD1Threads) d1q3_resident(const C* __restrict__ src, C* __restrict__ dst,
                                                            StepConsts<C> kc, int steps) {
  d1_resident_run<C, NL, TAU1, EA, EB>(src, dst, kc, steps);
}

// A batch of D1Q3 films, one workgroup per film (its constants, byte offset
// and layer count in the batch table), each held in LDS for `steps` steps;
// flip selects the source buffer (0: a -> b, 1: b -> a).  The workgroup is
// sized for the longest film and the dynamic LDS for the largest one.
template <typename C, bool TAU1, int EA, int EB>
__global__ void __launch_bounds__(kD1Threads) d1q3_resident_batch(const BatchFilm<C>* __restrict__ films,
                                                                  unsigned char* __restrict__ buf_a,
                                                                  unsigned char* __restrict__ buf_b, int flip,
                                                                  int steps) {
  const BatchFilm<C>& bf = films[blockIdx.x];
  const C* src = reinterpret_cast<const C*>((flip ? buf_b : buf_a) + bf.offset);
  C* dst = reinterpret_cast<C*>((flip ? buf_a : buf_b) + bf.offset);
  switch (bf.nl) {
    case 1: d1_resident_run<C, 1, TAU1, EA, EB>(src, dst, bf.kc, steps); break;
    case 2: d1_resident_run<C, 2, TAU1, EA, EB>(src, dst, bf.kc, steps); break;
    case 3: d1_resident_run<C, 3, TAU1, EA, EB>(src, dst, bf.kc, steps); break;
    default: d1_resident_run<C, 4, TAU1, EA, EB>(src, dst, bf.kc, steps); break;
  }
}

// ---- the resident step on a film split over several workgroups ----------
//
// A node's populations after a step depend on those of the nodes up to
// kD1Reach columns away before it (streaming into the moments, the
// neighbours' interface deviations in the pressure, the neighbours'
// pressures in the force).  A workgroup that holds its `core` nodes plus
// kD1Reach * s nodes on each side runs s steps alone: what the cut edges of
// its tile compute wrongly moves inwards kD1Reach nodes a step and never
// reaches the core.  One node per lane, each workgroup on its own CU; the
// halo nodes are computed redundantly.  Per-node arithmetic is that of
// d1_resident_run: results are bit-identical to it.
constexpr int kD1Reach = 3;
constexpr int kD1TileThreads = 128;  // lanes = tile nodes
constexpr int kD1TileSteps = 16;     // steps per launch
constexpr int kD1TileCore = kD1TileThreads - 2 * kD1Reach * kD1TileSteps;
static_assert(kD1TileCore > 0, "tile too narrow for its halo");

template <typename C>
__host__ __device__ constexpr size_t d1_tile_lds(int nl) {
  return (size_t)5 * nl * kD1TileThreads * sizeof(C);
}

// `steps` (1..kD1TileSteps) steps of a film whose nodes are split into tiles
// of `core` nodes (the last one may hold fewer), one workgroup of
// kD1TileThreads lanes each; src -> dst in the layout of d1_resident_run.
// The guard checks each node in the tile that owns it.
template <typename C, int NL, bool TAU1, int EA, int EB>
__global__ void __launch_bounds__(kD1TileThreads) d1q3_tiled(const C* __restrict__ src, C* __restrict__ dst,
                                                             StepConsts<C> kc, int steps, int core) {
  extern __shared__ unsigned char smem_raw[];
  const int nx = kc.nx;
  const int halo = kD1Reach * steps;
  const int w = core + 2 * halo;  // tile nodes, <= kD1TileThreads (host-checked)
  const int x0 = blockIdx.x * core;
  const int ncore = min(core, nx - x0);
  C* sf = reinterpret_cast<C*>(smem_raw);  // [3][w][NL]
  C* sz = sf + 3 * w * NL;                 // [w][NL]
  C* sp = sz + w * NL;                     // [w][NL]
  const long long plane = kc.plane;
  const int l = threadIdx.x;  // the lane's tile node
  const bool live = l < w;
  const bool owned = l >= halo && l < halo + ncore;
  for (int e = l; e < w * NL; e += kD1TileThreads) {
    const int c = e / NL, i = e - c * NL;
    int g = (x0 - halo + c) % nx;  // periodic; x0 - halo + c >= -halo
    if (g < 0) g += nx;
#pragma unroll
    for (int k = 0; k < 3; ++k) sf[(k * w + c) * NL + i] = src[k * plane * NL + (long long)g * NL + i];
  }
  __syncthreads();
  const int lm = max(l - 1, 0), lp = min(l + 1, w - 1);  // clamped at the cut edges
  int bad = 0;
  C f[NL][3];
  for (int s = 0; s < steps; ++s) {
    if (live) {
      // pre-collision populations: plane k keeps at node x the population
      // of node x + c_k
#pragma unroll
      for (int i = 0; i < NL; ++i) {
        f[i][0] = sf[(0 * w + l) * NL + i];
        f[i][1] = sf[(1 * w + lm) * NL + i];
        f[i][2] = sf[(2 * w + lp) * NL + i];
      }
      C dh[NL], q[NL], dz[NL];
      d1_moments<C, NL>(f, dh, q);
      d1_interfaces<C, NL>(dh, dz);
#pragma unroll
      for (int i = 0; i < NL; ++i) sz[l * NL + i] = dz[i];
    }
    __syncthreads();
    if (live) {
      C zm[NL], zc[NL], zp[NL], p[NL];
#pragma unroll
      for (int i = 0; i < NL; ++i) {
        zm[i] = sz[lm * NL + i];
        zc[i] = sz[l * NL + i];
        zp[i] = sz[lp * NL + i];
      }
      d1_pressure<C, NL, EA, EB>(kc, zm, zc, zp, p);
#pragma unroll
      for (int i = 0; i < NL; ++i) sp[l * NL + i] = p[i];
    }
    __syncthreads();
    if (live) {
      C pm[NL], pp[NL], fo[NL][3];
#pragma unroll
      for (int i = 0; i < NL; ++i) {
        pm[i] = sp[lm * NL + i];
        pp[i] = sp[lp * NL + i];
      }
      const int b = d1_collide<C, NL, TAU1>(kc, f, pm, pp, fo);
      if (owned) bad = b > bad ? b : bad;
#pragma unroll
      for (int i = 0; i < NL; ++i) {
        sf[(0 * w + l) * NL + i] = fo[i][0];
        sf[(1 * w + l) * NL + i] = fo[i][1];
        sf[(2 * w + l) * NL + i] = fo[i][2];
      }
    }
    __syncthreads();
  }
  for (int e = l; e < ncore * NL; e += kD1TileThreads) {
    const int c = e / NL, i = e - c * NL;
    const long long g = x0 + c;
#pragma unroll
    for (int k = 0; k < 3; ++k) dst[k * plane * NL + g * NL + i] = sf[(k * w + halo + c) * NL + i];
  }
  if (bad) kc.flag[0] = bad;
}

}  // namespace mlf
