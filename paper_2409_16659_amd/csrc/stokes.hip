// stokes.hip -- Stokes-limit layer velocities of a height field (FP64).
//
// In the Stokes limit the thin-film equation (Sec. II.B, Eq.
// thin_film_equation_n) has no flux inertia: every layer's flux is the one
// at which the pressure force -h_i grad p_i and the inter-layer friction
// 2 mu_i h_i a_i of Sec. II.A.2 cancel, q = K^-1 diag(h) grad p = -M grad Delta
// (M the mobility).  Restarting the lattice Boltzmann scheme from
// f^eq(h, U) with these velocities starts it on the trajectory it follows
// under strong friction, instead of from rest.
//
// Per node, with the same discretisation as the step (isotropic 9-point
// gradient and Laplacian, pressures p_i = sum_{j>=i} Delta_j with the
// Laplace and disjoining terms of Eqs. Laplace_pressure and
// disjoining_pressure) and the friction in interface velocities (v_0 = 0,
// g_i = mu_i / h_i, friction_i = 6 g_i (v_{i-1} + v_i - 2 U_i), stress
// continuity between layers, no stress at the gas), the balance
// friction_i = f_i := h_i d p_i is solved explicitly:
//   s_i = f_i / 2 + sum_{j>i} f_j,   v_i = v_{i-1} - s_i / g_i,
//   U_i = v_{i-1} - s_i / (2 g_i) - f_i / (12 g_i)
// (substituting U from the friction into the stress-continuity rows makes
// them g_i (v_{i-1} - v_i) - g_{i+1} (v_i - v_{i+1}) = (f_i + f_{i+1}) / 2,
// which telescope from the gas down).  No slip: films with slip lengths are
// rejected.
#include "../../include/mlfilm.h"

#include <hip/hip_runtime.h>

#include <cmath>

namespace {

constexpr int kMaxN = MLF_MAX_LAYERS;

struct StokesConsts {
  int n, nx, ny, ea, eb;
  double hstar;
  double gamma[kMaxN], mu[kMaxN];
  double spread[kMaxN][kMaxN];  // S_lk, [l][k-1]
};

__device__ inline double ipow(double r, int e) {
  double v = 1.0, b = r;
  while (e > 0) {
    if (e & 1) v *= b;
    b *= b;
    e >>= 1;
  }
  return v;
}

__device__ inline int wrapi(int v, int n) {
  v %= n;
  return v < 0 ? v + n : v;
}

// Pressures p_i at the centre of a 3x3 window of interface heights z[i][3][3]
// (z[i] is interface i = 1..N, rows dy = -1..1, columns dx = -1..1).
__device__ void pressures(const StokesConsts& k, const double (&z)[kMaxN][3][3], double (&p)[kMaxN]) {
  const int n = k.n;
  double zc[kMaxN + 1], lap[kMaxN + 1], qq[kMaxN + 1];
  zc[0] = 0.0, lap[0] = 0.0, qq[0] = 0.0;
  for (int i = 0; i < n; ++i) {
    const double(&w)[3][3] = z[i];
    const double gx = (w[1][2] - w[1][0]) / 3.0 + ((w[2][2] + w[0][2]) - (w[2][0] + w[0][0])) / 12.0;
    const double gy = (w[2][1] - w[0][1]) / 3.0 + ((w[2][2] + w[2][0]) - (w[0][2] + w[0][0])) / 12.0;
    lap[i + 1] = (4.0 * ((w[1][2] + w[1][0]) + (w[2][1] + w[0][1])) + ((w[2][2] + w[2][0]) + (w[0][2] + w[0][0])) -
                  20.0 * w[1][1]) / 6.0;
    qq[i + 1] = gx * gx + gy * gy;
    zc[i + 1] = w[1][1];
  }
  double sphi[kMaxN + 1], dup[kMaxN + 1], ddn[kMaxN + 1];
  for (int i = 0; i <= n; ++i) sphi[i] = dup[i] = ddn[i] = 0.0;
  const double a = k.ea, b = k.eb;
  for (int l = 0; l < n; ++l)
    for (int kk = 1; kk <= n - l; ++kk) {
      const double S = k.spread[l][kk - 1];
      if (S == 0.0) continue;
      const double d = zc[l + kk] - zc[l];
      const double r = kk * k.hstar / d;
      const double ra = ipow(r, k.ea), rb = ipow(r, k.eb);
      const double phi = S * (a * rb - b * ra) / (a - b);
      const double dphi = S * a * b * (ra - rb) / ((a - b) * d);
      sphi[l] += phi;
      dup[l] += dphi;
      ddn[l + kk] += dphi * (1.0 + 0.5 * qq[l]);
    }
  double acc = 0.0;
  for (int i = n; i >= 1; --i) {
    const double delta = -(k.gamma[i - 1] + sphi[i]) * lap[i] - dup[i] * (1.0 + 0.5 * qq[i]) + ddn[i];
    acc += delta;
    p[i - 1] = acc;
  }
}

__global__ void __launch_bounds__(256) stokes_kernel(const double* __restrict__ h, double* __restrict__ ux,
                                                     double* __restrict__ uy, StokesConsts k) {
  const long long plane = (long long)k.nx * k.ny;
  const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (t >= plane) return;
  const int x = (int)(t % k.nx), y = (int)(t / k.nx);
  const int n = k.n;
  // interface heights on the 5x5 window around the node
  double z5[kMaxN][5][5];
  for (int dy = 0; dy < 5; ++dy)
    for (int dx = 0; dx < 5; ++dx) {
      const long long e = (long long)wrapi(y + dy - 2, k.ny) * k.nx + wrapi(x + dx - 2, k.nx);
      double zz = 0.0;
      for (int i = 0; i < n; ++i) {
        zz += h[i * plane + e];
        z5[i][dy][dx] = zz;
      }
    }
  // pressures on the 3x3 window
  double p[3][3][kMaxN];
  for (int cy = 0; cy < 3; ++cy)
    for (int cx = 0; cx < 3; ++cx) {
      double w[kMaxN][3][3];
      for (int i = 0; i < n; ++i)
        for (int dy = 0; dy < 3; ++dy)
          for (int dx = 0; dx < 3; ++dx) w[i][dy][dx] = z5[i][cy + dy][cx + dx];
      double pc[kMaxN];
      pressures(k, w, pc);
      for (int i = 0; i < n; ++i) p[cy][cx][i] = pc[i];
    }
  double hc[kMaxN], fx[kMaxN], fy[kMaxN];
  for (int i = 0; i < n; ++i) {
    hc[i] = h[i * plane + t];
    const double gpx = (p[1][2][i] - p[1][0][i]) / 3.0 + ((p[2][2][i] + p[0][2][i]) - (p[2][0][i] + p[0][0][i])) / 12.0;
    const double gpy = (p[2][1][i] - p[0][1][i]) / 3.0 + ((p[2][2][i] + p[2][0][i]) - (p[0][2][i] + p[0][0][i])) / 12.0;
    fx[i] = hc[i] * gpx;
    fy[i] = hc[i] * gpy;
  }
  double tx = 0.0, ty = 0.0, sx[kMaxN], sy[kMaxN];
  for (int i = n - 1; i >= 0; --i) {
    sx[i] = 0.5 * fx[i] + tx;
    sy[i] = 0.5 * fy[i] + ty;
    tx += fx[i];
    ty += fy[i];
  }
  double vx = 0.0, vy = 0.0;
  for (int i = 0; i < n; ++i) {
    const double rg = hc[i] / k.mu[i];  // 1 / g_i
    ux[i * plane + t] = vx - 0.5 * sx[i] * rg - fx[i] * rg / 12.0;
    uy[i * plane + t] = vy - 0.5 * sy[i] * rg - fy[i] * rg / 12.0;
    vx -= sx[i] * rg;
    vy -= sy[i] * rg;
  }
}

}  // namespace

extern "C" mlf_status mlf_stokes_velocity(const mlf_params* p, const double* hgt, double* ux, double* uy,
                                          void* stream) {
  if (!p || !hgt || !ux || !uy) return MLF_EINVAL;
  const int n = p->n_layers;
  if (n < 1 || n > kMaxN || p->nx < 1 || p->ny < 1) return MLF_EINVAL;
  if (!(p->hstar > 0.0) || p->exp_b < 1 || p->exp_a <= p->exp_b) return MLF_EINVAL;
  StokesConsts k{};
  k.n = n, k.nx = p->nx, k.ny = p->ny, k.ea = p->exp_a, k.eb = p->exp_b, k.hstar = p->hstar;
  for (int i = 0; i < n; ++i) {
    if (!(p->mu[i] > 0.0) || !std::isfinite(p->gamma[i])) return MLF_EINVAL;
    if (p->slip[i] != 0.0) return MLF_EUNSUPPORTED;
    k.gamma[i] = p->gamma[i];
    k.mu[i] = p->mu[i];
  }
  int idx = 0;
  for (int l = 0; l < n; ++l)
    for (int kk = 1; kk <= n - l; ++kk) k.spread[l][kk - 1] = p->spread[idx++];
  const long long plane = (long long)p->nx * p->ny;
  const unsigned grid = (unsigned)((plane + 255) / 256);
  hipLaunchKernelGGL(stokes_kernel, dim3(grid), dim3(256), 0, static_cast<hipStream_t>(stream), hgt, ux, uy, k);
  return hipGetLastError() == hipSuccess ? MLF_OK : MLF_EDEVICE;
}
