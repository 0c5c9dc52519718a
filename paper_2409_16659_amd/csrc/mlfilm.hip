// mlfilm.hip -- C ABI of libmlfilm (declared in include/mlfilm.h): parameter
// handling, the fused step launch, initialisation, read-back, FP64 per-layer
// mass reduction and checkpoints.  All device memory is caller-owned.
#include "../../include/mlfilm.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "d1q3_kernel.hpp"
#include "d2q9_row_kernel.hpp"
#include "stream_probe.hpp"
#include "step_kernel.hpp"

using mlf::kMaxLayers;
using mlf::kQ;

namespace {

constexpr size_t kFlagOff = 0;          // int guard flag
constexpr size_t kRedOutOff = 256;      // double[64] reduction results
constexpr size_t kPartOff = 1024;       // double partials[kRedBlocks][kMaxLayers]
constexpr int kRedBlocks = 512;
constexpr size_t kStageOff = 64 * 1024; // staging for host <-> device fields
constexpr size_t kStageBytes = 16u << 20;
constexpr size_t kScratchBytes = kStageOff + kStageBytes;
constexpr int kPitchAlign = 64;  // elements
// x-components of the D2Q9 velocities; plane k stores the population of
// node x at column x - kCx[k] (see step_kernel.hpp)
constexpr int kCx[9] = {0, 1, 1, 0, -1, -1, -1, 0, 1};
constexpr int kCx3[3] = {0, 1, -1};  // D1Q3: rest, +x, -x

static_assert(offsetof(mlf_params, lattice) == 224 && sizeof(mlf_params) == 232, "mlf_params layout");

int nq_of(const mlf_params* p) { return p->lattice == MLF_D1Q3 ? 3 : kQ; }
int cx_of(int nq, int k) { return nq == 3 ? kCx3[k] : kCx[k]; }

// Element format of a population plane.
enum Fmt { kFmtF64, kFmtF32, kFmtF16, kFmtBF16 };

// Format of the rest plane and of the eight moving planes.
Fmt rest_fmt(int precision) {
  switch (precision) {
    case MLF_F64: return kFmtF64;
    case MLF_F16: return kFmtF16;
    case MLF_BF16: return kFmtBF16;
    default: return kFmtF32;  // F32 and both MIX formats
  }
}
Fmt move_fmt(int precision) {
  switch (precision) {
    case MLF_F64: return kFmtF64;
    case MLF_F32: return kFmtF32;
    case MLF_F16:
    case MLF_F16_MIX: return kFmtF16;
    default: return kFmtBF16;
  }
}
size_t fmt_size(Fmt f) { return f == kFmtF64 ? 8 : (f == kFmtF32 ? 4 : 2); }
bool fmt_scaled(Fmt f) { return f == kFmtF16 || f == kFmtBF16; }

// Population buffer layout: plane k (rest plane, then eight moving planes)
// of `plane` nodes (ny rows of `pitch`), each node holding the n layers'
// values next to each other.  Bytes per node of plane k, byte offset of
// plane k, and bytes of the whole buffer.
size_t node_bytes(int precision, int n, int k) {
  return (size_t)n * fmt_size(k == 0 ? rest_fmt(precision) : move_fmt(precision));
}
size_t plane_offset(int precision, int n, size_t plane, int k) {
  return k == 0 ? 0 : plane * (node_bytes(precision, n, 0) + (size_t)(k - 1) * node_bytes(precision, n, 1));
}
size_t buffer_bytes(int precision, int n, size_t plane, int nq) { return plane_offset(precision, n, plane, nq); }

int pitch_of(const mlf_params* p) { return (p->nx + kPitchAlign - 1) / kPitchAlign * kPitchAlign; }

int pair_index(int n, int l, int k) {  // packed S_lk, l-major, k = 1..n-l
  int idx = 0;
  for (int j = 0; j < l; ++j) idx += n - j;
  return idx + (k - 1);
}

mlf_status validate(const mlf_params* p, std::string* why) {
  auto bad = [&](const char* m) {
    if (why) *why = m;
    return MLF_EINVAL;
  };
  if (!p) return bad("null parameters");
  if (p->n_layers < 1 || p->n_layers > MLF_MAX_LAYERS) return bad("n_layers must be 1..4");
  if (p->nx < 1 || p->ny < 1) return bad("nx, ny must be >= 1");
  if (p->precision < MLF_F64 || p->precision > MLF_BF16_MIX) return bad("unknown precision");
  if (!(p->tau > 0.5) || !std::isfinite(p->tau)) return bad("tau must be > 0.5");
  if (!(p->hstar > 0.0) || !std::isfinite(p->hstar)) return bad("hstar must be > 0");
  if (!(p->exp_a > p->exp_b && p->exp_b >= 1) || p->exp_a > 64) return bad("need 64 >= exp_a > exp_b >= 1");
  for (int i = 0; i < p->n_layers; ++i) {
    if (!(p->mu[i] > 0.0) || !std::isfinite(p->mu[i])) return bad("mu must be > 0");
    if (!std::isfinite(p->gamma[i])) return bad("gamma must be finite");
  }
  int np = p->n_layers * (p->n_layers + 1) / 2;
  for (int j = 0; j < np; ++j)
    if (!std::isfinite(p->spread[j])) return bad("spread must be finite");
  size_t plane = (size_t)pitch_of(p) * (size_t)p->ny;
  if (plane * kQ * (size_t)p->n_layers > (size_t)1 << 40) return bad("grid too large");
  if (p->lattice != MLF_D2Q9 && p->lattice != MLF_D1Q3) return bad("unknown lattice");
  if (p->lattice == MLF_D1Q3) {
    if (p->ny != 1) return bad("the D1Q3 lattice needs ny == 1");
    if (p->precision != MLF_F64 && p->precision != MLF_F32) {
      if (why) *why = "the D1Q3 lattice supports F64 and F32 storage";
      return MLF_EUNSUPPORTED;
    }
  }
  // the step kernel addresses each group of three planes through a buffer
  // descriptor with 32-bit offsets and masks lanes with offset 2^31
  const size_t g0 = plane_offset(p->precision, p->n_layers, plane, 3);
  const size_t g1 = plane_offset(p->precision, p->n_layers, plane, 6) - g0;
  if (std::max(g0, g1) > (size_t)0x80000000u) {
    if (why) *why = "three population planes exceed 2 GiB";
    return MLF_EUNSUPPORTED;
  }
  for (int i = 0; i < p->n_layers; ++i)
    if (!(p->slip[i] >= 0.0) || !std::isfinite(p->slip[i])) return bad("slip lengths must be finite and >= 0");
  return MLF_OK;
}

// Friction matrix K (friction = K q) of one node from the interface-velocity
// form of the boundary conditions, column j being the response to a unit
// flux in layer j.  Layer i's Poiseuille profile is fixed by its bottom
// velocity w_i, top velocity v_i and mean U_i; with slip length beta_i the
// profile extrapolated to beta_i below the layer meets v_{i-1} (v_{-1} = 0),
// which with rho = beta_i / h_i gives
//   w_i = [v_{i-1} - rho (3 rho + 2) v_i + 6 rho (rho + 1) U_i] / ((1 + rho)(1 + 3 rho)),
// and stress continuity g_i (4 v_i + 2 w_i - 6 U_i) + g_{i+1} (4 w_{i+1} +
// 2 v_{i+1} - 6 U_{i+1}) = 0 (g = mu / h, g_N = 0 at the gas) is tridiagonal
// in v.  friction_i = 6 g_i (w_i + v_i - 2 U_i).
void friction_matrix(int n, const double* h, const double* mu, const double* slip, double* K) {
  double g[kMaxLayers + 1], A[kMaxLayers + 1], B[kMaxLayers + 1], E[kMaxLayers + 1];
  for (int i = 0; i < n; ++i) {
    g[i] = mu[i] / h[i];
    const double r = slip ? slip[i] / h[i] : 0.0, d = (1.0 + r) * (1.0 + 3.0 * r);
    A[i] = 1.0 / d;
    B[i] = -r * (3.0 * r + 2.0) / d;
    E[i] = 6.0 * r * (r + 1.0) / d;
  }
  g[n] = 0.0, A[n] = B[n] = E[n] = 0.0;
  for (int j = 0; j < n; ++j) {
    double U[kMaxLayers + 1] = {0, 0, 0, 0, 0}, v[kMaxLayers], c[kMaxLayers];
    U[j] = 1.0 / h[j];
    for (int i = 0; i < n; ++i) {
      const double sub = 2.0 * g[i] * A[i];
      const double diag = g[i] * (4.0 + 2.0 * B[i]) + 4.0 * g[i + 1] * A[i + 1];
      const double sup = g[i + 1] * (4.0 * B[i + 1] + 2.0);
      const double rhs = g[i] * (6.0 - 2.0 * E[i]) * U[i] + g[i + 1] * (6.0 - 4.0 * E[i + 1]) * U[i + 1];
      const double m = (i == 0) ? diag : diag - sub * c[i - 1];
      c[i] = sup / m;
      v[i] = (i == 0 ? rhs : rhs - sub * v[i - 1]) / m;
    }
    for (int i = n - 2; i >= 0; --i) v[i] -= c[i] * v[i + 1];
    for (int i = 0; i < n; ++i) {
      const double w = A[i] * (i > 0 ? v[i - 1] : 0.0) + B[i] * v[i] + E[i] * U[i];
      K[i * n + j] = 6.0 * g[i] * (w + v[i] - 2.0 * U[i]);
    }
  }
}

// Spectral radius of an n x n matrix M (n <= 4) by repeated squaring with
// renormalisation: rho(M) = lim |M^(2^k)|^(1/2^k), tracked in logarithms;
// valid for complex eigenvalue pairs too.
double spectral_radius(int n, const double* M) {
  double A[kMaxLayers * kMaxLayers], Bm[kMaxLayers * kMaxLayers];
  double s = 0.0;
  for (int i = 0; i < n * n; ++i) s = std::max(s, std::fabs(M[i]));
  if (s == 0.0 || !std::isfinite(s)) return s;
  for (int i = 0; i < n * n; ++i) A[i] = M[i] / s;
  double L = std::log(s);
  const int kSquarings = 40;
  for (int it = 1; it <= kSquarings; ++it) {
    double t = 0.0;
    for (int r = 0; r < n; ++r)
      for (int c = 0; c < n; ++c) {
        double v = 0.0;
        for (int k = 0; k < n; ++k) v += A[r * n + k] * A[k * n + c];
        Bm[r * n + c] = v;
        t = std::max(t, std::fabs(v));
      }
    if (t == 0.0) return 0.0;  // nilpotent
    for (int i = 0; i < n * n; ++i) A[i] = Bm[i] / t;
    L = 2.0 * L + std::log(t);
  }
  return std::exp(L / std::ldexp(1.0, kSquarings));
}

// Largest |eigenvalue| of -K (the largest friction rate; real and positive
// without slip).
double max_rate(int n, const double* K) {
  double M[kMaxLayers * kMaxLayers];
  for (int i = 0; i < n * n; ++i) M[i] = -K[i];
  return spectral_radius(n, M);
}

// Spectral radius of I + K: the per-step amplification of the fluxes by
// the explicit friction (q <- q + K q for every tau).
double friction_amplification(int n, const double* K) {
  double M[kMaxLayers * kMaxLayers];
  for (int r = 0; r < n; ++r)
    for (int c = 0; c < n; ++c) M[r * n + c] = K[r * n + c] + (r == c ? 1.0 : 0.0);
  return spectral_radius(n, M);
}

uint64_t fnv1a(const void* data, size_t n, uint64_t hsh = 1469598103934665603ull) {
  const unsigned char* p = static_cast<const unsigned char*>(data);
  for (size_t i = 0; i < n; ++i) {
    hsh ^= p[i];
    hsh *= 1099511628211ull;
  }
  return hsh;
}

uint64_t params_digest(const mlf_params* p) {
  mlf_params q = *p;
  q.check_every = 0;
  q.allow_unstable = 0;
  return fnv1a(&q, sizeof(q));
}

struct BlobHeader {
  char magic[8];
  uint32_t version;
  int32_t precision;
  int32_t n_layers, nx, ny, pitch;
  int64_t steps;
  double hbar[kMaxLayers];
  uint64_t digest;
  uint64_t payload;
};

// ---------------------------------------------------------------- kernels --
// Per-layer constants of the auxiliary kernels: reference heights and the
// storage scale of the 16-bit planes (they store scaled deviations).
struct Layers {
  double hb[kMaxLayers];
  double sc[kMaxLayers];
};

template <typename T>
constexpr bool kIs16 = sizeof(T) == 2;

template <typename S>
__device__ inline S to_store(double v) {
  return S((float)v);
}
template <>
__device__ inline double to_store<double>(double v) {
  return v;
}

// Populations: the rest plane (type R), then the eight moving planes (type
// S), each of `plane` nodes; a node holds the nl layers' values in a row.
template <typename R, typename S>
struct PopView {
  unsigned char* base;
  long long plane;
  int nl;
  int nq;  // directions: 9 (D2Q9) or 3 (D1Q3: rest, +x, -x)
  // unscaled value of layer i, direction k at node e
  __device__ double ld(int i, int k, long long e, const Layers& L) const {
    if (k == 0) return double(reinterpret_cast<const R*>(base)[e * nl + i]) / (kIs16<R> ? L.sc[i] : 1.0);
    const S* m = reinterpret_cast<const S*>(base + plane * nl * (long long)sizeof(R));
    return double(m[((long long)(k - 1) * plane + e) * nl + i]) / (kIs16<S> ? L.sc[i] : 1.0);
  }
  __device__ void st(int i, int k, long long e, double v, const Layers& L) const {
    if (k == 0) {
      reinterpret_cast<R*>(base)[e * nl + i] = to_store<R>(v * (kIs16<R> ? L.sc[i] : 1.0));
      return;
    }
    S* m = reinterpret_cast<S*>(base + plane * nl * (long long)sizeof(R));
    m[((long long)(k - 1) * plane + e) * nl + i] = to_store<S>(v * (kIs16<S> ? L.sc[i] : 1.0));
  }
};

// Populations at equilibrium f^eq(h, U) (Eq. equilibrium_distribution), rest
// population stored as deviation from hbar, for rows [ya, yb).
template <typename R, typename S>
__global__ void init_kernel(PopView<R, S> f, const double* __restrict__ hs, const double* __restrict__ uxs,
                            const double* __restrict__ uys, long long lstride, int yoff, int ya, int yb, int nx,
                            int pitch, int nl, Layers L) {
  long long n = (long long)(yb - ya) * nx;
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < n * nl;
       t += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(t / n);
    const long long rem = t % n;
    const int y = ya + (int)(rem / nx), x = (int)(rem % nx);
    const long long si = i * lstride + (long long)(y - yoff) * nx + x;
    const double h = hs[si], ux = uxs ? uxs[si] : 0.0, uy = uys ? uys[si] : 0.0;
    const double uu = ux * ux + uy * uy;
    const long long row = (long long)y * pitch;
    if (f.nq == 3) {  // D1Q3: f_0 = h (1 - U^2), f_+- = h (U^2 +- U) / 2
      f.st(i, 0, row + x, (h - L.hb[i]) - h * ux * ux, L);
      f.st(i, 1, row + mlf::wrap(x - 1, nx), 0.5 * h * (ux * ux + ux), L);
      f.st(i, 2, row + mlf::wrap(x + 1, nx), 0.5 * h * (ux * ux - ux), L);
      continue;
    }
    const int cx[9] = {0, 1, 1, 0, -1, -1, -1, 0, 1};
    const int cy[9] = {0, 0, 1, 1, 1, 0, -1, -1, -1};
    const double w[9] = {4.0 / 9, 1.0 / 9, 1.0 / 36, 1.0 / 9, 1.0 / 36, 1.0 / 9, 1.0 / 36, 1.0 / 9, 1.0 / 36};
    // plane k keeps at column x - c_kx the population of node x
    f.st(i, 0, row + x, (h - L.hb[i]) - h * (2.0 / 3.0) * uu, L);
    for (int k = 1; k < 9; ++k) {
      const double cu = cx[k] * ux + cy[k] * uy;
      f.st(i, k, row + mlf::wrap(x - cx[k], nx), w[k] * h * (3.0 * cu + 4.5 * cu * cu - 1.5 * uu), L);
    }
  }
}

// Height and flux of layer i at node x of the row starting at `row`: the
// moving planes keep node x's population at column x - c_kx.  One fixed
// summation order, so that read-back and the minimum see the same heights.
template <typename R, typename S>
__device__ inline void node_moments(const PopView<R, S>& f, int i, long long row, int x, int nx, const Layers& L,
                                    double& h, double& qx, double& qy) {
  if (f.nq == 3) {
    const double v0 = f.ld(i, 0, row + x, L), v1 = f.ld(i, 1, row + mlf::wrap(x - 1, nx), L),
                 v2 = f.ld(i, 2, row + mlf::wrap(x + 1, nx), L);
    qx = v1 - v2;
    qy = 0.0;
    h = L.hb[i] + (v0 + v1 + v2);
    return;
  }
  const int cx[9] = {0, 1, 1, 0, -1, -1, -1, 0, 1};
  double v[9];
  for (int k = 0; k < 9; ++k) v[k] = f.ld(i, k, row + mlf::wrap(x - cx[k], nx), L);
  const double dh = v[0] + v[1] + v[2] + v[3] + v[4] + v[5] + v[6] + v[7] + v[8];
  qx = (v[1] + v[2] + v[8]) - (v[4] + v[5] + v[6]);
  qy = (v[2] + v[3] + v[4]) - (v[6] + v[7] + v[8]);
  h = L.hb[i] + dh;
}

// h = hbar + sum_k f_k, U = q / h in FP64 for rows [ya, yb).
template <typename R, typename S>
__global__ void read_kernel(PopView<R, S> f, double* __restrict__ ho, double* __restrict__ uxo,
                            double* __restrict__ uyo, long long lstride, int yoff, int ya, int yb, int nx,
                            int pitch, int nl, Layers L) {
  long long n = (long long)(yb - ya) * nx;
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < n * nl;
       t += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(t / n);
    const long long rem = t % n;
    const int y = ya + (int)(rem / nx), x = (int)(rem % nx);
    double h, qx, qy;
    node_moments(f, i, (long long)y * pitch, x, nx, L, h, qx, qy);
    const long long di = i * lstride + (long long)(y - yoff) * nx + x;
    if (ho) ho[di] = h;
    if (uxo) uxo[di] = qx / h;
    if (uyo) uyo[di] = qy / h;
  }
}

// Block sums of sum_k f_ki (FP64, unscaled) per layer: partials[blockIdx.x][i].
template <typename R, typename S>
__global__ void __launch_bounds__(256) mass_partials(PopView<R, S> f, double* __restrict__ part, int nx,
                                                     int ny, int pitch, int nl, Layers L) {
  __shared__ double red[256 / 64][kMaxLayers];
  double acc[kMaxLayers] = {0, 0, 0, 0};
  const long long n = (long long)nx * ny;
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < n; t += (long long)gridDim.x * blockDim.x) {
    const int y = (int)(t / nx), x = (int)(t % nx);
    for (int i = 0; i < nl; ++i) {
      const long long e = (long long)y * pitch + x;
      double s = 0.0;
      for (int k = 0; k < f.nq; ++k) s += f.ld(i, k, e, L);  // power-of-two scales: exact
      acc[i] += s;
    }
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int i = 0; i < nl; ++i) {
    double v = acc[i];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if (lane == 0) red[wv][i] = v;
  }
  __syncthreads();
  if (threadIdx.x < nl) {
    double s = 0.0;
    for (int j = 0; j < (int)(blockDim.x >> 6); ++j) s += red[j][threadIdx.x];
    part[blockIdx.x * kMaxLayers + threadIdx.x] = s;
  }
}

// Sum of a FP64 field per layer (used for the reference heights of device
// inputs): partials[blockIdx.x][i].
__global__ void __launch_bounds__(256) field_partials(const double* __restrict__ a, double* __restrict__ part,
                                                      long long n, int nl) {
  __shared__ double red[256 / 64][kMaxLayers];
  double acc[kMaxLayers] = {0, 0, 0, 0};
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < n; t += (long long)gridDim.x * blockDim.x)
    for (int i = 0; i < nl; ++i) acc[i] += a[i * n + t];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int i = 0; i < nl; ++i) {
    double v = acc[i];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if (lane == 0) red[wv][i] = v;
  }
  __syncthreads();
  if (threadIdx.x < nl) {
    double s = 0.0;
    for (int j = 0; j < (int)(blockDim.x >> 6); ++j) s += red[j][threadIdx.x];
    part[blockIdx.x * kMaxLayers + threadIdx.x] = s;
  }
}

// Final fixed-order sum of the partials; one thread per layer.
// out[i] = sum over nblocks partials of layer i: each of the 256 threads
// sums a strided subset in order, then a tree in LDS (a fixed order).
__global__ void __launch_bounds__(256) finish_partials(const double* __restrict__ part, double* __restrict__ out,
                                                       int nblocks, int nl) {
  __shared__ double red[256];
  for (int i = 0; i < nl; ++i) {
    double s = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += 256) s += part[b * kMaxLayers + i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) out[i] = red[0];
    __syncthreads();
  }
}

__device__ inline double dmin(double a, double b) { return b < a ? b : a; }

// Minimum height per layer over the nodes t = first, first + stride, ...
// of one film, reduced over the workgroup; lane 0 of the result holds it.
template <typename R, typename S>
__device__ void block_min(const PopView<R, S>& f, int nx, int ny, int pitch, int nl, const Layers& L,
                          long long first, long long stride, double* __restrict__ out) {
  __shared__ double red[256 / 64][kMaxLayers];
  const double inf = __builtin_huge_val();
  double acc[kMaxLayers] = {inf, inf, inf, inf};
  const long long n = (long long)nx * ny;
  for (long long t = first; t < n; t += stride) {
    const int y = (int)(t / nx), x = (int)(t % nx);
    for (int i = 0; i < nl; ++i) {
      double h, qx, qy;
      node_moments(f, i, (long long)y * pitch, x, nx, L, h, qx, qy);
      acc[i] = dmin(acc[i], h);
    }
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int i = 0; i < nl; ++i) {
    double v = acc[i];
    for (int off = 32; off > 0; off >>= 1) v = dmin(v, __shfl_down(v, off, 64));
    if (lane == 0) red[wv][i] = v;
  }
  __syncthreads();
  if (threadIdx.x < kMaxLayers) {  // +inf past the film's layers
    double v = inf;
    if ((int)threadIdx.x < nl)
      for (int j = 0; j < (int)(blockDim.x >> 6); ++j) v = dmin(v, red[j][threadIdx.x]);
    out[threadIdx.x] = v;
  }
}

// Block minima of the heights per layer: partials[blockIdx.x][i].
template <typename R, typename S>
__global__ void __launch_bounds__(256) min_partials(PopView<R, S> f, double* __restrict__ part, int nx, int ny,
                                                    int pitch, int nl, Layers L) {
  block_min(f, nx, ny, pitch, nl, L, blockIdx.x * (long long)blockDim.x + threadIdx.x,
            (long long)gridDim.x * blockDim.x, part + blockIdx.x * kMaxLayers);
}

// Geometry and reference heights of one film of a batch for the minimum.
struct MinFilm {
  long long offset;  // bytes into the population buffer
  long long plane;   // nodes per plane (ny * pitch)
  int nx, ny, pitch, nl;
  int nq;            // directions (9 or 3)
  int pad;
  Layers L;
};

constexpr int kMinBlocksPerFilm = 8;

// Minima of every film of a batch: workgroup (x, film) covers nodes
// x, x + 8 * 256, ... of that film; partials[film][x][i].
template <typename R, typename S>
__global__ void __launch_bounds__(256) batch_min_partials(const MinFilm* __restrict__ films,
                                                          unsigned char* __restrict__ buf,
                                                          double* __restrict__ part) {
  const MinFilm m = films[blockIdx.y];
  const PopView<R, S> f{buf + m.offset, m.plane, m.nl, m.nq};
  block_min(f, m.nx, m.ny, m.pitch, m.nl, m.L, blockIdx.x * (long long)blockDim.x + threadIdx.x,
            (long long)gridDim.x * blockDim.x, part + ((size_t)blockIdx.y * gridDim.x + blockIdx.x) * kMaxLayers);
}

// out[g][i] = min over nblocks partials of group g (one thread per group and layer).
__global__ void finish_min(const double* __restrict__ part, double* __restrict__ out, int ngroups, int nblocks) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ngroups * kMaxLayers) return;
  const int g = t / kMaxLayers, i = t % kMaxLayers;
  double v = __builtin_huge_val();
  for (int b = 0; b < nblocks; ++b) v = dmin(v, part[((size_t)g * nblocks + b) * kMaxLayers + i]);
  out[t] = v;
}

}  // namespace

struct mlf_handle {
  mlf_params p;
  void* pop[2];
  int cur;
  unsigned char* scratch;
  hipStream_t stream;
  int pitch;
  size_t plane;
  size_t pop_bytes;
  double hbar[kMaxLayers];
  double scale[kMaxLayers];  // storage scale per layer (1 except IEEE half)
  int64_t steps;
  int block_w, seg_h;
  int ahead;  // rows of populations in flight in the step kernel (1 or 2)
  int sr;     // stochastic rounding of the rest plane (16-bit storage)
  bool initialised;
  hipGraphExec_t graph;  // captured step loop (constants baked in), or null
  int graph_steps, graph_parity;
  std::string err;
};

namespace {

// IEEE-half storage keeps the population deviations scaled by a power of two
// near 2^12 / hbar: values of order 1e-8 .. 1e-3 then stay in the normal
// range and deviations up to 16 hbar remain finite.  Other formats: 1.
double storage_scale(int precision, double hbar) {
  if (move_fmt(precision) != kFmtF16) return 1.0;
  int e = (int)std::floor(std::log2(4096.0 / std::max(hbar, 1e-30)));
  e = std::max(-30, std::min(30, e));
  return std::ldexp(1.0, e);
}

void set_scales(mlf_handle* h) {
  for (int i = 0; i < kMaxLayers; ++i)
    h->scale[i] = i < h->p.n_layers ? storage_scale(h->p.precision, h->hbar[i]) : 1.0;
}

// Host-side conversion of one stored element (population read/write);
// `raw` points at the element.
double host_load(Fmt fmt, const unsigned char* raw) {
  switch (fmt) {
    case kFmtF64: {
      double d;
      std::memcpy(&d, raw, 8);
      return d;
    }
    case kFmtF32: {
      float f;
      std::memcpy(&f, raw, 4);
      return f;
    }
    case kFmtF16: {
      _Float16 f;
      std::memcpy(&f, raw, 2);
      return (double)f;
    }
    default: {
      uint16_t u;
      std::memcpy(&u, raw, 2);
      uint32_t b = (uint32_t)u << 16;
      float f;
      std::memcpy(&f, &b, 4);
      return f;
    }
  }
}

void host_store(Fmt fmt, unsigned char* raw, double v) {
  switch (fmt) {
    case kFmtF64: std::memcpy(raw, &v, 8); break;
    case kFmtF32: {
      float f = (float)v;
      std::memcpy(raw, &f, 4);
      break;
    }
    case kFmtF16: {
      _Float16 f = (_Float16)v;
      std::memcpy(raw, &f, 2);
      break;
    }
    default: {
      float f = (float)v;
      uint32_t b;
      std::memcpy(&b, &f, 4);
      if ((b & 0x7f800000u) == 0x7f800000u && (b & 0x7fffffu))
        b = 0x7fc00000u;  // NaN stays NaN
      else
        b += 0x7fffu + ((b >> 16) & 1u);  // round to nearest even
      const uint16_t u = (uint16_t)(b >> 16);
      std::memcpy(raw, &u, 2);
    }
  }
}

Layers layers_of(const mlf_handle* h) {
  Layers L;
  for (int i = 0; i < kMaxLayers; ++i) {
    L.hb[i] = h->hbar[i];
    L.sc[i] = h->scale[i];
  }
  return L;
}

mlf_status fail(mlf_handle* h, mlf_status st, const std::string& m) {
  if (h) h->err = m;
  return st;
}

// The captured graph holds the step constants as kernel arguments: every
// change of reference heights, scales or launch shape drops it.
void drop_single_graph(mlf_handle* h) {
  if (h->graph) (void)hipGraphExecDestroy(h->graph);
  h->graph = nullptr;
  h->graph_steps = 0;
}

mlf_status hip_check(mlf_handle* h, hipError_t e, const char* what) {
  if (e == hipSuccess) return MLF_OK;
  return fail(h, MLF_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIPCHK(call)                                              \
  do {                                                            \
    mlf_status _s = hip_check(h, (call), #call);                  \
    if (_s != MLF_OK) return _s;                                  \
  } while (0)

int* flag_ptr(mlf_handle* h) { return reinterpret_cast<int*>(h->scratch + kFlagOff); }
double* redout_ptr(mlf_handle* h) { return reinterpret_cast<double*>(h->scratch + kRedOutOff); }
double* part_ptr(mlf_handle* h) { return reinterpret_cast<double*>(h->scratch + kPartOff); }
unsigned char* stage_ptr(mlf_handle* h) { return h->scratch + kStageOff; }

void default_launch(const mlf_params* p, int* bw, int* sh) {
  int w = p->nx + 4;
  *bw = w <= 64 ? 64 : (w <= 128 ? 128 : (w <= 192 ? 192 : 256));
  *sh = std::max(1, std::min(p->ny, 12));
}

template <typename C>
mlf::StepConsts<C> make_consts(const mlf_handle* h) {
  const mlf_params& p = h->p;
  mlf::StepConsts<C> k;
  std::memset(&k, 0, sizeof(k));
  k.nx = p.nx;
  k.ny = p.ny;
  k.pitch = h->pitch;
  k.plane = (long long)h->plane;
  const int W = h->block_w;
  k.wout = mlf::strip_width(p.nx, W);
  k.nstrip = mlf::strip_count(p.nx, W);
  k.seg_h = h->seg_h;
  k.nseg = (p.ny + k.seg_h - 1) / k.seg_h;
  const int n = p.n_layers;
  double z[kMaxLayers + 1];
  z[0] = 0.0;
  for (int i = 0; i < n; ++i) {
    k.hbar[i] = C(h->hbar[i]);
    z[i + 1] = z[i] + h->hbar[i];
    k.gamma[i] = C(p.gamma[i]);
    k.mu[i] = C(p.mu[i]);
  }
  for (int l = 0; l < n; ++l)
    for (int kk = 1; kk <= n - l; ++kk) {
      k.dbar[l][kk - 1] = C(z[l + kk] - z[l]);
      const double S = p.spread[pair_index(n, l, kk)];
      const double a = p.exp_a, b = p.exp_b;
      k.sa[l][kk - 1] = C(S * a / (a - b));
      k.sb[l][kk - 1] = C(S * b / (a - b));
      k.sab[l][kk - 1] = C(S * a * b / (a - b));
      if (S != 0.0) k.pairs |= 1u << (l * 4 + kk - 1);
    }
  for (int kk = 1; kk <= kMaxLayers; ++kk) k.khs[kk - 1] = C(kk * p.hstar);
  k.omega = C(1.0 / p.tau);
  for (int i = 0; i < n; ++i) {
    k.slip[i] = C(p.slip[i]);
    if (p.slip[i] != 0.0) k.slip_on = 1;
  }
  for (int i = 0; i < kMaxLayers; ++i) {
    k.scale[i] = C(h->scale[i]);
    k.iscale[i] = C(1.0 / h->scale[i]);
  }
  k.ea = p.exp_a;
  k.eb = p.exp_b;
  k.flag = flag_ptr(const_cast<mlf_handle*>(h));
  k.sr_on = h->sr;
  k.sr_step = (unsigned)h->steps;
  return k;
}

// Workgroups of the step kernel that fit on one CU at the handle's block
// width (0 if unknown).
template <typename R, typename S, typename C, int NL, bool T1, int EA, int EB, int AH>
int occupancy_ah(const mlf_handle* h) {
  int nb = 0;
  size_t lds = (size_t)8 * NL * h->block_w * sizeof(C);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, mlf::step_kernel<R, S, C, NL, T1, EA, EB, AH>, h->block_w,
                                                   lds) != hipSuccess)
    return 0;
  return nb;
}

template <typename R, typename S, typename C, int NL, bool T1, int EA, int EB, int AH>
hipError_t launch_ah(const mlf_handle* h, const void* src, void* dst) {
  mlf::StepConsts<C> kc = make_consts<C>(h);
  // grid padded to a multiple of the XCD count (tile_of_block)
  const int ntiles = kc.nstrip * kc.nseg;
  const int nblocks = (ntiles + mlf::kXcds - 1) / mlf::kXcds * mlf::kXcds;
  dim3 grid((unsigned)nblocks), block((unsigned)h->block_w);
  size_t lds = (size_t)8 * NL * h->block_w * sizeof(C);
  hipLaunchKernelGGL((mlf::step_kernel<R, S, C, NL, T1, EA, EB, AH>), grid, block, lds, h->stream,
                     static_cast<const unsigned char*>(src), static_cast<unsigned char*>(dst), kc);
  return hipGetLastError();
}

// Two rows ahead exist for tau = 1 with FP32 arithmetic only (prefetch_ok).
template <typename R, typename S, typename C, int NL, bool T1, int EA, int EB>
int occupancy_nl(const mlf_handle* h) {
  if constexpr (T1 && sizeof(C) == 4)
    if (h->ahead == 2) return occupancy_ah<R, S, C, NL, T1, EA, EB, 2>(h);
  return occupancy_ah<R, S, C, NL, T1, EA, EB, 1>(h);
}

template <typename R, typename S, typename C, int NL, bool T1, int EA, int EB>
hipError_t launch_nl(const mlf_handle* h, const void* src, void* dst) {
  if constexpr (T1 && sizeof(C) == 4)
    if (h->ahead == 2) return launch_ah<R, S, C, NL, T1, EA, EB, 2>(h, src, dst);
  return launch_ah<R, S, C, NL, T1, EA, EB, 1>(h, src, dst);
}

// Dispatch on (layers, tau == 1, exponents == (9, 3)); OCC selects the
// occupancy query instead of a launch.
template <typename R, typename S, typename C, bool T1, int EA, int EB>
hipError_t launch_t(const mlf_handle* h, const void* src, void* dst, int* occ) {
  switch (h->p.n_layers) {
    case 1:
      if (occ) return *occ = occupancy_nl<R, S, C, 1, T1, EA, EB>(h), hipSuccess;
      return launch_nl<R, S, C, 1, T1, EA, EB>(h, src, dst);
    case 2:
      if (occ) return *occ = occupancy_nl<R, S, C, 2, T1, EA, EB>(h), hipSuccess;
      return launch_nl<R, S, C, 2, T1, EA, EB>(h, src, dst);
    case 3:
      if (occ) return *occ = occupancy_nl<R, S, C, 3, T1, EA, EB>(h), hipSuccess;
      return launch_nl<R, S, C, 3, T1, EA, EB>(h, src, dst);
    default:
      if (occ) return *occ = occupancy_nl<R, S, C, 4, T1, EA, EB>(h), hipSuccess;
      return launch_nl<R, S, C, 4, T1, EA, EB>(h, src, dst);
  }
}

template <typename R, typename S, typename C>
hipError_t launch_sc(const mlf_handle* h, const void* src, void* dst, int* occ) {
  const bool t1 = h->p.tau == 1.0;
  const bool e93 = h->p.exp_a == 9 && h->p.exp_b == 3;
  if (t1 && e93) return launch_t<R, S, C, true, 9, 3>(h, src, dst, occ);
  if (t1) return launch_t<R, S, C, true, 0, 0>(h, src, dst, occ);
  if (e93) return launch_t<R, S, C, false, 9, 3>(h, src, dst, occ);
  return launch_t<R, S, C, false, 0, 0>(h, src, dst, occ);
}

// Calls f with typed null pointers of the handle's rest-plane and
// moving-plane storage types.
template <typename F>
void by_storage(const mlf_handle* h, F&& f) {
  switch (h->p.precision) {
    case MLF_F64: f((double*)nullptr, (double*)nullptr); break;
    case MLF_F32: f((float*)nullptr, (float*)nullptr); break;
    case MLF_F16: f((_Float16*)nullptr, (_Float16*)nullptr); break;
    case MLF_BF16: f((__bf16*)nullptr, (__bf16*)nullptr); break;
    case MLF_F16_MIX: f((float*)nullptr, (_Float16*)nullptr); break;
    default: f((float*)nullptr, (__bf16*)nullptr); break;
  }
}

hipError_t launch_step(const mlf_handle* h, const void* src, void* dst) {
  hipError_t e = hipSuccess;
  by_storage(h, [&](auto* rt, auto* st) {
    using R = std::remove_pointer_t<decltype(rt)>;
    using S = std::remove_pointer_t<decltype(st)>;
    using C = std::conditional_t<std::is_same_v<S, double>, double, float>;
    e = launch_sc<R, S, C>(h, src, dst, nullptr);
  });
  return e;
}

// ---- D1Q3 films (ny == 1): resident multi-step kernel or one step per launch

constexpr int kD1MaxStepsPerLaunch = 65536;  // keeps a resident launch to ~0.1 s

bool d1_resident(const mlf_params& p) {
  const size_t c = p.precision == MLF_F64 ? 8 : 4;
  return p.nx <= 2 * mlf::kD1Threads && (size_t)5 * p.n_layers * p.nx * c <= 65536;
}

int d1_threads(int nx) { return std::min(mlf::kD1Threads, std::max(64, (nx + 63) / 64 * 64)); }

// Single D1Q3 films longer than one tile run tiled over several workgroups
// (kD1TileSteps steps per launch); shorter ones are held by one workgroup of
// at most two waves.
bool d1_tiled(const mlf_params& p) { return p.lattice == MLF_D1Q3 && p.nx > mlf::kD1TileThreads; }

template <typename C, int NL, bool T1, int EA, int EB>
hipError_t d1_launch_nl(mlf_handle* h, int steps) {
  mlf::StepConsts<C> kc = make_consts<C>(h);
  const mlf_params& p = h->p;
  const C* src = static_cast<const C*>(h->pop[h->cur]);
  C* dst = static_cast<C*>(h->pop[h->cur ^ 1]);
  if (d1_tiled(p)) {
    if (steps < 1 || steps > mlf::kD1TileSteps) return hipErrorInvalidValue;
    const int tiles = (p.nx + mlf::kD1TileCore - 1) / mlf::kD1TileCore;
    hipLaunchKernelGGL((mlf::d1q3_tiled<C, NL, T1, EA, EB>), dim3((unsigned)tiles), dim3(mlf::kD1TileThreads),
                       mlf::d1_tile_lds<C>(NL), h->stream, src, dst, kc, steps, mlf::kD1TileCore);
    h->cur ^= 1;
    return hipGetLastError();
  }
  const size_t lds = mlf::d1_resident_lds<C>(p.nx, NL);
  hipLaunchKernelGGL((mlf::d1q3_resident<C, NL, T1, EA, EB>), dim3(1), dim3((unsigned)d1_threads(p.nx)), lds,
                     h->stream, src, dst, kc, steps);
  h->cur ^= 1;
  return hipGetLastError();
}

template <typename C, bool T1, int EA, int EB>
hipError_t d1_launch_t(mlf_handle* h, int steps) {
  switch (h->p.n_layers) {
    case 1: return d1_launch_nl<C, 1, T1, EA, EB>(h, steps);
    case 2: return d1_launch_nl<C, 2, T1, EA, EB>(h, steps);
    case 3: return d1_launch_nl<C, 3, T1, EA, EB>(h, steps);
    default: return d1_launch_nl<C, 4, T1, EA, EB>(h, steps);
  }
}

// Advances a D1Q3 film by `steps` (1..kD1MaxStepsPerLaunch; 1..kD1TileSteps
// when tiled); flips h->cur.
template <typename C>
hipError_t d1_advance_c(mlf_handle* h, int steps) {
  const bool t1 = h->p.tau == 1.0;
  const bool e93 = h->p.exp_a == 9 && h->p.exp_b == 3;
  if (t1 && e93) return d1_launch_t<C, true, 9, 3>(h, steps);
  if (t1) return d1_launch_t<C, true, 0, 0>(h, steps);
  if (e93) return d1_launch_t<C, false, 9, 3>(h, steps);
  return d1_launch_t<C, false, 0, 0>(h, steps);
}

hipError_t d1_advance(mlf_handle* h, int steps) {
  return h->p.precision == MLF_F64 ? d1_advance_c<double>(h, steps) : d1_advance_c<float>(h, steps);
}

// ---- D2Q9 films one row high: resident multi-step kernel ------------------

// One-row films wider than one tile run tiled over several workgroups
// (kRowTileSteps steps per launch); narrower ones fit one workgroup of at
// most two waves, which holds them for up to kD1MaxStepsPerLaunch steps per
// launch.
bool row_tiled(const mlf_params& p) {
  if (p.lattice != MLF_D2Q9 || p.ny != 1) return false;
  if (p.precision != MLF_F64 && p.precision != MLF_F32) return false;
  return p.nx > mlf::kRowTileThreads;
}

bool row_resident(const mlf_params& p) {
  if (p.lattice != MLF_D2Q9 || p.ny != 1) return false;
  if (p.precision != MLF_F64 && p.precision != MLF_F32) return false;
  if (row_tiled(p)) return true;
  const size_t c = p.precision == MLF_F64 ? 8 : 4;
  return p.nx <= mlf::kRowMaxPerThread * mlf::kRowThreads &&
         (size_t)11 * p.n_layers * p.nx * c <= mlf::kRowMaxLds;
}

template <typename C, int NL, bool T1, int EA, int EB>
hipError_t row_launch_nl(mlf_handle* h, int steps) {
  mlf::StepConsts<C> kc = make_consts<C>(h);
  const mlf_params& p = h->p;
  if (row_tiled(p)) {
    if (steps < 1 || steps > mlf::kRowTileSteps) return hipErrorInvalidValue;
    const size_t lds = mlf::row_tile_lds<C>(NL);
    auto kern = mlf::d2q9_row_tiled<C, NL, T1, EA, EB>;
    if (lds > 65536) {
      hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) return e;
    }
    const int tiles = (p.nx + mlf::kRowTileCore - 1) / mlf::kRowTileCore;
    hipLaunchKernelGGL(kern, dim3((unsigned)tiles), dim3(mlf::kRowTileThreads), lds, h->stream,
                       static_cast<const C*>(h->pop[h->cur]), static_cast<C*>(h->pop[h->cur ^ 1]), kc, steps,
                       mlf::kRowTileCore);
    h->cur ^= 1;
    return hipGetLastError();
  }
  const size_t lds = mlf::row_resident_lds<C>(p.nx, NL);
  auto kern = mlf::d2q9_row_resident<C, NL, T1, EA, EB>;
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  const int threads = std::min(mlf::kRowThreads, std::max(64, (p.nx + 63) / 64 * 64));
  hipLaunchKernelGGL(kern, dim3(1), dim3((unsigned)threads), lds, h->stream, static_cast<const C*>(h->pop[h->cur]),
                     static_cast<C*>(h->pop[h->cur ^ 1]), kc, steps);
  h->cur ^= 1;
  return hipGetLastError();
}

template <typename C, bool T1, int EA, int EB>
hipError_t row_launch_t(mlf_handle* h, int steps) {
  switch (h->p.n_layers) {
    case 1: return row_launch_nl<C, 1, T1, EA, EB>(h, steps);
    case 2: return row_launch_nl<C, 2, T1, EA, EB>(h, steps);
    case 3: return row_launch_nl<C, 3, T1, EA, EB>(h, steps);
    default: return row_launch_nl<C, 4, T1, EA, EB>(h, steps);
  }
}

// Advances a one-row D2Q9 film by `steps` (1..kD1MaxStepsPerLaunch; 1..kRowTileSteps when
// tiled); flips h->cur.
template <typename C>
hipError_t row_advance_c(mlf_handle* h, int steps) {
  const bool t1 = h->p.tau == 1.0;
  const bool e93 = h->p.exp_a == 9 && h->p.exp_b == 3;
  if (t1 && e93) return row_launch_t<C, true, 9, 3>(h, steps);
  if (t1) return row_launch_t<C, true, 0, 0>(h, steps);
  if (e93) return row_launch_t<C, false, 9, 3>(h, steps);
  return row_launch_t<C, false, 0, 0>(h, steps);
}

hipError_t row_advance(mlf_handle* h, int steps) {
  return h->p.precision == MLF_F64 ? row_advance_c<double>(h, steps) : row_advance_c<float>(h, steps);
}

int step_occupancy(const mlf_handle* h) {
  int occ = 0;
  by_storage(h, [&](auto* rt, auto* st) {
    using R = std::remove_pointer_t<decltype(rt)>;
    using S = std::remove_pointer_t<decltype(st)>;
    using C = std::conditional_t<std::is_same_v<S, double>, double, float>;
    (void)launch_sc<R, S, C>(h, nullptr, nullptr, &occ);  // occupancy query; 0 on error
  });
  return occ;
}

unsigned grid_for(long long n) {
  long long g = (n + 255) / 256;
  return (unsigned)std::max(1LL, std::min(g, 8192LL));
}

mlf_status launch_init(mlf_handle* h, const double* hs, const double* uxs, const double* uys, long long lstride,
                       int yoff, int ya, int yb) {
  const mlf_params& p = h->p;
  const long long n = (long long)(yb - ya) * p.nx * p.n_layers;
  const Layers L = layers_of(h);
  by_storage(h, [&](auto* rt, auto* st) {
    using R = std::remove_pointer_t<decltype(rt)>;
    using S = std::remove_pointer_t<decltype(st)>;
    const PopView<R, S> f{static_cast<unsigned char*>(h->pop[h->cur]), (long long)h->plane, p.n_layers,
                          nq_of(&p)};
    hipLaunchKernelGGL((init_kernel<R, S>), dim3(grid_for(n)), dim3(256), 0, h->stream, f, hs, uxs, uys, lstride,
                       yoff, ya, yb, p.nx, h->pitch, p.n_layers, L);
  });
  HIPCHK(hipGetLastError());
  return MLF_OK;
}

mlf_status launch_read(mlf_handle* h, double* ho, double* uxo, double* uyo, long long lstride, int yoff, int ya,
                       int yb) {
  const mlf_params& p = h->p;
  const long long n = (long long)(yb - ya) * p.nx * p.n_layers;
  const Layers L = layers_of(h);
  by_storage(h, [&](auto* rt, auto* st) {
    using R = std::remove_pointer_t<decltype(rt)>;
    using S = std::remove_pointer_t<decltype(st)>;
    const PopView<R, S> f{static_cast<unsigned char*>(h->pop[h->cur]), (long long)h->plane, p.n_layers,
                          nq_of(&p)};
    hipLaunchKernelGGL((read_kernel<R, S>), dim3(grid_for(n)), dim3(256), 0, h->stream, f, ho, uxo, uyo, lstride,
                       yoff, ya, yb, p.nx, h->pitch, p.n_layers, L);
  });
  HIPCHK(hipGetLastError());
  return MLF_OK;
}

int rows_per_chunk(const mlf_handle* h, int fields) {
  size_t row = (size_t)fields * h->p.n_layers * h->p.nx * sizeof(double);
  return (int)std::max<size_t>(0, kStageBytes / row);
}

mlf_status check_guard(mlf_handle* h) {
  int flag = 0;
  HIPCHK(hipMemcpyAsync(&flag, flag_ptr(h), sizeof(int), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  if (flag == 1)
    return fail(h, MLF_ENONPOSITIVE,
                "a layer height became <= 0 at or before step " + std::to_string(h->steps));
  if (flag != 0)
    return fail(h, MLF_ENONFINITE,
                "a layer height or flux became non-finite at or before step " + std::to_string(h->steps));
  return MLF_OK;
}

mlf_status check_stability(mlf_handle* h) {
  const mlf_params& p = h->p;
  if (p.allow_unstable) return MLF_OK;
  // explicit friction: the fluxes' per-step amplification I + K must have
  // spectral radius below 1 with each layer at h* or at its reference
  // thickness (without slip: every eigenvalue of -K below 2)
  double worst = 0.0, rate = 0.0;
  for (int mask = 0; mask < (1 << p.n_layers); ++mask) {
    double hh[kMaxLayers], K[kMaxLayers * kMaxLayers];
    for (int i = 0; i < p.n_layers; ++i) hh[i] = (mask >> i & 1) ? p.hstar : h->hbar[i];
    friction_matrix(p.n_layers, hh, p.mu, p.slip, K);
    worst = std::max(worst, friction_amplification(p.n_layers, K));
    rate = std::max(rate, max_rate(p.n_layers, K));
  }
  if (!(worst < 1.0)) {
    char buf[200];
    std::snprintf(buf, sizeof buf,
                  "explicit friction unstable: flux amplification %.4g >= 1 (largest friction rate %.4g)", worst,
                  rate);
    return fail(h, MLF_EUNSTABLE, buf);
  }
  return MLF_OK;
}

// Both population buffers start zeroed so that the row padding (never
// written by the kernels) is deterministic in checkpoints.
mlf_status zero_buffers(mlf_handle* h) {
  HIPCHK(hipMemsetAsync(h->pop[0], 0, h->pop_bytes, h->stream));
  HIPCHK(hipMemsetAsync(h->pop[1], 0, h->pop_bytes, h->stream));
  return MLF_OK;
}

mlf_status finish_init(mlf_handle* h) {
  HIPCHK(hipMemsetAsync(flag_ptr(h), 0, sizeof(int), h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  h->steps = 0;
  h->initialised = true;
  return MLF_OK;
}

}  // namespace

namespace {
template <int MODE, int AUX>
hipError_t stream_launch(const void* src, void* dst, uint32_t n16, uint32_t chunk, int blocks, hipStream_t s) {
  hipLaunchKernelGGL((mlf::stream_probe_kernel<MODE, AUX>), dim3((unsigned)blocks), dim3(mlf::kStreamThreads), 0, s,
                     static_cast<const unsigned char*>(src), static_cast<unsigned char*>(dst), n16, chunk);
  return hipGetLastError();
}
template <int MODE>
hipError_t stream_launch_m(bool nt, const void* src, void* dst, uint32_t n16, uint32_t chunk, int blocks,
                           hipStream_t s) {
  return nt ? stream_launch<MODE, 2>(src, dst, n16, chunk, blocks, s)
            : stream_launch<MODE, 0>(src, dst, n16, chunk, blocks, s);
}
}  // namespace

// ---- allocation-free per-layer mass -----------------------------------------
// Reduction partials of mlf_layer_mass_static live in this fixed array, one
// copy per GPU, for the life of the process.  Host code never uses the
// array's name as an address: it takes each device's address once with
// hipGetSymbolAddress and passes that pointer to the kernels.
namespace {
constexpr size_t kStaticScratchBytes = (size_t)kRedBlocks * kMaxLayers * sizeof(double);  // 16 KiB
constexpr int kStaticMaxDevices = 64;
}  // namespace

static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {
std::mutex g_static_mu;
void* g_static_ptr[kStaticMaxDevices];  // device address of `scratch` per device, null until taken

// Address of `scratch` on the current device; set-up on the first call per device.
hipError_t static_scratch(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kStaticMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_static_mu);
  if (!g_static_ptr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!ptr) return hipErrorInvalidSymbol;
    g_static_ptr[dev] = ptr;
  }
  *out = g_static_ptr[dev];
  return hipSuccess;
}

// out[i] = base[i] + fixed-order sum of the partials of layer i (the same
// order as finish_partials); base[i] = nx ny h_ref_i, formed on the host.
struct MassBase {
  double v[kMaxLayers];
};
__global__ void __launch_bounds__(256) finish_mass(const double* __restrict__ part, double* __restrict__ out,
                                                   int nblocks, int nl, MassBase base) {
  __shared__ double red[256];
  for (int i = 0; i < nl; ++i) {
    double s = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += 256) s += part[b * kMaxLayers + i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) out[i] = base.v[i] + red[0];
    __syncthreads();
  }
}
}  // namespace

// ================================================================ C ABI ====
extern "C" {

const char* mlf_version(void) { return "mlfilm 0.1 gfx950"; }


mlf_status mlf_stream_probe(int32_t mode, int32_t schedule, int32_t nontemporal, const void* src, void* dst,
                            uint64_t bytes, int32_t blocks, void* stream) {
  if (mode < MLF_STREAM_READ || mode > MLF_STREAM_COPY || (schedule != 0 && schedule != 1) || blocks < 0)
    return MLF_EINVAL;
  if (!dst || (mode != MLF_STREAM_WRITE && !src)) return MLF_EINVAL;
  if (bytes < 16 || bytes % 16 != 0 || bytes > 0xfffffff0ull) return MLF_EINVAL;
  const uint32_t n16 = (uint32_t)(bytes / 16);
  if (blocks == 0) {
    int dev = 0, ncu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      return MLF_EDEVICE;
    blocks = 64 * std::max(1, ncu);
  }
  // no more workgroups than 16-byte elements per lane group
  blocks = (int)std::min<uint64_t>((uint64_t)blocks, ((uint64_t)n16 + mlf::kStreamThreads - 1) / mlf::kStreamThreads);
  blocks = std::max(blocks, 1);
  const uint32_t chunk = schedule == 0 ? (uint32_t)(((uint64_t)n16 + blocks - 1) / blocks) : 0u;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e;
  if (mode == MLF_STREAM_READ) e = stream_launch_m<mlf::kStreamRead>(nontemporal != 0, src, dst, n16, chunk, blocks, s);
  else if (mode == MLF_STREAM_WRITE) e = stream_launch_m<mlf::kStreamWrite>(nontemporal != 0, dst, dst, n16, chunk, blocks, s);
  else e = stream_launch_m<mlf::kStreamCopy>(nontemporal != 0, src, dst, n16, chunk, blocks, s);
  return e == hipSuccess ? MLF_OK : MLF_EDEVICE;
}

mlf_status mlf_query_sizes(const mlf_params* p, size_t* pop_bytes, size_t* scratch_bytes) {
  mlf_status st = validate(p, nullptr);
  if (st != MLF_OK) return st;
  if (pop_bytes) *pop_bytes = buffer_bytes(p->precision, p->n_layers, (size_t)pitch_of(p) * p->ny, nq_of(p));
  if (scratch_bytes) *scratch_bytes = kScratchBytes;
  return MLF_OK;
}

mlf_status mlf_query_pitch(const mlf_params* p, int32_t* pitch) {
  mlf_status st = validate(p, nullptr);
  if (st != MLF_OK) return st;
  if (pitch) *pitch = pitch_of(p);
  return MLF_OK;
}

mlf_status mlf_create(const mlf_params* p, void* pop_a, void* pop_b, void* scratch, void* stream,
                      mlf_handle** out) {
  if (!out) return MLF_EINVAL;
  *out = nullptr;
  std::string why;
  mlf_status st = validate(p, &why);
  if (st != MLF_OK) return st;
  if (!pop_a || !pop_b || !scratch || pop_a == pop_b) return MLF_EINVAL;
  auto aligned = [](void* v) { return (reinterpret_cast<uintptr_t>(v) & 255) == 0; };
  if (!aligned(pop_a) || !aligned(pop_b) || !aligned(scratch)) return MLF_EINVAL;
  mlf_handle* h = new (std::nothrow) mlf_handle();
  if (!h) return MLF_EINVAL;
  h->p = *p;
  h->pop[0] = pop_a;
  h->pop[1] = pop_b;
  h->cur = 0;
  h->scratch = static_cast<unsigned char*>(scratch);
  h->stream = static_cast<hipStream_t>(stream);
  h->pitch = pitch_of(p);
  h->plane = (size_t)h->pitch * p->ny;
  h->pop_bytes = buffer_bytes(p->precision, p->n_layers, h->plane, nq_of(p));
  for (int i = 0; i < kMaxLayers; ++i) h->hbar[i] = 0.0, h->scale[i] = 1.0;
  h->steps = 0;
  h->initialised = false;
  h->graph = nullptr;
  h->graph_steps = 0;
  h->graph_parity = 0;
  default_launch(p, &h->block_w, &h->seg_h);
  h->ahead = 1;
  h->sr = 0;
  *out = h;
  return MLF_OK;
}

mlf_status mlf_destroy(mlf_handle* h) {
  if (!h) return MLF_EINVAL;
  drop_single_graph(h);
  delete h;
  return MLF_OK;
}

int64_t mlf_steps_done(const mlf_handle* h) { return h ? h->steps : -1; }

const char* mlf_last_error(const mlf_handle* h) { return h ? h->err.c_str() : "null handle"; }

// Widest strip the step kernel is compiled for with these parameters (the
// kernel's step_max_lanes: FP64 with four layers stops at 256 lanes).
int max_block_w(const mlf_params& p) { return (p.precision == MLF_F64 && p.n_layers == 4) ? 256 : 512; }

mlf_status mlf_set_launch(mlf_handle* h, int32_t block_w, int32_t seg_h) {
  if (!h) return MLF_EINVAL;
  drop_single_graph(h);
  int bw, sh;
  default_launch(&h->p, &bw, &sh);
  if (block_w != 0) {
    if (block_w != 64 && block_w != 128 && block_w != 192 && block_w != 256 && block_w != 512)
      return fail(h, MLF_EINVAL, "block_w must be 64, 128, 192, 256 or 512");
    if (block_w > max_block_w(h->p))
      return fail(h, MLF_EINVAL, "block_w 512 is not available for FP64 films of four layers");
    bw = block_w;
  }
  if (seg_h != 0) {
    if (seg_h < 1) return fail(h, MLF_EINVAL, "seg_h must be >= 1");
    sh = std::min(seg_h, h->p.ny);
  }
  h->block_w = bw;
  h->seg_h = sh;
  return MLF_OK;
}

mlf_status mlf_get_launch(const mlf_handle* h, int32_t* block_w, int32_t* seg_h) {
  if (!h) return MLF_EINVAL;
  if (block_w) *block_w = h->block_w;
  if (seg_h) *seg_h = h->seg_h;
  return MLF_OK;
}

// Two rows of populations in flight: D2Q9 films with tau = 1 and FP32
// arithmetic (every storage format but FP64).
bool prefetch_ok(const mlf_params& p) {
  return p.lattice == MLF_D2Q9 && p.tau == 1.0 && p.precision != MLF_F64;
}

mlf_status mlf_set_prefetch(mlf_handle* h, int32_t rows) {
  if (!h) return MLF_EINVAL;
  if (rows < 0 || rows > 2) return fail(h, MLF_EINVAL, "prefetch rows must be 0, 1 or 2");
  if (rows == 2 && !prefetch_ok(h->p))
    return fail(h, MLF_EINVAL, "two rows ahead needs a D2Q9 film with tau = 1 and non-FP64 storage");
  drop_single_graph(h);
  h->ahead = rows == 0 ? 1 : rows;
  return MLF_OK;
}

mlf_status mlf_get_prefetch(const mlf_handle* h, int32_t* rows) {
  if (!h || !rows) return MLF_EINVAL;
  *rows = h->ahead;
  return MLF_OK;
}

mlf_status mlf_set_rounding(mlf_handle* h, int32_t mode) {
  if (!h) return MLF_EINVAL;
  if (mode != MLF_ROUND_NEAREST && mode != MLF_ROUND_STOCHASTIC_REST)
    return fail(h, MLF_EINVAL, "unknown rounding mode");
  if (mode == MLF_ROUND_STOCHASTIC_REST &&
      !(h->p.lattice == MLF_D2Q9 && (h->p.precision == MLF_F16 || h->p.precision == MLF_BF16)))
    return fail(h, MLF_EINVAL, "stochastic rounding needs a D2Q9 film with MLF_F16 or MLF_BF16 storage");
  drop_single_graph(h);
  h->sr = mode == MLF_ROUND_STOCHASTIC_REST;
  return MLF_OK;
}

mlf_status mlf_get_rounding(const mlf_handle* h, int32_t* mode) {
  if (!h || !mode) return MLF_EINVAL;
  *mode = h->sr ? MLF_ROUND_STOCHASTIC_REST : MLF_ROUND_NEAREST;
  return MLF_OK;
}

mlf_status mlf_autotune(mlf_handle* h, int32_t reps, int32_t* block_w, int32_t* seg_h) {
  if (!h || reps < 1) return MLF_EINVAL;
  if (!h->initialised) return fail(h, MLF_EINVAL, "autotune before init");
  if (h->p.lattice == MLF_D1Q3) {  // the D1Q3 kernels have fixed shapes
    if (block_w) *block_w = h->block_w;
    if (seg_h) *seg_h = h->seg_h;
    return MLF_OK;
  }
  drop_single_graph(h);
  const mlf_params& p = h->p;
  int dev = 0, ncu = 0;
  HIPCHK(hipGetDevice(&dev));
  HIPCHK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  const int keep_w = h->block_w, keep_h = h->seg_h, keep_a = h->ahead;
  // candidates (block width, segment height, rows in flight)
  typedef std::array<int, 3> Cand;
  std::vector<Cand> cand;
  const int fixed[] = {2, 3, 4, 6, 8, 10, 12, 16, 20, 24, 32, 48, 64, 96, 128};
  for (int ah = 1; ah <= (prefetch_ok(p) ? 2 : 1); ++ah)
    for (int w : {64, 128, 192, 256, 512}) {
      if (w > max_block_w(p)) continue;
      h->block_w = w;
      h->ahead = ah;
      const int nstrip = mlf::strip_count(p.nx, w);
      for (int sh : fixed)
        if (sh <= p.ny) cand.push_back({w, sh, ah});
      // heights that fill 1..4 whole dispatch rounds
      const int slots = std::max(1, step_occupancy(h)) * std::max(1, ncu);
      for (int rounds = 1; rounds <= 4; ++rounds) {
        const int segs = std::max(1, rounds * slots / nstrip);
        const int sh = std::max(1, (p.ny + segs - 1) / segs);
        cand.push_back({w, std::min(sh, p.ny), ah});
      }
    }
  std::sort(cand.begin(), cand.end());
  cand.erase(std::unique(cand.begin(), cand.end()), cand.end());
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  mlf_status st = MLF_OK;
  // ms per launch of candidate c over n launches (current -> other buffer,
  // never swapped: the state is left unchanged)
  auto time_of = [&](const Cand& c, int n, float* ms) {
    h->block_w = c[0];
    h->seg_h = c[1];
    h->ahead = c[2];
    if ((st = hip_check(h, launch_step(h, h->pop[h->cur], h->pop[h->cur ^ 1]), "autotune launch")) != MLF_OK)
      return false;
    if ((st = hip_check(h, hipEventRecord(e0, h->stream), "hipEventRecord")) != MLF_OK) return false;
    for (int r = 0; r < n && st == MLF_OK; ++r)
      st = hip_check(h, launch_step(h, h->pop[h->cur], h->pop[h->cur ^ 1]), "autotune launch");
    if (st != MLF_OK) return false;
    if ((st = hip_check(h, hipEventRecord(e1, h->stream), "hipEventRecord")) != MLF_OK) return false;
    if ((st = hip_check(h, hipEventSynchronize(e1), "hipEventSynchronize")) != MLF_OK) return false;
    if ((st = hip_check(h, hipEventElapsedTime(ms, e0, e1), "hipEventElapsedTime")) != MLF_OK) return false;
    *ms /= (float)n;
    return true;
  };
  // a first pass over every candidate, then the four fastest re-timed in two
  // interleaved rounds of 4 x reps launches (the minimum counts): single
  // short timings are noisy at the few-percent level that separates shapes
  std::vector<std::pair<float, Cand>> timed;
  for (const auto& c : cand) {
    float ms = 0.f;
    if (!time_of(c, reps, &ms)) break;
    timed.emplace_back(ms, c);
  }
  int bw = keep_w, bh = keep_h, ba = keep_a;
  if (st == MLF_OK && !timed.empty()) {
    std::sort(timed.begin(), timed.end());
    timed.resize(std::min<size_t>(timed.size(), 4));
    std::vector<float> best(timed.size(), 1e30f);
    for (int round = 0; round < 2 && st == MLF_OK; ++round)
      for (size_t i = 0; i < timed.size() && st == MLF_OK; ++i) {
        float ms = 0.f;
        if (time_of(timed[i].second, 4 * reps, &ms)) best[i] = std::min(best[i], ms);
      }
    const size_t k = (size_t)(std::min_element(best.begin(), best.end()) - best.begin());
    bw = timed[k].second[0];
    bh = timed[k].second[1];
    ba = timed[k].second[2];
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  h->block_w = (st == MLF_OK) ? bw : keep_w;
  h->seg_h = (st == MLF_OK) ? bh : keep_h;
  h->ahead = (st == MLF_OK) ? ba : keep_a;
  if (st != MLF_OK) return st;
  if (block_w) *block_w = bw;
  if (seg_h) *seg_h = bh;
  return MLF_OK;
}

mlf_status mlf_init(mlf_handle* h, const double* hgt, const double* ux, const double* uy) {
  if (!h || !hgt) return MLF_EINVAL;
  drop_single_graph(h);
  const mlf_params& p = h->p;
  const long long nn = (long long)p.nx * p.ny;
  h->initialised = false;
  for (int i = 0; i < p.n_layers; ++i) {
    double s = 0.0;
    for (long long j = 0; j < nn; ++j) {
      const double v = hgt[i * nn + j];
      if (!std::isfinite(v) || (ux && !std::isfinite(ux[i * nn + j])) || (uy && !std::isfinite(uy[i * nn + j])))
        return fail(h, MLF_ENONFINITE, "initial field is not finite");
      if (!(v > 0.0)) return fail(h, MLF_ENONPOSITIVE, "initial height <= 0");
      s += v;
    }
    h->hbar[i] = s / (double)nn;
  }
  set_scales(h);
  mlf_status chk = check_stability(h);
  if (chk != MLF_OK) return chk;
  const int rows = rows_per_chunk(h, 3);
  if (rows < 1) return fail(h, MLF_EUNSUPPORTED, "grid rows too wide for the staging area");
  chk = zero_buffers(h);
  if (chk != MLF_OK) return chk;
  double* st = reinterpret_cast<double*>(stage_ptr(h));
  for (int ya = 0; ya < p.ny; ya += rows) {
    const int yb = std::min(p.ny, ya + rows);
    const long long cnt = (long long)(yb - ya) * p.nx, lstride = cnt;
    double* sh = st;
    double* sx = ux ? st + cnt * p.n_layers : nullptr;
    double* sy = uy ? st + 2 * cnt * p.n_layers : nullptr;
    for (int i = 0; i < p.n_layers; ++i) {
      HIPCHK(hipMemcpyAsync(sh + i * cnt, hgt + i * nn + (long long)ya * p.nx, cnt * sizeof(double),
                            hipMemcpyHostToDevice, h->stream));
      if (sx)
        HIPCHK(hipMemcpyAsync(sx + i * cnt, ux + i * nn + (long long)ya * p.nx, cnt * sizeof(double),
                              hipMemcpyHostToDevice, h->stream));
      if (sy)
        HIPCHK(hipMemcpyAsync(sy + i * cnt, uy + i * nn + (long long)ya * p.nx, cnt * sizeof(double),
                              hipMemcpyHostToDevice, h->stream));
    }
    mlf_status s = launch_init(h, sh, sx, sy, lstride, ya, ya, yb);
    if (s != MLF_OK) return s;
    HIPCHK(hipStreamSynchronize(h->stream));  // staging is reused
  }
  return finish_init(h);
}

mlf_status mlf_init_device(mlf_handle* h, const double* hgt, const double* ux, const double* uy) {
  if (!h || !hgt) return MLF_EINVAL;
  drop_single_graph(h);
  const mlf_params& p = h->p;
  const long long nn = (long long)p.nx * p.ny;
  h->initialised = false;
  hipLaunchKernelGGL(field_partials, dim3(kRedBlocks), dim3(256), 0, h->stream, hgt, part_ptr(h), nn, p.n_layers);
  HIPCHK(hipGetLastError());
  hipLaunchKernelGGL(finish_partials, dim3(1), dim3(256), 0, h->stream, part_ptr(h), redout_ptr(h), kRedBlocks,
                     p.n_layers);
  HIPCHK(hipGetLastError());
  double sums[kMaxLayers];
  HIPCHK(hipMemcpyAsync(sums, redout_ptr(h), p.n_layers * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  for (int i = 0; i < p.n_layers; ++i) {
    h->hbar[i] = sums[i] / (double)nn;
    if (!std::isfinite(h->hbar[i])) return fail(h, MLF_ENONFINITE, "initial field is not finite");
    if (!(h->hbar[i] > 0.0)) return fail(h, MLF_ENONPOSITIVE, "initial height <= 0");
  }
  set_scales(h);
  mlf_status s = check_stability(h);
  if (s != MLF_OK) return s;
  s = zero_buffers(h);
  if (s != MLF_OK) return s;
  s = launch_init(h, hgt, ux, uy, nn, 0, 0, p.ny);
  if (s != MLF_OK) return s;
  s = finish_init(h);
  if (s != MLF_OK) return s;
  // per-node validity of device inputs is checked by the first step's guard
  return MLF_OK;
}

mlf_status mlf_step(mlf_handle* h, int64_t nsteps) {
  if (!h || nsteps < 0) return MLF_EINVAL;
  if (!h->initialised) return fail(h, MLF_EINVAL, "mlf_step before mlf_init");
  const int every = h->p.check_every;
  // D1Q3 films, and D2Q9 films one row high without a captured graph, run
  // many steps per launch with the film held in LDS
  const bool row = !h->graph && row_resident(h->p);
  if (h->p.lattice == MLF_D1Q3 || row) {
    int64_t left = nsteps, since = 0;
    while (left > 0) {
      const int64_t per_launch = row ? (row_tiled(h->p) ? mlf::kRowTileSteps : kD1MaxStepsPerLaunch)
                                     : (d1_tiled(h->p) ? mlf::kD1TileSteps : kD1MaxStepsPerLaunch);
      int64_t chunk = std::min<int64_t>(left, per_launch);
      if (every > 0) chunk = std::min<int64_t>(chunk, every - since);
      HIPCHK(row ? row_advance(h, (int)chunk) : d1_advance(h, (int)chunk));
      left -= chunk;
      since += chunk;
      h->steps += chunk;
      if (every > 0 && since >= every && left > 0) {
        since = 0;
        mlf_status s = check_guard(h);
        if (s != MLF_OK) return s;
      }
    }
    return every >= 0 ? check_guard(h) : MLF_OK;
  }
  int64_t left = nsteps, since = 0;
  while (left > 0) {
    int64_t adv = 1;
    if (h->graph && h->cur == h->graph_parity && left >= h->graph_steps) {
      HIPCHK(hipGraphLaunch(h->graph, h->stream));
      adv = h->graph_steps;
    } else {
      HIPCHK(launch_step(h, h->pop[h->cur], h->pop[h->cur ^ 1]));
      h->cur ^= 1;
    }
    left -= adv;
    since += adv;
    h->steps += adv;
    if (every > 0 && since >= every && left > 0) {
      since = 0;
      mlf_status s = check_guard(h);
      if (s != MLF_OK) return s;
    }
  }
  if (every >= 0) return check_guard(h);
  return MLF_OK;
}

mlf_status mlf_capture(mlf_handle* h, int32_t steps) {
  if (!h) return MLF_EINVAL;
  drop_single_graph(h);
  if (steps == 0) return MLF_OK;
  if (steps < 0 || steps % 2 != 0) return fail(h, MLF_EINVAL, "graph steps must be even and >= 0");
  if (!h->initialised) return fail(h, MLF_EINVAL, "mlf_capture before mlf_init");
  if (h->p.lattice == MLF_D1Q3)
    return fail(h, MLF_EUNSUPPORTED, "D1Q3 films run many steps per launch; no graph needed");
  if (h->sr)
    return fail(h, MLF_EUNSUPPORTED, "stochastic rounding draws on the step count, which a graph would freeze");
  if (!h->stream) return fail(h, MLF_EUNSUPPORTED, "graph capture needs a non-default stream");
  HIPCHK(hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal));
  hipError_t le = hipSuccess;
  for (int t = 0; t < steps && le == hipSuccess; ++t) {
    const int c = (h->cur + t) & 1;
    le = launch_step(h, h->pop[c], h->pop[c ^ 1]);
  }
  hipGraph_t g = nullptr;
  hipError_t ee = hipStreamEndCapture(h->stream, &g);
  if (le != hipSuccess || ee != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return hip_check(h, le != hipSuccess ? le : ee, "graph capture");
  }
  hipGraphExec_t ex = nullptr;
  hipError_t ie = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (ie != hipSuccess) return hip_check(h, ie, "hipGraphInstantiate");
  h->graph = ex;
  h->graph_steps = steps;
  h->graph_parity = h->cur;
  return MLF_OK;
}

mlf_status mlf_read_device(mlf_handle* h, double* hgt, double* ux, double* uy) {
  if (!h) return MLF_EINVAL;
  if (!h->initialised) return fail(h, MLF_EINVAL, "read before init");
  if (!hgt && !ux && !uy) return MLF_OK;
  const long long nn = (long long)h->p.nx * h->p.ny;
  return launch_read(h, hgt, ux, uy, nn, 0, 0, h->p.ny);
}

mlf_status mlf_read(mlf_handle* h, double* hgt, double* ux, double* uy) {
  if (!h) return MLF_EINVAL;
  if (!h->initialised) return fail(h, MLF_EINVAL, "read before init");
  const mlf_params& p = h->p;
  const long long nn = (long long)p.nx * p.ny;
  const int rows = rows_per_chunk(h, 3);
  if (rows < 1) return fail(h, MLF_EUNSUPPORTED, "grid rows too wide for the staging area");
  double* st = reinterpret_cast<double*>(stage_ptr(h));
  for (int ya = 0; ya < p.ny; ya += rows) {
    const int yb = std::min(p.ny, ya + rows);
    const long long cnt = (long long)(yb - ya) * p.nx;
    double* sh = hgt ? st : nullptr;
    double* sx = ux ? st + cnt * p.n_layers : nullptr;
    double* sy = uy ? st + 2 * cnt * p.n_layers : nullptr;
    mlf_status s = launch_read(h, sh, sx, sy, cnt, ya, ya, yb);
    if (s != MLF_OK) return s;
    for (int i = 0; i < p.n_layers; ++i) {
      if (hgt)
        HIPCHK(hipMemcpyAsync(hgt + i * nn + (long long)ya * p.nx, sh + i * cnt, cnt * sizeof(double),
                              hipMemcpyDeviceToHost, h->stream));
      if (ux)
        HIPCHK(hipMemcpyAsync(ux + i * nn + (long long)ya * p.nx, sx + i * cnt, cnt * sizeof(double),
                              hipMemcpyDeviceToHost, h->stream));
      if (uy)
        HIPCHK(hipMemcpyAsync(uy + i * nn + (long long)ya * p.nx, sy + i * cnt, cnt * sizeof(double),
                              hipMemcpyDeviceToHost, h->stream));
    }
    HIPCHK(hipStreamSynchronize(h->stream));
  }
  return MLF_OK;
}

mlf_status mlf_layer_mass(mlf_handle* h, double* mass) {
  if (!h || !mass) return MLF_EINVAL;
  if (!h->initialised) return fail(h, MLF_EINVAL, "mass before init");
  const mlf_params& p = h->p;
  const Layers L = layers_of(h);
  by_storage(h, [&](auto* rt, auto* st) {
    using R = std::remove_pointer_t<decltype(rt)>;
    using S = std::remove_pointer_t<decltype(st)>;
    const PopView<R, S> f{static_cast<unsigned char*>(h->pop[h->cur]), (long long)h->plane, p.n_layers,
                          nq_of(&p)};
    hipLaunchKernelGGL((mass_partials<R, S>), dim3(kRedBlocks), dim3(256), 0, h->stream, f, part_ptr(h), p.nx, p.ny,
                       h->pitch, p.n_layers, L);
  });
  HIPCHK(hipGetLastError());
  hipLaunchKernelGGL(finish_partials, dim3(1), dim3(256), 0, h->stream, part_ptr(h), redout_ptr(h), kRedBlocks,
                     p.n_layers);
  HIPCHK(hipGetLastError());
  double dev[kMaxLayers];
  HIPCHK(hipMemcpyAsync(dev, redout_ptr(h), p.n_layers * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  const double nn = (double)p.nx * (double)p.ny;
  for (int i = 0; i < p.n_layers; ++i) mass[i] = nn * h->hbar[i] + dev[i];
  return MLF_OK;
}

mlf_status mlf_layer_mass_static(mlf_handle* h, double* mass_dev) {
  if (!h || !mass_dev) return MLF_EINVAL;
  if (!h->initialised) return fail(h, MLF_EINVAL, "mass before init");
  const mlf_params& p = h->p;
  void* sp = nullptr;
  HIPCHK(static_scratch(&sp));
  double* part = static_cast<double*>(sp);
  const Layers L = layers_of(h);
  by_storage(h, [&](auto* rt, auto* st) {
    using R = std::remove_pointer_t<decltype(rt)>;
    using S = std::remove_pointer_t<decltype(st)>;
    const PopView<R, S> f{static_cast<unsigned char*>(h->pop[h->cur]), (long long)h->plane, p.n_layers,
                          nq_of(&p)};
    hipLaunchKernelGGL((mass_partials<R, S>), dim3(kRedBlocks), dim3(256), 0, h->stream, f, part, p.nx, p.ny,
                       h->pitch, p.n_layers, L);
  });
  HIPCHK(hipGetLastError());
  MassBase base{};
  const double nn = (double)p.nx * (double)p.ny;
  for (int i = 0; i < p.n_layers; ++i) base.v[i] = nn * h->hbar[i];
  hipLaunchKernelGGL(finish_mass, dim3(1), dim3(256), 0, h->stream, part, mass_dev, kRedBlocks, p.n_layers, base);
  HIPCHK(hipGetLastError());
  return MLF_OK;
}

mlf_status mlf_layer_min(mlf_handle* h, double* hmin) {
  if (!h || !hmin) return MLF_EINVAL;
  if (!h->initialised) return fail(h, MLF_EINVAL, "minimum before init");
  const mlf_params& p = h->p;
  const Layers L = layers_of(h);
  by_storage(h, [&](auto* rt, auto* st) {
    using R = std::remove_pointer_t<decltype(rt)>;
    using S = std::remove_pointer_t<decltype(st)>;
    const PopView<R, S> f{static_cast<unsigned char*>(h->pop[h->cur]), (long long)h->plane, p.n_layers,
                          nq_of(&p)};
    hipLaunchKernelGGL((min_partials<R, S>), dim3(kRedBlocks), dim3(256), 0, h->stream, f, part_ptr(h), p.nx, p.ny,
                       h->pitch, p.n_layers, L);
  });
  HIPCHK(hipGetLastError());
  hipLaunchKernelGGL(finish_min, dim3(1), dim3(64), 0, h->stream, part_ptr(h), redout_ptr(h), 1, kRedBlocks);
  HIPCHK(hipGetLastError());
  double dev[kMaxLayers];
  HIPCHK(hipMemcpyAsync(dev, redout_ptr(h), sizeof(dev), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  for (int i = 0; i < p.n_layers; ++i) hmin[i] = dev[i];
  return MLF_OK;
}

mlf_status mlf_step_until(mlf_handle* h, int64_t max_steps, int32_t check_every, const double* threshold,
                          int64_t* steps_taken, int32_t* layer) {
  if (!h || !threshold || !steps_taken || !layer || max_steps < 0 || check_every < 1) return MLF_EINVAL;
  if (!h->initialised) return fail(h, MLF_EINVAL, "mlf_step_until before mlf_init");
  *steps_taken = 0;
  *layer = -1;
  double hmin[kMaxLayers];
  while (*steps_taken < max_steps) {
    const int64_t adv = std::min<int64_t>(check_every, max_steps - *steps_taken);
    mlf_status st = mlf_step(h, adv);
    *steps_taken += adv;
    if (st != MLF_OK) return st;
    if ((st = mlf_layer_min(h, hmin)) != MLF_OK) return st;
    for (int i = 0; i < h->p.n_layers; ++i)
      if (hmin[i] <= threshold[i]) {
        *layer = i;
        return MLF_OK;
      }
  }
  return MLF_OK;
}

mlf_status mlf_read_populations(mlf_handle* h, double* f) {
  if (!h || !f) return MLF_EINVAL;
  if (!h->initialised) return fail(h, MLF_EINVAL, "read before init");
  const mlf_params& p = h->p;
  std::vector<unsigned char> raw(h->pop_bytes);
  HIPCHK(hipMemcpyAsync(raw.data(), h->pop[h->cur], h->pop_bytes, hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  const int nq = nq_of(&p);
  for (int i = 0; i < p.n_layers; ++i)
    for (int k = 0; k < nq; ++k)
      for (int y = 0; y < p.ny; ++y)
        for (int x = 0; x < p.nx; ++x) {
          const Fmt fm = k == 0 ? rest_fmt(p.precision) : move_fmt(p.precision);
          const size_t e = (size_t)y * h->pitch + mlf::wrap(x - cx_of(nq, k), p.nx);
          const size_t b = plane_offset(p.precision, p.n_layers, h->plane, k) +
                           (e * p.n_layers + i) * fmt_size(fm);
          double v = host_load(fm, raw.data() + b) / (fmt_scaled(fm) ? h->scale[i] : 1.0);
          if (k == 0) v += h->hbar[i];
          f[(((size_t)i * nq + k) * p.ny + y) * p.nx + x] = v;
        }
  return MLF_OK;
}

mlf_status mlf_write_populations(mlf_handle* h, const double* f) {
  if (!h || !f) return MLF_EINVAL;
  if (!h->initialised) return fail(h, MLF_EINVAL, "write before init");
  const mlf_params& p = h->p;
  std::vector<unsigned char> raw(h->pop_bytes, 0);
  const int nq = nq_of(&p);
  for (int i = 0; i < p.n_layers; ++i)
    for (int k = 0; k < nq; ++k)
      for (int y = 0; y < p.ny; ++y)
        for (int x = 0; x < p.nx; ++x) {
          const Fmt fm = k == 0 ? rest_fmt(p.precision) : move_fmt(p.precision);
          const size_t e = (size_t)y * h->pitch + mlf::wrap(x - cx_of(nq, k), p.nx);
          const size_t b = plane_offset(p.precision, p.n_layers, h->plane, k) +
                           (e * p.n_layers + i) * fmt_size(fm);
          double v = f[(((size_t)i * nq + k) * p.ny + y) * p.nx + x];
          if (k == 0) v -= h->hbar[i];
          host_store(fm, raw.data() + b, v * (fmt_scaled(fm) ? h->scale[i] : 1.0));
        }
  HIPCHK(hipMemcpyAsync(h->pop[h->cur], raw.data(), h->pop_bytes, hipMemcpyHostToDevice, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  return MLF_OK;
}

mlf_status mlf_save(mlf_handle* h, void* blob, size_t* bytes) {
  if (!h || !bytes) return MLF_EINVAL;
  if (!h->initialised) return fail(h, MLF_EINVAL, "save before init");
  const size_t need = sizeof(BlobHeader) + h->pop_bytes;
  if (!blob) {
    *bytes = need;
    return MLF_OK;
  }
  if (*bytes < need) return fail(h, MLF_EINVAL, "checkpoint buffer too small");
  BlobHeader hd;
  std::memset(&hd, 0, sizeof hd);
  std::memcpy(hd.magic, "MLFILM01", 8);
  hd.version = 1;
  hd.precision = h->p.precision;
  hd.n_layers = h->p.n_layers;
  hd.nx = h->p.nx;
  hd.ny = h->p.ny;
  hd.pitch = h->pitch;
  hd.steps = h->steps;
  for (int i = 0; i < kMaxLayers; ++i) hd.hbar[i] = h->hbar[i];
  hd.digest = params_digest(&h->p);
  hd.payload = h->pop_bytes;
  std::memcpy(blob, &hd, sizeof hd);
  HIPCHK(hipMemcpyAsync(static_cast<unsigned char*>(blob) + sizeof hd, h->pop[h->cur], h->pop_bytes,
                        hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  *bytes = need;
  return MLF_OK;
}

mlf_status mlf_load(mlf_handle* h, const void* blob, size_t bytes) {
  if (!h || !blob) return MLF_EINVAL;
  drop_single_graph(h);
  if (bytes < sizeof(BlobHeader)) return fail(h, MLF_EINVAL, "checkpoint too small");
  BlobHeader hd;
  std::memcpy(&hd, blob, sizeof hd);
  if (std::memcmp(hd.magic, "MLFILM01", 8) != 0 || hd.version != 1) return fail(h, MLF_EINVAL, "not a checkpoint");
  if (hd.digest != params_digest(&h->p) || hd.pitch != h->pitch || hd.payload != h->pop_bytes ||
      bytes < sizeof hd + hd.payload)
    return fail(h, MLF_EINVAL, "checkpoint does not match these parameters");
  for (int i = 0; i < kMaxLayers; ++i) h->hbar[i] = hd.hbar[i];
  set_scales(h);
  mlf_status z = zero_buffers(h);
  if (z != MLF_OK) return z;
  HIPCHK(hipMemcpyAsync(h->pop[h->cur], static_cast<const unsigned char*>(blob) + sizeof hd, h->pop_bytes,
                        hipMemcpyHostToDevice, h->stream));
  HIPCHK(hipMemsetAsync(flag_ptr(h), 0, sizeof(int), h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  h->steps = hd.steps;
  h->initialised = true;
  return MLF_OK;
}

mlf_status mlf_spreading_from_tensions(int32_t n, const double* g, double* spread) {
  if (n < 1 || n > MLF_MAX_LAYERS || !g || !spread) return MLF_EINVAL;
  const int m = n + 2;
  auto G = [&](int a, int b) { return g[a * m + b]; };
  for (int j = 0; j < MLF_MAX_PAIRS; ++j) spread[j] = 0.0;
  for (int l = 0; l < n; ++l)
    for (int k = 1; k <= n - l; ++k) {
      double s = (k == 1) ? G(l, l + 2) - G(l, l + 1) - G(l + 1, l + 2)
                          : G(l, l + k + 1) + G(l + 1, l + k) - G(l, l + k) - G(l + 1, l + k + 1);
      spread[pair_index(n, l, k)] = s;
    }
  return MLF_OK;
}

mlf_status mlf_friction_matrix(int32_t n, const double* hh, const double* mu, double* K, double* rate) {
  if (n < 1 || n > MLF_MAX_LAYERS || !hh || !mu) return MLF_EINVAL;
  for (int i = 0; i < n; ++i)
    if (!(hh[i] > 0.0) || !(mu[i] > 0.0)) return MLF_EINVAL;
  double k[kMaxLayers * kMaxLayers];
  friction_matrix(n, hh, mu, nullptr, k);
  if (K) std::memcpy(K, k, sizeof(double) * n * n);
  if (rate) *rate = max_rate(n, k);
  return MLF_OK;
}

mlf_status mlf_friction_matrix_slip(int32_t n, const double* hh, const double* mu, const double* slip, double* K,
                                    double* rate) {
  if (n < 1 || n > MLF_MAX_LAYERS || !hh || !mu || !slip) return MLF_EINVAL;
  for (int i = 0; i < n; ++i)
    if (!(hh[i] > 0.0) || !(mu[i] > 0.0) || !(slip[i] >= 0.0) || !std::isfinite(slip[i])) return MLF_EINVAL;
  double k[kMaxLayers * kMaxLayers];
  friction_matrix(n, hh, mu, slip, k);
  if (K) std::memcpy(K, k, sizeof(double) * n * n);
  if (rate) *rate = max_rate(n, k);
  return MLF_OK;
}

}  // extern "C"

// ============================================================ batches ====
// Many independent films advanced together: one launch per step over a
// work list of (film, tile) items, per-film step constants in a device
// table, optionally replayed from a captured HIP graph.  Each film is
// served by an internal single-film handle on its slice of the batch
// buffers, which provides initialisation, read-back and mass.

namespace {

constexpr int kMaxFilms = 4096;
constexpr size_t kBatchFlagOff = (kScratchBytes + 255) / 256 * 256;        // int flags[kMaxFilms]
constexpr size_t kBatchTableOff = kBatchFlagOff + kMaxFilms * sizeof(int);  // BatchFilm<C>[n]
constexpr size_t kBatchTableBytes = 4u << 20;
constexpr size_t kBatchItemOff = kBatchTableOff + kBatchTableBytes;         // int2[n_items]
constexpr size_t kBatchItemBytes = 12u << 20;
constexpr size_t kBatchSumOff = kBatchItemOff + kBatchItemBytes;          // double sums[kMaxFilms][4]
constexpr size_t kBatchMinTabOff = kBatchSumOff + kMaxFilms * kMaxLayers * sizeof(double);  // MinFilm[n]
constexpr size_t kBatchMinPartOff = kBatchMinTabOff + (kMaxFilms * sizeof(MinFilm) + 255) / 256 * 256;
constexpr size_t kBatchScratchBytes =
    kBatchMinPartOff + (size_t)kMaxFilms * kMinBlocksPerFilm * kMaxLayers * sizeof(double);

size_t align256(size_t v) { return (v + 255) / 256 * 256; }

}  // namespace

struct mlf_batch {
  int n;
  mlf_params p0;                     // precision, tau and exponents shared by all films
  std::vector<mlf_handle*> film;
  std::vector<size_t> offset;        // byte offset of each film in a population buffer
  std::vector<int> order;            // films, most layer-node updates first
  std::vector<bool> ready;
  unsigned char* pop[2];
  int cur;
  unsigned char* scratch;
  hipStream_t stream;
  int block_w, seg_h, persistent;
  int ahead;  // rows of populations in flight in the batch kernel (1 or 2)
  int max_nl;
  int n_items;
  bool table_dirty;
  hipGraphExec_t graph;
  int graph_steps, graph_parity;
  int64_t steps;
  int failed;
  std::string err;
};

namespace {

mlf_status bfail(mlf_batch* b, mlf_status st, const std::string& m) {
  if (b) b->err = m;
  return st;
}

mlf_status bhip(mlf_batch* b, hipError_t e, const char* what) {
  if (e == hipSuccess) return MLF_OK;
  return bfail(b, MLF_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define BHIPCHK(call)                                             \
  do {                                                            \
    mlf_status _s = bhip(b, (call), #call);                       \
    if (_s != MLF_OK) return _s;                                  \
  } while (0)

mlf_status validate_batch(const mlf_params* films, int n, std::string* why) {
  if (!films || n < 1 || n > kMaxFilms) {
    if (why) *why = "need 1..4096 films";
    return MLF_EINVAL;
  }
  for (int f = 0; f < n; ++f) {
    mlf_status st = validate(&films[f], why);
    if (st != MLF_OK) return st;
    if (films[f].lattice != films[0].lattice) {
      if (why) *why = "films of a batch share the lattice";
      return MLF_EUNSUPPORTED;
    }
    if (films[f].lattice == MLF_D1Q3 && !d1_resident(films[f])) {
      if (why) *why = "batched D1Q3 films must fit one workgroup's LDS (nx <= 1024, 5 N nx values <= 64 KiB)";
      return MLF_EUNSUPPORTED;
    }
    if (films[f].precision != films[0].precision || films[f].tau != films[0].tau ||
        films[f].exp_a != films[0].exp_a || films[f].exp_b != films[0].exp_b) {
      if (why) *why = "films of a batch share precision, tau and exponents";
      return MLF_EUNSUPPORTED;
    }
  }
  return MLF_OK;
}

size_t film_bytes(const mlf_params* p) {
  return align256(buffer_bytes(p->precision, p->n_layers, (size_t)pitch_of(p) * p->ny, nq_of(p)));
}

bool batch_double(const mlf_batch* b) { return b->p0.precision == MLF_F64; }

size_t batch_table_entry(const mlf_batch* b) {
  return batch_double(b) ? sizeof(mlf::BatchFilm<double>) : sizeof(mlf::BatchFilm<float>);
}

int* batch_flags(mlf_batch* b) { return reinterpret_cast<int*>(b->scratch + kBatchFlagOff); }

// Tiles of film f under the batch's launch shape.
long long film_tiles(const mlf_batch* b, int f, int bw, int sh) {
  const mlf_params& p = b->film[f]->p;
  const int s = std::min(sh, p.ny);
  return (long long)mlf::strip_count(p.nx, bw) * ((p.ny + s - 1) / s);
}

long long batch_items(const mlf_batch* b, int bw, int sh) {
  long long t = 0;
  for (int f = 0; f < b->n; ++f) t += film_tiles(b, f, bw, sh);
  return t;
}

// Device table and work list for the current launch shape (synchronous).
template <typename C>
mlf_status upload_table_t(mlf_batch* b) {
  std::vector<mlf::BatchFilm<C>> tab(b->n);
  std::vector<int2> items;
  items.reserve((size_t)b->n_items);
  for (int f = 0; f < b->n; ++f) {
    mlf_handle* h = b->film[f];
    h->block_w = b->block_w;
    h->seg_h = std::min(b->seg_h, h->p.ny);
    std::memset(&tab[f], 0, sizeof(tab[f]));
    tab[f].kc = make_consts<C>(h);
    tab[f].kc.flag = batch_flags(b) + f;
    tab[f].offset = (long long)b->offset[f];
    tab[f].nl = h->p.n_layers;
  }
  for (int f : b->order) {
    const int nt = tab[f].kc.nstrip * tab[f].kc.nseg;
    for (int t = 0; t < nt; ++t) items.push_back(make_int2(f, t));
  }
  BHIPCHK(hipMemcpyAsync(b->scratch + kBatchTableOff, tab.data(), tab.size() * sizeof(tab[0]),
                         hipMemcpyHostToDevice, b->stream));
  BHIPCHK(hipMemcpyAsync(b->scratch + kBatchItemOff, items.data(), items.size() * sizeof(int2),
                         hipMemcpyHostToDevice, b->stream));
  BHIPCHK(hipStreamSynchronize(b->stream));
  b->n_items = (int)items.size();
  b->table_dirty = false;
  return MLF_OK;
}

mlf_status upload_table(mlf_batch* b) {
  b->n_items = (int)batch_items(b, b->block_w, b->seg_h);
  return batch_double(b) ? upload_table_t<double>(b) : upload_table_t<float>(b);
}

template <typename R, typename S, typename C, bool T1, int EA, int EB, int AH>
hipError_t launch_batch_ah(const mlf_batch* b, int flip, int* occ) {
  auto kern = mlf::batch_kernel<R, S, C, T1, EA, EB, AH>;
  const size_t lds = (size_t)8 * b->max_nl * b->block_w * sizeof(C);
  if (occ) {
    int nb = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kern, b->block_w, lds);
    *occ = nb;
    return e;
  }
  int grid = (b->n_items + mlf::kXcds - 1) / mlf::kXcds * mlf::kXcds;
  if (b->persistent) {
    int nb = 0, dev = 0, ncu = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kern, b->block_w, lds);
    if (e != hipSuccess) return e;
    if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
    if ((e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) return e;
    const int slots = std::max(1, nb) * std::max(1, ncu) / mlf::kXcds * mlf::kXcds;
    grid = std::max(mlf::kXcds, std::min(grid, slots));
  }
  hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3((unsigned)b->block_w), lds, b->stream,
                     reinterpret_cast<const mlf::BatchFilm<C>*>(b->scratch + kBatchTableOff),
                     reinterpret_cast<const int2*>(b->scratch + kBatchItemOff), b->n_items, b->pop[0], b->pop[1],
                     flip, (uint32_t)b->steps);
  return hipGetLastError();
}

template <typename R, typename S, typename C, bool T1, int EA, int EB>
hipError_t launch_batch_t(const mlf_batch* b, int flip, int* occ) {
  if constexpr (T1 && sizeof(C) == 4)
    if (b->ahead == 2) return launch_batch_ah<R, S, C, T1, EA, EB, 2>(b, flip, occ);
  return launch_batch_ah<R, S, C, T1, EA, EB, 1>(b, flip, occ);
}

template <typename R, typename S, typename C>
hipError_t launch_batch_sc(const mlf_batch* b, int flip, int* occ) {
  const bool t1 = b->p0.tau == 1.0;
  const bool e93 = b->p0.exp_a == 9 && b->p0.exp_b == 3;
  if (t1 && e93) return launch_batch_t<R, S, C, true, 9, 3>(b, flip, occ);
  if (t1) return launch_batch_t<R, S, C, true, 0, 0>(b, flip, occ);
  if (e93) return launch_batch_t<R, S, C, false, 9, 3>(b, flip, occ);
  return launch_batch_t<R, S, C, false, 0, 0>(b, flip, occ);
}

// One step of every film from buffer `flip` into the other one.
// D1Q3 batch: one workgroup per film, `steps` steps held in LDS.
template <typename C, bool T1, int EA, int EB>
hipError_t d1_batch_launch_t(const mlf_batch* b, int steps) {
  size_t lds = 0;
  int threads = 64;
  for (const mlf_handle* h : b->film) {
    lds = std::max(lds, mlf::d1_resident_lds<C>(h->p.nx, h->p.n_layers));
    threads = std::max(threads, d1_threads(h->p.nx));
  }
  hipLaunchKernelGGL((mlf::d1q3_resident_batch<C, T1, EA, EB>), dim3((unsigned)b->n), dim3((unsigned)threads), lds,
                     b->stream, reinterpret_cast<const mlf::BatchFilm<C>*>(b->scratch + kBatchTableOff), b->pop[0],
                     b->pop[1], b->cur, steps);
  return hipGetLastError();
}

template <typename C>
hipError_t d1_batch_launch_c(const mlf_batch* b, int steps) {
  const bool t1 = b->p0.tau == 1.0;
  const bool e93 = b->p0.exp_a == 9 && b->p0.exp_b == 3;
  if (t1 && e93) return d1_batch_launch_t<C, true, 9, 3>(b, steps);
  if (t1) return d1_batch_launch_t<C, true, 0, 0>(b, steps);
  if (e93) return d1_batch_launch_t<C, false, 9, 3>(b, steps);
  return d1_batch_launch_t<C, false, 0, 0>(b, steps);
}

hipError_t d1_batch_launch(const mlf_batch* b, int steps) {
  return b->p0.precision == MLF_F64 ? d1_batch_launch_c<double>(b, steps) : d1_batch_launch_c<float>(b, steps);
}

hipError_t launch_batch(const mlf_batch* b, int flip) {
  hipError_t e = hipSuccess;
  by_storage(b->film[0], [&](auto* rt, auto* st) {
    using R = std::remove_pointer_t<decltype(rt)>;
    using S = std::remove_pointer_t<decltype(st)>;
    using C = std::conditional_t<std::is_same_v<S, double>, double, float>;
    e = launch_batch_sc<R, S, C>(b, flip, nullptr);
  });
  return e;
}

void drop_graph(mlf_batch* b) {
  if (b->graph) (void)hipGraphExecDestroy(b->graph);
  b->graph = nullptr;
  b->graph_steps = 0;
}

mlf_status batch_ready(mlf_batch* b) {
  for (int f = 0; f < b->n; ++f)
    if (!b->ready[f]) return bfail(b, MLF_EINVAL, "film " + std::to_string(f) + " is not initialised");
  if (b->table_dirty) return upload_table(b);
  return MLF_OK;
}

mlf_status batch_guard(mlf_batch* b) {
  std::vector<int> flags(b->n);
  BHIPCHK(hipMemcpyAsync(flags.data(), batch_flags(b), b->n * sizeof(int), hipMemcpyDeviceToHost, b->stream));
  BHIPCHK(hipStreamSynchronize(b->stream));
  for (int f = 0; f < b->n; ++f)
    if (flags[f] != 0) {
      b->failed = f;
      const std::string where = "film " + std::to_string(f) + " at or before step " + std::to_string(b->steps);
      if (flags[f] == 1) return bfail(b, MLF_ENONPOSITIVE, "a layer height became <= 0 in " + where);
      return bfail(b, MLF_ENONFINITE, "a layer height or flux became non-finite in " + where);
    }
  return MLF_OK;
}

mlf_status film_index(mlf_batch* b, int f) {
  if (f < 0 || f >= b->n) return bfail(b, MLF_EINVAL, "film index out of range");
  return MLF_OK;
}

}  // namespace

extern "C" {

mlf_status mlf_batch_query_sizes(const mlf_params* films, int32_t n, size_t* pop_bytes, size_t* scratch_bytes) {
  mlf_status st = validate_batch(films, n, nullptr);
  if (st != MLF_OK) return st;
  size_t total = 0;
  for (int f = 0; f < n; ++f) total += film_bytes(&films[f]);
  if (pop_bytes) *pop_bytes = total;
  if (scratch_bytes) *scratch_bytes = kBatchScratchBytes;
  return MLF_OK;
}

mlf_status mlf_batch_create(const mlf_params* films, int32_t n, void* pop_a, void* pop_b, void* scratch,
                            void* stream, mlf_batch** out) {
  if (!out) return MLF_EINVAL;
  *out = nullptr;
  std::string why;
  mlf_status st = validate_batch(films, n, &why);
  if (st != MLF_OK) return st;
  if (!pop_a || !pop_b || !scratch || pop_a == pop_b) return MLF_EINVAL;
  auto aligned = [](void* v) { return (reinterpret_cast<uintptr_t>(v) & 255) == 0; };
  if (!aligned(pop_a) || !aligned(pop_b) || !aligned(scratch)) return MLF_EINVAL;
  mlf_batch* b = new (std::nothrow) mlf_batch();
  if (!b) return MLF_EINVAL;
  b->n = n;
  b->p0 = films[0];
  b->pop[0] = static_cast<unsigned char*>(pop_a);
  b->pop[1] = static_cast<unsigned char*>(pop_b);
  b->cur = 0;
  b->scratch = static_cast<unsigned char*>(scratch);
  b->stream = static_cast<hipStream_t>(stream);
  b->max_nl = 1;
  size_t off = 0;
  for (int f = 0; f < n; ++f) {
    mlf_handle* h = nullptr;
    st = mlf_create(&films[f], b->pop[0] + off, b->pop[1] + off, scratch, stream, &h);
    if (st != MLF_OK) {
      for (mlf_handle* g : b->film) mlf_destroy(g);
      delete b;
      return st;
    }
    b->film.push_back(h);
    b->offset.push_back(off);
    off += film_bytes(&films[f]);
    b->max_nl = std::max(b->max_nl, films[f].n_layers);
  }
  b->ready.assign(n, false);
  b->order.resize(n);
  for (int f = 0; f < n; ++f) b->order[f] = f;
  std::stable_sort(b->order.begin(), b->order.end(), [&](int a, int c) {
    auto lu = [&](int f) { return (long long)films[f].n_layers * films[f].nx * films[f].ny; };
    return lu(a) > lu(c);
  });
  b->block_w = 256;
  b->seg_h = 8;
  b->persistent = 0;
  b->ahead = 1;
  if (batch_items(b, b->block_w, b->seg_h) * (long long)sizeof(int2) > (long long)kBatchItemBytes ||
      (size_t)n * batch_table_entry(b) > kBatchTableBytes) {
    for (mlf_handle* g : b->film) mlf_destroy(g);
    delete b;
    return MLF_EUNSUPPORTED;
  }
  b->table_dirty = true;
  b->graph = nullptr;
  b->graph_steps = 0;
  b->graph_parity = 0;
  b->steps = 0;
  b->failed = -1;
  *out = b;
  return MLF_OK;
}

mlf_status mlf_batch_init(mlf_batch* b, int32_t film, const double* hgt, const double* ux, const double* uy) {
  if (!b) return MLF_EINVAL;
  mlf_status st = film_index(b, film);
  if (st != MLF_OK) return st;
  mlf_handle* h = b->film[film];
  h->cur = b->cur;
  b->ready[film] = false;
  st = mlf_init(h, hgt, ux, uy);
  if (st != MLF_OK) return bfail(b, st, "film " + std::to_string(film) + ": " + h->err);
  BHIPCHK(hipMemsetAsync(batch_flags(b) + film, 0, sizeof(int), b->stream));
  BHIPCHK(hipStreamSynchronize(b->stream));
  b->ready[film] = true;
  b->table_dirty = true;  // reference heights and scales changed
  return MLF_OK;
}

mlf_status mlf_batch_init_device(mlf_batch* b, int32_t film, const double* hgt, const double* ux, const double* uy) {
  if (!b) return MLF_EINVAL;
  mlf_status st = film_index(b, film);
  if (st != MLF_OK) return st;
  mlf_handle* h = b->film[film];
  h->cur = b->cur;
  b->ready[film] = false;
  st = mlf_init_device(h, hgt, ux, uy);
  if (st != MLF_OK) return bfail(b, st, "film " + std::to_string(film) + ": " + h->err);
  BHIPCHK(hipMemsetAsync(batch_flags(b) + film, 0, sizeof(int), b->stream));
  BHIPCHK(hipStreamSynchronize(b->stream));
  b->ready[film] = true;
  b->table_dirty = true;
  return MLF_OK;
}

mlf_status mlf_batch_init_device_all_u(mlf_batch* b, const double* const* hgts, const double* const* uxs,
                                       const double* const* uys) {
  if (!b || !hgts || (!uxs) != (!uys)) return MLF_EINVAL;
  if (uxs)
    for (int f = 0; f < b->n; ++f)
      if (!uxs[f] || !uys[f]) return bfail(b, MLF_EINVAL, "null velocity array");
  double* sums = reinterpret_cast<double*>(b->scratch + kBatchSumOff);
  for (int f = 0; f < b->n; ++f) {
    if (!hgts[f]) return bfail(b, MLF_EINVAL, "null height array");
    mlf_handle* h = b->film[f];
    const long long nn = (long long)h->p.nx * h->p.ny;
    b->ready[f] = false;
    h->initialised = false;
    drop_single_graph(h);
    // per-film sums: the partials area is reused in stream order
    hipLaunchKernelGGL(field_partials, dim3(kRedBlocks), dim3(256), 0, b->stream, hgts[f], part_ptr(h), nn,
                       h->p.n_layers);
    BHIPCHK(hipGetLastError());
    hipLaunchKernelGGL(finish_partials, dim3(1), dim3(256), 0, b->stream, part_ptr(h), sums + (size_t)f * kMaxLayers,
                       kRedBlocks, h->p.n_layers);
    BHIPCHK(hipGetLastError());
  }
  std::vector<double> hs((size_t)b->n * kMaxLayers);
  BHIPCHK(hipMemcpyAsync(hs.data(), sums, hs.size() * sizeof(double), hipMemcpyDeviceToHost, b->stream));
  BHIPCHK(hipStreamSynchronize(b->stream));
  for (int f = 0; f < b->n; ++f) {
    mlf_handle* h = b->film[f];
    const long long nn = (long long)h->p.nx * h->p.ny;
    for (int i = 0; i < h->p.n_layers; ++i) {
      h->hbar[i] = hs[(size_t)f * kMaxLayers + i] / (double)nn;
      if (!std::isfinite(h->hbar[i])) return bfail(b, MLF_ENONFINITE, "film " + std::to_string(f) + ": not finite");
      if (!(h->hbar[i] > 0.0)) return bfail(b, MLF_ENONPOSITIVE, "film " + std::to_string(f) + ": height <= 0");
    }
    set_scales(h);
    mlf_status st = check_stability(h);
    if (st != MLF_OK) return bfail(b, st, "film " + std::to_string(f) + ": " + h->err);
  }
  for (int f = 0; f < b->n; ++f) {
    mlf_handle* h = b->film[f];
    h->cur = b->cur;
    mlf_status st = zero_buffers(h);
    if (st == MLF_OK)
      st = launch_init(h, hgts[f], uxs ? uxs[f] : nullptr, uys ? uys[f] : nullptr, (long long)h->p.nx * h->p.ny, 0,
                       0, h->p.ny);
    if (st != MLF_OK) return bfail(b, st, h->err);
  }
  BHIPCHK(hipMemsetAsync(batch_flags(b), 0, b->n * sizeof(int), b->stream));
  BHIPCHK(hipStreamSynchronize(b->stream));
  for (int f = 0; f < b->n; ++f) {
    b->film[f]->steps = 0;
    b->film[f]->initialised = true;
    b->ready[f] = true;
  }
  b->table_dirty = true;
  return MLF_OK;
}

mlf_status mlf_batch_init_device_all(mlf_batch* b, const double* const* hgts) {
  return mlf_batch_init_device_all_u(b, hgts, nullptr, nullptr);
}

mlf_status mlf_batch_read_device_all(mlf_batch* b, double* const* outs) {
  if (!b || !outs) return MLF_EINVAL;
  for (int f = 0; f < b->n; ++f) {
    if (!b->ready[f]) return bfail(b, MLF_EINVAL, "film " + std::to_string(f) + " is not initialised");
    if (!outs[f]) return bfail(b, MLF_EINVAL, "null output array");
    mlf_handle* h = b->film[f];
    h->cur = b->cur;
    const long long nn = (long long)h->p.nx * h->p.ny;
    mlf_status st = launch_read(h, outs[f], nullptr, nullptr, nn, 0, 0, h->p.ny);
    if (st != MLF_OK) return bfail(b, st, h->err);
  }
  return MLF_OK;
}

mlf_status mlf_batch_step(mlf_batch* b, int64_t nsteps) {
  if (!b || nsteps < 0) return MLF_EINVAL;
  mlf_status st = batch_ready(b);
  if (st != MLF_OK) return st;
  b->failed = -1;
  if (b->p0.lattice == MLF_D1Q3) {
    for (int64_t left = nsteps; left > 0;) {
      const int chunk = (int)std::min<int64_t>(left, kD1MaxStepsPerLaunch);
      BHIPCHK(d1_batch_launch(b, chunk));
      b->cur ^= 1;
      left -= chunk;
      b->steps += chunk;
    }
    return batch_guard(b);
  }
  int64_t left = nsteps;
  while (left > 0) {
    if (b->graph && b->cur == b->graph_parity && left >= b->graph_steps) {
      BHIPCHK(hipGraphLaunch(b->graph, b->stream));
      left -= b->graph_steps;
      b->steps += b->graph_steps;
    } else {
      BHIPCHK(launch_batch(b, b->cur));
      b->cur ^= 1;
      left -= 1;
      b->steps += 1;
    }
  }
  return batch_guard(b);
}

mlf_status mlf_batch_capture(mlf_batch* b, int32_t steps) {
  if (!b) return MLF_EINVAL;
  drop_graph(b);
  if (steps == 0) return MLF_OK;
  if (steps < 0 || steps % 2 != 0) return bfail(b, MLF_EINVAL, "graph steps must be even and >= 0");
  if (b->p0.lattice == MLF_D1Q3)
    return bfail(b, MLF_EUNSUPPORTED, "D1Q3 batches run many steps per launch; no graph needed");
  if (!b->stream) return bfail(b, MLF_EUNSUPPORTED, "graph capture needs a non-default stream");
  if (!b->film.empty() && b->film[0]->sr)
    return bfail(b, MLF_EUNSUPPORTED, "stochastic rounding draws from the step count, which a graph would freeze");
  mlf_status st = batch_ready(b);
  if (st != MLF_OK) return st;
  BHIPCHK(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
  hipError_t le = hipSuccess;
  for (int t = 0; t < steps && le == hipSuccess; ++t) le = launch_batch(b, (b->cur + t) & 1);
  hipGraph_t g = nullptr;
  hipError_t ee = hipStreamEndCapture(b->stream, &g);
  if (le != hipSuccess || ee != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return bhip(b, le != hipSuccess ? le : ee, "graph capture");
  }
  hipGraphExec_t ex = nullptr;
  hipError_t ie = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (ie != hipSuccess) return bhip(b, ie, "hipGraphInstantiate");
  b->graph = ex;
  b->graph_steps = steps;
  b->graph_parity = b->cur;
  return MLF_OK;
}

mlf_status mlf_batch_read(mlf_batch* b, int32_t film, double* hgt, double* ux, double* uy) {
  if (!b) return MLF_EINVAL;
  mlf_status st = film_index(b, film);
  if (st != MLF_OK) return st;
  mlf_handle* h = b->film[film];
  h->cur = b->cur;
  st = mlf_read(h, hgt, ux, uy);
  return st == MLF_OK ? st : bfail(b, st, h->err);
}

mlf_status mlf_batch_read_device(mlf_batch* b, int32_t film, double* hgt, double* ux, double* uy) {
  if (!b) return MLF_EINVAL;
  mlf_status st = film_index(b, film);
  if (st != MLF_OK) return st;
  mlf_handle* h = b->film[film];
  h->cur = b->cur;
  st = mlf_read_device(h, hgt, ux, uy);
  return st == MLF_OK ? st : bfail(b, st, h->err);
}

mlf_status mlf_batch_layer_mass(mlf_batch* b, int32_t film, double* mass) {
  if (!b) return MLF_EINVAL;
  mlf_status st = film_index(b, film);
  if (st != MLF_OK) return st;
  mlf_handle* h = b->film[film];
  h->cur = b->cur;
  st = mlf_layer_mass(h, mass);
  return st == MLF_OK ? st : bfail(b, st, h->err);
}

mlf_status mlf_batch_layer_min(mlf_batch* b, int32_t film, double* hmin) {
  if (!b) return MLF_EINVAL;
  mlf_status st = film_index(b, film);
  if (st != MLF_OK) return st;
  mlf_handle* h = b->film[film];
  h->cur = b->cur;
  st = mlf_layer_min(h, hmin);
  return st == MLF_OK ? st : bfail(b, st, h->err);
}

mlf_status mlf_batch_layer_min_all(mlf_batch* b, double* hmin) {
  if (!b || !hmin) return MLF_EINVAL;
  mlf_status st = batch_ready(b);
  if (st != MLF_OK) return st;
  std::vector<MinFilm> tab(b->n);
  for (int f = 0; f < b->n; ++f) {
    const mlf_handle* h = b->film[f];
    tab[f] = MinFilm{(long long)b->offset[f], (long long)h->plane, h->p.nx,    h->p.ny,
                     h->pitch,                 h->p.n_layers,          nq_of(&h->p), 0, layers_of(h)};
  }
  MinFilm* dtab = reinterpret_cast<MinFilm*>(b->scratch + kBatchMinTabOff);
  double* part = reinterpret_cast<double*>(b->scratch + kBatchMinPartOff);
  double* out = reinterpret_cast<double*>(b->scratch + kBatchSumOff);
  BHIPCHK(hipMemcpyAsync(dtab, tab.data(), tab.size() * sizeof(MinFilm), hipMemcpyHostToDevice, b->stream));
  const dim3 grid(kMinBlocksPerFilm, (unsigned)b->n);
  unsigned char* buf = b->pop[b->cur];
  by_storage(b->film[0], [&](auto* rt, auto* st) {  // all films share the storage format
    using R = std::remove_pointer_t<decltype(rt)>;
    using S = std::remove_pointer_t<decltype(st)>;
    hipLaunchKernelGGL((batch_min_partials<R, S>), grid, dim3(256), 0, b->stream, dtab, buf, part);
  });
  BHIPCHK(hipGetLastError());
  const int nt = b->n * kMaxLayers;
  hipLaunchKernelGGL(finish_min, dim3((nt + 255) / 256), dim3(256), 0, b->stream, part, out, b->n, kMinBlocksPerFilm);
  BHIPCHK(hipGetLastError());
  BHIPCHK(hipMemcpyAsync(hmin, out, (size_t)nt * sizeof(double), hipMemcpyDeviceToHost, b->stream));
  BHIPCHK(hipStreamSynchronize(b->stream));
  return MLF_OK;
}

mlf_status mlf_batch_step_until(mlf_batch* b, int64_t max_steps, int32_t check_every, const double* threshold,
                                int64_t* t_hit, int32_t* layer_hit, int64_t* steps_taken) {
  if (!b || !threshold || !t_hit || !layer_hit || !steps_taken || max_steps < 0 || check_every < 1)
    return MLF_EINVAL;
  mlf_status st = batch_ready(b);
  if (st != MLF_OK) return st;
  for (int f = 0; f < b->n; ++f) {
    t_hit[f] = -1;
    layer_hit[f] = -1;
  }
  *steps_taken = 0;
  std::vector<double> hmin((size_t)b->n * kMaxLayers);
  int open = b->n;
  while (open > 0 && *steps_taken < max_steps) {
    const int64_t adv = std::min<int64_t>(check_every, max_steps - *steps_taken);
    st = mlf_batch_step(b, adv);
    *steps_taken += adv;
    if (st != MLF_OK) return st;
    if ((st = mlf_batch_layer_min_all(b, hmin.data())) != MLF_OK) return st;
    for (int f = 0; f < b->n; ++f) {
      if (t_hit[f] >= 0) continue;
      for (int i = 0; i < b->film[f]->p.n_layers; ++i)
        if (hmin[(size_t)f * kMaxLayers + i] <= threshold[(size_t)f * kMaxLayers + i]) {
          t_hit[f] = b->steps;
          layer_hit[f] = i;
          --open;
          break;
        }
    }
  }
  return MLF_OK;
}

mlf_status mlf_batch_set_launch(mlf_batch* b, int32_t block_w, int32_t seg_h, int32_t persistent) {
  if (!b) return MLF_EINVAL;
  const int bw = block_w == 0 ? 256 : block_w, sh = seg_h == 0 ? 8 : seg_h;
  if (bw != 64 && bw != 128 && bw != 192 && bw != 256)
    return bfail(b, MLF_EINVAL, "block_w must be 64, 128, 192 or 256");
  if (sh < 1) return bfail(b, MLF_EINVAL, "seg_h must be >= 1");
  if (batch_items(b, bw, sh) * (long long)sizeof(int2) > (long long)kBatchItemBytes)
    return bfail(b, MLF_EINVAL, "launch shape gives too many work items");
  b->block_w = bw;
  b->seg_h = sh;
  b->persistent = persistent != 0;
  b->table_dirty = true;
  drop_graph(b);
  return MLF_OK;
}

mlf_status mlf_batch_set_prefetch(mlf_batch* b, int32_t rows) {
  if (!b) return MLF_EINVAL;
  if (rows < 0 || rows > 2) return bfail(b, MLF_EINVAL, "prefetch rows must be 0, 1 or 2");
  if (rows == 2 && !prefetch_ok(b->p0))
    return bfail(b, MLF_EINVAL, "two rows ahead needs D2Q9 films with tau = 1 and non-FP64 storage");
  b->ahead = rows == 0 ? 1 : rows;
  drop_graph(b);
  return MLF_OK;
}

mlf_status mlf_batch_get_prefetch(const mlf_batch* b, int32_t* rows) {
  if (!b || !rows) return MLF_EINVAL;
  *rows = b->ahead;
  return MLF_OK;
}

mlf_status mlf_batch_set_rounding(mlf_batch* b, int32_t mode) {
  if (!b) return MLF_EINVAL;
  if (mode != MLF_ROUND_NEAREST && mode != MLF_ROUND_STOCHASTIC_REST)
    return bfail(b, MLF_EINVAL, "unknown rounding mode");
  if (mode == MLF_ROUND_STOCHASTIC_REST &&
      !(b->p0.lattice == MLF_D2Q9 && (b->p0.precision == MLF_F16 || b->p0.precision == MLF_BF16)))
    return bfail(b, MLF_EINVAL, "stochastic rounding needs D2Q9 films with MLF_F16 or MLF_BF16 storage");
  drop_graph(b);
  for (mlf_handle* h : b->film) h->sr = mode == MLF_ROUND_STOCHASTIC_REST;
  b->table_dirty = true;
  return MLF_OK;
}

mlf_status mlf_batch_get_rounding(const mlf_batch* b, int32_t* mode) {
  if (!b || !mode) return MLF_EINVAL;
  *mode = (!b->film.empty() && b->film[0]->sr) ? MLF_ROUND_STOCHASTIC_REST : MLF_ROUND_NEAREST;
  return MLF_OK;
}

mlf_status mlf_batch_get_launch(const mlf_batch* b, int32_t* block_w, int32_t* seg_h, int32_t* persistent) {
  if (!b) return MLF_EINVAL;
  if (block_w) *block_w = b->block_w;
  if (seg_h) *seg_h = b->seg_h;
  if (persistent) *persistent = b->persistent;
  return MLF_OK;
}

mlf_status mlf_batch_autotune(mlf_batch* b, int32_t reps, int32_t* block_w, int32_t* seg_h, int32_t* persistent) {
  if (!b || reps < 1) return MLF_EINVAL;
  mlf_status st = batch_ready(b);
  if (st != MLF_OK) return st;
  if (b->p0.lattice == MLF_D1Q3) {  // fixed shape: one workgroup per film
    if (block_w) *block_w = b->block_w;
    if (seg_h) *seg_h = b->seg_h;
    if (persistent) *persistent = b->persistent;
    return MLF_OK;
  }
  drop_graph(b);
  const int keep_w = b->block_w, keep_h = b->seg_h, keep_p = b->persistent, keep_a = b->ahead;
  struct Cand {
    int w, h, p, a;
  };
  std::vector<Cand> cand;
  for (int a = 1; a <= (prefetch_ok(b->p0) ? 2 : 1); ++a)
    for (int w : {64, 128, 192, 256})
      for (int h : {2, 4, 6, 8, 12, 16, 24, 32, 48, 64, 96})
        for (int pp : {0, 1})
          if (batch_items(b, w, h) * (long long)sizeof(int2) <= (long long)kBatchItemBytes)
            cand.push_back({w, h, pp, a});
  hipEvent_t e0, e1;
  BHIPCHK(hipEventCreate(&e0));
  BHIPCHK(hipEventCreate(&e1));
  float best = 1e30f;
  Cand pick{keep_w, keep_h, keep_p, keep_a};
  for (const Cand& c : cand) {
    b->block_w = c.w;
    b->seg_h = c.h;
    b->persistent = c.p;
    b->ahead = c.a;
    if ((st = upload_table(b)) != MLF_OK) break;
    // current -> other buffer, never swapped: the state is left unchanged
    if ((st = bhip(b, launch_batch(b, b->cur), "autotune launch")) != MLF_OK) break;
    if ((st = bhip(b, hipEventRecord(e0, b->stream), "hipEventRecord")) != MLF_OK) break;
    for (int r = 0; r < reps && st == MLF_OK; ++r) st = bhip(b, launch_batch(b, b->cur), "autotune launch");
    if (st != MLF_OK) break;
    if ((st = bhip(b, hipEventRecord(e1, b->stream), "hipEventRecord")) != MLF_OK) break;
    if ((st = bhip(b, hipEventSynchronize(e1), "hipEventSynchronize")) != MLF_OK) break;
    float ms = 0.f;
    if ((st = bhip(b, hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime")) != MLF_OK) break;
    if (ms < best) {
      best = ms;
      pick = c;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st == MLF_OK) {
    b->block_w = pick.w;
    b->seg_h = pick.h;
    b->persistent = pick.p;
    b->ahead = pick.a;
  } else {
    b->block_w = keep_w;
    b->seg_h = keep_h;
    b->persistent = keep_p;
    b->ahead = keep_a;
  }
  b->table_dirty = true;
  mlf_status up = upload_table(b);
  if (st != MLF_OK) return st;
  if (up != MLF_OK) return up;
  if (block_w) *block_w = pick.w;
  if (seg_h) *seg_h = pick.h;
  if (persistent) *persistent = pick.p;
  return MLF_OK;
}

int64_t mlf_batch_steps_done(const mlf_batch* b) { return b ? b->steps : -1; }

int32_t mlf_batch_failed_film(const mlf_batch* b) { return b ? b->failed : -1; }

const char* mlf_batch_last_error(const mlf_batch* b) { return b ? b->err.c_str() : "null batch"; }

mlf_status mlf_batch_destroy(mlf_batch* b) {
  if (!b) return MLF_EINVAL;
  drop_graph(b);
  for (mlf_handle* h : b->film) mlf_destroy(h);
  delete b;
  return MLF_OK;
}

}  // extern "C"
