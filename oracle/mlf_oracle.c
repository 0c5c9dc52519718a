/*
 * mlf_oracle.c -- plain FP64 CPU oracle of the N-layer thin-film
 * shallow-water lattice Boltzmann step (Richter, Malgaretti & Harting,
 * arXiv 2409.16659).
 *
 * TEST INFRASTRUCTURE ONLY: written to be read against the paper, not to be
 * fast.  It shares no code with the HIP implementation and the product
 * never calls it.
 *
 * One step t -> t+1, in the paper's order (Sec. III plus the pressure and
 * friction of Sec. II):
 *   O1  moments h_i = sum_k f_ki, q_i = h_i U_i = sum_k c_k f_ki
 *   O2  interfaces z_0 = 0, z_i = z_{i-1} + h_i                     (Sec. II)
 *   O3  grad z_i and lap z_i (isotropic stencils; the paper is silent)
 *   O4  wetting potentials phi_lk = S_lk phi_k(z_{l+k} - z_l) and phi'_lk
 *   O5  jumps Delta_i = Lambda_i + Pi_i, pressures p_i = sum_{j>=i} Delta_j
 *   O6  grad p_i
 *   O7  friction 2 mu_i h_i a_i from the boundary-condition system
 *   O8  force F_i = -h_i grad p_i + 2 mu_i h_i a_i                (Eq. force)
 *   O9  BGK collision with the shallow-water equilibrium and forcing
 *   O10 streaming f_ki(x + c_k, t+1) = f*_ki(x), periodic
 * Each stage is a separate loop over all nodes; the per-node arithmetic has a
 * fixed order, so results do not depend on the number of OpenMP threads.
 */
#include "mlf_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Lattices (Sec. III).  D1Q3: c = 0, +1, -1 with w = 2/3, 1/6, 1/6.
 * D2Q9: c_0 = 0, then counter-clockwise starting east; the diagonal vectors
 * are (+-1, +-1) -- they must connect lattice nodes, and their weight 1/36
 * is the standard one for that vector set.  c_s^2 = 1/3 on both. */
static const int D2Q9_CX[9] = {0, 1, 1, 0, -1, -1, -1, 0, 1};
static const int D2Q9_CY[9] = {0, 0, 1, 1, 1, 0, -1, -1, -1};
static const double D2Q9_W[9] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 36.0,
                                 1.0 / 9.0,  1.0 / 36.0, 1.0 / 9.0,
                                 1.0 / 36.0, 1.0 / 9.0,  1.0 / 36.0};
static const int D1Q3_CX[3] = {0, 1, -1};
static const int D1Q3_CY[3] = {0, 0, 0};
static const double D1Q3_W[3] = {2.0 / 3.0, 1.0 / 6.0, 1.0 / 6.0};
static const double CS2 = 1.0 / 3.0;

int orc_lattice(int lattice, int *cx, int *cy, double *w) {
  int q = (lattice == ORC_D1Q3) ? 3 : 9;
  const int *sx = (q == 3) ? D1Q3_CX : D2Q9_CX;
  const int *sy = (q == 3) ? D1Q3_CY : D2Q9_CY;
  const double *sw = (q == 3) ? D1Q3_W : D2Q9_W;
  for (int k = 0; k < q; ++k) {
    if (cx) cx[k] = sx[k];
    if (cy) cy[k] = sy[k];
    if (w) w[k] = sw[k];
  }
  return q;
}

static int g_threads = 0;
void orc_set_threads(int n) { g_threads = n; }
int orc_get_threads(void) {
#ifdef _OPENMP
  return g_threads > 0 ? g_threads : omp_get_max_threads();
#else
  return 1;
#endif
}

static int wrap(int v, int n) { return ((v % n) + n) % n; }

/* ------------------------------------------------------------------------ */
/* Eq. (wetting_potential): phi_k(d) = (a r^b - b r^a) / (a - b), r = k hstar / d,
 * with a > b (the paper's n > m).  Powers are plain repeated products. */
static double ipow(double r, int n) {
  double v = 1.0;
  for (int j = 0; j < n; ++j) v *= r;
  return v;
}

double orc_phi(int k, double d, double hstar, int a, int b) {
  double r = k * hstar / d;
  return (a * ipow(r, b) - b * ipow(r, a)) / (double)(a - b);
}

/* d phi_k / d d = a b (r^a - r^b) / ((a - b) d), since dr/dd = -r/d. */
double orc_dphi(int k, double d, double hstar, int a, int b) {
  double r = k * hstar / d;
  return (double)a * b * (ipow(r, a) - ipow(r, b)) / ((double)(a - b) * d);
}

/* Eq. (spreading_parameters):
 *   S_i1 = g_{i,i+2} - g_{i,i+1} - g_{i+1,i+2}
 *   S_ik = g_{i,i+k+1} + g_{i+1,i+k} - g_{i,i+k} - g_{i+1,i+k+1}   (k >= 2) */
void orc_spreading_from_tensions(int n, const double *g,
                                 double spread[ORC_MAX_LAYERS][ORC_MAX_LAYERS]) {
  int m = n + 2;
#define G(a, b) g[(a) * m + (b)]
  for (int l = 0; l < ORC_MAX_LAYERS; ++l)
    for (int k = 0; k < ORC_MAX_LAYERS; ++k) spread[l][k] = 0.0;
  for (int i = 0; i < n; ++i)
    for (int k = 1; k <= n - i; ++k) {
      if (k == 1)
        spread[i][0] = G(i, i + 2) - G(i, i + 1) - G(i + 1, i + 2);
      else
        spread[i][k - 1] = G(i, i + k + 1) + G(i + 1, i + k) - G(i, i + k) - G(i + 1, i + k + 1);
    }
#undef G
}

/* ------------------------------------------------------------------------ */
/* Gradient and Laplacian of a periodic field.  The paper does not state its
 * discretisation; the oracle uses the isotropic lattice stencils built from
 * the lattice weights:  grad f = (1/c_s^2) sum_k w_k c_k (f(x + c_k) - f(x)),
 * lap f = (2/c_s^2) sum_k w_k (f(x + c_k) - f(x)).  (Since sum_k w_k c_k = 0
 * the gradient is the usual central difference; written with differences a
 * uniform field gives exactly zero.)  Both are exact on quadratic
 * polynomials; on D1Q3 they are the 3-point central differences. */
void orc_grad(int lattice, int nx, int ny, const double *f, double *gx, double *gy) {
  int cx[9], cy[9];
  double w[9];
  int q = orc_lattice(lattice, cx, cy, w);
#pragma omp parallel for num_threads(orc_get_threads())
  for (long n = 0; n < (long)nx * ny; ++n) {
    int y = (int)(n / nx), x = (int)(n % nx);
    double sx = 0.0, sy = 0.0;
    for (int k = 0; k < q; ++k) {
      double v = f[(long)wrap(y + cy[k], ny) * nx + wrap(x + cx[k], nx)] - f[n];
      sx += w[k] * cx[k] * v;
      sy += w[k] * cy[k] * v;
    }
    gx[n] = sx / CS2;
    if (gy) gy[n] = sy / CS2;
  }
}

void orc_lap(int lattice, int nx, int ny, const double *f, double *lap) {
  int cx[9], cy[9];
  double w[9];
  int q = orc_lattice(lattice, cx, cy, w);
#pragma omp parallel for num_threads(orc_get_threads())
  for (long n = 0; n < (long)nx * ny; ++n) {
    int y = (int)(n / nx), x = (int)(n % nx);
    double s = 0.0;
    for (int k = 0; k < q; ++k) {
      double v = f[(long)wrap(y + cy[k], ny) * nx + wrap(x + cx[k], nx)];
      s += w[k] * (v - f[n]);
    }
    lap[n] = 2.0 * s / CS2;
  }
}

/* ------------------------------------------------------------------------ */
/* O2-O5.  Pressures from heights h[N][ny][nx].
 *   Lambda_i = -(gamma_{i,i+1} + sum_{k=1}^{N-i} phi_ik(z_{i+k} - z_i)) lap z_i
 *   Pi_i     = -sum_{k=1}^{N-i} phi'_ik(z_{i+k} - z_i)(1 + (grad z_i)^2/2)
 *              + sum_{l=0}^{i-1} phi'_{l,i-l}(z_i - z_l)(1 + (grad z_l)^2/2)
 *   p_i - p_atm = sum_{j=i}^{N} (Lambda_j + Pi_j)
 * (Eqs. Laplace_pressure and disjoining_pressure; the surface element is
 * 1 + (grad z)^2/2 as in the free-energy appendix; grad z_0 = 0.) */
int orc_pressure(const orc_params *p, const double *h, double *pres, double *jump) {
  const int N = p->n_layers, nx = p->nx, ny = p->ny;
  const long nn = (long)nx * ny;
  double *z = malloc(sizeof(double) * N * nn);
  double *gx = malloc(sizeof(double) * N * nn);
  double *gy = malloc(sizeof(double) * N * nn);
  double *lz = malloc(sizeof(double) * N * nn);
  if (!z || !gx || !gy || !lz) {
    free(z); free(gx); free(gy); free(lz);
    return ORC_EINVAL;
  }
  /* O2: interface heights, z_i stored at index i-1 */
  for (long n = 0; n < nn; ++n) {
    double zz = 0.0;
    for (int i = 0; i < N; ++i) {
      zz += h[i * nn + n];
      z[i * nn + n] = zz;
    }
  }
  /* O3: stencils of every interface z_1..z_N */
  for (int i = 0; i < N; ++i) {
    orc_grad(p->lattice, nx, ny, z + i * nn, gx + i * nn, gy + i * nn);
    orc_lap(p->lattice, nx, ny, z + i * nn, lz + i * nn);
  }
#pragma omp parallel for num_threads(orc_get_threads())
  for (long n = 0; n < nn; ++n) {
    double zf[ORC_MAX_LAYERS + 1], sq[ORC_MAX_LAYERS + 1];
    double ph[ORC_MAX_LAYERS][ORC_MAX_LAYERS + 1], dph[ORC_MAX_LAYERS][ORC_MAX_LAYERS + 1];
    double dl[ORC_MAX_LAYERS + 1];
    zf[0] = 0.0;
    sq[0] = 0.0; /* flat substrate: grad z_0 = 0 */
    for (int i = 1; i <= N; ++i) {
      zf[i] = z[(i - 1) * nn + n];
      double a = gx[(i - 1) * nn + n], b = gy[(i - 1) * nn + n];
      sq[i] = a * a + b * b;
    }
    /* O4: wetting potentials of every pair (l, l+k) */
    for (int l = 0; l < N; ++l)
      for (int k = 1; k <= N - l; ++k) {
        double d = zf[l + k] - zf[l];
        ph[l][k] = p->spread[l][k - 1] * orc_phi(k, d, p->hstar, p->exp_a, p->exp_b);
        dph[l][k] = p->spread[l][k - 1] * orc_dphi(k, d, p->hstar, p->exp_a, p->exp_b);
      }
    /* O5: jumps across interface i = 1..N */
    for (int i = 1; i <= N; ++i) {
      double ten = p->gamma[i - 1];
      for (int k = 1; k <= N - i; ++k) ten += ph[i][k];
      double lam = -ten * lz[(i - 1) * nn + n];
      double pi = 0.0;
      for (int k = 1; k <= N - i; ++k) pi -= dph[i][k] * (1.0 + sq[i] / 2.0);
      for (int l = 0; l <= i - 1; ++l) pi += dph[l][i - l] * (1.0 + sq[l] / 2.0);
      dl[i] = lam + pi;
    }
    double acc = 0.0;
    for (int i = N; i >= 1; --i) {
      acc += dl[i];
      if (pres) pres[(i - 1) * nn + n] = acc;
      if (jump) jump[(i - 1) * nn + n] = dl[i];
    }
  }
  free(z); free(gx); free(gy); free(lz);
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* O7.  Friction force (Sec. II.A.2).  In each layer the horizontal velocity
 * is a Poiseuille profile u_i = a_i s^2 + b_i s + c_i.  The layer-local
 * coordinate s = z - z_{i-1} in [0, h_i] is used instead of z itself: the
 * quadratic coefficient a_i -- the only one the friction needs -- is the
 * same, and the system is far better conditioned.  Unknowns are ordered
 * (a_1, b_1, c_1, ..., a_N, b_N, c_N); the three rows of layer i are
 *   Eq. (no_slip):  u_i(-beta_i) = u_{i-1}(h_{i-1})   (u_0 = 0)
 *   Eq. (flux):     int_0^{h_i} u_i ds = h_i U_i = q_i
 *   Eq. (viscous_boundary): u_i'(h_i) = (mu_{i+1}/mu_i) u_{i+1}'(0),
 *                   with mu_{N+1} = 0 at the gas.
 * Solved by Gaussian elimination with partial pivoting for nrhs right-hand
 * sides at once; friction_i = 2 mu_i h_i a_i (Eq. friction_force). */
static int friction_solve(int n, const double *h, const double *mu, const double *slip,
                          int nrhs, const double *const *q, double *const *fr) {
  enum { MX = 3 * ORC_MAX_LAYERS };
  double D[MX][MX], R[MX][2], X[MX][2];
  int m = 3 * n;
  for (int r = 0; r < m; ++r) {
    for (int c = 0; c < m; ++c) D[r][c] = 0.0;
    R[r][0] = R[r][1] = 0.0;
  }
  for (int i = 0; i < n; ++i) {
    int a = 3 * i, b = 3 * i + 1, c = 3 * i + 2;
    double hi = h[i], be = slip ? slip[i] : 0.0;
    /* no-slip / slip: a_i be^2 - b_i be + c_i - u_{i-1}(h_{i-1}) = 0 */
    D[a][a] = be * be;
    D[a][b] = -be;
    D[a][c] = 1.0;
    if (i > 0) {
      double hp = h[i - 1];
      D[a][3 * (i - 1) + 0] = -hp * hp;
      D[a][3 * (i - 1) + 1] = -hp;
      D[a][3 * (i - 1) + 2] = -1.0;
    }
    /* flux */
    D[b][a] = hi * hi * hi / 3.0;
    D[b][b] = hi * hi / 2.0;
    D[b][c] = hi;
    for (int j = 0; j < nrhs; ++j) R[b][j] = q[j][i];
    /* stress continuity: 2 a_i h_i + b_i - (mu_{i+1}/mu_i) b_{i+1} = 0 */
    D[c][a] = 2.0 * hi;
    D[c][b] = 1.0;
    if (i + 1 < n) D[c][3 * (i + 1) + 1] = -mu[i + 1] / mu[i];
  }
  /* forward elimination with partial pivoting */
  for (int col = 0; col < m; ++col) {
    int piv = col;
    for (int r = col + 1; r < m; ++r)
      if (fabs(D[r][col]) > fabs(D[piv][col])) piv = r;
    if (D[piv][col] == 0.0 || !isfinite(D[piv][col])) return ORC_EINVAL;
    if (piv != col) {
      for (int c = 0; c < m; ++c) {
        double t = D[col][c];
        D[col][c] = D[piv][c];
        D[piv][c] = t;
      }
      for (int j = 0; j < nrhs; ++j) {
        double t = R[col][j];
        R[col][j] = R[piv][j];
        R[piv][j] = t;
      }
    }
    for (int r = col + 1; r < m; ++r) {
      double f = D[r][col] / D[col][col];
      if (f == 0.0) continue;
      for (int c = col; c < m; ++c) D[r][c] -= f * D[col][c];
      for (int j = 0; j < nrhs; ++j) R[r][j] -= f * R[col][j];
    }
  }
  /* back substitution */
  for (int j = 0; j < nrhs; ++j)
    for (int r = m - 1; r >= 0; --r) {
      double s = R[r][j];
      for (int c = r + 1; c < m; ++c) s -= D[r][c] * X[c][j];
      X[r][j] = s / D[r][r];
    }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < nrhs; ++j) fr[j][i] = 2.0 * mu[i] * h[i] * X[3 * i][j];
  return ORC_OK;
}

int orc_friction(int n, const double *h, const double *mu, const double *slip,
                 const double *q, double *fr) {
  if (n < 1 || n > ORC_MAX_LAYERS) return ORC_EINVAL;
  const double *qq[1] = {q};
  double *ff[1] = {fr};
  return friction_solve(n, h, mu, slip, 1, qq, ff);
}

/* ------------------------------------------------------------------------ */
/* O9 pieces.  Eq. (equilibrium_distribution) with c_s^2 = 1/3 (the printed
 * "c_2" is read as c_s):
 *   f^eq_0 = h (1 - w_0 U^2 / (2 c_s^2))
 *   f^eq_k = w_k h (c_k.U / c_s^2 + (c_k.U)^2 / (2 c_s^4) - U^2 / (2 c_s^2))
 * and the forcing term w_k c_k.F / c_s^2 of Eq. (BGK). */
void orc_equilibrium(int lattice, double h, double ux, double uy, double *feq) {
  int cx[9], cy[9];
  double w[9];
  int q = orc_lattice(lattice, cx, cy, w);
  double uu = ux * ux + uy * uy;
  feq[0] = h * (1.0 - w[0] * uu / (2.0 * CS2));
  for (int k = 1; k < q; ++k) {
    double cu = cx[k] * ux + cy[k] * uy;
    feq[k] = w[k] * h * (cu / CS2 + cu * cu / (2.0 * CS2 * CS2) - uu / (2.0 * CS2));
  }
}

void orc_forcing(int lattice, double fx, double fy, double *out) {
  int cx[9], cy[9];
  double w[9];
  int q = orc_lattice(lattice, cx, cy, w);
  for (int k = 0; k < q; ++k) out[k] = w[k] * (cx[k] * fx + cy[k] * fy) / CS2;
}

/* ------------------------------------------------------------------------ */
struct orc_state {
  orc_params p;
  int Q;
  int cx[9], cy[9];
  double w[9];
  long nn;
  double *f, *fn;                       /* [N][Q][ny][nx] */
  double *h, *qx, *qy, *pr, *gpx, *gpy; /* [N][ny][nx] */
  long steps;
};

#define FIDX(s, i, k, n) ((((long)(i) * (s)->Q + (k)) * (s)->nn) + (n))

static int params_ok(const orc_params *p) {
  if (p->n_layers < 1 || p->n_layers > ORC_MAX_LAYERS) return 0;
  if (p->nx < 1 || p->ny < 1) return 0;
  if (p->lattice != ORC_D2Q9 && p->lattice != ORC_D1Q3) return 0;
  if (p->lattice == ORC_D1Q3 && p->ny != 1) return 0;
  if (!(p->tau > 0.0) || !(p->hstar > 0.0)) return 0;
  if (!(p->exp_a > p->exp_b && p->exp_b > 0)) return 0;
  for (int i = 0; i < p->n_layers; ++i)
    if (!(p->mu[i] > 0.0)) return 0;
  return 1;
}

orc_state *orc_create(const orc_params *p) {
  if (!p || !params_ok(p)) return NULL;
  orc_state *s = calloc(1, sizeof(orc_state));
  if (!s) return NULL;
  s->p = *p;
  s->Q = orc_lattice(p->lattice, s->cx, s->cy, s->w);
  s->nn = (long)p->nx * p->ny;
  long nf = (long)p->n_layers * s->Q * s->nn, nm = (long)p->n_layers * s->nn;
  s->f = calloc(nf, sizeof(double));
  s->fn = calloc(nf, sizeof(double));
  s->h = calloc(nm, sizeof(double));
  s->qx = calloc(nm, sizeof(double));
  s->qy = calloc(nm, sizeof(double));
  s->pr = calloc(nm, sizeof(double));
  s->gpx = calloc(nm, sizeof(double));
  s->gpy = calloc(nm, sizeof(double));
  if (!s->f || !s->fn || !s->h || !s->qx || !s->qy || !s->pr || !s->gpx || !s->gpy) {
    orc_destroy(s);
    return NULL;
  }
  return s;
}

void orc_destroy(orc_state *s) {
  if (!s) return;
  free(s->f); free(s->fn); free(s->h); free(s->qx); free(s->qy);
  free(s->pr); free(s->gpx); free(s->gpy);
  free(s);
}

long orc_steps_done(const orc_state *s) { return s->steps; }

int orc_init(orc_state *s, const double *h, const double *ux, const double *uy) {
  const int N = s->p.n_layers;
  for (long j = 0; j < (long)N * s->nn; ++j) {
    if (!isfinite(h[j]) || (ux && !isfinite(ux[j])) || (uy && !isfinite(uy[j]))) return ORC_ENONFINITE;
    if (!(h[j] > 0.0)) return ORC_ENONPOSITIVE;
  }
  for (int i = 0; i < N; ++i)
    for (long n = 0; n < s->nn; ++n) {
      double feq[9];
      long j = (long)i * s->nn + n;
      orc_equilibrium(s->p.lattice, h[j], ux ? ux[j] : 0.0, uy ? uy[j] : 0.0, feq);
      for (int k = 0; k < s->Q; ++k) s->f[FIDX(s, i, k, n)] = feq[k];
    }
  s->steps = 0;
  return ORC_OK;
}

/* O1: moments of the current populations */
static int moments(const orc_state *s, double *h, double *qx, double *qy) {
  const int N = s->p.n_layers;
  int err = ORC_OK;
#pragma omp parallel for num_threads(orc_get_threads()) reduction(max : err)
  for (long n = 0; n < s->nn; ++n)
    for (int i = 0; i < N; ++i) {
      double hs = 0.0, xs = 0.0, ys = 0.0;
      for (int k = 0; k < s->Q; ++k) {
        double v = s->f[FIDX(s, i, k, n)];
        hs += v;
        xs += s->cx[k] * v;
        ys += s->cy[k] * v;
      }
      long j = (long)i * s->nn + n;
      h[j] = hs;
      qx[j] = xs;
      qy[j] = ys;
      if (!isfinite(hs) || !isfinite(xs) || !isfinite(ys)) {
        if (err < ORC_ENONFINITE) err = ORC_ENONFINITE;
      } else if (!(hs > 0.0)) {
        if (err < ORC_ENONPOSITIVE) err = ORC_ENONPOSITIVE;
      }
    }
  return err;
}

static int one_step(orc_state *s) {
  const orc_params *p = &s->p;
  const int N = p->n_layers, nx = p->nx, ny = p->ny;
  const long nn = s->nn;
  /* O1 */
  int err = moments(s, s->h, s->qx, s->qy);
  if (err) return err;
  /* O2-O5 */
  err = orc_pressure(p, s->h, s->pr, NULL);
  if (err) return err;
  /* O6 */
  for (int i = 0; i < N; ++i)
    orc_grad(p->lattice, nx, ny, s->pr + i * nn, s->gpx + i * nn, s->gpy + i * nn);
  /* O7-O10 per node */
#pragma omp parallel for num_threads(orc_get_threads()) reduction(max : err)
  for (long n = 0; n < nn; ++n) {
    double hn[ORC_MAX_LAYERS], qxn[ORC_MAX_LAYERS], qyn[ORC_MAX_LAYERS];
    double frx[ORC_MAX_LAYERS], fry[ORC_MAX_LAYERS];
    for (int i = 0; i < N; ++i) {
      hn[i] = s->h[i * nn + n];
      qxn[i] = s->qx[i * nn + n];
      qyn[i] = s->qy[i * nn + n];
    }
    /* O7: the same matrix serves the x and y flux components */
    const double *qq[2] = {qxn, qyn};
    double *ff[2] = {frx, fry};
    if (friction_solve(N, hn, p->mu, p->slip, 2, qq, ff) != ORC_OK) {
      err = ORC_ENONFINITE;
      continue;
    }
    int y = (int)(n / nx), x = (int)(n % nx);
    for (int i = 0; i < N; ++i) {
      /* O8 */
      double Fx = -hn[i] * s->gpx[i * nn + n] + frx[i];
      double Fy = -hn[i] * s->gpy[i * nn + n] + fry[i];
      /* O9: U = q/h, collide towards f^eq(h, U), add the forcing */
      double ux = qxn[i] / hn[i], uy = qyn[i] / hn[i];
      double feq[9], frc[9];
      orc_equilibrium(p->lattice, hn[i], ux, uy, feq);
      orc_forcing(p->lattice, Fx, Fy, frc);
      for (int k = 0; k < s->Q; ++k) {
        double fk = s->f[FIDX(s, i, k, n)];
        double fstar = fk - (fk - feq[k]) / p->tau + frc[k];
        /* O10: push to the neighbour x + c_k */
        long dst = (long)wrap(y + s->cy[k], ny) * nx + wrap(x + s->cx[k], nx);
        s->fn[FIDX(s, i, k, dst)] = fstar;
      }
    }
  }
  if (err) return err;
  double *t = s->f;
  s->f = s->fn;
  s->fn = t;
  s->steps += 1;
  return ORC_OK;
}

int orc_step(orc_state *s, long nsteps) {
  for (long t = 0; t < nsteps; ++t) {
    int err = one_step(s);
    if (err) return err;
  }
  return ORC_OK;
}

void orc_read(const orc_state *s, double *h, double *ux, double *uy) {
  const long nm = (long)s->p.n_layers * s->nn;
  double *hh = malloc(sizeof(double) * nm * 3);
  if (!hh) return;
  double *qx = hh + nm, *qy = hh + 2 * nm;
  moments(s, hh, qx, qy);
  for (long j = 0; j < nm; ++j) {
    if (h) h[j] = hh[j];
    if (ux) ux[j] = qx[j] / hh[j];
    if (uy) uy[j] = qy[j] / hh[j];
  }
  free(hh);
}

/* Neumaier-compensated per-layer sum of h over all nodes */
void orc_mass(const orc_state *s, double *mass) {
  const long nm = (long)s->p.n_layers * s->nn;
  double *hh = malloc(sizeof(double) * nm * 3);
  if (!hh) return;
  moments(s, hh, hh + nm, hh + 2 * nm);
  for (int i = 0; i < s->p.n_layers; ++i) {
    double sum = 0.0, c = 0.0;
    for (long n = 0; n < s->nn; ++n) {
      double v = hh[(long)i * s->nn + n], t = sum + v;
      if (fabs(sum) >= fabs(v))
        c += (sum - t) + v;
      else
        c += (v - t) + sum;
      sum = t;
    }
    mass[i] = sum + c;
  }
  free(hh);
}

void orc_get_f(const orc_state *s, double *f) {
  memcpy(f, s->f, sizeof(double) * (size_t)s->p.n_layers * s->Q * s->nn);
}

void orc_set_f(orc_state *s, const double *f) {
  memcpy(s->f, f, sizeof(double) * (size_t)s->p.n_layers * s->Q * s->nn);
}
