/*
 * mlf_oracle.h -- plain FP64 CPU oracle for the N-layer thin-film
 * shallow-water lattice Boltzmann step of Richter, Malgaretti & Harting,
 * "Modeling of thin liquid films with arbitrary many layers"
 * (arXiv 2409.16659).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the HIP
 * implementation; it is slow on purpose and shares no code with it.
 * Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load it.  The product path never calls it.
 *
 * Notation follows the paper: N layers i = 1..N on a flat substrate
 * (index 0), gas above layer N; h_i layer thickness, z_i interface height
 * (z_0 = 0, z_i = z_{i-1} + h_i, Sec. II, Fig. 1); q_i = h_i U_i the layer
 * flux.  Lattice units dx = dt = 1.
 *
 * Parity notes: every function here is pinned by the CPU tests, except the
 * choice of gradient/Laplacian stencil, which the paper does not state
 * (the oracle uses the isotropic D2Q9-weight stencils; that this equals
 * the authors' stencil is parity unpinned).
 */
#ifndef MLF_ORACLE_H
#define MLF_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_MAX_LAYERS 4

enum { ORC_D2Q9 = 0, ORC_D1Q3 = 1 };
enum { ORC_OK = 0, ORC_ENONPOSITIVE = 1, ORC_ENONFINITE = 2, ORC_EINVAL = 3 };

typedef struct {
  int n_layers;          /* N, 1..ORC_MAX_LAYERS                          */
  int nx, ny;            /* periodic grid; D1Q3 requires ny == 1          */
  int lattice;           /* ORC_D2Q9 or ORC_D1Q3                          */
  double tau;            /* BGK relaxation time, Eq. (BGK)                */
  double hstar;          /* precursor thickness h*, Eq. (wetting_potential) */
  int exp_a, exp_b;      /* wetting exponents, a > b > 0 (the paper's n, m) */
  double gamma[ORC_MAX_LAYERS];  /* gamma_{i,i+1}, i = 1..N (gamma_N: layer N / gas) */
  double mu[ORC_MAX_LAYERS];     /* viscosities mu_1..mu_N                  */
  double slip[ORC_MAX_LAYERS];   /* slip lengths beta_1..beta_N, Eq. (no_slip) */
  /* spreading coefficients S_{l,k}: spread[l][k-1], l = 0..N-1, k = 1..N-l */
  double spread[ORC_MAX_LAYERS][ORC_MAX_LAYERS];
} orc_params;

typedef struct orc_state orc_state;

/* ---- whole-step driver ------------------------------------------------ */
orc_state *orc_create(const orc_params *p);
void orc_destroy(orc_state *s);
/* h, ux, uy: [N][ny][nx] host FP64; ux/uy may be NULL (U = 0).
 * Populations start at equilibrium f = f^eq(h, U). */
int orc_init(orc_state *s, const double *h, const double *ux, const double *uy);
/* Advance nsteps steps.  Returns ORC_OK or the error of the first step whose
 * moments were non-positive / non-finite (state then undefined). */
int orc_step(orc_state *s, long nsteps);
long orc_steps_done(const orc_state *s);
/* h, ux, uy [N][ny][nx]; any may be NULL.  U = q / h (moment definition). */
void orc_read(const orc_state *s, double *h, double *ux, double *uy);
/* per-layer mass sum_x h_i, Neumaier-compensated */
void orc_mass(const orc_state *s, double *mass);
/* population access, layout f[i][k][y][x] with Q = 9 (D2Q9) or 3 (D1Q3) */
void orc_get_f(const orc_state *s, double *f);
void orc_set_f(orc_state *s, const double *f);
void orc_set_threads(int nthreads);
int orc_get_threads(void);

/* ---- individual pieces, exposed for the pins -------------------------- */
/* lattice tables: Q, c_k (cx, cy) and w_k */
int orc_lattice(int lattice, int *cx, int *cy, double *w);
/* Eq. (wetting_potential): phi_k(d) and its derivative, without S */
double orc_phi(int k, double d, double hstar, int a, int b);
double orc_dphi(int k, double d, double hstar, int a, int b);
/* Eq. (spreading_parameters) from a full symmetric tension table
 * g[(N+2)*(N+2)] (index 0 = substrate, N+1 = gas). */
void orc_spreading_from_tensions(int n, const double *g, double spread[ORC_MAX_LAYERS][ORC_MAX_LAYERS]);
/* gradient and Laplacian of a periodic field f[ny][nx] */
void orc_grad(int lattice, int nx, int ny, const double *f, double *gx, double *gy);
void orc_lap(int lattice, int nx, int ny, const double *f, double *lap);
/* pressures p_i - p_atm and jumps Delta_i = p_i - p_{i+1} for heights
 * h[N][ny][nx] (Eqs. Laplace_pressure, disjoining_pressure). */
int orc_pressure(const orc_params *p, const double *h, double *pres, double *jump);
/* friction 2 mu_i h_i a_i of one node for flux vectors q (Eq. friction_force),
 * from the boundary-condition system (Eqs. no_slip, flux, viscous_boundary). */
int orc_friction(int n, const double *h, const double *mu, const double *slip,
                 const double *q, double *fr);
/* Eq. (equilibrium_distribution) and the forcing term of Eq. (BGK) */
void orc_equilibrium(int lattice, double h, double ux, double uy, double *feq);
void orc_forcing(int lattice, double fx, double fy, double *out);

#ifdef __cplusplus
}
#endif
#endif
