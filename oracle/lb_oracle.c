/* lb_oracle.c -- plain FP64 CPU oracle of the fine-box lattice-Boltzmann step.
 *
 * TEST INFRASTRUCTURE ONLY (see lb_oracle.h).  Written for clarity, not
 * speed: every step follows the method's order with whole-lattice passes
 * (moments, chain, spreading, collision, boundary equilibrium, streaming),
 * OpenMP only over z-planes.
 *
 * Sources of each part:
 *   lattice, equilibrium          standard D3Q19 model (Sec. 3); second-order
 *                                 equilibrium w_i rho [1 + 3 c.u + 9/2 (c.u)^2 - 3/2 u^2]
 *   BGK collision + forcing       Guo, Zheng, Shi (2002) forcing with u = (j + g/2)/rho
 *   MRT collision                 weighted-orthogonal basis of Duenweg, Schiller
 *                                 and Ladd (the LB review cited for the model in Sec. 3)
 *   equilibrium initial state and
 *   equilibrium boundary          Sec. 2 (populations set to local equilibrium;
 *                                 all sites at t = 0, boundary only afterwards)
 *   boundary interpolation        Sec. 2-3 (linear in space on the face grid,
 *                                 linear in time between samples)
 *   bead-spring chain, friction   Sec. 1 (Stokes friction coupling of beads,
 *                                 Ahlrichs-Duenweg), FENE springs
 *   centre-of-mass pinning        Sec. 2 (polymer centre of mass fixed at the tracer)
 */
#include "lb_oracle.h"

#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdlib.h>
#include <string.h>

/* ---------------------------------------------------------------- lattice */
static const int C[OR_Q][3] = {
    {0, 0, 0},
    {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},  {0, -1, 0}, {0, 0, 1},  {0, 0, -1},
    {1, 1, 0},  {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},
    {1, 0, 1},  {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
    {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};

static double W[OR_Q];
static double E[OR_Q][OR_Q]; /* E[k][i] = e_k(c_i) */
static double B[OR_Q];       /* B[k] = sum_i w_i e_k(c_i)^2 */
static int tables_ready = 0;

static void basis_row(const int c[3], double e[OR_Q]) {
  const double cx = c[0], cy = c[1], cz = c[2];
  const double c2 = cx * cx + cy * cy + cz * cz;
  e[0] = 1.0;
  e[1] = cx;
  e[2] = cy;
  e[3] = cz;
  e[4] = c2 - 1.0;
  e[5] = 3.0 * cx * cx - c2;
  e[6] = cy * cy - cz * cz;
  e[7] = cx * cy;
  e[8] = cy * cz;
  e[9] = cx * cz;
  e[10] = (3.0 * c2 - 5.0) * cx;
  e[11] = (3.0 * c2 - 5.0) * cy;
  e[12] = (3.0 * c2 - 5.0) * cz;
  e[13] = (cy * cy - cz * cz) * cx;
  e[14] = (cz * cz - cx * cx) * cy;
  e[15] = (cx * cx - cy * cy) * cz;
  e[16] = 3.0 * c2 * c2 - 6.0 * c2 + 1.0;
  e[17] = (2.0 * c2 - 3.0) * (3.0 * cx * cx - c2);
  e[18] = (2.0 * c2 - 3.0) * (cy * cy - cz * cz);
}

static void init_tables(void) {
  if (tables_ready) return;
  for (int i = 0; i < OR_Q; i++) {
    int c2 = C[i][0] * C[i][0] + C[i][1] * C[i][1] + C[i][2] * C[i][2];
    W[i] = (c2 == 0) ? 1.0 / 3.0 : (c2 == 1) ? 1.0 / 18.0 : 1.0 / 36.0;
  }
  for (int i = 0; i < OR_Q; i++) {
    double e[OR_Q];
    basis_row(C[i], e);
    for (int k = 0; k < OR_Q; k++) E[k][i] = e[k];
  }
  for (int k = 0; k < OR_Q; k++) {
    double s = 0.0;
    for (int i = 0; i < OR_Q; i++) s += W[i] * E[k][i] * E[k][i];
    B[k] = s;
  }
  tables_ready = 1;
}

int or_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void or_lattice(int c[OR_Q][3], double w[OR_Q]) {
  init_tables();
  for (int i = 0; i < OR_Q; i++) {
    for (int a = 0; a < 3; a++) c[i][a] = C[i][a];
    w[i] = W[i];
  }
}

void or_mrt_basis(double e[OR_Q][OR_Q], double b[OR_Q]) {
  init_tables();
  for (int k = 0; k < OR_Q; k++) {
    b[k] = B[k];
    for (int i = 0; i < OR_Q; i++) e[k][i] = E[k][i];
  }
}

/* ------------------------------------------------------- node primitives */
void or_equilibrium(double rho, const double u[3], double feq[OR_Q]) {
  init_tables();
  const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  for (int i = 0; i < OR_Q; i++) {
    const double cu = C[i][0] * u[0] + C[i][1] * u[1] + C[i][2] * u[2];
    feq[i] = W[i] * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
  }
}

/* Guo forcing population w_i [3 (c_i - u).g + 9 (c_i.u)(c_i.g)] */
static void forcing_pops(const double u[3], const double g[3], double F[OR_Q]) {
  for (int i = 0; i < OR_Q; i++) {
    const double cu = C[i][0] * u[0] + C[i][1] * u[1] + C[i][2] * u[2];
    const double cg = C[i][0] * g[0] + C[i][1] * g[1] + C[i][2] * g[2];
    double s = 0.0;
    for (int a = 0; a < 3; a++) s += 3.0 * (C[i][a] - u[a]) * g[a];
    F[i] = W[i] * (s + 9.0 * cu * cg);
  }
}

void or_collide(const or_params* p, const double f[OR_Q], const double g[3], double out[OR_Q]) {
  init_tables();
  double rho = 0.0, j[3] = {0.0, 0.0, 0.0};
  for (int i = 0; i < OR_Q; i++) {
    rho += f[i];
    for (int a = 0; a < 3; a++) j[a] += C[i][a] * f[i];
  }
  double u[3];
  for (int a = 0; a < 3; a++) u[a] = (j[a] + 0.5 * g[a]) / rho;
  double feq[OR_Q], F[OR_Q];
  or_equilibrium(rho, u, feq);
  forcing_pops(u, g, F);
  if (p->collision == OR_BGK) {
    const double om = 1.0 / p->tau;
    for (int i = 0; i < OR_Q; i++)
      out[i] = f[i] - om * (f[i] - feq[i]) + (1.0 - 0.5 * om) * F[i];
    return;
  }
  /* MRT: m = E f; m* = m_eq + gamma (m - m_eq) + (1 + gamma)/2 m_F; f* = W E^T B^-1 m* */
  double gam[OR_Q];
  for (int k = 0; k < OR_Q; k++) {
    if (k < 4) gam[k] = 1.0;                       /* mass and momentum: conserved */
    else if (k == 4) gam[k] = 1.0 - 1.0 / p->tau_bulk;
    else if (k < 10) gam[k] = 1.0 - 1.0 / p->tau;  /* five shear modes */
    else gam[k] = 1.0 - p->ghost_rate;             /* nine ghost modes */
  }
  double ms[OR_Q];
  for (int k = 0; k < OR_Q; k++) {
    double m = 0.0, meq = 0.0, mf = 0.0;
    for (int i = 0; i < OR_Q; i++) {
      m += E[k][i] * f[i];
      meq += E[k][i] * feq[i];
      mf += E[k][i] * F[i];
    }
    ms[k] = meq + gam[k] * (m - meq) + 0.5 * (1.0 + gam[k]) * mf;
  }
  for (int i = 0; i < OR_Q; i++) {
    double s = 0.0;
    for (int k = 0; k < OR_Q; k++) s += E[k][i] * ms[k] / B[k];
    out[i] = W[i] * s;
  }
}

/* ------------------------------------------------ counter-based RNG */
/* Philox4x32-10 (Salmon, Moraes, Dror and Shaw, "Parallel random numbers:
 * as easy as 1, 2, 3", SC 2011): ten rounds of two 32x32->64-bit products
 * mixed into a 128-bit counter under a 64-bit key that is bumped by the Weyl
 * constants between rounds. */
void or_philox4x32(const unsigned ctr[4], const unsigned key[2], unsigned out[4]) {
  unsigned c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  unsigned k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; r++) {
    const unsigned long long p0 = (unsigned long long)0xD2511F53u * c0;
    const unsigned long long p1 = (unsigned long long)0xCD9E8D57u * c2;
    const unsigned hi0 = (unsigned)(p0 >> 32), lo0 = (unsigned)p0;
    const unsigned hi1 = (unsigned)(p1 >> 32), lo1 = (unsigned)p1;
    c0 = hi1 ^ c1 ^ k0;
    c1 = lo1;
    c2 = hi0 ^ c3 ^ k1;
    c3 = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  out[0] = c0;
  out[1] = c1;
  out[2] = c2;
  out[3] = c3;
}

/* 32 random bits -> uniform on (-sqrt 3, sqrt 3): mean 0, variance 1 */
double or_unit_uniform(unsigned u) {
  return ((double)u - 2147483647.5) * (1.7320508075688772 / 2147483648.0);
}

/* Fluctuating MRT (Duenweg, Schiller and Ladd; the LB review the paper cites
 * for its coupling): the same relaxation as or_collide, plus on every
 * non-conserved mode k >= 4 the noise sqrt(mu rho b_k (1 - gamma_k^2)) r_k,
 * mu = 3 kT (k_B T in lattice units over c_s^2), rho the node's density and
 * r_k of zero mean and unit variance.  It keeps the mode fluctuations at
 * their equilibrium variance mu rho b_k. */
void or_collide_noise(const or_params* p, const double f[OR_Q], const double g[3], double mu,
                      const double r[OR_Q], double out[OR_Q]) {
  init_tables();
  double rho = 0.0, j[3] = {0.0, 0.0, 0.0};
  for (int i = 0; i < OR_Q; i++) {
    rho += f[i];
    for (int a = 0; a < 3; a++) j[a] += C[i][a] * f[i];
  }
  double u[3];
  for (int a = 0; a < 3; a++) u[a] = (j[a] + 0.5 * g[a]) / rho;
  double feq[OR_Q], F[OR_Q];
  or_equilibrium(rho, u, feq);
  forcing_pops(u, g, F);
  double gam[OR_Q];
  for (int k = 0; k < OR_Q; k++) {
    if (k < 4) gam[k] = 1.0;
    else if (k == 4) gam[k] = 1.0 - 1.0 / p->tau_bulk;
    else if (k < 10) gam[k] = 1.0 - 1.0 / p->tau;
    else gam[k] = 1.0 - p->ghost_rate;
  }
  double ms[OR_Q];
  for (int k = 0; k < OR_Q; k++) {
    double m = 0.0, meq = 0.0, mf = 0.0;
    for (int i = 0; i < OR_Q; i++) {
      m += E[k][i] * f[i];
      meq += E[k][i] * feq[i];
      mf += E[k][i] * F[i];
    }
    ms[k] = meq + gam[k] * (m - meq) + 0.5 * (1.0 + gam[k]) * mf;
    if (k >= 4) ms[k] += sqrt(mu * rho * B[k] * (1.0 - gam[k] * gam[k])) * r[k];
  }
  for (int i = 0; i < OR_Q; i++) {
    double s = 0.0;
    for (int k = 0; k < OR_Q; k++) s += E[k][i] * ms[k] / B[k];
    out[i] = W[i] * s;
  }
}

int or_chain_md(int nb, int substeps, int fix_com, double zeta, double mass, double fene_k,
                double fene_r0, const double anchor[3], double* pos, double* vel,
                const double* ubead, double* dp) {
  return or_chain_md_noise(nb, substeps, fix_com, zeta, mass, fene_k, fene_r0, anchor, pos, vel,
                           ubead, 0.0, NULL, dp);
}

int or_chain_md_noise(int nb, int substeps, int fix_com, double zeta, double mass, double fene_k,
                      double fene_r0, const double anchor[3], double* pos, double* vel,
                      const double* ubead, double kT, const double* rnd, double* dp) {
  const double h = 1.0 / substeps;
  const double decay = exp(-zeta * h / mass);
  /* Langevin noise of the exact friction update: the velocity of a bead
   * relaxing toward u + F/zeta over a substep takes the Ornstein-Uhlenbeck
   * increment of standard deviation sqrt(kT/m (1 - e^{-2 zeta h/m})) */
  const double kick = kT > 0.0 ? sqrt(kT / mass * (1.0 - exp(-2.0 * zeta * h / mass))) : 0.0;
  const double r02 = fene_r0 * fene_r0;
  double* F = (double*)calloc((size_t)nb * 3, sizeof(double));
  if (!F) return OR_ERR_OOM;
  for (int j = 0; j < nb * 3; j++) dp[j] = 0.0;
  int status = OR_OK;
  for (int s = 0; s < substeps && status == OR_OK; s++) {
    /* FENE bond forces, each bond once, applied with opposite signs */
    for (int j = 0; j < nb * 3; j++) F[j] = 0.0;
    for (int j = 0; j + 1 < nb; j++) {
      double r[3], r2 = 0.0;
      for (int a = 0; a < 3; a++) {
        r[a] = pos[3 * (j + 1) + a] - pos[3 * j + a];
        r2 += r[a] * r[a];
      }
      if (r2 >= r02) { status = OR_ERR_FENE; break; }
      const double fac = fene_k / (1.0 - r2 / r02);
      for (int a = 0; a < 3; a++) {
        F[3 * j + a] += fac * r[a];
        F[3 * (j + 1) + a] -= fac * r[a];
      }
    }
    if (status != OR_OK) break;
    /* friction: exact solution of m dV/dt = -zeta (V - u) + F with u, F fixed */
    for (int j = 0; j < nb; j++) {
      for (int a = 0; a < 3; a++) {
        const double u = ubead[3 * j + a];
        const double fz = F[3 * j + a] / zeta;
        const double v0 = vel[3 * j + a];
        double v1 = u + fz + (v0 - u - fz) * decay;
        if (kick > 0.0) v1 += kick * rnd[((size_t)s * nb + j) * 3 + a];
        dp[3 * j + a] += mass * (v1 - v0) - F[3 * j + a] * h;
        vel[3 * j + a] = v1;
        pos[3 * j + a] += h * v1;
      }
    }
    if (fix_com) {
      double vb[3] = {0, 0, 0}, rb[3] = {0, 0, 0};
      for (int j = 0; j < nb; j++)
        for (int a = 0; a < 3; a++) {
          vb[a] += vel[3 * j + a];
          rb[a] += pos[3 * j + a];
        }
      for (int a = 0; a < 3; a++) {
        vb[a] /= nb;
        rb[a] /= nb;
      }
      for (int j = 0; j < nb; j++)
        for (int a = 0; a < 3; a++) {
          vel[3 * j + a] -= vb[a];
          pos[3 * j + a] = pos[3 * j + a] - rb[a] + anchor[a];
        }
    }
  }
  free(F);
  return status;
}

/* ------------------------------------------------------------------ box */
typedef struct {
  int nb, substeps, fix_com;
  double zeta, mass, fene_k, fene_r0, anchor[3];
  double *pos, *vel;
} chain_t;

struct or_box {
  or_params p;
  long nn;                  /* nodes */
  double *f, *fs, *fn;      /* pre-collision, post-collision, next pre-collision */
  double *g;                /* [nn][3] force density of the current step */
  long step;
  int err_code;
  long err_step;
  int has_bc, bc_mode, bc_dt, bc_ns, bc_res;
  long bc_t0;
  double* bc;
  int n_chains;
  chain_t* chains;
  double mass_mom[5];
  /* accelerated-frame body force: tracer acceleration samples [ns][3] */
  int has_body, body_dt, body_ns;
  long body_t0;
  double* body;
  /* thermal fluctuations: kT, Philox key, the box's index in the counter */
  double kT;
  unsigned key[2];
  unsigned box_index;
};

static long nidx(const or_box* b, int x, int y, int z) {
  return ((long)z * b->p.ny + y) * b->p.nx + x;
}

static int axis_n(const or_box* b, int a) {
  return a == 0 ? b->p.nx : (a == 1 ? b->p.ny : b->p.nz);
}

static int is_periodic(const or_box* b, int a) { return (b->p.periodic_mask >> a) & 1u; }

static int in_interior(const or_box* b, const int q[3]) {
  for (int a = 0; a < 3; a++) {
    if (is_periodic(b, a)) continue;
    if (q[a] < 1 || q[a] > axis_n(b, a) - 2) return 0;
  }
  return 1;
}

static int wrap(int v, int n) { return ((v % n) + n) % n; }

or_box* or_create(const or_params* p) {
  init_tables();
  if (!p || p->nx < 1 || p->ny < 1 || p->nz < 1 || p->tau <= 0.5) return NULL;
  for (int a = 0; a < 3; a++) {
    int n = a == 0 ? p->nx : (a == 1 ? p->ny : p->nz);
    if (!((p->periodic_mask >> a) & 1u) && n < 3) return NULL;
  }
  or_box* b = (or_box*)calloc(1, sizeof(or_box));
  if (!b) return NULL;
  b->p = *p;
  b->nn = (long)p->nx * p->ny * p->nz;
  b->f = (double*)calloc((size_t)b->nn * OR_Q, sizeof(double));
  b->fs = (double*)calloc((size_t)b->nn * OR_Q, sizeof(double));
  b->fn = (double*)calloc((size_t)b->nn * OR_Q, sizeof(double));
  b->g = (double*)calloc((size_t)b->nn * 3, sizeof(double));
  if (!b->f || !b->fs || !b->fn || !b->g) {
    or_destroy(b);
    return NULL;
  }
  or_set_initial(b, NULL);
  return b;
}

void or_destroy(or_box* b) {
  if (!b) return;
  free(b->f);
  free(b->fs);
  free(b->fn);
  free(b->g);
  free(b->bc);
  free(b->body);
  for (int c = 0; c < b->n_chains; c++) {
    free(b->chains[c].pos);
    free(b->chains[c].vel);
  }
  free(b->chains);
  free(b);
}

int or_set_initial(or_box* b, const double* u) {
  for (int z = 0; z < b->p.nz; z++)
    for (int y = 0; y < b->p.ny; y++)
      for (int x = 0; x < b->p.nx; x++) {
        const long n = nidx(b, x, y, z);
        double uu[3] = {0.0, 0.0, 0.0}, feq[OR_Q];
        const int q[3] = {x, y, z};
        if (u && in_interior(b, q))
          for (int a = 0; a < 3; a++) uu[a] = u[3 * n + a];
        or_equilibrium(b->p.rho0, uu, feq);
        for (int i = 0; i < OR_Q; i++) b->f[i * b->nn + n] = feq[i];
      }
  b->step = 0;
  b->err_code = OR_OK;
  b->err_step = -1;
  memset(b->mass_mom, 0, sizeof(b->mass_mom));
  return OR_OK;
}

int or_set_populations(or_box* b, const double* f) {
  memcpy(b->f, f, sizeof(double) * (size_t)b->nn * OR_Q);
  return OR_OK;
}

int or_set_boundary(or_box* b, int mode, long t0, int dt, int n_samples, int res, const double* data) {
  if (dt < 1 || n_samples < 1 || !data) return OR_ERR_ARG;
  if (mode != OR_BC_AFFINE && mode != OR_BC_SAMPLED) return OR_ERR_ARG;
  if (mode == OR_BC_SAMPLED && res < 2) return OR_ERR_ARG;
  size_t per = mode == OR_BC_AFFINE ? 9 : (size_t)6 * res * res * 3;
  free(b->bc);
  b->bc = (double*)malloc(sizeof(double) * per * n_samples);
  if (!b->bc) return OR_ERR_OOM;
  memcpy(b->bc, data, sizeof(double) * per * n_samples);
  b->has_bc = 1;
  b->bc_mode = mode;
  b->bc_t0 = t0;
  b->bc_dt = dt;
  b->bc_ns = n_samples;
  b->bc_res = res;
  return OR_OK;
}

int or_add_chain(or_box* b, int nb, int substeps, int fix_com, double zeta, double mass,
                 double fene_k, double fene_r0, const double anchor[3], const double* pos,
                 const double* vel) {
  if (nb < 1 || substeps < 1 || zeta <= 0 || mass <= 0 || fene_r0 <= 0 || !pos) return OR_ERR_ARG;
  chain_t* nc = (chain_t*)realloc(b->chains, sizeof(chain_t) * (b->n_chains + 1));
  if (!nc) return OR_ERR_OOM;
  b->chains = nc;
  chain_t* c = &b->chains[b->n_chains];
  c->nb = nb;
  c->substeps = substeps;
  c->fix_com = fix_com;
  c->zeta = zeta;
  c->mass = mass;
  c->fene_k = fene_k;
  c->fene_r0 = fene_r0;
  for (int a = 0; a < 3; a++) c->anchor[a] = anchor[a];
  c->pos = (double*)malloc(sizeof(double) * 3 * nb);
  c->vel = (double*)calloc((size_t)3 * nb, sizeof(double));
  if (!c->pos || !c->vel) return OR_ERR_OOM;
  memcpy(c->pos, pos, sizeof(double) * 3 * nb);
  if (vel) memcpy(c->vel, vel, sizeof(double) * 3 * nb);
  b->n_chains++;
  return OR_OK;
}

int or_set_body_force(or_box* b, long t0, int dt, int n_samples, const double* accel) {
  if (n_samples == 0 || !accel) {
    free(b->body);
    b->body = NULL;
    b->has_body = 0;
    return OR_OK;
  }
  if (dt < 1 || n_samples < 1) return OR_ERR_ARG;
  double* a = (double*)malloc(sizeof(double) * 3 * (size_t)n_samples);
  if (!a) return OR_ERR_OOM;
  memcpy(a, accel, sizeof(double) * 3 * (size_t)n_samples);
  free(b->body);
  b->body = a;
  b->has_body = 1;
  b->body_t0 = t0;
  b->body_dt = dt;
  b->body_ns = n_samples;
  return OR_OK;
}

int or_set_thermal(or_box* b, double kT, unsigned long long seed, unsigned box_index) {
  if (!(kT >= 0.0)) return OR_ERR_ARG;
  if (kT > 0.0 && b->p.collision != OR_MRT) return OR_ERR_ARG;
  b->kT = kT;
  b->key[0] = (unsigned)(seed & 0xffffffffu);
  b->key[1] = (unsigned)(seed >> 32);
  b->box_index = box_index;
  return OR_OK;
}

/* tracer acceleration at step n, linear in time between samples */
static int body_accel(const or_box* b, long n, double a[3]) {
  const long rel = n - b->body_t0;
  if (rel < 0) return OR_ERR_ARG;
  const long k = rel / b->body_dt;
  const long rem = rel - k * b->body_dt;
  if (k >= b->body_ns || (rem > 0 && k + 1 >= b->body_ns)) return OR_ERR_ARG;
  const double th = (double)rem / (double)b->body_dt;
  for (int c = 0; c < 3; c++)
    a[c] = rem > 0 ? (1.0 - th) * b->body[3 * k + c] + th * b->body[3 * (k + 1) + c] : b->body[3 * k + c];
  return OR_OK;
}

/* the 16 unit-variance numbers of node m at step n: four Philox draws with
 * counter (node, box, step, draw) */
static void node_noise(const or_box* b, long m, long n, double r[16]) {
  for (unsigned d = 0; d < 4; d++) {
    const unsigned ctr[4] = {(unsigned)m, b->box_index, (unsigned)n, d};
    unsigned o[4];
    or_philox4x32(ctr, b->key, o);
    for (int q = 0; q < 4; q++) r[4 * d + q] = or_unit_uniform(o[q]);
  }
}

/* First face, in the order -x, +x, -y, +y, -z, +z, that contains node q; -1 if none. */
static int node_face(const or_box* b, const int q[3]) {
  for (int f = 0; f < 6; f++) {
    const int a = f / 2;
    if (is_periodic(b, a)) continue;
    const int at = (f % 2 == 0) ? 0 : axis_n(b, a) - 1;
    if (q[a] == at) return f;
  }
  return -1;
}

/* bilinear value of sample k on face f at tangential node coordinates (iu, iv) */
static void face_bilinear(const or_box* b, int k, int f, int iu, int iv, int nu, int nv, double out[3]) {
  const int R = b->bc_res;
  /* corner-aligned grid: point p sits at node coordinate p (n-1)/(R-1) */
  const long su = (long)iu * (R - 1), sv = (long)iv * (R - 1);
  const int p = (int)(su / (nu - 1)), q = (int)(sv / (nv - 1));
  const double al = (double)(su - (long)p * (nu - 1)) / (double)(nu - 1);
  const double be = (double)(sv - (long)q * (nv - 1)) / (double)(nv - 1);
  const int p1 = p + 1 < R ? p + 1 : p, q1 = q + 1 < R ? q + 1 : q;
  const double* S = b->bc + ((size_t)k * 6 + f) * R * R * 3;
  for (int c = 0; c < 3; c++) {
    const double s00 = S[((size_t)q * R + p) * 3 + c], s01 = S[((size_t)q * R + p1) * 3 + c];
    const double s10 = S[((size_t)q1 * R + p) * 3 + c], s11 = S[((size_t)q1 * R + p1) * 3 + c];
    out[c] = (1.0 - al) * (1.0 - be) * s00 + al * (1.0 - be) * s01 + (1.0 - al) * be * s10 + al * be * s11;
  }
}

/* time slot of step n: k, theta; returns OR_ERR_ARG outside the sampled window */
static int time_slot(const or_box* b, long n, long* k, double* th, int* need2) {
  const long rel = n - b->bc_t0;
  if (rel < 0) return OR_ERR_ARG;
  *k = rel / b->bc_dt;
  const long rem = rel - *k * b->bc_dt;
  *th = (double)rem / (double)b->bc_dt;
  *need2 = rem > 0;
  if (*k >= b->bc_ns || (*need2 && *k + 1 >= b->bc_ns)) return OR_ERR_ARG;
  return OR_OK;
}

int or_boundary_velocity(const or_box* b, int x, int y, int z, long n, double u[3]) {
  if (!b->has_bc) return OR_ERR_STATE;
  long k;
  double th;
  int need2;
  int st = time_slot(b, n, &k, &th, &need2);
  if (st) return st;
  const int q[3] = {x, y, z};
  if (b->bc_mode == OR_BC_AFFINE) {
    double A[9];
    for (int e = 0; e < 9; e++)
      A[e] = need2 ? (1.0 - th) * b->bc[9 * k + e] + th * b->bc[9 * (k + 1) + e] : b->bc[9 * k + e];
    double r[3];
    for (int a = 0; a < 3; a++) r[a] = q[a] - 0.5 * (axis_n(b, a) - 1);
    for (int a = 0; a < 3; a++) u[a] = A[3 * a] * r[0] + A[3 * a + 1] * r[1] + A[3 * a + 2] * r[2];
    return OR_OK;
  }
  const int f = node_face(b, q);
  if (f < 0) return OR_ERR_ARG;
  const int au = (f / 2 == 0) ? 1 : 0;
  const int av = (f / 2 == 2) ? 1 : 2;
  double v0[3], v1[3] = {0, 0, 0};
  face_bilinear(b, (int)k, f, q[au], q[av], axis_n(b, au), axis_n(b, av), v0);
  if (need2) face_bilinear(b, (int)k + 1, f, q[au], q[av], axis_n(b, au), axis_n(b, av), v1);
  for (int c = 0; c < 3; c++) u[c] = need2 ? (1.0 - th) * v0[c] + th * v1[c] : v0[c];
  return OR_OK;
}

static int has_boundary_layer(const or_box* b) {
  return (b->p.periodic_mask & 7u) != 7u;
}

/* trilinear stencil of position r: nodes[8], weights[8]; OR_ERR_BEAD_OUT if a
 * node leaves the interior (periodic axes wrap) */
static int stencil(const or_box* b, const double r[3], long nodes[8], double w8[8]) {
  int base[3];
  double d[3];
  for (int a = 0; a < 3; a++) {
    const double fl = floor(r[a]);
    base[a] = (int)fl;
    d[a] = r[a] - fl;
    if (!is_periodic(b, a) && (base[a] < 1 || base[a] + 1 > axis_n(b, a) - 2)) return OR_ERR_BEAD_OUT;
  }
  for (int c = 0; c < 8; c++) {
    const int o[3] = {c & 1, (c >> 1) & 1, (c >> 2) & 1};
    int q[3];
    double w = 1.0;
    for (int a = 0; a < 3; a++) {
      q[a] = wrap(base[a] + o[a], axis_n(b, a));
      w *= o[a] ? d[a] : 1.0 - d[a];
    }
    nodes[c] = nidx(b, q[0], q[1], q[2]);
    w8[c] = w;
  }
  return OR_OK;
}

int or_step(or_box* b, int nsteps) {
  const long nn = b->nn;
  const int nx = b->p.nx, ny = b->p.ny, nz = b->p.nz;
  if (has_boundary_layer(b) && !b->has_bc) return OR_ERR_STATE;
  for (int s = 0; s < nsteps; s++) {
    if (b->err_code) return b->err_code;
    const long n = b->step;
    if (has_boundary_layer(b)) {
      long k;
      double th;
      int need2;
      if (time_slot(b, n, &k, &th, &need2)) return OR_ERR_ARG;
    }
    double acc[3] = {0.0, 0.0, 0.0};
    if (b->has_body && body_accel(b, n, acc)) return OR_ERR_ARG;

    /* 1-4: chain against the pre-collision moments at t_n; force density g */
    memset(b->g, 0, sizeof(double) * (size_t)nn * 3);
    int err = OR_OK;
    chain_t* nxt = NULL;
    if (b->n_chains) {
      nxt = (chain_t*)calloc((size_t)b->n_chains, sizeof(chain_t));
      unsigned bead0 = 0; /* index of the chain's first bead among the box's beads */
      for (int c = 0; c < b->n_chains && !err; bead0 += (unsigned)b->chains[c].nb, c++) {
        const chain_t* ch = &b->chains[c];
        nxt[c] = *ch;
        nxt[c].pos = (double*)malloc(sizeof(double) * 3 * ch->nb);
        nxt[c].vel = (double*)malloc(sizeof(double) * 3 * ch->nb);
        memcpy(nxt[c].pos, ch->pos, sizeof(double) * 3 * ch->nb);
        memcpy(nxt[c].vel, ch->vel, sizeof(double) * 3 * ch->nb);
        double* ub = (double*)calloc((size_t)3 * ch->nb, sizeof(double));
        double* dp = (double*)calloc((size_t)3 * ch->nb, sizeof(double));
        long* nodes = (long*)malloc(sizeof(long) * 8 * ch->nb);
        double* wts = (double*)malloc(sizeof(double) * 8 * ch->nb);
        for (int j = 0; j < ch->nb && !err; j++) {
          err = stencil(b, &ch->pos[3 * j], &nodes[8 * j], &wts[8 * j]);
          if (err) break;
          for (int cc = 0; cc < 8; cc++) {
            const long m = nodes[8 * j + cc];
            double rho = 0.0, jj[3] = {0, 0, 0};
            for (int i = 0; i < OR_Q; i++) {
              const double fi = b->f[i * nn + m];
              rho += fi;
              for (int a = 0; a < 3; a++) jj[a] += C[i][a] * fi;
            }
            for (int a = 0; a < 3; a++) ub[3 * j + a] += wts[8 * j + cc] * jj[a] / rho;
          }
        }
        /* bead noise: one Philox draw per bead and substep, counter
         * (bead index in the box, box, step, 16 + substep), three numbers used */
        double* rnd = NULL;
        if (!err && b->kT > 0.0) {
          rnd = (double*)malloc(sizeof(double) * 3 * (size_t)ch->nb * ch->substeps);
          for (int s2 = 0; s2 < ch->substeps; s2++)
            for (int j = 0; j < ch->nb; j++) {
              const unsigned ctr[4] = {bead0 + (unsigned)j, b->box_index, (unsigned)n, 16u + (unsigned)s2};
              unsigned o[4];
              or_philox4x32(ctr, b->key, o);
              for (int a = 0; a < 3; a++) rnd[((size_t)s2 * ch->nb + j) * 3 + a] = or_unit_uniform(o[a]);
            }
        }
        if (!err)
          err = or_chain_md_noise(ch->nb, ch->substeps, ch->fix_com, ch->zeta, ch->mass, ch->fene_k,
                                  ch->fene_r0, ch->anchor, nxt[c].pos, nxt[c].vel, ub, b->kT, rnd, dp);
        free(rnd);
        if (!err)
          for (int j = 0; j < ch->nb; j++)
            for (int cc = 0; cc < 8; cc++)
              for (int a = 0; a < 3; a++)
                b->g[3 * nodes[8 * j + cc] + a] -= wts[8 * j + cc] * dp[3 * j + a];
        free(ub);
        free(dp);
        free(nodes);
        free(wts);
      }
    }
    if (err) {
      if (nxt) {
        for (int c = 0; c < b->n_chains; c++) {
          free(nxt[c].pos);
          free(nxt[c].vel);
        }
        free(nxt);
      }
      b->err_code = err;
      b->err_step = n;
      return err;
    }

    /* 5-6: collide on the interior; boundary nodes take f_eq(rho0, u_b(t_n)) */
    int bc_err = OR_OK;
#pragma omp parallel for schedule(static) reduction(min : bc_err)
    for (int z = 0; z < nz; z++)
      for (int y = 0; y < ny; y++)
        for (int x = 0; x < nx; x++) {
          const long m = nidx(b, x, y, z);
          const int q[3] = {x, y, z};
          double fin[OR_Q], fout[OR_Q];
          if (in_interior(b, q)) {
            double rho = 0.0;
            for (int i = 0; i < OR_Q; i++) {
              fin[i] = b->f[i * nn + m];
              rho += fin[i];
            }
            /* accelerated frame: force density -rho dv/dt on top of the chains' */
            double gt[3];
            for (int a = 0; a < 3; a++) gt[a] = b->g[3 * m + a] - rho * acc[a];
            if (b->kT > 0.0) {
              double r16[16], r[OR_Q] = {0};
              node_noise(b, m, n, r16);
              for (int k = 4; k < OR_Q; k++) r[k] = r16[k - 4];
              or_collide_noise(&b->p, fin, gt, 3.0 * b->kT, r, fout);
            } else {
              or_collide(&b->p, fin, gt, fout);
            }
          } else {
            double ubv[3];
            int st = or_boundary_velocity(b, x, y, z, n, ubv);
            if (st < bc_err) bc_err = st;
            or_equilibrium(b->p.rho0, ubv, fout);
          }
          for (int i = 0; i < OR_Q; i++) b->fs[i * nn + m] = fout[i];
        }
    if (bc_err) return bc_err;

    /* 7: stream (pull), f_i(x, t+1) = f*_i(x - c_i, t), periodic axes wrap */
#pragma omp parallel for schedule(static)
    for (int z = 0; z < nz; z++)
      for (int y = 0; y < ny; y++)
        for (int x = 0; x < nx; x++) {
          const long m = nidx(b, x, y, z);
          const int q[3] = {x, y, z};
          if (!in_interior(b, q)) {
            for (int i = 0; i < OR_Q; i++) b->fn[i * nn + m] = W[i] * b->p.rho0;
            continue;
          }
          for (int i = 0; i < OR_Q; i++) {
            const int sx = wrap(x - C[i][0], nx), sy = wrap(y - C[i][1], ny), sz = wrap(z - C[i][2], nz);
            b->fn[i * nn + m] = b->fs[i * nn + nidx(b, sx, sy, sz)];
          }
        }

    /* 8: mass and momentum of the interior at t_{n+1} every K steps */
    double rec[5] = {0, 0, 0, 0, 0};
    int record = b->p.reduce_every > 0 && (n + 1) % b->p.reduce_every == 0;
    if (record) {
      double M = 0.0, P[3] = {0, 0, 0};
      for (int z = 0; z < nz; z++)
        for (int y = 0; y < ny; y++)
          for (int x = 0; x < nx; x++) {
            const int q[3] = {x, y, z};
            if (!in_interior(b, q)) continue;
            const long m = nidx(b, x, y, z);
            for (int i = 0; i < OR_Q; i++) {
              const double fi = b->fn[i * nn + m];
              M += fi;
              for (int a = 0; a < 3; a++) P[a] += C[i][a] * fi;
            }
          }
      rec[0] = (double)(n + 1);
      rec[1] = M;
      rec[2] = P[0];
      rec[3] = P[1];
      rec[4] = P[2];
      if (!isfinite(M) || !isfinite(P[0]) || !isfinite(P[1]) || !isfinite(P[2])) {
        if (nxt) {
          for (int c = 0; c < b->n_chains; c++) {
            free(nxt[c].pos);
            free(nxt[c].vel);
          }
          free(nxt);
        }
        b->err_code = OR_ERR_UNSTABLE;
        b->err_step = n;
        return OR_ERR_UNSTABLE;
      }
    }

    /* commit */
    double* t = b->f;
    b->f = b->fn;
    b->fn = t;
    if (nxt) {
      for (int c = 0; c < b->n_chains; c++) {
        free(b->chains[c].pos);
        free(b->chains[c].vel);
        b->chains[c].pos = nxt[c].pos;
        b->chains[c].vel = nxt[c].vel;
      }
      free(nxt);
    }
    if (record) memcpy(b->mass_mom, rec, sizeof(rec));
    b->step = n + 1;
  }
  return OR_OK;
}

long or_get_step(const or_box* b) { return b->step; }

void or_get_error(const or_box* b, int* code, long* step) {
  *code = b->err_code;
  *step = b->err_step;
}

void or_read_pop(const or_box* b, double* f) {
  memcpy(f, b->f, sizeof(double) * (size_t)b->nn * OR_Q);
}

void or_read_rho_u(const or_box* b, double* rho, double* u) {
  for (int z = 0; z < b->p.nz; z++)
    for (int y = 0; y < b->p.ny; y++)
      for (int x = 0; x < b->p.nx; x++) {
        const long m = nidx(b, x, y, z);
        const int q[3] = {x, y, z};
        if (!in_interior(b, q)) {
          if (rho) rho[m] = b->p.rho0;
          if (u) u[3 * m] = u[3 * m + 1] = u[3 * m + 2] = 0.0;
          continue;
        }
        double r = 0.0, j[3] = {0, 0, 0};
        for (int i = 0; i < OR_Q; i++) {
          const double fi = b->f[i * b->nn + m];
          r += fi;
          for (int a = 0; a < 3; a++) j[a] += C[i][a] * fi;
        }
        if (rho) rho[m] = r;
        if (u)
          for (int a = 0; a < 3; a++) u[3 * m + a] = j[a] / r;
      }
}

int or_n_beads(const or_box* b) {
  int n = 0;
  for (int c = 0; c < b->n_chains; c++) n += b->chains[c].nb;
  return n;
}

void or_read_beads(const or_box* b, double* pos, double* vel) {
  long o = 0;
  for (int c = 0; c < b->n_chains; c++) {
    const chain_t* ch = &b->chains[c];
    if (pos) memcpy(pos + o, ch->pos, sizeof(double) * 3 * ch->nb);
    if (vel) memcpy(vel + o, ch->vel, sizeof(double) * 3 * ch->nb);
    o += 3 * ch->nb;
  }
}

void or_read_mass_mom(const or_box* b, double out[5]) { memcpy(out, b->mass_mom, sizeof(b->mass_mom)); }

void or_read_last_force(const or_box* b, double* g) {
  memcpy(g, b->g, sizeof(double) * (size_t)b->nn * 3);
}

/* ------------------------------------------------------------- vorticity */
/* The paper validates the fine box against the DNS through the vorticity
 * magnitude |omega| = |curl u|, averaged over a control volume around the
 * tracer (Sec. 3, Figs. 1 and 2).  Here u = j/rho is the velocity of the
 * pre-collision moments at t_n (the readout's u), and each derivative is the
 * second-order central difference (d u_c/d x_a)(q) = (u_c(q + e_a) -
 * u_c(q - e_a)) / 2.  It is defined at nodes whose six axis neighbours are
 * interior (periodic axes wrap). */
static void node_u(const or_box* b, long m, double u[3]) {
  double r = 0.0, j[3] = {0, 0, 0};
  for (int i = 0; i < OR_Q; i++) {
    const double fi = b->f[i * b->nn + m];
    r += fi;
    for (int a = 0; a < 3; a++) j[a] += C[i][a] * fi;
  }
  for (int a = 0; a < 3; a++) u[a] = j[a] / r;
}

static int vort_defined(const or_box* b, const int q[3]) {
  if (!in_interior(b, q)) return 0;
  for (int a = 0; a < 3; a++)
    for (int s = -1; s <= 1; s += 2) {
      int n[3] = {q[0], q[1], q[2]};
      n[a] = is_periodic(b, a) ? wrap(n[a] + s, axis_n(b, a)) : n[a] + s;
      if (!in_interior(b, n)) return 0;
    }
  return 1;
}

/* |curl u| at a defined node q */
static double node_vorticity(const or_box* b, const int q[3]) {
  double du[3][3]; /* du[c][a] = d u_c / d x_a */
  for (int a = 0; a < 3; a++) {
    int qp[3] = {q[0], q[1], q[2]}, qm[3] = {q[0], q[1], q[2]};
    qp[a] = wrap(q[a] + 1, axis_n(b, a));
    qm[a] = wrap(q[a] - 1, axis_n(b, a));
    double up[3], um[3];
    node_u(b, nidx(b, qp[0], qp[1], qp[2]), up);
    node_u(b, nidx(b, qm[0], qm[1], qm[2]), um);
    for (int c = 0; c < 3; c++) du[c][a] = 0.5 * (up[c] - um[c]);
  }
  const double wx = du[2][1] - du[1][2];
  const double wy = du[0][2] - du[2][0];
  const double wz = du[1][0] - du[0][1];
  return sqrt(wx * wx + wy * wy + wz * wz);
}

int or_vorticity(const or_box* b, double* out) {
  int count = 0;
  for (int z = 0; z < b->p.nz; z++)
    for (int y = 0; y < b->p.ny; y++)
      for (int x = 0; x < b->p.nx; x++) {
        const int q[3] = {x, y, z};
        const long m = nidx(b, x, y, z);
        if (vort_defined(b, q)) {
          out[m] = node_vorticity(b, q);
          count++;
        } else {
          out[m] = 0.0;
        }
      }
  return count;
}

int or_vorticity_mean(const or_box* b, const int lo[3], const int hi[3], double* mean) {
  for (int a = 0; a < 3; a++)
    if (lo[a] > hi[a] || lo[a] < 0 || hi[a] >= axis_n(b, a)) return OR_ERR_ARG;
  double s = 0.0;
  long n = 0;
  for (int z = lo[2]; z <= hi[2]; z++)
    for (int y = lo[1]; y <= hi[1]; y++)
      for (int x = lo[0]; x <= hi[0]; x++) {
        const int q[3] = {x, y, z};
        if (!vort_defined(b, q)) return OR_ERR_ARG;
        s += node_vorticity(b, q);
        n++;
      }
  *mean = s / (double)n;
  return OR_OK;
}
