/* lb_oracle.h -- plain FP64 CPU oracle of the fine-box lattice-Boltzmann step.
 *
 * TEST INFRASTRUCTURE ONLY.  This oracle exists to check the GPU library; the
 * tests, the smoke check and the benchmark's CPU-baseline leg are the only
 * code allowed to load it.  It shares no source with the GPU path.
 *
 * What it computes (Lee, Duenweg, Schumacher, "Multiscale modelling strategy
 * using the lattice Boltzmann method for polymer dynamics in a turbulent
 * flow"):
 *   - the standard D3Q19 lattice Boltzmann model (Sec. 3), with BGK or the
 *     weighted-orthogonal multiple-relaxation-time collision of the LB review
 *     the paper cites for its model, with Guo-type forcing;
 *   - a prescribed initial field on all sites and a time-dependent velocity on
 *     the boundary only, both enforced by setting populations to local
 *     equilibrium (Sec. 2);
 *   - a bead-spring (FENE) chain coupled to the fluid by a Stokes friction
 *     coefficient (Sec. 1), with its centre of mass pinned (Sec. 2).
 *
 * Layout: populations f[i][z][y][x] (x fastest), i in the lattice order of
 * or_lattice().  Every function returns 0 or a negative status code.
 */
#ifndef LB_ORACLE_H
#define LB_ORACLE_H
#ifdef __cplusplus
extern "C" {
#endif

#define OR_Q 19

enum { OR_OK = 0, OR_ERR_ARG = -1, OR_ERR_OOM = -2, OR_ERR_FENE = -4,
       OR_ERR_BEAD_OUT = -5, OR_ERR_UNSTABLE = -6, OR_ERR_STATE = -7 };
enum { OR_BGK = 0, OR_MRT = 1 };
enum { OR_BC_AFFINE = 0, OR_BC_SAMPLED = 1 };

typedef struct {
  int nx, ny, nz;            /* nodes per axis, boundary layer included */
  unsigned periodic_mask;    /* bit a set: axis a is periodic (no boundary layer) */
  int collision;             /* OR_BGK or OR_MRT */
  double tau;                /* shear relaxation time, nu = (tau - 1/2)/3 */
  double tau_bulk;           /* MRT bulk relaxation time */
  double ghost_rate;         /* MRT ghost-mode relaxation rate */
  double rho0;               /* rest density, also the boundary density */
  int reduce_every;          /* K: record mass and momentum every K steps (0: never) */
} or_params;

typedef struct or_box or_box;

/* lattice tables: c[19][3] and w[19] */
void or_lattice(int c[OR_Q][3], double w[OR_Q]);
/* number of OpenMP threads a step uses (the oracle's host cores) */
int or_threads(void);
/* weighted-orthogonal MRT basis: e[k][i] = e_k(c_i), norms b[k] = sum_i w_i e_k(c_i)^2 */
void or_mrt_basis(double e[OR_Q][OR_Q], double b[OR_Q]);
/* node-level primitives */
void or_equilibrium(double rho, const double u[3], double feq[OR_Q]);
void or_collide(const or_params* p, const double f[OR_Q], const double g[3], double out[OR_Q]);
/* one LB step of a chain's molecular dynamics given the fluid velocity at each
 * bead (ubead[nb][3]); pos/vel updated in place, dp[nb][3] receives the
 * friction impulse per bead.  Returns OR_ERR_FENE on an overstretched bond
 * (pos/vel then hold partial results). */
int or_chain_md(int nb, int substeps, int fix_com, double zeta, double mass, double fene_k,
                double fene_r0, const double anchor[3], double* pos, double* vel,
                const double* ubead, double* dp);

/* or_chain_md with Langevin noise at temperature kT: rnd[substeps][nb][3]
 * unit-variance numbers (NULL when kT = 0) */
int or_chain_md_noise(int nb, int substeps, int fix_com, double zeta, double mass, double fene_k,
                      double fene_r0, const double anchor[3], double* pos, double* vel,
                      const double* ubead, double kT, const double* rnd, double* dp);
/* fluctuating MRT collision: mu = 3 kT, r[k] (k >= 4) unit-variance numbers */
void or_collide_noise(const or_params* p, const double f[OR_Q], const double g[3], double mu,
                      const double r[OR_Q], double out[OR_Q]);
/* Philox4x32-10 counter-based generator, and its map of 32 bits to a uniform
 * number of mean 0 and variance 1 */
void or_philox4x32(const unsigned ctr[4], const unsigned key[2], unsigned out[4]);
double or_unit_uniform(unsigned u);

or_box* or_create(const or_params* p);
void or_destroy(or_box* b);
/* f(x,0) = f_eq(rho0, u(x)) on interior nodes; u = [nz][ny][nx][3] or NULL (rest) */
int or_set_initial(or_box* b, const double* u);
/* overwrite the pre-collision populations at the current step, [19][nz][ny][nx] */
int or_set_populations(or_box* b, const double* f);
/* boundary source: AFFINE data = [n_samples][9] (row-major A), SAMPLED data =
 * [n_samples][6][res][res][3]; sample k belongs to step t0 + k dt */
int or_set_boundary(or_box* b, int mode, long t0, int dt, int n_samples, int res, const double* data);
/* append a chain; pos[nb][3] (lattice units), vel[nb][3] or NULL */
int or_add_chain(or_box* b, int nb, int substeps, int fix_com, double zeta, double mass,
                 double fene_k, double fene_r0, const double anchor[3], const double* pos,
                 const double* vel);
/* accelerated-frame body force (Sec. 2): the tracer acceleration a = dv/dt,
 * accel[n_samples][3] (lattice units) at steps t0 + k dt, linear in time
 * between samples; every interior node receives -rho a.  n_samples = 0 clears */
int or_set_body_force(or_box* b, long t0, int dt, int n_samples, const double* accel);
/* thermal fluctuations at kT (MRT only): fluctuating collision and bead
 * Langevin noise from Philox4x32-10 with key = seed and counters (node, box,
 * step, draw 0..3) for the fluid and (bead, box, step, 16 + substep) for beads */
int or_set_thermal(or_box* b, double kT, unsigned long long seed, unsigned box_index);
/* advance n steps; stops at and latches the first error */
int or_step(or_box* b, int n);
long or_get_step(const or_box* b);
void or_get_error(const or_box* b, int* code, long* step);
int or_boundary_velocity(const or_box* b, int x, int y, int z, long n, double u[3]);
void or_read_pop(const or_box* b, double* f);
void or_read_rho_u(const or_box* b, double* rho, double* u);
int or_n_beads(const or_box* b);
void or_read_beads(const or_box* b, double* pos, double* vel);
/* latest mass/momentum record: step, M, Px, Py, Pz */
void or_read_mass_mom(const or_box* b, double out[5]);
/* force density g[nz][ny][nx][3] spread onto the lattice in the last step */
void or_read_last_force(const or_box* b, double* g);
/* vorticity magnitude |curl u| of u = j/rho at t_n by central differences
 * (Sec. 3, Figs. 1-2): out[nz][ny][nx], 0 where a node's six axis neighbours
 * are not all interior; returns the number of nodes where it is defined */
int or_vorticity(const or_box* b, double* out);
/* its mean over the node range lo..hi (inclusive, x y z); OR_ERR_ARG if the
 * range holds a node where it is not defined */
int or_vorticity_mean(const or_box* b, const int lo[3], const int hi[3], double* mean);

#ifdef __cplusplus
}
#endif
#endif
