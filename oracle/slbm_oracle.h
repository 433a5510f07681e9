/*
 * slbm_oracle.h -- plain CPU reference of the solid lattice-Boltzmann step.
 *
 * TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg load this library.  It shares no source with
 * the HIP library and is never a fallback for it.
 *
 * Method: Faust, Schlueter, H. Mueller, R. Mueller, "Dirichlet and Neumann
 * boundary conditions in a Lattice Boltzmann Method for Elastodynamics"
 * (2022), sections 2-4.  One time step is, in the paper's order:
 * moments (eq:moments) -> source term S with the density gradient
 * (eq:sourceterm) -> equilibrium (eq:fieq) -> BGK collision with forcing
 * (eq:coll) -> displacement integration of j -> streaming (eq:stream) ->
 * local boundary rules on cut links (eq:bbcon/eq:bbnoncon for Dirichlet,
 * eq:abbcon/eq:abbnoncon for Neumann, boundary Poisson stress from
 * eq:trafocauchy, eq:bcchainneum, eq:approxdiv).
 *
 * Units: inputs are user units with dx = 1 cell; internally the lattice has
 * dx = dt = 1, rho0 = 1 and c_s^2 = 1/3, so dt_user = sqrt(rho/(3 mu)).
 *
 * All functions are single-threaded per call except that loops over rows may
 * run under OpenMP; results do not depend on the thread count.
 */
#ifndef SLBM_ORACLE_H
#define SLBM_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORACLE_DIRICHLET = 1, ORACLE_NEUMANN = 2 };
enum { ORACLE_PROFILE_STEP = 0, ORACLE_PROFILE_RAMP = 1 };

typedef struct {
    int32_t nx, ny;
    double lam, mu, rho;          /* Lame parameters and density, user units */
    double tau;                   /* relaxation time in units of dt, > 1/2 */
    double force[2];              /* body force per volume, user units */
    int32_t periodic_x, periodic_y;
    int32_t neumann_order;        /* 1: rho_bd and sigma_tt extrapolated along
                                   * the link as in the paper; 0: taken at x */
    const uint8_t* mask;          /* [ny*nx], 1 = material site */
    int32_t n_links;              /* cut links (x, k), see slbm_workloads */
    const int32_t* link_site;     /* [n_links] iy*nx + ix */
    const int32_t* link_dir;      /* [n_links] k in 1..8 */
    const double* link_q;         /* [n_links] s/l in (0, 1] */
    const int32_t* link_group;    /* [n_links] */
    const int32_t* link_group2;   /* [n_links] second wall at a corner, or -1 */
    const double* link_normal;    /* [n_links][2] outward unit normal */
    const double* link_normal2;   /* [n_links][2] */
    int32_t n_groups;
    const int32_t* group_kind;    /* [n_groups] ORACLE_DIRICHLET | ORACLE_NEUMANN */
    const double* group_value;    /* [n_groups][2] wall velocity or traction */
    const int32_t* group_profile; /* [n_groups] */
    const double* group_ramp_time;/* [n_groups] user time units */
} oracle_problem;

typedef struct oracle_s oracle_t;

/* Returns NULL and writes a message into err on invalid input. */
oracle_t* oracle_create(const oracle_problem* p, char* err, int errlen);
void oracle_destroy(oracle_t* o);

/* Initial state from fields in user units (any pointer may be NULL: rest
 * value).  rho [n], vel [2][n], sigma [3][n] (xx, yy, xy), u [2][n] cells.
 * The populations are set to the equilibrium of (rho, j, P) with P from the
 * Poisson-stress relation and the divergence approximation. */
int oracle_init_fields(oracle_t* o, const double* rho, const double* vel,
                       const double* sigma, const double* u);

void oracle_step(oracle_t* o, int64_t nsteps);
int64_t oracle_step_count(const oracle_t* o);

/* Moments of the current state in user units; any pointer may be NULL.
 * rho [n], j [2][n] (with the S/2 correction), P [3][n], sigma [3][n].
 * Void sites get zeros. */
void oracle_moments(const oracle_t* o, double* rho, double* j, double* P, double* sigma);
/* Displacement in cells, trapezoid readout of the integrated velocity. */
void oracle_displacement(const oracle_t* o, double* u);

/* Lattice-unit access for unit tests: populations f [9][n]. */
void oracle_get_populations(const oracle_t* o, double* f);
void oracle_set_populations(oracle_t* o, const double* f);
/* lattice parameters: {lam_L, mu_L, tau, dt_user, stress scale, velocity scale} */
void oracle_lattice_params(const oracle_t* o, double* out6);
/* The equilibrium of eq:fieq in lattice units, P = {xx, yy, xy}. */
void oracle_equilibrium(double rho, const double* j, const double* P, double* feq9);

/* Number of OpenMP threads later calls may use (0 or less: the runtime's
 * default).  Returns the number in effect.  Results do not depend on it. */
int oracle_set_threads(int n);

#ifdef __cplusplus
}
#endif
#endif
