/*
 * slbm3.h -- C ABI of the three-dimensional (D3Q19) solid lattice-Boltzmann
 * step in libslbm.so.
 *
 * The paper (Faust, Schlueter, H. Mueller, R. Mueller, 2022) states its
 * method in two dimensions and notes that its local boundary rules carry
 * over to three (section 1).  This is that three-dimensional form: the same
 * moments (eq:moments), source term with the density gradient
 * (eq:sourceterm), equilibrium with the populations' own second moment
 * (eq:fieq), BGK collision with forcing (eq:coll), streaming (eq:stream) and
 * displacement integration, on the D3Q19 lattice (c_s^2 = 1/3, weights 1/3,
 * 1/18, 1/36).
 *
 * Geometry
 *   A box of nx x ny x nz sites at integer coordinates, periodic in y and z.
 *   In x it is either periodic or closed by two walls, planes normal to x
 *   that cross every link leaving the material at the fraction q of its
 *   length (section 4: q = 1/2 gives the lattice-conforming planes
 *   x = -1/2 and x = nx - 1/2; in general the planes are x = -q and
 *   x = nx - 1 + q).  A Dirichlet wall carries a wall velocity, with the
 *   rule of eq:bbcon (q = 1/2) or eq:bbnoncon (j* = rho(x) v*).  A Neumann
 *   wall carries a traction t* (the stress times the outward normal of the
 *   material: -x at the first wall, +x at the second), with the rule of
 *   eq:abbcon or eq:abbnoncon.  That rule's boundary Cauchy stress is
 *   sigma* = Pi sigma_b Pi + n t* + t* n - (t*.n) n n, with Pi = I - n n; its
 *   tangential block sigma_b, and rho_bd, are those at the boundary site
 *   (neumann_order 0) or extrapolated along the link from the site behind,
 *   (1 + q) X(x) - q X(x - c_i) (neumann_order 1, the paper's form).  The
 *   rules at q != 1/2 read the population at x - c_i, the next site inward;
 *   a one-site-wide slab has none and takes kappa = 0, beta = 1.  A wall's or
 *   group's value is on from the first step (SLBM_PROFILE_STEP) or ramped,
 *   scaled by min(t_n / ramp_time, 1) where t_n is the time of the
 *   post-collision state the rule reads (the rule that completes step n + 1).
 *
 *   Directions c_i (D3Q19): 0 rest; 1-6 +x -x +y -y +z -z; 7-10 (1,1,0)
 *   (-1,-1,0) (1,-1,0) (-1,1,0); 11-14 (1,0,1) (-1,0,-1) (1,0,-1) (-1,0,1);
 *   15-18 (0,1,1) (0,-1,-1) (0,1,-1) (0,-1,1).
 *
 *   General geometry: a box periodic on every axis with a material mask;
 *   void sites (cavities, notches) hold no material.  Each link from a
 *   material site into the void is cut where it leaves the material, at its
 *   own fraction q, with its own outward normal and boundary group; a link
 *   between two material sites may be cut too (a crack of zero thickness),
 *   listed from both sides, each face with its own q, normal and group.  A
 *   cut link takes the rule of its group as above (Dirichlet: eq:bbcon / eq:bbnoncon;
 *   Neumann: eq:abbcon / eq:abbnoncon with the traction t* = value -
 *   pressure n).  Where the opposite link at the same site is cut too there
 *   is no site behind: kappa = 0, beta = 1 and no extrapolation.  The density
 *   gradient takes 2 rho(x) - rho(x - c_i) across a cut link (rho(x) if both
 *   are cut).  Void sites report zero density, momentum, stress and
 *   displacement.
 *
 * Host arrays
 *   Arrays are [component][nz][ny][nx] of doubles, x fastest.  The site index
 *   is (iz*ny + iy)*nx + ix.  Vectors have three components (x, y, z).
 *   Symmetric tensors have six, in the order xx, yy, zz, xy, xz, yz.
 *
 * Units, ownership, threading and errors
 *   As in slbm.h: user units with dx = 1 and dt = sqrt(rho/(3 mu)); every
 *   input is copied and the library owns its device memory.  A handle is not
 *   shared between threads.  Work is queued on the handle's stream, and calls
 *   that return host data synchronise it.  The status codes and
 *   slbm_last_error() are those of slbm.h.
 */
#ifndef SLBM3_H
#define SLBM3_H

#include <stddef.h>
#include <stdint.h>

#include "slbm.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct slbm3_s* slbm3_handle;

typedef struct {
    int32_t kind;                /* SLBM_DIRICHLET (value: wall velocity) or SLBM_NEUMANN (value: traction) */
    double value[3];             /* user units */
    double q;                    /* fraction of a cut link inside the material, (0, 1]; 1/2: lattice-conforming */
    int32_t profile;             /* SLBM_PROFILE_STEP (on from t = 0) or SLBM_PROFILE_RAMP */
    double ramp_time;            /* RAMP: value scaled by min(t / ramp_time, 1), user units, > 0 */
} slbm3_wall;

/* One cut link of a general geometry (80 bytes): the link from the material
 * site x to x + c_dir, whose far end is void (or material across a crack),
 * crossing the boundary at the fraction q of its length.  A link that leaves
 * through the edge where two faces meet (both crossed at the same point)
 * carries the second face too: there the Dirichlet face wins, and two
 * Neumann faces fix the rows of both normals of sigma* (in the frame n, n2,
 * e = n x n2, the shear between them averaged), sigma*_ee taken from the
 * material as the tangential block is for one face. */
typedef struct {
    int32_t site;                /* (iz*ny + iy)*nx + ix of x, a material site */
    int32_t dir;                 /* direction i of the link, 1..18 (order above) */
    double q;                    /* (0, 1] */
    int32_t group;               /* index into slbm3_params.groups */
    double normal[3];            /* outward unit normal of the material where the link crosses */
    int32_t group2;              /* the second face's group at an edge, or -1 */
    double normal2[3];           /* its outward unit normal, orthogonal to normal (ignored when group2 = -1) */
} slbm3_link;

/* Boundary data shared by a group of cut links, user units. */
typedef struct {
    int32_t kind;                /* SLBM_DIRICHLET (value: wall velocity) or SLBM_NEUMANN */
    double value[3];             /* Dirichlet: wall velocity; Neumann: traction, t* = value - pressure n */
    double pressure;             /* Neumann: uniform pressure on the boundary (0: none); ignored for Dirichlet */
    int32_t profile;             /* SLBM_PROFILE_STEP or SLBM_PROFILE_RAMP (value and pressure scaled) */
    double ramp_time;            /* RAMP: min(t / ramp_time, 1), user units, > 0 */
} slbm3_bc_group;

typedef struct {
    int32_t nx, ny, nz;          /* sites, each >= 1; at most 2^29 in total */
    double lambda, mu, rho;      /* user units; mu > 0, rho > 0, lambda > -mu */
    double tau_bar;              /* relaxation time in units of dt, > 1/2 */
    double body_force[3];        /* per volume, user units */
    int32_t periodic_x;          /* 1: periodic in x; 0: the two walls below */
    slbm3_wall walls[2];         /* crossing the links of the first and the last sites in x (ignored when periodic_x) */
    int32_t neumann_order;       /* 0: rho_bd and the tangential stress at the boundary site; 1: extrapolated */
    /* General geometry (needs periodic_x = 1; NULL mask: none): */
    const uint8_t* mask;         /* [nz][ny][nx], nonzero: material, 0: void */
    int64_t n_links;             /* every link from a material site into the void, and both sides of each crack, once */
    const slbm3_link* links;     /* any order */
    int32_t n_groups;
    const slbm3_bc_group* groups;
    int32_t precision;           /* SLBM_FP64, or SLBM_FP32 (fp32 populations and arithmetic, fp64 U) */
    int32_t device;              /* HIP device ordinal */
    void* stream;                /* hipStream_t to queue work on; NULL: a stream owned by the handle */
} slbm3_params;

/* Creates a box at rest (f = f_eq(rho, 0, 0), U = 0, step 0).  SLBM_E_INVAL
 * for invalid parameters, SLBM_E_UNSUPPORTED above 2^29 sites or with more
 * than 15 distinct ramp times among the groups, SLBM_E_NOMEM or
 * SLBM_E_DEVICE if allocation fails; *out is NULL on failure.  With a mask
 * SLBM_E_INVAL also names the first invalid link: a site out of range or
 * void, a direction out of 1..18, q outside (0, 1], a group out of range, a
 * normal that is not a unit vector (to 1e-9), a second group out of range
 * or its normal not a unit vector orthogonal to the first, the two faces of
 * an edge with different time profiles, a link listed twice, a link into the
 * material whose link back is not listed, or a link from the material into
 * the void that is not listed; and a group with an invalid kind, a bad
 * profile or a ramp time that is not positive.
 * The arrays are copied. */
int slbm3_create(const slbm3_params* params, slbm3_handle* out);

/* Sets the state from fields (any pointer may be NULL: density rho, velocity
 * 0, stress 0, displacement 0):
 *   f = f_eq(rho, rho v - S/2, P), with P = -sigma + (lambda - mu)(1 - rho/rho0) I;
 *   U = u - (j/rho)/2.
 * The step count is reset to 0.  Arrays: rho [n], vel [3][n], sigma [6][n],
 * u [3][n].  SLBM_E_INVAL for a non-positive density.  Synchronises. */
int slbm3_init_fields(slbm3_handle h, const double* rho, const double* vel, const double* sigma,
                      const double* u);

/* Queues nsteps time steps (two launches each). */
int slbm3_step(slbm3_handle h, int64_t nsteps);

/* Waits for queued work.  SLBM_E_DIVERGED if a step produced a non-finite
 * value, or a site with |drho| + |j| >= rho0 (lattice units, far outside
 * linear elasticity), since creation or the last slbm3_init_fields. */
int slbm3_sync(slbm3_handle h);

/* Moments of the current state, in user units.  These are the density rho
 * [n], the momentum j [3][n] (with the half source term, eq:moments), the
 * second moment P [6][n] and the Cauchy stress sigma [6][n]
 * (eq:poissonstress with eq:approxdiv).  Any output pointer may be NULL.
 * Synchronises. */
int slbm3_moments(slbm3_handle h, double* rho, double* j, double* P, double* sigma);

/* Displacement u [3][n] in cells: U + (j/rho)/2, the trapezoid rule for the
 * integral of j/rho.  Synchronises. */
int slbm3_displacement(slbm3_handle h, double* u);

/* Same as slbm3_displacement into device memory u_dev ([3][n] doubles) on
 * the handle's stream, without synchronising; u_dev belongs to the caller and
 * must stay valid until the queued work has run. */
int slbm3_displacement_device(slbm3_handle h, void* u_dev);

/* Same as slbm3_moments into device memory on the handle's stream, without
 * synchronising: rho [n], j [3][n], P [6][n], sigma [6][n] (any pointer may be
 * NULL), each an array of doubles (dtype SLBM_FP64) or floats (SLBM_FP32, the
 * double values rounded to nearest).  SLBM_E_INVAL for another dtype. */
int slbm3_moments_device(slbm3_handle h, void* rho_dev, void* j_dev, void* P_dev, void* sigma_dev, int dtype);

/* Steps taken since creation or the last slbm3_init_fields, and that time in
 * user units. */
int slbm3_time(slbm3_handle h, int64_t* step, double* t_user);

/* Device memory held by the handle, in bytes. */
int slbm3_device_bytes(slbm3_handle h, int64_t* bytes);

/* Checkpoint and resume: slbm3_save writes the whole state (populations,
 * the displacement sums, the step count, the divergence flag and, with cut
 * links, the rule values the next step reads) into the caller's host buffer
 * of *bytes bytes and sets *bytes to the size used; with buf NULL it only
 * reports the size.  SLBM_E_INVAL when *bytes is too small.  slbm3_load
 * restores a checkpoint on a handle created with the same box, geometry and
 * precision (SLBM_E_INVAL otherwise: the checkpoint carries a fingerprint of
 * the mask and the cut links, or of the walls), so that stepping on gives
 * results bit-identical to an uninterrupted run.  Loads and time profiles
 * may differ; the rule values saved with the state were formed with the
 * saving handle's.  Both synchronise. */
int slbm3_save(slbm3_handle h, void* buf, size_t* bytes);
int slbm3_load(slbm3_handle h, const void* buf, size_t bytes);

/* Frees the handle and its device memory after the queued work; NULL is a
 * no-op. */
int slbm3_destroy(slbm3_handle h);

#ifdef __cplusplus
}
#endif

#endif
