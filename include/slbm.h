/*
 * slbm.h -- C ABI of the MI355X solid lattice-Boltzmann library (libslbm.so).
 *
 * The library advances plates of isotropic linear-elastic material with the
 * lattice-Boltzmann method of Faust, Schlueter, H. Mueller and R. Mueller,
 * "Dirichlet and Neumann boundary conditions in a Lattice Boltzmann Method
 * for Elastodynamics" (2022).  The problem it accepts is the paper's
 * statement in section 2: a domain, Lame parameters lambda and mu, density
 * rho, a body force F, and Dirichlet (eq:bcdir, given as the wall velocity
 * d(u*)/dt, eq:bcchaindir) or Neumann (eq:bcneu, traction t*) data on the
 * boundary.  One time step (section 3) is: moments (eq:moments), source term
 * with the density gradient (eq:sourceterm), equilibrium (eq:fieq), BGK
 * collision with forcing (eq:coll), streaming (eq:stream), integration of
 * the displacement from j, and the local boundary rules of section 4 on
 * every cut link (eq:bbcon/eq:bbnoncon, eq:abbcon/eq:abbnoncon, with the
 * boundary Poisson stress of eq:trafocauchy, eq:bcchainneum, eq:approxdiv).
 *
 * Conventions
 *   Sites sit at integer coordinates (ix, iy), 0 <= ix < nx, 0 <= iy < ny;
 *   host arrays are row-major with site index iy*nx + ix.  D2Q9 directions:
 *   0 (0,0), 1 (1,0), 2 (0,1), 3 (-1,0), 4 (0,-1), 5 (1,1), 6 (-1,1),
 *   7 (-1,-1), 8 (1,-1).  A link (x, k) is cut when the segment from x to
 *   x + c_k crosses a wall; q = s_k/l_k in (0, 1] is the fraction of the link
 *   between x and the wall (1/2 for a straight wall half-way between sites).
 *
 * Units
 *   User units with dx = 1 cell.  The lattice runs at c_s^2 = 1/3, so the
 *   time step is dt = sqrt(rho/(3 mu)) (paper, section 5.1).  Stresses and
 *   tractions scale with 3 mu, velocities with dx/dt.  Displacements are
 *   returned in cells.
 *
 * Ownership and threading
 *   The library copies every input during slbm_create; the caller may free
 *   them on return.  It owns all device memory and frees it in slbm_destroy.
 *   Output buffers belong to the caller.  A handle must not be used from two
 *   threads at once.  Work is queued on the handle's HIP stream; calls that
 *   return data to the host synchronise that stream.
 *
 * Errors
 *   Every function returns an slbm_status.  Nothing throws across the ABI.
 *   slbm_last_error() gives a thread-local message for the last failure.
 */
#ifndef SLBM_H
#define SLBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SLBM_OK = 0,
    SLBM_E_INVAL = -1,       /* invalid argument or inconsistent geometry */
    SLBM_E_NOMEM = -2,       /* device or host allocation failed */
    SLBM_E_DEVICE = -3,      /* a HIP call failed */
    SLBM_E_DIVERGED = -4,    /* a non-finite value, or |drho| + |j| >= rho0 (lattice units), appeared */
    SLBM_E_UNSUPPORTED = -5, /* valid request the library does not handle */
    SLBM_E_BUDGET = -6       /* a batch has no room for the plate */
} slbm_status;

typedef enum {
    SLBM_FP64 = 0,           /* fp64 populations and arithmetic */
    SLBM_FP32 = 1            /* fp32 populations and arithmetic, fp64 displacement */
} slbm_precision;

typedef enum { SLBM_DIRICHLET = 1, SLBM_NEUMANN = 2 } slbm_bc_kind;
typedef enum { SLBM_PROFILE_STEP = 0, SLBM_PROFILE_RAMP = 1 } slbm_profile;

/* A boundary-condition group.  DIRICHLET: value = wall velocity d(u*)/dt;
 * NEUMANN: value = traction t* = sigma n.  Both in user units.  STEP: on
 * from t = 0.  RAMP: scaled by min(t/ramp_time, 1). */
typedef struct {
    int32_t kind;
    int32_t profile;
    double value[2];
    double ramp_time;
} slbm_bc_group;

/* A cut link (x, dir).  normal is the outward unit normal of the material at
 * the crossing.  A link through the meeting point of two walls (a plate
 * corner, the mouth of an edge crack) names the second wall in group2 and
 * normal2; otherwise group2 = -1.  At such a link a Dirichlet wall wins over
 * a Neumann one; two Neumann walls fix the whole boundary stress,
 * sigma* = sym(t_A n_A + t_B n_B). */
typedef struct {
    int32_t site;            /* iy*nx + ix of the material site x */
    int32_t dir;             /* 1..8 */
    double q;                /* (0, 1] */
    int32_t group;
    int32_t group2;
    double normal[2];
    double normal2[2];
} slbm_link;

typedef struct {
    int32_t nx, ny;          /* sites, each >= 1; at most 2^28 in total */
    double lambda, mu, rho;  /* user units, dx = 1 cell */
    double tau;              /* BGK relaxation time in units of dt, > 1/2 */
    double body_force[2];    /* uniform body force per volume, user units */
    int32_t periodic_x, periodic_y;  /* 1: wrap; cut links never cross a periodic seam */
    int32_t precision;       /* slbm_precision */
    int32_t neumann_order;   /* 1: boundary density and tangential stress
                                extrapolated along the link (the paper's rule);
                                0: taken at the boundary site */
    const uint8_t* mask;     /* [ny*nx] 1 = material */
    int32_t n_links;
    const slbm_link* links;  /* every cut link of every material site, any order */
    int32_t n_groups;
    const slbm_bc_group* groups;
    int32_t device;          /* HIP device ordinal */
    void* stream;            /* hipStream_t to queue work on; NULL: the library's own */
} slbm_params;

typedef struct slbm_s* slbm_handle;

/* Validates and copies the problem, uploads it and sets the rest state
 * (zero displacement and velocity, unstressed).  SLBM_E_INVAL when a cut link
 * names a void site, an uncut link leaves the material, q is outside (0, 1],
 * a normal is not a unit vector, a group index is out of range, a material
 * site has all 8 links cut (an isolated site: the kernels keep one flag byte
 * per site, whose all-ones value marks a void site), tau <= 1/2, or mu,
 * rho <= 0.  SLBM_E_UNSUPPORTED above 2^28 sites; SLBM_E_NOMEM or
 * SLBM_E_DEVICE if allocation fails. */
int slbm_create(const slbm_params* params, slbm_handle* out);

/* Replaces the state by the equilibrium of given fields (section 2: P from
 * eq:poissonstress with div u from eq:approxdiv; j = rho v).  Host arrays in
 * user units, each may be NULL for its rest value: rho [n], vel [2][n],
 * sigma [3][n] (xx, yy, xy), u [2][n] cells.  Resets the step counter. */
int slbm_init_fields(slbm_handle h, const double* rho, const double* vel,
                     const double* sigma, const double* u);

/* Queues nsteps time steps on the handle's stream and returns.  One step is
 * the lattice-Boltzmann equation eq:LBE of section 3 -- moments
 * (eq:moments), source term (eq:sourceterm), equilibrium (eq:fieq), BGK
 * collision with forcing (eq:coll), streaming (eq:stream) -- with the rules
 * of section 4 on the cut links and the displacement advanced by j/rho
 * (section 2, u obtained by integrating j).  SLBM_E_INVAL for nsteps < 0 or
 * a plate owned by a batch. */
int slbm_step(slbm_handle h, int64_t nsteps);

/* Waits for queued work; SLBM_E_DIVERGED once any step produced a value
 * that is not finite, or a site whose density deviation and momentum reach
 * the rest density, |drho| + |j| >= rho0 in lattice units -- far outside
 * linear elasticity (checked on every site at every step).  The method is
 * explicit and conditionally stable (section 3 sets tau_bar for stability;
 * the Neumann rule of section 4 can grow a surface mode on traction-free
 * walls), so a run can overflow; the flag stays set until slbm_init_fields
 * or slbm_load. */
int slbm_sync(slbm_handle h);

/* Moments of the current state in user units, host arrays [n] / [2][n] /
 * [3][n] (xx, yy, xy); any pointer may be NULL.  j includes the S/2 part of
 * eq:moments; sigma = -P + (lambda - mu)(rho0 - rho)/rho0 I.  Void sites
 * read zero.  Synchronises. */
int slbm_moments(slbm_handle h, double* rho, double* j, double* P, double* sigma);

/* Displacement [2][n] in cells, host array: u is not a variable of the
 * lattice-Boltzmann state (section 2: it is obtained by integrating
 * j = rho du/dt), so the library sums j/rho every step and reads out with
 * the trapezoid rule, u^n = U^n + j^n/(2 rho^n).  Void sites read zero.
 * Synchronises. */
int slbm_displacement(slbm_handle h, double* u);

/* Same as slbm_displacement into device memory u_dev ([2][n] doubles) on
 * the handle's stream, without synchronising. */
int slbm_displacement_device(slbm_handle h, void* u_dev);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * displacement as slbm_displacement_device, into device memory u_dev
 * ([2][n] doubles, the caller's), queued on the handle's stream, without
 * synchronising, and with no device allocation or free: its density
 * scratch is a fixed 144 MiB array in the library's code object, one per
 * device, so plates whose padded plane ((ny + 2) rows of nx + 65 sites
 * rounded up to a multiple of 64) exceeds 18874368 sites return
 * SLBM_E_INVAL (a 4096 x 4096 plate fits).  Every call on a device uses
 * that device's one array: calls that may overlap on one device (on
 * different streams, or from different threads) race and must be ordered by
 * the caller.  SLBM_E_INVAL for a null pointer. */
int slbm_displacement_device_noalloc(slbm_handle h, void* u_dev);

/* Same as slbm_moments into device memory on the handle's stream, without
 * synchronising: rho_dev [n], j_dev [2][n], P_dev [3][n], sigma_dev [3][n]
 * (any pointer may be NULL), each an array of doubles (dtype SLBM_FP64) or
 * floats (SLBM_FP32, the double values rounded to nearest).  The arrays
 * belong to the caller and must be device memory on the handle's device,
 * valid until the queued work has run.  SLBM_E_INVAL for another dtype. */
int slbm_moments_device(slbm_handle h, void* rho_dev, void* j_dev, void* P_dev, void* sigma_dev, int dtype);

/* Step count and physical time of the current state: t = step * dt with
 * dt = sqrt(rho/(3 mu)) (section 5.1, c_s = dx/(sqrt(3) dt)); either pointer
 * may be NULL. */
int slbm_time(slbm_handle h, int64_t* step, double* t_user);

/* Launch shape of the fused step.  A workgroup advances a tile of seg_rows
 * rows (one wave per row, plus two waves for the density-halo rows) of one
 * strip of columns; strip is the strip width (62: two halo lanes per wave;
 * 64: aligned columns, the halo columns gathered by each wave).  strip 58
 * takes two time steps per launch: the tile's first step is kept in LDS and
 * the state is read and written once per two steps (seg_rows + 6 waves per
 * tile, 58 output columns; an odd step count ends with one single step).
 * seg_rows is at most 14 (10 with strip 58); 0 keeps the library's choice.
 * With strip 58 the library also lists, per tile, the plate's cut links in
 * the tile's reach (slbm_boundary_lists), so that the tile evaluates the
 * section 4 rules of all of them together; it allocates device memory for
 * the lists (SLBM_E_NOMEM if none is left).  SLBM_E_INVAL beyond the limits.
 * Results do not depend on the shape. */
int slbm_set_launch(slbm_handle h, int32_t seg_rows, int32_t strip);

/* The per-tile cut-link lists of the two-steps-per-launch step (strip 58):
 * the rows per tile they were built for (0: none, and the step evaluates the
 * boundary rules of section 4 site by site), the records in all lists, and
 * the most in one tile.  Lists are kept only when every tile's fits the
 * tile's LDS and workgroup (576 records, and one per thread: 64 (rows + 6))
 * and the plate has at most 64 BC groups; a cut link appears in every tile
 * whose rows and columns, halo included, reach its site.  Any pointer may be
 * NULL. */
int slbm_boundary_lists(slbm_handle h, int32_t* rows, int64_t* records, int32_t* max_per_tile);

/* Host only (no device call): the layout of those lists for an nx x ny grid
 * (periodic_x, periodic_y as in slbm_params) and tiles of `rows` rows (1 to
 * 10) of 58-column strips.  Tile t (strip fastest) reaches rows y0 - 3 ..
 * y0 + rows + 2 and columns xs - 3 .. xs + 60 (y0 = rows (t / strips),
 * xs = 58 (t mod strips)), wrapping on periodic axes; wave w and lane l of the
 * tile hold row y0 - 3 + w and column xs - 3 + l.  Every cut link i (its site
 * link_sites[i] = y nx + x, as slbm_link.site) appears in each tile whose
 * reach holds its site, once per image of the site there.  Writes
 * tile_start[0 .. n_tiles] (tile t's records are tile_start[t] ..
 * tile_start[t + 1]), and for each record the link index (rec_link) and the
 * position w << 8 | l (rec_pos), `capacity` entries at most (SLBM_E_INVAL if
 * there are more; pass NULL arrays to get the counts first).  Any pointer may
 * be NULL.  SLBM_E_INVAL for a bad grid, rows or site. */
int slbm_tile_list_layout(int32_t nx, int32_t ny, int32_t periodic_x, int32_t periodic_y, int32_t rows,
                          int32_t n_links, const int32_t* link_sites, int32_t* tile_start, int32_t* rec_link,
                          int32_t* rec_pos, int64_t capacity, int64_t* n_tiles, int64_t* n_records,
                          int32_t* max_per_tile);

/* How the step's workgroups are dealt to the GPU's 8 XCDs: 0 (the default)
 * gives each XCD one contiguous band of tiles; group g, a power of two up to
 * 64, gives each XCD groups of g consecutive workgroups, the groups of the
 * XCDs interleaved.
 * Bands keep the rows neighbouring tiles share in one L2; interleaved groups
 * spread clusters of expensive boundary tiles (a hole, a crack) over all
 * XCDs.  Results do not depend on it.  SLBM_E_INVAL for other values. */
int slbm_set_xcd_group(slbm_handle h, int32_t group);

/* The launch configuration in use: rows per tile (0: the library's choice),
 * strip (0 default, 58, 62 or 64, as in slbm_set_launch) and XCD group (as in
 * slbm_set_xcd_group); any pointer may be NULL. */
int slbm_get_launch(slbm_handle h, int32_t* seg_rows, int32_t* strip, int32_t* xcd_group);

/* Times the fused step on this plate for each strip width (62, 64 and the
 * two-steps-per-launch 58) and a range of rows per tile (short bursts of
 * launches, the state restored after each) and keeps the fastest; then times
 * that shape with interleaved XCD groups of 8 and keeps them if they are at
 * least 1 % faster (else bands).  Reports the shape and its time per step in
 * microseconds (any pointer may be NULL); slbm_get_launch gives the XCD
 * group.  Synchronises.  The state and step count are unchanged. */
int slbm_autotune(slbm_handle h, int32_t* seg_rows, int32_t* strip, double* us_per_step);

/* Checkpoint of the full state of the time stepping of section 3 (the
 * populations, the displacement sum, the step count and the divergence
 * flag) in an opaque host buffer the caller owns.  With buf = NULL,
 * slbm_save only reports the size in *bytes; SLBM_E_INVAL when *bytes is
 * too small.  slbm_load restores it on a plate of the same size and
 * precision (SLBM_E_INVAL otherwise), so that stepping on gives results
 * bit-identical to an uninterrupted run.  Both synchronise. */
int slbm_save(slbm_handle h, void* buf, size_t* bytes);
int slbm_load(slbm_handle h, const void* buf, size_t bytes);

/* HBM bytes the handle holds on the device (populations, displacement,
 * geometry, link records and any readout scratch). */
int slbm_device_bytes(slbm_handle h, int64_t* bytes);

/* Waits for the handle's work and frees its device memory and stream (if
 * the library created it).  NULL is a no-op; SLBM_E_INVAL for a plate owned
 * by a batch (slbm_batch_remove frees those). */
int slbm_destroy(slbm_handle h);

/* ---------------------------------------------------------------- batches
 *
 * Many plates of uneven size and geometry, each the problem of sections 2-4
 * with its own geometry, material and loads, advanced together: one kernel
 * launch takes a step (or two, with strip 58) of every plate still running,
 * launches are queued as replays of a captured HIP graph, and each plate
 * keeps its own step count.  Plates join and leave between calls
 * (continuous batching).  Every plate of a batch has the batch's precision
 * and no periodic axis.  A plate's results are those it would have alone
 * (the arithmetic of each site does not depend on the batch).
 *
 * Device memory: the batch reserves its whole budget at creation and carves
 * every plate, and one readout scratch the plates share (sized for the
 * displacement readout of the largest plate; the full moments readout grows
 * it on demand), out of it, so slbm_batch_add fails rather than exceed the
 * budget, and no call while steps run allocates or frees device memory (a
 * removed plate's memory is reused once the work queued before its removal
 * has run).  Tables of a few bytes per tile and per plate sit outside the
 * budget.
 *
 * Streams: steps go to the batch's stream; plate creation and readouts of
 * batch plates to a second stream of the batch's, a readout after the
 * plate's last queued step, so admitting and reading out plates overlaps the
 * steps of the others.
 *
 * Divergence: from the launch after a plate's state turns non-finite, the
 * kernels skip its arithmetic (its steps are still counted); it is retired
 * (its remaining steps set to zero, so slbm_batch_poll lists it) at a later
 * batch call, once the copy of the divergence words queued with each step
 * call has arrived; slbm_sync on its handle reports SLBM_E_DIVERGED.  Not
 * thread-safe.
 */
typedef struct slbm_batch_s* slbm_batch;

/* hbm_budget_bytes of device memory, reserved now, hold the batch's plates;
 * stream as in slbm_params (NULL: the batch's own).  SLBM_E_NOMEM when the
 * budget cannot be reserved. */
int slbm_batch_create(int64_t hbm_budget_bytes, int32_t device, void* stream, slbm_batch* out);

/* Creates the plate (as slbm_create, on the batch's device, in its budget)
 * with nsteps steps to take, and returns its slot.  SLBM_E_BUDGET when the
 * plate, or the readout scratch its displacement needs, does not fit the
 * budget (nothing stays allocated then). */
int slbm_batch_add(slbm_batch b, const slbm_params* params, int64_t nsteps, int32_t* slot);

/* Queues k steps: every plate advances by min(k, its remaining steps)
 * (eq:LBE, sections 3-4).  Does not wait for the device. */
int slbm_batch_step(slbm_batch b, int64_t k);

/* Slots whose steps are all queued, or that were retired as diverged (up to
 * capacity written; *n_done = all).  Does not wait for the device. */
int slbm_batch_poll(slbm_batch b, int32_t* done_slots, int32_t capacity, int32_t* n_done);

/* The plate's handle, owned by the batch, for the readouts slbm_displacement,
 * slbm_displacement_device, slbm_moments, slbm_moments_device, slbm_sync,
 * slbm_save and slbm_time (queued behind the plate's steps); valid until the
 * plate is removed.  Calls that step or change the plate (slbm_step,
 * slbm_init_fields, slbm_load, slbm_autotune, slbm_set_launch,
 * slbm_set_xcd_group, slbm_destroy) return SLBM_E_INVAL on it. */
int slbm_batch_handle(slbm_batch b, int32_t slot, slbm_handle* h);
int slbm_batch_remaining(slbm_batch b, int32_t slot, int64_t* steps);

/* The plate's displacement [2][n] in cells, into a host array (slbm_displacement
 * of the slot's handle).  SLBM_E_INVAL for an empty slot.  Waits for the
 * plate's queued steps and its readout only. */
int slbm_batch_displacement(slbm_batch b, int32_t slot, double* u);

/* Removes the plate; its slot is reused at once and its memory once the work
 * queued before the call has run.  Does not wait for the device. */
int slbm_batch_remove(slbm_batch b, int32_t slot);

/* Launch shape of the batched step, for every plate: rows per tile (1..14,
 * 1..10 with strip 58) and strip width (62, 64, or 58: two steps per launch,
 * a plate with one step left taking one) as in slbm_set_launch.
 * SLBM_E_INVAL beyond the limits. */
int slbm_batch_set_launch(slbm_batch b, int32_t rows, int32_t strip);

/* How the batched launch deals its workgroups to the XCDs, as
 * slbm_set_xcd_group for one plate: 0 (the default) contiguous bands, g a
 * power of two up to 64 interleaved groups of g.  Results do not depend on
 * it.  SLBM_E_INVAL for other values. */
int slbm_batch_set_xcd_group(slbm_batch b, int32_t group);

/* The batched launch shape in use (any pointer may be NULL). */
int slbm_batch_get_launch(slbm_batch b, int32_t* rows, int32_t* strip, int32_t* xcd_group);

/* Picks the batched launch shape on the plates resident now: times a set of
 * shapes (two steps per launch at 4, 6, 8 and 10 rows, one step at 6, 10 and
 * 14 rows), then the best with XCD groups of 8 (kept when 1 % faster), each
 * over 32 steps after 32 that rebuild its tables and graph, while budget
 * steps last, comparing the time per material-site update of the plates
 * running in the timed steps.  The trial steps are real: every plate advances
 * by them (at most its remaining steps), exactly as it would in any shape.
 * Keeps and reports the fastest shape and its time per step of the whole
 * batch in microseconds (any pointer may be NULL).  Synchronises. */
int slbm_batch_autotune(slbm_batch b, int64_t max_steps, int32_t* rows, int32_t* strip, int32_t* xcd_group,
                        double* us_per_step);

/* Waits for everything queued on the batch's streams. */
int slbm_batch_sync(slbm_batch b);

/* Waits until at most in_flight of the batch's slbm_batch_step calls are
 * still queued or running (0: all have run), and retires the plates found
 * diverged meanwhile.  A loop that queues the next call before it waits
 * keeps the device busy while bounding how far the host runs ahead.
 * SLBM_E_INVAL for in_flight < 0. */
int slbm_batch_wait(slbm_batch b, int32_t in_flight);

/* Device memory in use in the budget (plates and readout scratch, including
 * blocks of removed plates not yet reusable) and the budget. */
int slbm_batch_bytes(slbm_batch b, int64_t* used, int64_t* budget);

/* Waits for the batch's work, then frees every plate and the budget.  NULL
 * is a no-op. */
int slbm_batch_destroy(slbm_batch b);

/* Plain device-to-device copy of `bytes` (a multiple of 16, 16-byte aligned
 * pointers) queued on `stream` (NULL: the null stream) of `device`.  The
 * streaming reference the fused step's bandwidth is quoted against; not part
 * of the method. */
int slbm_copy(void* dst, const void* src, size_t bytes, int32_t device, void* stream);

const char* slbm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
