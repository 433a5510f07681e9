/*
 * slbm_oracle.c -- plain CPU reference of the solid lattice-Boltzmann step.
 *
 * TEST INFRASTRUCTURE (see slbm_oracle.h).  Written for a reader holding the
 * paper: every block names the equation it evaluates.  No blocking, no fusion
 * and no reordering beyond what the equations state; whole-lattice arrays are
 * written out between the stages of the algorithm.
 *
 * Populations f_i are stored unshifted, as in the paper.  `real` is double,
 * or long double with -DORACLE_EXTENDED (used where the comparison needs the
 * small deviation from the rest state resolved to better than fp64 allows).
 */
#ifdef _OPENMP
#include <omp.h>
#endif
#include "slbm_oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#ifdef ORACLE_EXTENDED
typedef long double real;
#else
typedef double real;
#endif

/* D2Q9 (paper, section 3, figure "lattice"): c_0 = 0, then the four axis
 * links and the four diagonals.  With this numbering the opposite of 5 is 7,
 * as in the paper's bounce-back example.  Weights are the standard D2Q9
 * ones, which give the isotropy c_s^2 = 1/3 the time-step rule relies on. */
static const int CX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int CY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const int OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};

static real W(int i)
{
    if (i == 0) return (real)4 / (real)9;
    if (i <= 4) return (real)1 / (real)9;
    return (real)1 / (real)36;
}

static const real CS2 = (real)1 / (real)3;   /* c_s^2 in lattice units */

struct oracle_s {
    int nx, ny, n, px, py, norder;
    /* lattice units */
    real lam, mu, tau, F[2];
    /* unit scales */
    double rho_user, mu_user, dt_user, s_sigma, s_v;
    uint8_t* mat;          /* [n] */
    int32_t* link_at;      /* [9][n]: index of cut link (x,k), else -1 */
    uint8_t* cutm;         /* [n]: bit k-1 set when link (x,k) is cut */
    int nl;
    int32_t *lsite, *ldir, *lgroup, *lgroup2;
    real *lq, *ln, *ln2;   /* q, normal [nl][2], normal2 [nl][2] */
    int ng;
    int32_t *gkind, *gprof;
    real* gval;            /* [ng][2] lattice units */
    double* gramp;         /* ramp length in steps */
    real *f, *fnew, *fcol; /* [9][n] */
    real* U;               /* [2][n] integrated velocity (cells) */
    real *rho, *jx, *jy, *Pxx, *Pyy, *Pxy, *Sx, *Sy;  /* [n] */
    int64_t step;
};

/* neighbour of site (x, y) along +c_k (sign = 1) or -c_k (sign = -1);
 * -1 outside the grid */
static int neighbour_xy(const oracle_t* o, int x, int y, int k, int sign)
{
    x += sign * CX[k];
    y += sign * CY[k];
    if (o->px) x = (x + o->nx) % o->nx;
    if (o->py) y = (y + o->ny) % o->ny;
    if (x < 0 || x >= o->nx || y < 0 || y >= o->ny) return -1;
    return y * o->nx + x;
}

static int neighbour(const oracle_t* o, int s, int k, int sign)
{
    return neighbour_xy(o, s % o->nx, s / o->nx, k, sign);
}

static void* xcalloc(size_t n, size_t sz)
{
    void* p = calloc(n ? n : 1, sz);
    if (!p) { fprintf(stderr, "oracle: out of memory\n"); abort(); }
    return p;
}

/* ------------------------------------------------------------------------
 * eq:fieq  f_i^eq = w_i ( rho + c_i.j / c_s^2
 *                         + (P - rho c_s^2 I):(c_i c_i - c_s^2 I) / (2 c_s^4) )
 */
static real feq_i(int i, real rho, real jx, real jy, real pxx, real pyy, real pxy)
{
    real cx = CX[i], cy = CY[i];
    real cj = cx * jx + cy * jy;
    real second = (pxx - rho * CS2) * (cx * cx - CS2)
                + (pyy - rho * CS2) * (cy * cy - CS2)
                + 2 * pxy * cx * cy;
    return W(i) * (rho + cj / CS2 + second / (2 * CS2 * CS2));
}

void oracle_equilibrium(double rho, const double* j, const double* P, double* feq9)
{
    for (int i = 0; i < 9; i++)
        feq9[i] = (double)feq_i(i, rho, j[0], j[1], P[0], P[1], P[2]);
}

/* Time profile of a boundary group at step m (the rule applied after the
 * collision of step m uses the value at t_m = m dt). */
static real profile(const oracle_t* o, int g, int64_t m)
{
    if (o->gprof[g] == ORACLE_PROFILE_RAMP) {
        real r = (real)m / (real)o->gramp[g];
        return r < 1 ? r : 1;
    }
    return 1;
}

/* ------------------------------------------------------------------------ */

oracle_t* oracle_create(const oracle_problem* p, char* err, int errlen)
{
#define FAIL(...) do { if (err) snprintf(err, errlen, __VA_ARGS__); oracle_destroy(o); return NULL; } while (0)
    oracle_t* o = (oracle_t*)xcalloc(1, sizeof(oracle_t));
    if (p->nx < 1 || p->ny < 1) FAIL("grid must be at least 1x1");
    if (!(p->mu > 0) || !(p->rho > 0)) FAIL("mu and rho must be positive");
    if (!(p->tau > 0.5)) FAIL("tau must exceed 1/2");
    o->nx = p->nx; o->ny = p->ny; o->n = p->nx * p->ny;
    o->px = p->periodic_x != 0; o->py = p->periodic_y != 0;
    if (p->neumann_order != 0 && p->neumann_order != 1) FAIL("neumann_order must be 0 or 1");
    o->norder = p->neumann_order;
    /* unit mapping: c_s = sqrt(mu/rho) = dx/(sqrt(3) dt) (paper, section 5.1) */
    o->rho_user = p->rho; o->mu_user = p->mu;
    o->dt_user = sqrt(p->rho / (3.0 * p->mu));
    o->s_sigma = 3.0 * p->mu;                 /* stress: rho dx^2/dt^2 */
    o->s_v = 1.0 / o->dt_user;                /* velocity: dx/dt */
    o->mu = (real)p->mu / (real)o->s_sigma;   /* = 1/3 */
    o->lam = (real)p->lam / (real)o->s_sigma;
    o->tau = (real)p->tau;
    o->F[0] = (real)p->force[0] / (real)o->s_sigma;
    o->F[1] = (real)p->force[1] / (real)o->s_sigma;

    int n = o->n;
    o->mat = (uint8_t*)xcalloc(n, 1);
    for (int s = 0; s < n; s++) o->mat[s] = p->mask[s] ? 1 : 0;

    o->ng = p->n_groups;
    o->gkind = (int32_t*)xcalloc(o->ng, sizeof(int32_t));
    o->gprof = (int32_t*)xcalloc(o->ng, sizeof(int32_t));
    o->gval = (real*)xcalloc(2 * o->ng, sizeof(real));
    o->gramp = (double*)xcalloc(o->ng, sizeof(double));
    for (int g = 0; g < o->ng; g++) {
        o->gkind[g] = p->group_kind[g];
        o->gprof[g] = p->group_profile[g];
        if (o->gkind[g] != ORACLE_DIRICHLET && o->gkind[g] != ORACLE_NEUMANN) FAIL("group %d: bad kind", g);
        double scale = o->gkind[g] == ORACLE_DIRICHLET ? o->s_v : o->s_sigma;
        o->gval[2 * g] = (real)p->group_value[2 * g] / (real)scale;
        o->gval[2 * g + 1] = (real)p->group_value[2 * g + 1] / (real)scale;
        if (o->gprof[g] == ORACLE_PROFILE_RAMP) {
            if (!(p->group_ramp_time[g] > 0)) FAIL("group %d: ramp time must be positive", g);
            o->gramp[g] = p->group_ramp_time[g] / o->dt_user;
        } else if (o->gprof[g] != ORACLE_PROFILE_STEP) {
            FAIL("group %d: bad profile", g);
        }
    }

    o->link_at = (int32_t*)xcalloc((size_t)9 * n, sizeof(int32_t));
    for (size_t i = 0; i < (size_t)9 * n; i++) o->link_at[i] = -1;
    o->cutm = (uint8_t*)xcalloc(n, 1);
    o->nl = p->n_links;
    o->lsite = (int32_t*)xcalloc(o->nl, sizeof(int32_t));
    o->ldir = (int32_t*)xcalloc(o->nl, sizeof(int32_t));
    o->lgroup = (int32_t*)xcalloc(o->nl, sizeof(int32_t));
    o->lgroup2 = (int32_t*)xcalloc(o->nl, sizeof(int32_t));
    o->lq = (real*)xcalloc(o->nl, sizeof(real));
    o->ln = (real*)xcalloc(2 * o->nl, sizeof(real));
    o->ln2 = (real*)xcalloc(2 * o->nl, sizeof(real));
    for (int l = 0; l < o->nl; l++) {
        int s = p->link_site[l], k = p->link_dir[l];
        if (s < 0 || s >= n || !o->mat[s]) FAIL("link %d: site is not material", l);
        if (k < 1 || k > 8) FAIL("link %d: direction must be 1..8", l);
        if (!(p->link_q[l] > 0 && p->link_q[l] <= 1)) FAIL("link %d: q outside (0,1]", l);
        if (p->link_group[l] < 0 || p->link_group[l] >= o->ng) FAIL("link %d: bad group", l);
        if (p->link_group2[l] < -1 || p->link_group2[l] >= o->ng) FAIL("link %d: bad second group", l);
        if (o->link_at[(size_t)k * n + s] >= 0) FAIL("link %d: duplicate", l);
        double nn = p->link_normal[2 * l] * p->link_normal[2 * l] + p->link_normal[2 * l + 1] * p->link_normal[2 * l + 1];
        if (fabs(nn - 1.0) > 1e-9) FAIL("link %d: normal is not a unit vector", l);
        if (p->link_group2[l] >= 0) {
            double n2 = p->link_normal2[2 * l] * p->link_normal2[2 * l] + p->link_normal2[2 * l + 1] * p->link_normal2[2 * l + 1];
            if (fabs(n2 - 1.0) > 1e-9) FAIL("link %d: second normal is not a unit vector", l);
        }
        o->link_at[(size_t)k * n + s] = l;
        o->cutm[s] |= (uint8_t)(1u << (k - 1));
        o->lsite[l] = s; o->ldir[l] = k;
        o->lq[l] = (real)p->link_q[l];
        o->lgroup[l] = p->link_group[l]; o->lgroup2[l] = p->link_group2[l];
        o->ln[2 * l] = (real)p->link_normal[2 * l]; o->ln[2 * l + 1] = (real)p->link_normal[2 * l + 1];
        o->ln2[2 * l] = (real)p->link_normal2[2 * l]; o->ln2[2 * l + 1] = (real)p->link_normal2[2 * l + 1];
    }
    /* every population arriving at a material site must come from exactly one
     * place: streamed along an uncut link, or set by a boundary rule */
    for (int s = 0; s < n; s++) {
        if (!o->mat[s]) continue;
        for (int k = 1; k < 9; k++) {
            int cut = o->link_at[(size_t)k * n + s] >= 0;
            int t = neighbour(o, s, k, +1);
            if (!cut && (t < 0 || !o->mat[t])) FAIL("site %d: uncut link %d leaves the material", s, k);
            if (!cut && o->link_at[(size_t)OPP[k] * n + t] >= 0) FAIL("site %d: link %d cut from one end only", s, k);
        }
    }

    o->f = (real*)xcalloc((size_t)9 * n, sizeof(real));
    o->fnew = (real*)xcalloc((size_t)9 * n, sizeof(real));
    o->fcol = (real*)xcalloc((size_t)9 * n, sizeof(real));
    o->U = (real*)xcalloc((size_t)2 * n, sizeof(real));
    o->rho = (real*)xcalloc(n, sizeof(real));
    o->jx = (real*)xcalloc(n, sizeof(real));
    o->jy = (real*)xcalloc(n, sizeof(real));
    o->Pxx = (real*)xcalloc(n, sizeof(real));
    o->Pyy = (real*)xcalloc(n, sizeof(real));
    o->Pxy = (real*)xcalloc(n, sizeof(real));
    o->Sx = (real*)xcalloc(n, sizeof(real));
    o->Sy = (real*)xcalloc(n, sizeof(real));
    /* rest state: rho = 1, j = 0, P = 0 (no stress, no displacement) */
    for (int s = 0; s < n; s++)
        if (o->mat[s])
            for (int i = 0; i < 9; i++) o->f[(size_t)i * n + s] = feq_i(i, 1, 0, 0, 0, 0, 0);
    o->step = 0;
    return o;
#undef FAIL
}

void oracle_destroy(oracle_t* o)
{
    if (!o) return;
    free(o->mat); free(o->link_at); free(o->cutm);
    free(o->lsite); free(o->ldir); free(o->lgroup); free(o->lgroup2);
    free(o->lq); free(o->ln); free(o->ln2);
    free(o->gkind); free(o->gprof); free(o->gval); free(o->gramp);
    free(o->f); free(o->fnew); free(o->fcol); free(o->U);
    free(o->rho); free(o->jx); free(o->jy);
    free(o->Pxx); free(o->Pyy); free(o->Pxy); free(o->Sx); free(o->Sy);
    free(o);
}

/* ------------------------------------------------------------------------
 * eq:moments  rho = sum f_i,  j_raw = sum f_i c_i,  P = sum f_i c_i c_i
 * (j gets + S/2 once S is known, see source_term)
 */
static void moments(oracle_t* o, const real* f)
{
    int n = o->n;
#pragma omp parallel for schedule(static)
    for (int s = 0; s < n; s++) {
        if (!o->mat[s]) continue;
        real r = 0, jx = 0, jy = 0, pxx = 0, pyy = 0, pxy = 0;
        for (int i = 0; i < 9; i++) {
            real fi = f[(size_t)i * n + s];
            r += fi;
            jx += fi * CX[i];
            jy += fi * CY[i];
            pxx += fi * CX[i] * CX[i];
            pyy += fi * CY[i] * CY[i];
            pxy += fi * CX[i] * CY[i];
        }
        o->rho[s] = r; o->jx[s] = jx; o->jy[s] = jy;
        o->Pxx[s] = pxx; o->Pyy[s] = pyy; o->Pxy[s] = pxy;
    }
}

/* ------------------------------------------------------------------------
 * eq:sourceterm  S = F + (mu - lambda)/rho grad(rho).
 * The paper does not name a gradient stencil; this uses the isotropic D2Q9
 * one, d_a rho = (1/c_s^2) sum_i w_i c_ia rho(x + c_i).  Across a cut link the
 * missing neighbour value is extrapolated linearly from the opposite side,
 * 2 rho(x) - rho(x - c_i), or taken as rho(x) when that side is cut too.
 * Then j = j_raw + S/2 (eq:moments).
 */
static void source_term(oracle_t* o)
{
    int n = o->n;
#pragma omp parallel for schedule(static)
    for (int s = 0; s < n; s++) {
        if (!o->mat[s]) continue;
        int x = s % o->nx, y = s / o->nx;
        real gx = 0, gy = 0;
        for (int i = 1; i < 9; i++) {
            real r;
            if (!(o->cutm[s] >> (i - 1) & 1)) {
                r = o->rho[neighbour_xy(o, x, y, i, +1)];
            } else if (!(o->cutm[s] >> (OPP[i] - 1) & 1)) {
                r = 2 * o->rho[s] - o->rho[neighbour_xy(o, x, y, i, -1)];
            } else {
                r = o->rho[s];
            }
            gx += W(i) * CX[i] * r;
            gy += W(i) * CY[i] * r;
        }
        gx /= CS2;
        gy /= CS2;
        real c = (o->mu - o->lam) / o->rho[s];
        o->Sx[s] = o->F[0] + c * gx;
        o->Sy[s] = o->F[1] + c * gy;
        o->jx[s] += o->Sx[s] / 2;
        o->jy[s] += o->Sy[s] / 2;
    }
}

/* Cauchy stress from the Poisson stress (eq:poissonstress) with the
 * divergence approximation div u = (rho0 - rho)/rho0 (eq:approxdiv), rho0 = 1. */
static void cauchy(const oracle_t* o, int s, real* sxx, real* syy, real* sxy)
{
    real div = 1 - o->rho[s];
    *sxx = -o->Pxx[s] + (o->lam - o->mu) * div;
    *syy = -o->Pyy[s] + (o->lam - o->mu) * div;
    *sxy = -o->Pxy[s];
}

/* ------------------------------------------------------------------------
 * Boundary rule for the cut link (x, k): sets f_kbar(x, t+dt) from the
 * post-collision populations of time t (section 4).
 */
static void boundary_rule(oracle_t* o, int l, int64_t m)
{
    int n = o->n;
    int x = o->lsite[l], k = o->ldir[l], kb = OPP[k];
    real q = o->lq[l];
    /* a link whose opposite neighbour is cut too has no site behind it: the
     * terms that need x - c_k are dropped (q taken as 1/2) */
    int thin = o->link_at[(size_t)kb * n + x] >= 0;
    int y = thin ? -1 : neighbour(o, x, k, -1);
    real kappa = thin ? 0 : (1 - 2 * q) / (1 + 2 * q);      /* (l - 2s)/(l + 2s) */
    real beta = thin ? 1 : 2 / (1 + 2 * q);                  /* 2l/(l + 2s) */
    real fk = o->fcol[(size_t)k * n + x];
    real fkb = o->fcol[(size_t)kb * n + x];
    real fk_behind = thin ? 0 : o->fcol[(size_t)k * n + y];
    real cx = CX[k], cy = CY[k];

    int g1 = o->lgroup[l], g2 = o->lgroup2[l];
    int gd = -1;      /* Dirichlet wins where a corner meets both kinds */
    if (o->gkind[g1] == ORACLE_DIRICHLET) gd = g1;
    else if (g2 >= 0 && o->gkind[g2] == ORACLE_DIRICHLET) gd = g2;

    real out;
    if (gd >= 0) {
        /* eq:bbcon / eq:bbnoncon with j* = rho(x) times the wall velocity (eq:bcchaindir) */
        real a = profile(o, gd, m);
        real jsx = o->rho[x] * o->gval[2 * gd] * a;
        real jsy = o->rho[x] * o->gval[2 * gd + 1] * a;
        out = fk + kappa * (fk_behind - fkb)
            - beta * (2 / CS2) * W(k) * (cx * jsx + cy * jsy);
    } else {
        /* eq:abbcon / eq:abbnoncon */
        /* rho_bd: linear interpolation along the link (paper, section 4.2;
         * 3/2 rho(x) - 1/2 rho(x - c_k) at q = 1/2), or rho(x) at order 0 */
        int extrap = !thin && o->norder == 1;
        real rbd = extrap ? (1 + q) * o->rho[x] - q * o->rho[y] : o->rho[x];
        real sxx, syy, sxy;    /* boundary Cauchy stress sigma* */
        if (g2 >= 0) {
            /* two walls meet on this link: both tractions fix sigma* fully,
             * sigma* = sym(t_A n_A + t_B n_B) */
            real a1 = profile(o, g1, m), a2 = profile(o, g2, m);
            real tax = o->gval[2 * g1] * a1, tay = o->gval[2 * g1 + 1] * a1;
            real tbx = o->gval[2 * g2] * a2, tby = o->gval[2 * g2 + 1] * a2;
            real nax = o->ln[2 * l], nay = o->ln[2 * l + 1];
            real nbx = o->ln2[2 * l], nby = o->ln2[2 * l + 1];
            sxx = tax * nax + tbx * nbx;
            syy = tay * nay + tby * nby;
            sxy = ((tax * nay + tbx * nby) + (tay * nax + tby * nbx)) / 2;
        } else {
            /* eq:trafocauchy: in the frame (n, e_t) the traction fixes
             * sigma_nn = t.n and sigma_nt = t.e_t; sigma_tt is extrapolated
             * along the link from the material, with the weights of rho_bd */
            real a = profile(o, g1, m);
            real tx = o->gval[2 * g1] * a, ty = o->gval[2 * g1 + 1] * a;
            real nx_ = o->ln[2 * l], ny_ = o->ln[2 * l + 1];
            real ex = -ny_, ey = nx_;
            real cxx, cyy, cxy;
            cauchy(o, x, &cxx, &cyy, &cxy);
            real stt = ex * ex * cxx + 2 * ex * ey * cxy + ey * ey * cyy;
            if (extrap) {
                cauchy(o, y, &cxx, &cyy, &cxy);
                real stt_y = ex * ex * cxx + 2 * ex * ey * cxy + ey * ey * cyy;
                stt = (1 + q) * stt - q * stt_y;
            }
            real tn = tx * nx_ + ty * ny_;
            real tt = tx * ex + ty * ey;
            sxx = tn * nx_ * nx_ + tt * 2 * nx_ * ex + stt * ex * ex;
            syy = tn * ny_ * ny_ + tt * 2 * ny_ * ey + stt * ey * ey;
            sxy = tn * nx_ * ny_ + tt * (nx_ * ey + ex * ny_) + stt * ex * ey;
        }
        /* eq:bcchainneum with eq:approxdiv at rho_bd */
        real div = 1 - rbd;
        real pxx = -sxx + (o->lam - o->mu) * div;
        real pyy = -syy + (o->lam - o->mu) * div;
        real pxy = -sxy;
        real second = (pxx - rbd * CS2) * (cx * cx - CS2)
                    + (pyy - rbd * CS2) * (cy * cy - CS2)
                    + 2 * pxy * cx * cy;
        real E = 2 * W(k) * (rbd + second / (2 * CS2 * CS2));
        out = -fk - kappa * (fk_behind + fkb) + beta * E;
    }
    o->fnew[(size_t)kb * n + x] = out;
}

/* ------------------------------------------------------------------------ */

void oracle_step(oracle_t* o, int64_t nsteps)
{
    int n = o->n;
    for (int64_t it = 0; it < nsteps; it++) {
        moments(o, o->f);
        source_term(o);
        /* eq:coll  f_col = f - (f - f_eq)/tau + (1 - 1/(2 tau)) psi,
         * eq:sourceterm  psi_i = w_i c_i.S / c_s^2  (dt = 1) */
#pragma omp parallel for schedule(static)
        for (int s = 0; s < n; s++) {
            if (!o->mat[s]) continue;
            for (int i = 0; i < 9; i++) {
                real fi = o->f[(size_t)i * n + s];
                real fe = feq_i(i, o->rho[s], o->jx[s], o->jy[s], o->Pxx[s], o->Pyy[s], o->Pxy[s]);
                real psi = W(i) * (CX[i] * o->Sx[s] + CY[i] * o->Sy[s]) / CS2;
                o->fcol[(size_t)i * n + s] = fi - (fi - fe) / o->tau + (1 - 1 / (2 * o->tau)) * psi;
            }
            /* displacement: integrate du/dt = j/rho (left sum, read out with
             * the trapezoid correction in oracle_displacement) */
            o->U[s] += o->jx[s] / o->rho[s];
            o->U[(size_t)n + s] += o->jy[s] / o->rho[s];
        }
        /* eq:stream  f_i(x + c_i, t + 1) = f_col_i(x, t) along uncut links */
#pragma omp parallel for schedule(static)
        for (int s = 0; s < n; s++) {
            if (!o->mat[s]) continue;
            int x = s % o->nx, y = s / o->nx;
            o->fnew[s] = o->fcol[s];
            for (int i = 1; i < 9; i++)
                if (!(o->cutm[s] >> (i - 1) & 1))
                    o->fnew[(size_t)i * n + neighbour_xy(o, x, y, i, +1)] = o->fcol[(size_t)i * n + s];
        }
        /* section 4: cut links get their returning population from the rules */
#pragma omp parallel for schedule(static)
        for (int l = 0; l < o->nl; l++) boundary_rule(o, l, o->step);
        real* t = o->f; o->f = o->fnew; o->fnew = t;
        o->step++;
    }
}

int64_t oracle_step_count(const oracle_t* o) { return o->step; }

/* ------------------------------------------------------------------------ */

void oracle_moments(const oracle_t* oc, double* rho, double* j, double* P, double* sigma)
{
    oracle_t* o = (oracle_t*)oc;   /* scratch arrays only */
    int n = o->n;
    moments(o, o->f);
    source_term(o);
    double sv = o->rho_user * o->s_v;
    for (int s = 0; s < n; s++) {
        int m = o->mat[s];
        if (rho) rho[s] = m ? (double)o->rho[s] * o->rho_user : 0.0;
        if (j) {
            j[s] = m ? (double)o->jx[s] * sv : 0.0;
            j[(size_t)n + s] = m ? (double)o->jy[s] * sv : 0.0;
        }
        if (P) {
            P[s] = m ? (double)o->Pxx[s] * o->s_sigma : 0.0;
            P[(size_t)n + s] = m ? (double)o->Pyy[s] * o->s_sigma : 0.0;
            P[(size_t)2 * n + s] = m ? (double)o->Pxy[s] * o->s_sigma : 0.0;
        }
        if (sigma) {
            real a = 0, b = 0, c = 0;
            if (m) cauchy(o, s, &a, &b, &c);
            sigma[s] = (double)a * o->s_sigma;
            sigma[(size_t)n + s] = (double)b * o->s_sigma;
            sigma[(size_t)2 * n + s] = (double)c * o->s_sigma;
        }
    }
}

void oracle_displacement(const oracle_t* oc, double* u)
{
    oracle_t* o = (oracle_t*)oc;
    int n = o->n;
    moments(o, o->f);
    source_term(o);
    /* U holds u0 - v0/2 + sum_{m<n} v^m, so u^n = U + v^n/2 is the trapezoid
     * rule for the integral of v = j/rho */
    for (int s = 0; s < n; s++) {
        if (!o->mat[s]) { u[s] = 0; u[(size_t)n + s] = 0; continue; }
        u[s] = (double)(o->U[s] + o->jx[s] / o->rho[s] / 2);
        u[(size_t)n + s] = (double)(o->U[(size_t)n + s] + o->jy[s] / o->rho[s] / 2);
    }
}

int oracle_init_fields(oracle_t* o, const double* rho, const double* vel,
                       const double* sigma, const double* u)
{
    int n = o->n;
    /* density first: the source term needs its gradient */
    for (int s = 0; s < n; s++) {
        if (!o->mat[s]) continue;
        o->rho[s] = rho ? (real)rho[s] / (real)o->rho_user : 1;
        if (!(o->rho[s] > 0)) return -1;
    }
    for (int s = 0; s < n; s++) { o->jx[s] = 0; o->jy[s] = 0; }
    source_term(o);   /* adds S/2 to j = 0: j now holds S/2 */
    for (int s = 0; s < n; s++) {
        if (!o->mat[s]) continue;
        real r = o->rho[s];
        real jx = 0, jy = 0;
        if (vel) {
            jx = r * (real)vel[s] / (real)o->s_v;
            jy = r * (real)vel[(size_t)n + s] / (real)o->s_v;
        }
        real sxx = 0, syy = 0, sxy = 0;
        if (sigma) {
            sxx = (real)sigma[s] / (real)o->s_sigma;
            syy = (real)sigma[(size_t)n + s] / (real)o->s_sigma;
            sxy = (real)sigma[(size_t)2 * n + s] / (real)o->s_sigma;
        }
        /* eq:poissonstress with eq:approxdiv */
        real div = 1 - r;
        real pxx = -sxx + (o->lam - o->mu) * div;
        real pyy = -syy + (o->lam - o->mu) * div;
        real pxy = -sxy;
        /* populations carry j - S/2 so that the j moment (with + S/2) is j */
        real jrx = jx - o->jx[s], jry = jy - o->jy[s];
        for (int i = 0; i < 9; i++) o->f[(size_t)i * n + s] = feq_i(i, r, jrx, jry, pxx, pyy, pxy);
        real u0x = u ? (real)u[s] : 0, u0y = u ? (real)u[(size_t)n + s] : 0;
        o->U[s] = u0x - jx / r / 2;
        o->U[(size_t)n + s] = u0y - jy / r / 2;
    }
    o->step = 0;
    return 0;
}

void oracle_get_populations(const oracle_t* o, double* f)
{
    for (size_t i = 0; i < (size_t)9 * o->n; i++) f[i] = (double)o->f[i];
}

void oracle_set_populations(oracle_t* o, const double* f)
{
    for (size_t i = 0; i < (size_t)9 * o->n; i++) o->f[i] = (real)f[i];
}

void oracle_lattice_params(const oracle_t* o, double* out6)
{
    out6[0] = (double)o->lam;
    out6[1] = (double)o->mu;
    out6[2] = (double)o->tau;
    out6[3] = o->dt_user;
    out6[4] = o->s_sigma;
    out6[5] = o->s_v;
}

int oracle_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}
