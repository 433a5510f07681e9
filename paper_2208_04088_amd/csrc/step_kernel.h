// step_kernel.h -- device code of the fused solid-LBM time step (gfx950).
//
// Included by slbm.hip (single-plate and batched paths).
// Method: Faust, Schlueter, H. Mueller, R. Mueller, "Dirichlet and Neumann
// boundary conditions in a Lattice Boltzmann Method for Elastodynamics"
// (2022), sections 3 and 4.  The data layout is described in slbm.hip.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "slbm.h"

namespace slbm_dev {

// ----------------------------------------------------------------- lattice

// D2Q9 velocities, paper section 3 (numbering as in include/slbm.h).
__host__ __device__ constexpr int CX(int i) { return (i == 1 || i == 5 || i == 8) ? 1 : ((i == 3 || i == 6 || i == 7) ? -1 : 0); }
__host__ __device__ constexpr int CY(int i) { return (i == 2 || i == 5 || i == 6) ? 1 : ((i == 4 || i == 7 || i == 8) ? -1 : 0); }
__host__ __device__ constexpr int OPP(int i) { return i == 0 ? 0 : (i <= 4 ? ((i + 1) & 3) + 1 : ((i - 3) & 3) + 5); }
__host__ __device__ constexpr double WD(int i) { return i == 0 ? 4.0 / 9.0 : (i <= 4 ? 1.0 / 9.0 : 1.0 / 36.0); }

constexpr int kPadL = 64;      // padding columns left of the grid: keeps wide strips 256-byte aligned

// Two strip shapes for the fused step (the autotuner picks per plate):
//   wide   64 output columns per wave, 256-byte aligned; each wave also
//          gathers the densities of the two halo columns (HaloGather);
//   narrow 62 output columns per wave (lanes 1..62); lanes 0 and 63 sit on
//          the halo columns and only supply density.
template <bool WIDE> constexpr int strip_width() { return WIDE ? 64 : 62; }
constexpr unsigned kVoid = 0xFFu;

// A site update is flagged as diverged when |drho| + |j| (lattice units,
// rest density 1) reaches this bound -- a density deviation as large as the
// rest density itself, far outside linear elasticity -- or is not finite.
// An unstable mode is caught long before it overflows.
constexpr double kDivergeBound = 1.0;

struct GroupDev {
    int32_t profile;           // SLBM_PROFILE_*
    int32_t pad;
    double ramp_steps;         // ramp length in steps
};

// Coefficients of the boundary rule of one cut link (x, k); see build_links.
template <typename real>
struct LinkDev {
    real kappa;                // (l - 2s)/(l + 2s), 0 with no site behind x
    real wx, wy;               // weights of rho and sigma_tt at x and x - c_k
    real D;                    // Dirichlet: -beta (2/c_s^2) w_k c_k.v
    real be[4];                // Neumann: beta d(E_k - 2 r_k)/d(drho_bd, Pxx*, Pyy*, Pxy*)
    real K1[3], K2[3], E3[3];  // Neumann: known boundary stress per unit profile; e_t e_t
    int32_t g1, g2;            // groups whose profiles scale D or K1, K2
    int32_t kind;              // SLBM_DIRICHLET | SLBM_NEUMANN
    int32_t behind;            // 1: x - c_k is a material site reached by an uncut link
    int32_t k, dx, dy, pad;
};

// A cut link in a tile's list (the two-step kernel's cooperative rules): the
// link record's coefficients, with its direction, kind, the site-behind flag
// and its groups packed into meta (k | kind << 4 | behind << 6 | (g1 + 1) << 8
// | (g2 + 1) << 16, groups below 255) and its position in the tile.
template <typename real>
struct TileRec {
    real kappa, wx, wy, D;
    real be[4];
    real K1[3], K2[3], E3[3];
    int32_t meta;
    int32_t pos;               // the site's wave << 8 | lane in the tile
};

template <typename real>
__host__ __device__ inline int link_kind(const LinkDev<real>& L) { return L.kind; }
template <typename real>
__host__ __device__ inline int link_kind(const TileRec<real>& R) { return (R.meta >> 4) & 3; }

template <typename real>
struct StepArgs {
    const real* src;
    real* dst;
    double* U;
    const uint8_t* flags;
    const int32_t* bidx;
    const LinkDev<real>* links;
    const GroupDev* groups;
    unsigned int* diverged;
    // cut links per tile of the two-step kernel (null: none built for this
    // launch shape): tile t's are recs[rec_start[t] .. rec_start[t + 1])
    const int32_t* rec_start;
    const TileRec<real>* recs;
    long long plane;           // ny * ld
    long long t_prev;          // step whose post-collision state src holds
    int nx, ny, ld;
    int seg, nstrips, ntiles;
    int px, py;
    int ngroups;               // entries of groups
    int local;                 // src holds the populations themselves
    int group_shift;           // workgroups to XCDs: -1 contiguous bands, s >= 0 interleaved groups of 2^s
    real omega;                // 1/tau
    real lm, ml;               // lambda - mu, mu - lambda (lattice units)
    real Fx, Fy;
};

template <typename real>
__device__ __forceinline__ real profile_of(const GroupDev& G, long long t)
{
    if (G.profile == SLBM_PROFILE_RAMP) {
        real r = real((double)t / G.ramp_steps);
        return r < real(1) ? r : real(1);
    }
    return real(1);
}

template <typename real>
__device__ __forceinline__ real profile_at(const GroupDev* g, int gi, long long t)
{
    return profile_of<real>(g[gi], t);
}

// Shifted equilibrium g_eq,i = f_eq,i - r_i of eq:fieq, drho = rho - 1:
// w_i [drho (2 - 3|c|^2/2) + 3 c.j + 9/2 (Pxx (cx^2 - 1/3) + Pyy (cy^2 - 1/3) + 2 Pxy cx cy)]
template <int i, typename real>
__device__ __forceinline__ real geq(real dr, real jx, real jy, real pxx, real pyy, real pxy)
{
    constexpr int cx = CX(i), cy = CY(i);
    constexpr double w = WD(i);
    constexpr double a0 = w * (2.0 - 1.5 * (cx * cx + cy * cy));
    constexpr double ax = 3.0 * w * cx, ay = 3.0 * w * cy;
    constexpr double axx = 4.5 * w * (cx * cx - 1.0 / 3.0);
    constexpr double ayy = 4.5 * w * (cy * cy - 1.0 / 3.0);
    constexpr double axy = 9.0 * w * cx * cy;
    real v = real(a0) * dr;
    if (cx != 0) v += real(ax) * jx;
    if (cy != 0) v += real(ay) * jy;
    v += real(axx) * pxx + real(ayy) * pyy;
    if (cx * cy != 0) v += real(axy) * pxy;
    return v;
}

template <typename real>
__device__ __forceinline__ void moments9(const real g[9], real& dr, real& jx, real& jy,
                                         real& pxx, real& pyy, real& pxy)
{
    // eq:moments on shifted populations (the rest state has rho = 1, j = 0, P = 0)
    const real d57 = g[5] + g[7], d68 = g[6] + g[8];
    dr = g[0] + g[1] + g[2] + g[3] + g[4] + d57 + d68;
    jx = g[1] - g[3] + g[5] - g[6] - g[7] + g[8];
    jy = g[2] - g[4] + g[5] + g[6] - g[7] - g[8];
    pxx = g[1] + g[3] + d57 + d68;
    pyy = g[2] + g[4] + d57 + d68;
    pxy = d57 - d68;
}

// Element e of a plane: a uniform base pointer plus a 32-bit byte offset, so
// that loads and stores address through a scalar base register and one
// vector register (a plane holds far fewer than 2^32 bytes; checked at
// creation).
// The empty asm pins the base in scalar registers and keeps the compiler
// from folding the plane offset into per-lane 64-bit address arithmetic.
template <typename T>
using gptr = __attribute__((address_space(1))) T*;

template <typename T>
__device__ __forceinline__ gptr<T> sbase(T* p)
{
    gptr<T> q = (gptr<T>)p;
    asm("" : "+s"(q));
    return q;
}
template <typename T>
__device__ __forceinline__ T ldu(const T* base, unsigned e)       // base uniform over the wave
{
    return *(gptr<const T>)((gptr<const char>)sbase(base) + e * (unsigned)sizeof(T));
}
template <typename T>
__device__ __forceinline__ void stu(T* base, unsigned e, T v)     // base uniform over the wave
{
    *(gptr<T>)((gptr<char>)sbase(base) + e * (unsigned)sizeof(T)) = v;
}
template <typename T>
__device__ __forceinline__ T ldg(const T* base, unsigned e)       // any base
{
    return *(const T*)((const char*)base + e * (unsigned)sizeof(T));
}

// Offset of site (x, y) in a padded plane.
__host__ __device__ __forceinline__ int sidx(int x, int y, int ld) { return (y + 1) * ld + (x + kPadL); }

// Offset of the site at (x + dx, y + dy), wrapped on periodic axes.
template <bool PER>
__device__ __forceinline__ int wrap_off(int x, int y, int dx, int dy, int nx, int ny, int ld, int px, int py)
{
    int xx = x + dx, yy = y + dy;
    if (PER) {
        if (px) xx = xx < 0 ? xx + nx : (xx >= nx ? xx - nx : xx);
        if (py) yy = yy < 0 ? yy + ny : (yy >= ny ? yy - ny : yy);
    }
    return sidx(xx, yy, ld);
}

// The previous step's post-collision populations around a site, read as
// prev(i, dx, dy) = population i at (x + dx, y + dy): from the state buffer in
// global memory (wrapped on periodic axes) ...
template <typename real, bool PER>
struct GlobalPrev {
    const real* src;
    long long plane;
    int x, y, nx, ny, ld, px, py;
    __device__ __forceinline__ real operator()(int i, int dx, int dy) const
    {
        return ldg(src + i * plane, wrap_off<PER>(x, y, dx, dy, nx, ny, ld, px, py));
    }
    // all nine populations at one site (plane bases uniform over the wave)
    __device__ __forceinline__ void all(int dx, int dy, real h[9]) const
    {
        const int off = wrap_off<PER>(x, y, dx, dy, nx, ny, ld, px, py);
#pragma unroll
        for (int j = 0; j < 9; ++j) h[j] = ldu(src + j * plane, off);
    }
};

// ... or from a tile of them in LDS, post[row][i][lane] (two-step kernel).
template <typename real>
struct LdsPrev {
    const real (*post)[9][64];
    int r, l;
    __device__ __forceinline__ real operator()(int i, int dx, int dy) const { return post[r + dy][i][l + dx]; }
    __device__ __forceinline__ void all(int dx, int dy, real h[9]) const
    {
#pragma unroll
        for (int j = 0; j < 9; ++j) h[j] = post[r + dy][j][l + dx];
    }
};

// Moments of the post-collision populations at (x + dx, y + dy).
template <typename real, class Prev>
__device__ __forceinline__ void stored_moments(const Prev& prev, int dx, int dy, real& dr, real& pxx, real& pyy,
                                               real& pxy)
{
    real h[9];
    prev.all(dx, dy, h);
    real jx, jy;
    moments9(h, dr, jx, jy, pxx, pyy, pxy);
}

// The boundary rule of section 4 for the cut link (x, k): the population
// arriving at x in direction kbar at the current step, from the previous
// post-collision state -- gk, gkb its populations k and kbar at x, gky its
// population k at x - c_k (0 with no site behind x), (drx, pxxx, pyyx, pxyx)
// its moments at x and (dry, pxxy, pyyy, pxyy) at x - c_k (read only when the
// rule extrapolates, L.wy != 0), p1 and p2 the profiles of the link's groups
// at that step (p2 = 0 without a second group).
template <typename real, class Rec>
__device__ real rule_value(const StepArgs<real>& a, const Rec& L, real gk, real gkb, real gky,
                           real drx, real pxxx, real pyyx, real pxyx, real dry, real pxxy, real pyyy, real pxyy,
                           real p1, real p2)
{
    if (link_kind(L) == SLBM_DIRICHLET) {
        // eq:bbcon / eq:bbnoncon, j* = rho(x) d(u*)/dt (eq:bcchaindir)
        return gk + L.kappa * (gky - gkb) + L.D * (real(1) + drx) * p1;
    }
    // eq:abbcon / eq:abbnoncon.  Cauchy stress from the Poisson stress with the
    // divergence approximation (eq:poissonstress, eq:approxdiv):
    // sigma = -P - (lambda - mu) drho I.
    real drbd = L.wx * drx;
    real stt = L.wx * (L.E3[0] * (-pxxx - a.lm * drx) + L.E3[1] * (-pyyx - a.lm * drx)
                       - real(2) * L.E3[2] * pxyx);
    if (L.wy != real(0)) {
        drbd += L.wy * dry;
        stt += L.wy * (L.E3[0] * (-pxxy - a.lm * dry) + L.E3[1] * (-pyyy - a.lm * dry)
                       - real(2) * L.E3[2] * pxyy);
    }
    // boundary Cauchy stress (eq:trafocauchy) and Poisson stress (eq:bcchainneum)
    const real sxx = p1 * L.K1[0] + p2 * L.K2[0] + stt * L.E3[0];
    const real syy = p1 * L.K1[1] + p2 * L.K2[1] + stt * L.E3[1];
    const real sxy = p1 * L.K1[2] + p2 * L.K2[2] + stt * L.E3[2];
    const real Pxx = -sxx - a.lm * drbd;
    const real Pyy = -syy - a.lm * drbd;
    const real Pxy = -sxy;
    return -gk - L.kappa * (gky + gkb) + L.be[0] * drbd + L.be[1] * Pxx + L.be[2] * Pyy + L.be[3] * Pxy;
}

// rule_value with the state read through prev (time t_prev) and the
// profiles from the group table.
template <typename real, class Prev>
__device__ real boundary_value(const StepArgs<real>& a, const LinkDev<real>& L, const Prev& prev, long long t_prev,
                               real drx, real pxxx, real pyyx, real pxyx)
{
    const int k = L.k, kb = OPP(k);
    const real gk = prev(k, 0, 0);
    const real gkb = prev(kb, 0, 0);
    real gky = real(0);
    if (L.behind) gky = prev(k, -L.dx, -L.dy);
    if (L.kind == SLBM_DIRICHLET) {
        const real p = profile_at<real>(a.groups, L.g1, t_prev);
        return rule_value<real>(a, L, gk, gkb, gky, drx, pxxx, pyyx, pxyx, real(0), real(0), real(0), real(0), p,
                                real(0));
    }
    real dry = real(0), pxxy = real(0), pyyy = real(0), pxyy = real(0);
    if (L.wy != real(0)) stored_moments<real>(prev, -L.dx, -L.dy, dry, pxxy, pyyy, pxyy);
    const real p1 = profile_at<real>(a.groups, L.g1, t_prev);
    const real p2 = L.g2 >= 0 ? profile_at<real>(a.groups, L.g2, t_prev) : real(0);
    return rule_value<real>(a, L, gk, gkb, gky, drx, pxxx, pyyx, pxyx, dry, pxxy, pyyy, pxyy, p1, p2);
}

// Replaces the populations of cut links of a boundary site (grid offset s) by
// the section 4 rules.  g already holds the pulls along uncut links.
template <typename real, class Prev>
__device__ void boundary_fixup(const StepArgs<real>& a, const Prev& prev, int s, unsigned fl, long long t_prev,
                               real g[9])
{
    real drx, pxxx, pyyx, pxyx;
    stored_moments<real>(prev, 0, 0, drx, pxxx, pyyx, pxyx);
    int li = ldu(a.bidx, s);
    unsigned m = fl;
    while (m) {
        const int k = __builtin_ctz(m) + 1;
        m &= m - 1;
        const LinkDev<real> L = a.links[li++];
        const real v = boundary_value<real>(a, L, prev, t_prev, drx, pxxx, pyyx, pxyx);
        const int i = OPP(k);
#pragma unroll
        for (int j = 1; j < 9; ++j)
            if (j == i) g[j] = v;
    }
}

template <typename real, bool PER>
__device__ __forceinline__ GlobalPrev<real, PER> global_prev(const StepArgs<real>& a, int x, int y)
{
    return GlobalPrev<real, PER>{a.src, a.plane, x, y, a.nx, a.ny, a.ld, a.px, a.py};
}

// Populations at site (x, y) for the current step (x, y in the grid, wrapped
// by the caller on periodic axes).  Returns false for sites without state.
template <typename real, bool PER>
__device__ __forceinline__ bool fetch_site(const StepArgs<real>& a, int x, int y, real g[9], unsigned& flo)
{
    const int s = sidx(x, y, a.ld);
    const unsigned fl = ldu(a.flags, s);
    flo = fl;
    if (fl == kVoid) {
#pragma unroll
        for (int i = 0; i < 9; ++i) g[i] = real(0);
        return false;
    }
#pragma unroll
    for (int i = 0; i < 9; ++i)
        g[i] = a.local ? ldu(a.src + i * a.plane, s)
                       : ldu(a.src + i * a.plane, wrap_off<PER>(x, y, -CX(i), -CY(i), a.nx, a.ny, a.ld, a.px, a.py));
    if (!a.local && fl != 0) boundary_fixup<real>(a, global_prev<real, PER>(a, x, y), s, fl, a.t_prev, g);
    return true;
}

// Site coordinates of a row or halo site: wrapped on periodic axes (any
// distance: tiles reach up to three sites past a plate narrower than that),
// clamped into the grid otherwise -- so that every pull address stays in the
// allocation -- and then marked outside.
template <bool PER>
__device__ __forceinline__ void place(int nx, int ny, int px, int py, int& x, int& y, bool& in)
{
    in = true;
    if (x < 0 || x >= nx) {
        if (PER && px) {
            x %= nx;
            if (x < 0) x += nx;
        } else {
            in = false;
            x = x < 0 ? 0 : nx - 1;
        }
    }
    if (y < 0 || y >= ny) {
        if (PER && py) {
            y %= ny;
            if (y < 0) y += ny;
        } else {
            in = false;
            y = y < 0 ? 0 : ny - 1;
        }
    }
}

// Loads of one site, unconditional: a site outside the grid loads from a
// clamped in-grid site and is masked when completed (a conditional load
// would make the compiler wait for earlier loads before initialising its
// target registers).  The padding ring keeps the pull addresses of any
// in-grid site inside the allocation.
template <typename real, bool PER>
__device__ __forceinline__ void site_issue(const StepArgs<real>& a, int x, int y, real g[9], unsigned& fl,
                                           int& ys, bool& in, int& s_out)
{
    place<PER>(a.nx, a.ny, a.px, a.py, x, y, in);
    ys = y;
    const int s = sidx(x, y, a.ld);
    s_out = s;
    fl = ldu(a.flags, s);
    if (a.local) {
#pragma unroll
        for (int i = 0; i < 9; ++i) g[i] = ldu(a.src + i * a.plane, s);
    } else {
#pragma unroll
        for (int i = 0; i < 9; ++i)
            g[i] = ldu(a.src + i * a.plane, wrap_off<PER>(x, y, -CX(i), -CY(i), a.nx, a.ny, a.ld, a.px, a.py));
    }
}

// Completes one site: boundary rules on cut links, nothing for void sites.
// Returns delta-rho (0 without state).
template <typename real, bool PER>
__device__ __forceinline__ real site_finish(const StepArgs<real>& a, int x, int y, bool in, bool want,
                                            unsigned& fl, real g[9])
{
    if (!in) fl = kVoid;
    const bool live = fl != kVoid;
    if (want && live && !a.local && fl != 0) {
        int xx = x, yy = y;
        bool in2;
        place<PER>(a.nx, a.ny, a.px, a.py, xx, yy, in2);
        boundary_fixup<real>(a, global_prev<real, PER>(a, xx, yy), sidx(xx, yy, a.ld), fl, a.t_prev, g);
    }
#pragma unroll
    for (int i = 0; i < 9; ++i) g[i] = live ? g[i] : real(0);
    return g[0] + g[1] + g[2] + g[3] + g[4] + g[5] + g[6] + g[7] + g[8];
}

// 1/x: the hardware reciprocal in single precision (within one ulp), a
// correctly rounded division in double precision.
__device__ __forceinline__ float recip(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double recip(double x) { return 1.0 / x; }

// Whether any site of the wave has a cut link (void sites carry kVoid);
// called where the whole wave is active.
__device__ __forceinline__ bool wave_has_cuts(unsigned fl) { return __any(fl != 0u && fl != kVoid); }

// Density stencil of the source term below and at a site: delta-rho of row
// y-1 (m) and row y (c) at the site's column and its two neighbours.
template <typename real>
struct Window {
    real m, m_l, m_r;
    real c, c_l, c_r;
};

// Collision and source term of one site, given the densities of its eight
// neighbours (w and the row above, rp): the post-collision populations o and
// the site's j (with S/2) and rho.
//
// eq:coll with eq:fieq, in the closure where the equilibrium's second moment
// is the populations' own: collision leaves rho and P unchanged, adds S to j
// and relaxes the three ghost moments.  The update is therefore written as
//   g_i <- g_i + T_i(S) + a_x vx_i + a_y vy_i + a_e ve_i
// with integer ghost vectors vx = cx (3 cy^2 - 2), vy = cy (3 cx^2 - 2),
// ve = (4, -2 x4, 1 x4) and T(S) = (S_x/2)(e_1 - e_3) + (S_y/2)(e_2 - e_4),
// whose zeroth, first and second moments are exact in floating point.  In
// exact arithmetic this is the BGK update with the source psi_i = w_i c_i.S/c_s^2
// (the projection of the BGK change onto the ghost vectors gives a_x, a_y,
// a_e below).  Rounded equilibrium weights would instead scale the conserved
// moments by (1 + omega eps) each step, a drift of ~5e-4 after 10^4 steps in
// single precision.
//
// CUTS = false: no site of the wave has a cut link (a wave-uniform fast path;
// the substitution below is then the identity).
template <typename real, bool CUTS>
__device__ __forceinline__ bool collide_core(const StepArgs<real>& a, const real g[9], unsigned fl,
                                             const Window<real>& w, real rp, real rp_l, real rp_r, real o[9],
                                             real& jx_out, real& jy_out, real& ir_out)
{
    const real A4 = g[1] + g[2] + g[3] + g[4];
    const real B4 = g[5] + g[6] + g[7] + g[8];
    const real Dx = g[5] - g[6] - g[7] + g[8];
    const real Dy = g[5] + g[6] - g[7] - g[8];
    const real g13 = g[1] - g[3], g24 = g[2] - g[4];
    const real dr = g[0] + A4 + B4;
    // eq:sourceterm: isotropic D2Q9 gradient of rho; across a cut link the
    // neighbour is extrapolated from the opposite side
    real nb[9];
    nb[1] = w.c_r; nb[2] = rp; nb[3] = w.c_l; nb[4] = w.m;
    nb[5] = rp_r; nb[6] = rp_l; nb[7] = w.m_l; nb[8] = w.m_r;
    real rt[9];
#pragma unroll
    for (int i = 1; i < 9; ++i) {
        if constexpr (CUTS) {
            const bool ci = (fl >> (i - 1)) & 1u;
            const bool co = (fl >> (OPP(i) - 1)) & 1u;
            rt[i] = ci ? (co ? dr : real(2) * dr - nb[OPP(i)]) : nb[i];
        } else {
            rt[i] = nb[i];
        }
    }
    const real gx = real(1.0 / 3.0) * (rt[1] - rt[3]) + real(1.0 / 12.0) * (rt[5] - rt[6] - rt[7] + rt[8]);
    const real gy = real(1.0 / 3.0) * (rt[2] - rt[4]) + real(1.0 / 12.0) * (rt[5] + rt[6] - rt[7] - rt[8]);
    const real rho = real(1) + dr;
    const real ir = recip(rho);
    const real c = a.ml * ir;
    const real Sx = a.Fx + c * gx, Sy = a.Fy + c * gy;
    const real hx = real(0.5) * Sx, hy = real(0.5) * Sy;
    // j of eq:moments with the half-step source
    const real jx = g13 + Dx + hx;
    const real jy = g24 + Dy + hy;
    const real ax = (a.omega * (g13 - real(2) * Dx) + Sx) * real(1.0 / 12.0);
    const real ay = (a.omega * (g24 - real(2) * Dy) + Sy) * real(1.0 / 12.0);
    const real ae = a.omega * (real(2) * A4 - real(4) * B4 - g[0]) * real(1.0 / 36.0);
    const real ae2 = real(2) * ae;
    const real ax2 = real(2) * ax, ay2 = real(2) * ay;
    o[0] = g[0] + real(4) * ae;
    o[1] = g[1] + ((hx - ax2) - ae2);
    o[3] = g[3] + ((ax2 - hx) - ae2);
    o[2] = g[2] + ((hy - ay2) - ae2);
    o[4] = g[4] + ((ay2 - hy) - ae2);
    o[5] = g[5] + ((ax + ay) + ae);
    o[6] = g[6] + ((ay - ax) + ae);
    o[7] = g[7] + (ae - (ax + ay));
    o[8] = g[8] + ((ax - ay) + ae);
    jx_out = jx;
    jy_out = jy;
    ir_out = ir;
    return !(fabs(dr) + fabs(jx) + fabs(jy) < real(kDivergeBound));
}

// displacement: U += j/rho, the increment in the populations' precision
// (ir = 1/rho), the sum in fp64
template <typename real>
__device__ __forceinline__ void advance_u(double& ux, double& uy, real jx, real jy, real ir)
{
    ux = ux + (double)(jx * ir);
    uy = uy + (double)(jy * ir);
}

// collide_core, then the populations and the displacement stored at (x, y).
template <typename real, bool CUTS>
__device__ __forceinline__ bool collide_site(const StepArgs<real>& a, int x, int y, const real g[9], unsigned fl,
                                             double ux, double uy, const Window<real>& w, real rp, real rp_l,
                                             real rp_r)
{
    real o[9], jx, jy, ir;
    const bool bad = collide_core<real, CUTS>(a, g, fl, w, rp, rp_l, rp_r, o, jx, jy, ir);
    const int s = sidx(x, y, a.ld);
#pragma unroll
    for (int i = 0; i < 9; ++i) stu(a.dst + i * a.plane, s, o[i]);
    advance_u(ux, uy, jx, jy, ir);
    stu(a.U, s, ux);
    stu(a.U + a.plane, s, uy);
    return bad;
}

// ------------------------------------------------------------------ tiles
//
// A workgroup advances a tile of R rows (R <= kMaxTileRows) of one strip: one
// wave per output row plus two waves for the density-halo rows below and
// above the tile.
// Every wave issues all loads of its row at once, completes the pulls with
// the boundary rules and puts the density in LDS; after a barrier the output
// waves read the 3x3 density stencil of the source term from LDS and collide.
constexpr int kMaxTileRows = 14;

template <bool WIDE> constexpr int tile_waves(int rows) { return rows + 2; }
template <bool WIDE> constexpr int max_tile_rows() { return kMaxTileRows; }

// Workgroups are dealt round-robin to the 8 XCDs; this gives each XCD a
// contiguous band of tile numbers so that the halo rows and columns tiles
// share stay in one L2.  nb (the grid size) is a multiple of 8.
__device__ __forceinline__ int xcd_banded(int b, int nb) { return (b & 7) * (nb >> 3) + (b >> 3); }

// The step kernels can instead give each XCD groups of 2^s consecutive
// workgroups, the groups of the 8 XCDs interleaved (the grid is then a
// multiple of 8 2^s).  Tiles with boundary work cluster (a hole, a crack);
// bands hand such a cluster to one XCD, which finishes last, while
// interleaved groups spread it.  Which is faster depends on the plate, so the
// autotuner measures both.  Both maps are formed without a branch, so a wave
// needs its arguments only once before its first loads.
__device__ __forceinline__ int xcd_map(int b, int nb, int shift)
{
    const int x = b & 7, l = b >> 3;
    const int band = x * (nb >> 3) + l;
    const int s = shift < 0 ? 0 : shift;
    const int grouped = ((((l >> s) << 3) + x) << s) + (l & ((1 << s) - 1));
    return shift < 0 ? band : grouped;
}

// Densities of the two halo columns of a wide strip in row y (left: column
// xs - 1, right: xs + 64).  Lanes 0-8 pull the nine populations of the left
// site, lanes 32-40 those of the right one (one load each), and the sums are
// formed in the order site_finish uses, so they equal what the wave owning
// the site computes.  A halo site with cut links takes the full site path
// (boundary rules), all lanes of a half-wave on its side.
template <typename real, bool PER>
struct HaloGather {
    real v;
    unsigned fl;
    int x, y;
    bool in;

    __device__ __forceinline__ void issue(const StepArgs<real>& a, int lane, int xs, int yrow)
    {
        const int side = lane >> 5, i = lane & 31;
        const int d = i < 9 ? i : 0;
        x = side ? xs + 64 : xs - 1;
        y = yrow;
        place<PER>(a.nx, a.ny, a.px, a.py, x, y, in);
        const int hs = sidx(x, y, a.ld);
        fl = ldu(a.flags, hs);
        const int off = a.local ? hs : wrap_off<PER>(x, y, -CX(d), -CY(d), a.nx, a.ny, a.ld, a.px, a.py);
        v = ldg(a.src + d * a.plane, off);
    }

    __device__ __forceinline__ void finish(const StepArgs<real>& a, int lane, int xs, int yrow, real& dl, real& dr)
    {
        const unsigned fl_l = __shfl(fl, 0), fl_r = __shfl(fl, 32);
        const bool live_l = __shfl((int)in, 0) && fl_l != kVoid;
        const bool live_r = __shfl((int)in, 32) && fl_r != kVoid;
        real sl = __shfl(v, 0), sr = __shfl(v, 32);
#pragma unroll
        for (int i = 1; i < 9; ++i) {
            sl += __shfl(v, i);
            sr += __shfl(v, 32 + i);
        }
        dl = live_l ? sl : real(0);
        dr = live_r ? sr : real(0);
        const bool slow_l = live_l && fl_l != 0 && !a.local, slow_r = live_r && fl_r != 0 && !a.local;
        if (slow_l || slow_r) {
            real g[9];
            unsigned f;
            bool in2;
            int ys2, s2;
            const int hx = (lane >> 5) ? xs + 64 : xs - 1;
            site_issue<real, PER>(a, hx, yrow, g, f, ys2, in2, s2);
            const real d = site_finish<real, PER>(a, hx, ys2, in2, true, f, g);
            const real d_l = __shfl(d, 0), d_r = __shfl(d, 32);
            if (slow_l) dl = d_l;
            if (slow_r) dr = d_r;
        }
    }
};

template <typename real, bool PER, bool WIDE>
__device__ __forceinline__ bool step_tile(const StepArgs<real>& a, int tile, real (*dens)[66])
{
    constexpr int W = strip_width<WIDE>();
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int R = a.seg;
    const int strip = tile % a.nstrips;            // strip fastest: rows stream through memory in order
    const int y0 = (tile / a.nstrips) * R;
    const int xs = strip * W;                      // first output column of the strip
    // wave w holds row y0 - 1 + w; narrow strips put the halo columns on
    // lanes 0 and 63, wide ones gather them (HaloGather)
    const int x = WIDE ? xs + lane : xs - 1 + lane;
    const int y = y0 - 1 + wave;
    real g[9];
    unsigned fl;
    bool in;
    int ys, s;
    site_issue<real, PER>(a, x, y, g, fl, ys, in, s);
    HaloGather<real, PER> hg;
    if constexpr (WIDE) hg.issue(a, lane, xs, y);
    const double ux = ldu(a.U, s), uy = ldu(a.U + a.plane, s);
    const int c = WIDE ? lane + 1 : lane;
    dens[wave][c] = site_finish<real, PER>(a, x, ys, in, true, fl, g);
    if constexpr (WIDE) {
        real dl, dr;
        hg.finish(a, lane, xs, y, dl, dr);
        if (lane == 0) dens[wave][0] = dl;
        if (lane == 63) dens[wave][W + 1] = dr;
    }
    __syncthreads();
    const bool cuts = wave_has_cuts(fl);
    const bool out = wave >= 1 && wave <= R && y < a.ny && x < a.nx && (WIDE || (lane >= 1 && lane <= 62));
    if (!out || fl == kVoid) return false;
    Window<real> w;
    w.m = dens[wave - 1][c]; w.m_l = dens[wave - 1][c - 1]; w.m_r = dens[wave - 1][c + 1];
    w.c_l = dens[wave][c - 1]; w.c_r = dens[wave][c + 1];
    return cuts ? collide_site<real, true>(a, x, y, g, fl, ux, uy, w, dens[wave + 1][c], dens[wave + 1][c - 1],
                                           dens[wave + 1][c + 1])
                : collide_site<real, false>(a, x, y, g, fl, ux, uy, w, dens[wave + 1][c], dens[wave + 1][c - 1],
                                            dens[wave + 1][c + 1]);
}

// Sets the plate's divergence word when any lane of the wave saw a
// non-finite value: one atomic per wave, none once the word is set (a plate
// that has blown up would otherwise send an atomic from every site, every
// step, to one address).
__device__ __forceinline__ void flag_divergence(unsigned int* word, bool bad)
{
    if (__any(bad) && (threadIdx.x & 63) == 0 && *(volatile unsigned int*)word == 0u) atomicOr(word, 1u);
}

// One time step of one plate: one workgroup of tile_waves(seg) waves per tile.
template <typename real, bool PER, bool WIDE>
__global__ __launch_bounds__(1024) void k_step(StepArgs<real> a)
{
    __shared__ real dens[kMaxTileRows + 2][66];
    const int tile = xcd_map(blockIdx.x, gridDim.x, a.group_shift);
    if (tile >= a.ntiles) return;                 // uniform over the workgroup
    flag_divergence(a.diverged, step_tile<real, PER, WIDE>(a, tile, dens));
}

// ---------------------------------------------------- two steps per launch
//
// A workgroup of R + 6 waves (R <= kMaxTileRows2) advances a tile of R rows
// of a 58-column strip by two time steps, reading the state once and writing
// it once.  A step at a site depends on the previous state within two sites
// (the pulls one, the density stencil one more), so the first step is taken
// on the tile widened by two rows and two columns on each side -- wave w
// holds row y0 - 3 + w, lane l column xs - 3 + l -- and its post-collision
// populations stay in LDS, from where the second step pulls.  Every site's
// arithmetic is that of two single steps, so the state is bit-identical to
// theirs.
constexpr int kMaxTileRows2 = 10;
constexpr int kStrip2 = 58;

// Cut links whose rules a tile of the two-step kernel evaluates together
// (below), and the BC groups whose profiles it tabulates: the host uses the
// cooperative kernel only when every tile's records (at most one per thread
// of the workgroup) and the plate's groups fit.  The records fill what is
// left of the LDS two single-precision workgroups share on a compute unit.
constexpr int kTileRecCap = 576;
constexpr int kTileGroupCap = 64;

// LDS of a two-step tile.  post holds the first step's post-collision
// populations (rows 0..R+3).  In the cooperative kernel the same words first
// carry the first step's rule values, plane k - 1 of row w those of the cut
// links k of wave w (rows 0..R+5); they are read before the first step's
// collision writes post.
template <typename real, bool COOP>
struct TileLds {
    real post_[kMaxTileRows2 + 4][9][64];
    real dens[kMaxTileRows2 + 6][66];
    __device__ real (*post())[9][64] { return post_; }
};
template <typename real>
struct TileLds<real, true> {
    static constexpr int kWords = (kMaxTileRows2 + 6) * 8 * 64 > (kMaxTileRows2 + 4) * 9 * 64
                                      ? (kMaxTileRows2 + 6) * 8 * 64 : (kMaxTileRows2 + 4) * 9 * 64;
    real buf[kWords];
    real dens[kMaxTileRows2 + 6][66];
    TileRec<real> recs[kTileRecCap];
    real prof[2][kTileGroupCap];
    __device__ real (*post())[9][64] { return reinterpret_cast<real (*)[9][64]>(buf); }
    __device__ real (*rule1())[8][64] { return reinterpret_cast<real (*)[8][64]>(buf); }
};

// Population k of h[0..8] for a k known only at run time, by bit masks (a
// dynamically indexed register array would go through scratch memory).
__device__ __forceinline__ float pick9(const float h[9], int k)
{
    unsigned v = 0u;
#pragma unroll
    for (int j = 0; j < 9; ++j) v |= __float_as_uint(h[j]) & (0u - (unsigned)(k == j));
    return __uint_as_float(v);
}
__device__ __forceinline__ double pick9(const double h[9], int k)
{
    unsigned long long v = 0ull;
#pragma unroll
    for (int j = 0; j < 9; ++j) v |= (unsigned long long)__double_as_longlong(h[j]) & (0ull - (unsigned long long)(k == j));
    return __longlong_as_double((long long)v);
}

// TWO = false: only the first step, stored like a single step (a plate in a
// batch with one step left).
//
// The rules of section 4 at the tile's cut links, two ways.  COOP = false:
// site by site, each site with cut links pulling, from global memory (first
// step) or LDS (second), the state its links read and the links'
// coefficients, one link after the other.  COOP = true (the plate carries
// per-tile record lists, rec_start, each of at most kTileRecCap records):
// together -- the workgroup copies the tile's records into LDS with its first
// loads, one thread per record gathers the state its rule reads (one round of
// loads for all records), evaluates it and leaves the value in LDS where the
// site's lane picks it up (first step) or in the LDS slot the site's pull
// reads (second step).  Both compute every rule value from the same inputs
// with rule_value, so the state is the same to the bit.
template <typename real, bool PER, bool TWO, bool COOP>
__device__ __forceinline__ bool step_tile2(const StepArgs<real>& a, int tile, TileLds<real, COOP>& lds)
{
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int R = a.seg;
    const int strip = tile % a.nstrips;
    const int y0 = (tile / a.nstrips) * R;
    const int xs = strip * kStrip2 - 3;
    const int x = xs + lane, y = y0 - 3 + wave;
    real (*const post)[9][64] = lds.post();
    // first step, from the state buffer
    real g[9];
    unsigned fl;
    bool in;
    int ys, s;
    site_issue<real, PER>(a, x, y, g, fl, ys, in, s);
    const bool out_row = wave >= 3 && wave <= R + 2;        // uniform over the wave
    double ux = 0.0, uy = 0.0;
    if (out_row) {
        ux = ldu(a.U, s);
        uy = ldu(a.U + a.plane, s);
    }
    int r0 = 0, nrec = 0;
    if constexpr (COOP) {
        r0 = a.rec_start[tile];
        nrec = a.rec_start[tile + 1] - r0;                  // uniform over the workgroup
    }
    // the tile's records and the groups' profiles into LDS, and the first
    // step's rules (none when src holds the populations themselves)
    if constexpr (COOP) if (nrec > 0) {
        // the record this thread evaluates: where it is and which link
        int rpos = 0, rk = 1;
        const bool rec = tid < nrec;
        if (rec) {
            rpos = a.recs[r0 + tid].pos;
            rk = a.recs[r0 + tid].meta & 15;
        }
        // the tile's records into LDS, 8 words per thread in flight
        {
            constexpr int RW = (int)(sizeof(TileRec<real>) / 4);
            const uint32_t* gw = reinterpret_cast<const uint32_t*>(a.recs + r0);
            uint32_t* lw = reinterpret_cast<uint32_t*>(lds.recs);
            const int n = nrec * RW;
            for (int base = 0; base < n; base += 8 * nthr) {
                uint32_t t[8];
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const int i = base + tid + j * nthr;
                    t[j] = gw[i < n ? i : 0];
                }
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const int i = base + tid + j * nthr;
                    if (i < n) lw[i] = t[j];
                }
            }
        }
        // profiles of the groups at the first and the second step
        if (tid < a.ngroups) {
            const GroupDev G = a.groups[tid];
            lds.prof[0][tid] = profile_of<real>(G, a.t_prev);
            lds.prof[1][tid] = profile_of<real>(G, a.t_prev + 1);
        }
        // the state the record's rule reads: the nine populations at its site
        // x and at x - c_k
        real h0[9], hb[9];
        const bool rule1 = rec && !a.local;
        if (rule1) {
            int rx = xs + (rpos & 255), ry = y0 - 3 + (rpos >> 8);
            bool rin;
            place<PER>(a.nx, a.ny, a.px, a.py, rx, ry, rin);
            const int so = sidx(rx, ry, a.ld);
            const int sb = wrap_off<PER>(rx, ry, -CX(rk), -CY(rk), a.nx, a.ny, a.ld, a.px, a.py);
#pragma unroll
            for (int j = 0; j < 9; ++j) {
                h0[j] = ldu(a.src + j * a.plane, so);
                hb[j] = ldu(a.src + j * a.plane, sb);
            }
        }
        __syncthreads();
        if (rule1) {
            const TileRec<real>& L = lds.recs[tid];
            const int meta = L.meta, kind = link_kind(L);
            const int g1 = ((meta >> 8) & 255) - 1, g2 = ((meta >> 16) & 255) - 1;
            real drx, jx, jy, pxxx, pyyx, pxyx;
            moments9(h0, drx, jx, jy, pxxx, pyyx, pxyx);
            real dry = real(0), pxxy = real(0), pyyy = real(0), pxyy = real(0);
            if (kind != SLBM_DIRICHLET && L.wy != real(0)) moments9(hb, dry, jx, jy, pxxy, pyyy, pxyy);
            const real gk = pick9(h0, rk), gkb = pick9(h0, OPP(rk));
            const real gky = ((meta >> 6) & 1) ? pick9(hb, rk) : real(0);
            const real p1 = lds.prof[0][g1];
            const real p2 = (kind != SLBM_DIRICHLET && g2 >= 0) ? lds.prof[0][g2] : real(0);
            lds.rule1()[rpos >> 8][rk - 1][rpos & 255] =
                rule_value<real>(a, L, gk, gkb, gky, drx, pxxx, pyyx, pxyx, dry, pxxy, pyyy, pxyy, p1, p2);
        }
        if (!a.local) {                                 // uniform over the workgroup
            __syncthreads();
            // the site's pulls along its cut links are the rule values
            if (in && fl != kVoid && fl != 0u) {
#pragma unroll
                for (int k = 1; k < 9; ++k)
                    if ((fl >> (k - 1)) & 1u) g[OPP(k)] = lds.rule1()[wave][k - 1][lane];
            }
        }
    }
    lds.dens[wave][lane] = site_finish<real, PER>(a, x, ys, in, !COOP, fl, g);
    __syncthreads();
    const bool cuts = wave_has_cuts(fl);
    const bool out = out_row && lane >= 3 && lane <= 60 && y < a.ny && x < a.nx && fl != kVoid;
    bool bad = false;
    if (wave >= 1 && wave <= R + 4) {
        real o[9];
        if (lane >= 1 && lane <= 62 && fl != kVoid) {
            Window<real> w;
            w.m = lds.dens[wave - 1][lane]; w.m_l = lds.dens[wave - 1][lane - 1]; w.m_r = lds.dens[wave - 1][lane + 1];
            w.c_l = lds.dens[wave][lane - 1]; w.c_r = lds.dens[wave][lane + 1];
            real jx, jy, ir;
            const bool b = cuts ? collide_core<real, true>(a, g, fl, w, lds.dens[wave + 1][lane],
                                                           lds.dens[wave + 1][lane - 1], lds.dens[wave + 1][lane + 1],
                                                           o, jx, jy, ir)
                                : collide_core<real, false>(a, g, fl, w, lds.dens[wave + 1][lane],
                                                            lds.dens[wave + 1][lane - 1], lds.dens[wave + 1][lane + 1],
                                                            o, jx, jy, ir);
            if (out) {
                bad = b;
                advance_u(ux, uy, jx, jy, ir);
            }
        } else {
#pragma unroll
            for (int i = 0; i < 9; ++i) o[i] = real(0);
        }
        if constexpr (!TWO) {
            if (out) {
#pragma unroll
                for (int i = 0; i < 9; ++i) stu(a.dst + i * a.plane, s, o[i]);
                stu(a.U, s, ux);
                stu(a.U + a.plane, s, uy);
            }
            return bad;
        }
#pragma unroll
        for (int i = 0; i < 9; ++i) post[wave - 1][i][lane] = o[i];
    }
    if constexpr (!TWO) return bad;
    __syncthreads();
    // second step, from the first step's post-collision populations
    if constexpr (COOP) if (nrec > 0) {
        // every rule value from the unmodified state first, then each into the
        // slot its site pulls from (a slot another rule reads -- across a
        // crack -- is overwritten only after all have read it)
        real v = real(0);
        int vr = 0, vi = 0, vl = 0;
        bool put = false;
        if (tid < nrec) {
            const TileRec<real>& L = lds.recs[tid];
            const int w = L.pos >> 8, l = L.pos & 255;
            if (w >= 2 && w <= R + 3 && l >= 2 && l <= 61) {
                const int meta = L.meta, kind = link_kind(L);
                const int g1 = ((meta >> 8) & 255) - 1, g2 = ((meta >> 16) & 255) - 1;
                const int k = meta & 15, kb = OPP(k), dx = CX(k), dy = CY(k);
                const LdsPrev<real> prev{post, w - 1, l};
                real drx, pxxx, pyyx, pxyx;
                stored_moments<real>(prev, 0, 0, drx, pxxx, pyyx, pxyx);
                const real gk = prev(k, 0, 0), gkb = prev(kb, 0, 0);
                const real gky = ((meta >> 6) & 1) ? prev(k, -dx, -dy) : real(0);
                real dry = real(0), pxxy = real(0), pyyy = real(0), pxyy = real(0);
                if (kind != SLBM_DIRICHLET && L.wy != real(0)) stored_moments<real>(prev, -dx, -dy, dry, pxxy, pyyy, pxyy);
                const real p1 = lds.prof[1][g1];
                const real p2 = (kind != SLBM_DIRICHLET && g2 >= 0) ? lds.prof[1][g2] : real(0);
                v = rule_value<real>(a, L, gk, gkb, gky, drx, pxxx, pyyx, pxyx, dry, pxxy, pyyy, pxyy, p1, p2);
                vr = w - 1 + dy;
                vi = kb;
                vl = l + dx;
                put = true;
            }
        }
        __syncthreads();
        if (put) post[vr][vi][vl] = v;
        __syncthreads();
    }
    if (wave >= 2 && wave <= R + 3) {
        const int r = wave - 1;
        const int lc = lane < 2 ? 2 : (lane > 61 ? 61 : lane);   // lanes 0, 1, 62, 63: no second-step site
#pragma unroll
        for (int i = 0; i < 9; ++i) g[i] = post[r - CY(i)][i][lc - CX(i)];
        const bool live = fl != kVoid;
        if constexpr (!COOP)
            if (live && fl != 0) boundary_fixup<real>(a, LdsPrev<real>{post, r, lc}, s, fl, a.t_prev + 1, g);
#pragma unroll
        for (int i = 0; i < 9; ++i) g[i] = live ? g[i] : real(0);
        lds.dens[wave][lane] = g[0] + g[1] + g[2] + g[3] + g[4] + g[5] + g[6] + g[7] + g[8];
    }
    __syncthreads();
    if (out) {
        Window<real> w;
        w.m = lds.dens[wave - 1][lane]; w.m_l = lds.dens[wave - 1][lane - 1]; w.m_r = lds.dens[wave - 1][lane + 1];
        w.c_l = lds.dens[wave][lane - 1]; w.c_r = lds.dens[wave][lane + 1];
        real o[9], jx, jy, ir;
        bad |= cuts ? collide_core<real, true>(a, g, fl, w, lds.dens[wave + 1][lane], lds.dens[wave + 1][lane - 1],
                                               lds.dens[wave + 1][lane + 1], o, jx, jy, ir)
                    : collide_core<real, false>(a, g, fl, w, lds.dens[wave + 1][lane], lds.dens[wave + 1][lane - 1],
                                                lds.dens[wave + 1][lane + 1], o, jx, jy, ir);
#pragma unroll
        for (int i = 0; i < 9; ++i) stu(a.dst + i * a.plane, s, o[i]);
        advance_u(ux, uy, jx, jy, ir);
        stu(a.U, s, ux);
        stu(a.U + a.plane, s, uy);
    }
    return bad;
}

// Waves per SIMD the two-step kernels are compiled for: in single precision
// enough for two workgroups of rows + 6 waves on a compute unit (7: at most 72
// VGPRs, up to 8 rows; 8: at most 64 VGPRs, 9 or 10 rows); in double
// precision no bound (one workgroup).
template <typename real>
constexpr int k2_waves(int rows) { return sizeof(real) == 4 ? (rows > 8 ? 8 : 7) : 1; }

// Two time steps of one plate: one workgroup of seg + 6 waves per tile
// (W = k2_waves(seg)); COOP: the boundary rules tile by tile from the
// plate's tile record lists.
template <typename real, bool PER, int W, bool COOP>
__global__ __launch_bounds__(1024, W) void k_step2(StepArgs<real> a)
{
    __shared__ TileLds<real, COOP> lds;
    const int tile = xcd_map(blockIdx.x, gridDim.x, a.group_shift);
    if (tile >= a.ntiles) return;                 // uniform over the workgroup
    flag_divergence(a.diverged, step_tile2<real, PER, true, COOP>(a, tile, lds));
}

// Per-plate state of the batched step, in device memory so that a captured
// graph of steps stays valid from one replay to the next.  The table holds
// two copies, one per launch parity: a launch reads its plates from copy
// `parity`, and the workgroup of each plate's first tile writes the plate's
// state for the next launch into copy parity ^ 1 (its buffers swapped, its
// clock and countdown advanced), so consecutive launches need no separate
// bookkeeping kernel.
template <typename real>
struct BatchPlate {
    StepArgs<real> args;       // src/dst and t_prev as of this launch
    long long remaining;       // steps still to take; 0: idle
    int active;                // 1 while remaining > 0
    int halted;                // 1 once the plate's divergence word was set: its tiles skip the arithmetic
};

// The plate's state after a launch of up to maxk steps: an active plate
// takes min(maxk, remaining) steps, reading one buffer and writing the other.
// A plate whose state overflowed in an earlier launch is halted: its steps
// are still counted (the host's account of every plate stays exact) but no
// longer computed, until the host retires it.
template <typename real>
__device__ __forceinline__ BatchPlate<real> batch_next(BatchPlate<real> B, int maxk)
{
    if (B.active && !B.halted && *(volatile unsigned int*)B.args.diverged) B.halted = 1;
    if (B.active) {
        const long long k = B.remaining < maxk ? B.remaining : maxk;
        real* t = const_cast<real*>(B.args.src);
        B.args.src = B.args.dst;
        B.args.dst = t;
        B.args.t_prev += k;
        B.args.local = 0;
        B.remaining -= k;
        B.active = B.remaining > 0 ? 1 : 0;
    }
    return B;
}

// One time step of every active plate of a batch in one launch.  The tiles of
// all plates (of one height, the launch's) are numbered consecutively
// (tile_start[p] is plate p's first); one workgroup per tile (the grid holds
// at least ntiles workgroups), tiles of a plate that is done return at once.
// plates points at 2 * cap descriptors (copy `parity` is read).
template <typename real, bool WIDE>
__global__ __launch_bounds__(1024) void k_step_batch(BatchPlate<real>* __restrict__ plates, int cap, int parity,
                                                     const int* __restrict__ tile_plate,
                                                     const int* __restrict__ tile_start, int ntiles, int group_shift)
{
    __shared__ real dens[kMaxTileRows + 2][66];
    const int t = xcd_map(blockIdx.x, gridDim.x, group_shift);
    if (t >= ntiles) return;                      // uniform over the workgroup
    const int p = tile_plate[t];
    const BatchPlate<real> B = plates[parity * cap + p];
    const int lt = t - tile_start[p];
    // the plate's first tile hands the next launch its state
    if (lt == 0 && threadIdx.x == 0) plates[(parity ^ 1) * cap + p] = batch_next(B, 1);
    if (!B.active || B.halted) return;
    flag_divergence(B.args.diverged, step_tile<real, false, WIDE>(B.args, lt, dens));
}

// Up to two time steps of every active plate of a batch in one launch (the
// tiles of the two-step kernel): each plate takes min(maxk, remaining).
// COOP: every plate carries tile lists (the boundary rules tile by tile).
template <typename real, int W, bool COOP>
__global__ __launch_bounds__(1024, W) void k_step2_batch(BatchPlate<real>* __restrict__ plates, int cap, int parity,
                                                      const int* __restrict__ tile_plate,
                                                      const int* __restrict__ tile_start, int ntiles, int maxk,
                                                      int group_shift)
{
    __shared__ TileLds<real, COOP> lds;
    const int t = xcd_map(blockIdx.x, gridDim.x, group_shift);
    if (t >= ntiles) return;                      // uniform over the workgroup
    const int p = tile_plate[t];
    const BatchPlate<real> B = plates[parity * cap + p];
    const int lt = t - tile_start[p];
    // the plate's first tile hands the next launch its state
    if (lt == 0 && threadIdx.x == 0) plates[(parity ^ 1) * cap + p] = batch_next(B, maxk);
    if (!B.active || B.halted) return;
    if (maxk >= 2 && B.remaining >= 2)
        flag_divergence(B.args.diverged, step_tile2<real, false, true, COOP>(B.args, lt, lds));
    else
        flag_divergence(B.args.diverged, step_tile2<real, false, false, COOP>(B.args, lt, lds));
}

}  // namespace slbm_dev
