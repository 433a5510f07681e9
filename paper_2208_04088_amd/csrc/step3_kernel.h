// Device code of the three-dimensional (D3Q19) solid lattice-Boltzmann step.
//
// The paper's method (sections 2-4) is two-dimensional; its rules are local
// to a link, and this is their D3Q19 form: the same moments (eq:moments),
// source term (eq:sourceterm), equilibrium with the populations' own second
// moment (eq:fieq) and forced BGK collision (eq:coll), with c_s^2 = 1/3 and
// weights 1/3, 1/18, 1/36.  Boundaries: either two planes normal to x that
// cut the links leaving the material at a fraction q (y and z periodic), or
// (GEO) a general geometry periodic on every axis -- a material mask and cut
// links, each with its own q, outward normal and group (cavities, cracks).
// The Dirichlet rule is eq:bbcon / eq:bbnoncon, the Neumann rule eq:abbcon /
// eq:abbnoncon with the boundary stress
// sigma* = Pi sigma_b Pi + n t* + t* n - (t*.n) n n (Pi = I - n n).
//
// State: shifted post-collision populations g = f - r (r the rest state),
// SoA planes g[i][z][y][x], site offset (z ny + y) nx + x; consecutive planes
// are `stride` elements apart, a little more than a plane, so that the 19
// streams of a pull do not all start on the same HBM channel.  One step is two
// launches: k3_density (delta-rho of the pulled state, needed by the
// gradient stencil of every neighbour) and k3_step (pull with the rules,
// moments, source term, collision, U, store; with a general geometry also
// the next step's rule values at the cut links), and with extrapolating
// Neumann links k3_links_ext before them.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace slbm3_dev {

// D3Q19: rest; +x -x +y -y +z -z; (1,1,0) (-1,-1,0) (1,-1,0) (-1,1,0);
// (1,0,1) (-1,0,-1) (1,0,-1) (-1,0,1); (0,1,1) (0,-1,-1) (0,1,-1) (0,-1,1).
// Opposite directions are adjacent: opp(i) = i + 1 for odd i.
constexpr int kQ = 19;

// A site update is flagged as diverged when |drho| + |j| (lattice units,
// rest density 1) reaches this bound -- a density deviation as large as the
// rest density itself, far outside linear elasticity -- or is not finite.
constexpr double kDivergeBound = 1.0;
constexpr int kCX[kQ] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
constexpr int kCY[kQ] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
constexpr int kCZ[kQ] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
__host__ __device__ constexpr int opp3(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }
__host__ __device__ constexpr double w3(int i) { return i == 0 ? 1.0 / 3.0 : (i <= 6 ? 1.0 / 18.0 : 1.0 / 36.0); }
__host__ __device__ constexpr int c2_3(int i) { return kCX[i] * kCX[i] + kCY[i] * kCY[i] + kCZ[i] * kCZ[i]; }

enum { kWallNone = 0, kWallDirichlet = 1, kWallNeumann = 2 };

// Site flags of a box with cut links (general geometry): bit i - 1 set when
// link i of the site is cut, kVoid3 for a void site.
constexpr uint32_t kVoid3 = 0x80000000u;
constexpr uint32_t kCutMask3 = 0x3FFFFu;

// One cut link (x, i) of a general geometry, in lattice units, with the
// rule's constants folded on the host.  Dirichlet (eq:bbcon / eq:bbnoncon):
//   g_ib = g_i + kappa (g_i(x - c_i) - g_ib) - rho(x) a c0,  c0 = beta 6 w_i c_i.v*.
// Neumann (eq:abbcon / eq:abbnoncon): g_ib = -g_i - kappa (g_i(x - c_i) + g_ib)
// + 2 beta e, with e = g_eq,i(rho_bd, 0, P*) the shifted equilibrium at the
// boundary stress sigma* = Pi sigma_b Pi + n t* + t* n - (t*.n) n n.  With
// A = c_i c_i - I/3 and sigma_b = -P_b - (lambda - mu) drho_bd I this is
// linear in the site's (or the extrapolated) drho_bd and P_b:
//   e = c0 drho_bd + sum_k B_k P_b,k - a K,
//   c0 = w_i [5/2 - 3/2 |c_i|^2 + 9/2 (lambda - mu)(tr(Pi A Pi) - |c_i|^2 + 1)],
//   B  = 9/2 w_i Pi A Pi (xx yy zz, then xy xz yz doubled),
//   K  = 9/2 w_i [2 n.A.t* - (t*.n) n.A.n].
// a is the time profile of the link's group (1, or a ramp: slot s of the
// launch's factor tables).  kappa and beta are 0 and 1 when the opposite link
// is cut too (no site behind); ext: Neumann with rho_bd and sigma_b
// extrapolated along the link, (1 + q) X(x) - q X(x - c_i).
template <typename real>
struct Link3 {
    real kap, bet2, q1, q;         // kappa, 2 beta, 1 + q, q
    real c0;
    real B[6];
    real K;
    uint32_t meta;                 // link3_meta
    int32_t site;                  // (z ny + y) nx + x of the material site x
};
// meta: direction k (5 bits), opposite (5), kind (2), ext (1), c + 1 per axis
// (2 each), time-profile slot (4)
constexpr int kProfileSlots3 = 16;          // slot 0: constant; 1..15: ramps
__host__ __device__ constexpr uint32_t link3_meta(int k, int kb, int kind, int ext, int cx, int cy, int cz, int slot)
{
    return (uint32_t)k | (uint32_t)kb << 5 | (uint32_t)kind << 10 | (uint32_t)ext << 12 |
           (uint32_t)(cx + 1) << 13 | (uint32_t)(cy + 1) << 15 | (uint32_t)(cz + 1) << 17 | (uint32_t)slot << 19;
}

template <typename real>
struct Step3Args {
    const real* src;           // post-collision state (pulled), or the populations themselves (local)
    real* dst;
    double* U;                 // [3] planes
    real* dens;                // delta-rho of the pulled state (written by k3_density)
    unsigned int* diverged;
    long long plane;           // sites per plane
    long long stride;          // elements from one plane of src, dst or U to the next (>= plane)
    int nx, ny, nz;
    int px;                    // periodic in x (else walls)
    int local;                 // src holds the populations at the sites themselves
    int ntiles;                // 64-site row chunks
    int wkind[2];              // walls crossing the first and the last site's x links
    real wval[2][3];           // lattice units: wall velocity (Dirichlet) or traction (Neumann)
    // per wall, from its q: kappa = (1 - 2q)/(1 + 2q), beta = 2/(1 + 2q)
    // (0 and 1 with no site behind, nx = 1); wext: Neumann with rho_bd and
    // the tangential stress extrapolated along the link, weights 1 + q, -q
    real wkap[2], wbeta[2], wq1[2], wq[2];
    int wext[2];
    // general geometry (periodic on every axis): site flags, each cut site's
    // first link record, the records (sorted by site and direction)
    const uint32_t* flags;
    const int32_t* bidx;
    const Link3<real>* links;
    real* lval;                // per record: (A, s_kappa), see cut_links3
    const int32_t* wrec;       // per workgroup of k3_step: its first record (one more: the count)
    // the groups' time profiles per slot, at the time of the state the pulls
    // read (pf_pull) and of the state the step produces (pf_next)
    real pf_pull[kProfileSlots3], pf_next[kProfileSlots3];
    real omega, omega_h;       // 1/tau, 1 - 1/(2 tau)
    real ml, lm;               // mu - lambda, lambda - mu (lattice units)
    real F[3];
};

// Shifted equilibrium g_eq,i = f_eq,i - r_i of eq:fieq, drho = rho - 1:
// w_i [drho (5/2 - 3|c|^2/2) + 3 c.j + 9/2 (P : (c c - I/3))].
template <int i, typename real>
__device__ __forceinline__ real geq3(real dr, const real j[3], const real P[6])
{
    constexpr int cx = kCX[i], cy = kCY[i], cz = kCZ[i];
    constexpr double w = w3(i);
    constexpr double a0 = w * (2.5 - 1.5 * c2_3(i));
    real v = real(a0) * dr;
    if (cx != 0) v += real(3.0 * w * cx) * j[0];
    if (cy != 0) v += real(3.0 * w * cy) * j[1];
    if (cz != 0) v += real(3.0 * w * cz) * j[2];
    v += real(4.5 * w * (cx * cx - 1.0 / 3.0)) * P[0];
    v += real(4.5 * w * (cy * cy - 1.0 / 3.0)) * P[1];
    v += real(4.5 * w * (cz * cz - 1.0 / 3.0)) * P[2];
    if (cx * cy != 0) v += real(9.0 * w * cx * cy) * P[3];
    if (cx * cz != 0) v += real(9.0 * w * cx * cz) * P[4];
    if (cy * cz != 0) v += real(9.0 * w * cy * cz) * P[5];
    return v;
}

// ------------------------------------------------------ ghost moments
//
// The collision of eq:coll leaves rho and P unchanged and adds S to j (the
// equilibrium carries the populations' own second moment).  It is applied as
//   g_i <- g_i + T_i(S) + sum_k a_k n_k,i
// with T(S) = (S_a/2)(e_{+a} - e_{-a}) on the axis links, whose zeroth,
// first and second moments are exactly 0, S and 0 in floating point, and nine
// integer ghost vectors n_k orthogonal to 1, c and c c (an orthogonal D3Q19
// moment basis: epsilon, q_x, q_y, q_z, 3 pi_xx, pi_ww, m_x, m_y, m_z).  The
// coefficients a_k are the projections of the BGK change onto the n_k:
//   a_k = [omega (E_k - m_k) + (1 - omega/2) Psi_k - tau_k] / N_k,
// m_k = n_k.g, E_k = n_k.g_eq, Psi_k = n_k.psi, tau_k = n_k.T, N_k = n_k.n_k.
// In exact arithmetic this is the BGK update; in floating point the conserved
// moments change only by unbiased rounding, whereas rounded equilibrium
// weights would scale them by (1 + omega eps) every step.
__host__ __device__ constexpr int ghost3(int k, int i)
{
    const int cx = kCX[i], cy = kCY[i], cz = kCZ[i];
    const int c2 = cx * cx + cy * cy + cz * cz;
    switch (k) {
    case 0: return (21 * c2 * c2 - 53 * c2 + 24) / 2;             // epsilon
    case 1: return (5 * c2 - 9) * cx;                             // q_x
    case 2: return (5 * c2 - 9) * cy;                             // q_y
    case 3: return (5 * c2 - 9) * cz;                             // q_z
    case 4: return (3 * c2 - 5) * (3 * cx * cx - c2);             // 3 pi_xx
    case 5: return (3 * c2 - 5) * (cy * cy - cz * cz);            // pi_ww
    case 6: return cx * (cy * cy - cz * cz);                      // m_x
    case 7: return cy * (cz * cz - cx * cx);                      // m_y
    default: return cz * (cx * cx - cy * cy);                     // m_z
    }
}
constexpr int kGhosts3 = 9;

// sum_i n_k,i f(i) for the lattice tables, at compile time
__host__ __device__ constexpr int ghost_dot_poly(int k, int px, int py, int pz)
{
    int s = 0;
    for (int i = 0; i < kQ; ++i) {
        int m = 1;
        for (int e = 0; e < px; ++e) m *= kCX[i];
        for (int e = 0; e < py; ++e) m *= kCY[i];
        for (int e = 0; e < pz; ++e) m *= kCZ[i];
        s += ghost3(k, i) * m;
    }
    return s;
}
__host__ __device__ constexpr bool ghosts_orthogonal()
{
    for (int k = 0; k < kGhosts3; ++k)
        for (int px = 0; px <= 2; ++px)
            for (int py = 0; py <= 2 - px; ++py)
                for (int pz = 0; pz <= 2 - px - py; ++pz)
                    if (ghost_dot_poly(k, px, py, pz) != 0) return false;
    for (int k = 0; k < kGhosts3; ++k)
        for (int l = 0; l < k; ++l) {
            int s = 0;
            for (int i = 0; i < kQ; ++i) s += ghost3(k, i) * ghost3(l, i);
            if (s != 0) return false;
        }
    return true;
}
static_assert(ghosts_orthogonal(), "ghost vectors must be orthogonal to 1, c, c c and to each other");

__host__ __device__ constexpr double ghost_norm(int k)
{
    double s = 0;
    for (int i = 0; i < kQ; ++i) s += double(ghost3(k, i)) * ghost3(k, i);
    return s;
}
// E_k = n_k.g_eq = er(k) drho + sum_a ej(k, a) j_a + sum_c ep(k, c) P_c (c: xx yy zz xy xz yz)
__host__ __device__ constexpr double ghost_er(int k)
{
    double s = 0;
    for (int i = 0; i < kQ; ++i) s += ghost3(k, i) * w3(i) * (2.5 - 1.5 * c2_3(i));
    return s;
}
__host__ __device__ constexpr double ghost_ej(int k, int a)      // also Psi_k per S_a
{
    double s = 0;
    for (int i = 0; i < kQ; ++i) s += ghost3(k, i) * 3.0 * w3(i) * (a == 0 ? kCX[i] : (a == 1 ? kCY[i] : kCZ[i]));
    return s;
}
__host__ __device__ constexpr double ghost_ep(int k, int c)
{
    double s = 0;
    for (int i = 0; i < kQ; ++i) {
        const int cx = kCX[i], cy = kCY[i], cz = kCZ[i];
        double t = 0;
        switch (c) {
        case 0: t = cx * cx - 1.0 / 3.0; break;
        case 1: t = cy * cy - 1.0 / 3.0; break;
        case 2: t = cz * cz - 1.0 / 3.0; break;
        case 3: t = 2.0 * cx * cy; break;
        case 4: t = 2.0 * cx * cz; break;
        default: t = 2.0 * cy * cz; break;
        }
        s += ghost3(k, i) * 4.5 * w3(i) * t;
    }
    return s;
}
// tau_k per S_a: T puts +S_a/2 on link +a (1, 3, 5) and -S_a/2 on -a (2, 4, 6)
__host__ __device__ constexpr double ghost_et(int k, int a) { return 0.5 * (ghost3(k, 1 + 2 * a) - ghost3(k, 2 + 2 * a)); }

// Coefficient of one ghost from the site's moments (drho, j with S/2, P),
// its populations and S.
template <int k, typename real>
__device__ __forceinline__ real ghost_coef3(const real g[kQ], real dr, const real j[3], const real P[6],
                                            const real S[3], real omega, real omega_h)
{
    real m = real(0);
#pragma unroll
    for (int i = 0; i < kQ; ++i) {
        const int n = ghost3(k, i);
        if (n == 1) m += g[i];
        else if (n == -1) m -= g[i];
        else if (n != 0) m += real(n) * g[i];
    }
    real e = real(ghost_er(k)) * dr;
#pragma unroll
    for (int a = 0; a < 3; ++a)
        if (ghost_ej(k, a) != 0.0) e += real(ghost_ej(k, a)) * j[a];
#pragma unroll
    for (int c = 0; c < 6; ++c)
        if (ghost_ep(k, c) != 0.0) e += real(ghost_ep(k, c)) * P[c];
    real src = real(0);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (ghost_ej(k, a) != 0.0) src += omega_h * (real(ghost_ej(k, a)) * S[a]);
        if (ghost_et(k, a) != 0.0) src -= real(ghost_et(k, a)) * S[a];
    }
    return (omega * (e - m) + src) * real(1.0 / ghost_norm(k));
}

// Post-collision populations o from g, the moments (j with S/2) and S.
template <typename real>
__device__ __forceinline__ void collide_ghost3(const real g[kQ], real dr, const real j[3], const real P[6],
                                               const real S[3], real omega, real omega_h, real o[kQ])
{
    real ak[kGhosts3];
    ak[0] = ghost_coef3<0>(g, dr, j, P, S, omega, omega_h);
    ak[1] = ghost_coef3<1>(g, dr, j, P, S, omega, omega_h);
    ak[2] = ghost_coef3<2>(g, dr, j, P, S, omega, omega_h);
    ak[3] = ghost_coef3<3>(g, dr, j, P, S, omega, omega_h);
    ak[4] = ghost_coef3<4>(g, dr, j, P, S, omega, omega_h);
    ak[5] = ghost_coef3<5>(g, dr, j, P, S, omega, omega_h);
    ak[6] = ghost_coef3<6>(g, dr, j, P, S, omega, omega_h);
    ak[7] = ghost_coef3<7>(g, dr, j, P, S, omega, omega_h);
    ak[8] = ghost_coef3<8>(g, dr, j, P, S, omega, omega_h);
    const real h[3] = {real(0.5) * S[0], real(0.5) * S[1], real(0.5) * S[2]};
#pragma unroll
    for (int i = 0; i < kQ; ++i) {
        real d = real(0);
#pragma unroll
        for (int k = 0; k < kGhosts3; ++k) {
            const int n = ghost3(k, i);
            if (n == 1) d += ak[k];
            else if (n == -1) d -= ak[k];
            else if (n != 0) d += real(n) * ak[k];
        }
        if (i >= 1 && i <= 6) d += (i & 1) ? h[(i - 1) >> 1] : -h[(i - 1) >> 1];
        o[i] = g[i] + d;
    }
}

// delta-rho, j and P (xx yy zz xy xz yz) of shifted populations.
template <typename real>
__device__ __forceinline__ void moments3(const real g[kQ], real& dr, real j[3], real P[6])
{
    dr = real(0);
    j[0] = j[1] = j[2] = real(0);
    for (int k = 0; k < 6; ++k) P[k] = real(0);
#pragma unroll
    for (int i = 0; i < kQ; ++i) {
        dr += g[i];
        if (kCX[i]) j[0] += kCX[i] > 0 ? g[i] : -g[i];
        if (kCY[i]) j[1] += kCY[i] > 0 ? g[i] : -g[i];
        if (kCZ[i]) j[2] += kCZ[i] > 0 ? g[i] : -g[i];
        if (kCX[i]) P[0] += g[i];
        if (kCY[i]) P[1] += g[i];
        if (kCZ[i]) P[2] += g[i];
        if (kCX[i] * kCY[i]) P[3] += kCX[i] * kCY[i] > 0 ? g[i] : -g[i];
        if (kCX[i] * kCZ[i]) P[4] += kCX[i] * kCZ[i] > 0 ? g[i] : -g[i];
        if (kCY[i] * kCZ[i]) P[5] += kCY[i] * kCZ[i] > 0 ? g[i] : -g[i];
    }
}

__device__ __forceinline__ int wrap(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

// Site (x, y, z) of a 64-site row chunk: tile t -> (chunk, y, z), chunks
// fastest; lanes past nx are outside.
struct Site3 {
    int x, y, z;
    bool in;
};

__device__ __forceinline__ Site3 site_of(int tile, int lane, int nx, int ny)
{
    const int chunks = (nx + 63) >> 6;
    const int c = tile % chunks, r = tile / chunks;
    Site3 s;
    s.x = (c << 6) + lane;
    s.y = r % ny;
    s.z = r / ny;
    s.in = s.x < nx;
    if (!s.in) s.x = nx - 1;                   // keep addresses in the grid
    return s;
}

__device__ __forceinline__ unsigned sidx3(int x, int y, int z, int nx, int ny)
{
    return ((unsigned)z * (unsigned)ny + (unsigned)y) * (unsigned)nx + (unsigned)x;
}

// The populations of the step at a site: pulled from the neighbours'
// post-collision values along uncut links; on a link cut by a wall the
// returning population comes from the wall rule, from the site's own
// post-collision populations (rho and P are those of the previous step,
// conserved by the collision).
// The rules of section 4 at the cut links of a general geometry.  The value
// a cut link (x, i) returns to x in direction ibar is A + s_kappa g_i(x - c_i):
// A takes only the post-collision state at x, s_kappa is kappa (Dirichlet) or
// -kappa (Neumann), and g_i(x - c_i) is the population the pull of direction
// i brings to x anyway (a thin link has kappa = 0 and needs none).  k3_step
// evaluates A at every cut link of its workgroup's sites as soon as it has
// their post-collision populations (one thread per link, through LDS), so
// the rules take no pass of their own over the state.  A link whose Neumann
// data are extrapolated along it (ext) needs the state at x - c_i as well:
// k3_links_ext evaluates its whole value, with s_kappa = 0.  lval holds
// (A, s_kappa) per record; s_kappa is set on the host.
//
// A from the record's folded constants (its own q, normal and group), g_i
// and g_ib at x, drho and (or, ext, rho_bd and P_b) at x.
template <typename real>
__device__ __forceinline__ real link_part3(const Link3<real>& L, real hi, real hib, real dr, real drb, const real Pb[6],
                                           real at)
{
    if (((L.meta >> 10) & 3u) == kWallDirichlet) return hi - L.kap * hib - (real(1) + dr) * (at * L.c0);
    const real e = L.c0 * drb + (L.B[0] * Pb[0] + L.B[1] * Pb[1] + L.B[2] * Pb[2]) +
                   (L.B[3] * Pb[3] + L.B[4] * Pb[4] + L.B[5] * Pb[5]) - at * L.K;
    return -hi - L.kap * hib + L.bet2 * e;
}

// The whole value of each ext link from the post-collision state, one thread
// per link (elink: the records' indices).
template <typename real>
__global__ __launch_bounds__(256) void k3_links_ext(Step3Args<real> a, const int32_t* elink, int n_ext)
{
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (t >= n_ext) return;
    const int l = elink[t];
    const Link3<real> L = a.links[l];
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const unsigned s = (unsigned)L.site;
    const int x = (int)(s % (unsigned)nx), y = (int)((s / (unsigned)nx) % (unsigned)ny),
              z = (int)(s / ((unsigned)nx * (unsigned)ny));
    const int i = (int)(L.meta & 31u), ib = (int)((L.meta >> 5) & 31u);
    const int cx = (int)((L.meta >> 13) & 3u) - 1, cy = (int)((L.meta >> 15) & 3u) - 1, cz = (int)((L.meta >> 17) & 3u) - 1;
    // the site behind x along the link, x - c_i (periodic axes)
    const unsigned sb = sidx3(wrap(x - cx, nx), wrap(y - cy, ny), wrap(z - cz, nz), nx, ny);
    real h[kQ];
#pragma unroll
    for (int k = 0; k < kQ; ++k) h[k] = a.src[k * a.stride + s];
    real dr, j[3], P[6];
    moments3(h, dr, j, P);
    const real hi = a.src[i * a.stride + s], hib = a.src[ib * a.stride + s], hy = a.src[i * a.stride + sb];
#pragma unroll
    for (int k = 0; k < kQ; ++k) h[k] = a.src[k * a.stride + sb];
    real dry, Py[6];
    moments3(h, dry, j, Py);
    const real drb = L.q1 * dr - L.q * dry;
#pragma unroll
    for (int c = 0; c < 6; ++c) P[c] = L.q1 * P[c] - L.q * Py[c];
    a.lval[2 * l] = link_part3(L, hi, hib, dr, drb, P, a.pf_pull[(L.meta >> 19) & 15u]) - L.kap * hy;
}

// A cut site's pulls along its cut links (the site's records are consecutive,
// in direction order, from bidx): A + s_kappa g_i(x - c_i), every value
// formed from the pulled populations before any is replaced.
template <typename real>
__device__ __forceinline__ void cut_links3(const Step3Args<real>& a, unsigned s, uint32_t fl, real g[kQ])
{
    const int li = a.bidx[s];
    const uint32_t m = fl & kCutMask3;
    real v[kQ];
#pragma unroll
    for (int k = 1; k < kQ; ++k)
        if ((m >> (k - 1)) & 1u) {
            const int l = li + __builtin_popcount(m & ((1u << (k - 1)) - 1u));
            v[k] = a.lval[2 * l] + a.lval[2 * l + 1] * g[k];
        }
#pragma unroll
    for (int k = 1; k < kQ; ++k)
        if ((m >> (k - 1)) & 1u) g[opp3(k)] = v[k];
}

template <typename real, bool PX, bool GEO = false>
__device__ __forceinline__ void pull3(const Step3Args<real>& a, const Site3& st, real g[kQ], uint32_t& fl)
{
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const unsigned s = sidx3(st.x, st.y, st.z, nx, ny);
    fl = GEO ? a.flags[s] : 0u;
    if (a.local) {
#pragma unroll
        for (int i = 0; i < kQ; ++i) g[i] = a.src[i * a.stride + s];
        if (GEO && (fl & kVoid3)) {
#pragma unroll
            for (int i = 0; i < kQ; ++i) g[i] = real(0);
        }
        return;
    }
    const int ym = wrap(st.y - 1, ny), yp = wrap(st.y + 1, ny);
    const int zm = wrap(st.z - 1, nz), zp = wrap(st.z + 1, nz);
    int xm = st.x - 1, xp = st.x + 1;
    if (PX) {
        xm = wrap(xm, nx);
        xp = wrap(xp, nx);
    } else {
        xm = xm < 0 ? 0 : xm;                  // cut links: replaced below
        xp = xp >= nx ? nx - 1 : xp;
    }
#pragma unroll
    for (int i = 0; i < kQ; ++i) {
        const int xx = kCX[i] > 0 ? xm : (kCX[i] < 0 ? xp : st.x);
        const int yy = kCY[i] > 0 ? ym : (kCY[i] < 0 ? yp : st.y);
        const int zz = kCZ[i] > 0 ? zm : (kCZ[i] < 0 ? zp : st.z);
        g[i] = a.src[i * a.stride + sidx3(xx, yy, zz, nx, ny)];
    }
    if constexpr (GEO) {
        // the pulls above are issued for every lane (in-grid addresses), so
        // that they do not wait for the flags
        if (fl & kVoid3) {                      // void: nothing to pull
#pragma unroll
            for (int i = 0; i < kQ; ++i) g[i] = real(0);
        } else if ((fl & kCutMask3) != 0u) {
            cut_links3<real>(a, s, fl, g);
        }
        return;
    }
    if (!PX && (st.x == 0 || st.x == nx - 1)) {
        real h[kQ];
#pragma unroll
        for (int i = 0; i < kQ; ++i) h[i] = a.src[i * a.stride + s];
        real dr, j[3], P[6];
        moments3(h, dr, j, P);
        // both walls when nx == 1
#pragma unroll
        for (int side = 0; side < 2; ++side) {
            if (side == 0 ? st.x != 0 : st.x != nx - 1) continue;
            const int kind = a.wkind[side];
            const real n = side == 0 ? real(-1) : real(1);
            const real* v = a.wval[side];
            const real kap = a.wkap[side], bet = a.wbeta[side];
            // the site behind x along a cut link, x - c_i, is the next site
            // inward (none in a one-site-wide slab, where kappa = 0)
            const int bx = nx == 1 ? st.x : (side == 0 ? st.x + 1 : st.x - 1);
            const real rho = real(1) + dr;
            const real jz[3] = {real(0), real(0), real(0)};
#pragma unroll
            for (int i = 1; i < kQ; ++i) {
                // link i leaves through this wall; its opposite returns
                if (kCX[i] != (side == 0 ? -1 : 1)) continue;
                const unsigned sb = sidx3(bx, wrap(st.y - kCY[i], ny), wrap(st.z - kCZ[i], nz), nx, ny);
                const real hy = a.src[i * a.stride + sb];    // f_i at x - c_i
                real val;
                if (kind == kWallDirichlet) {
                    // eq:bbcon / eq:bbnoncon: f_ib = f_i + kappa (f_i(x - c_i) - f_ib)
                    // - beta 6 w_i c_i.j*, j* = rho(x) v*
                    const real cv = real(kCX[i]) * v[0] + real(kCY[i]) * v[1] + real(kCZ[i]) * v[2];
                    val = h[i] + kap * (hy - h[opp3(i)]) - bet * (real(6.0 * w3(i)) * rho * cv);
                } else {
                    // eq:abbcon / eq:abbnoncon: f_ib = -f_i - kappa (f_i(x - c_i) + f_ib)
                    // + beta 2 f_eq,i(rho_bd, 0, P*); shifted: g_eq in place of f_eq.
                    // Boundary Poisson stress P* = -sigma* - (lambda - mu) drho_bd I with
                    // sigma = -P - (lambda - mu) drho I: its normal row from the traction,
                    // its tangential block that of P at the site, or extrapolated along
                    // the link, (1 + q) X(x) - q X(x - c_i)
                    real drb = dr, Pb1 = P[1], Pb2 = P[2], Pb5 = P[5];
                    if (a.wext[side]) {
                        real hb[kQ];
#pragma unroll
                        for (int k = 0; k < kQ; ++k) hb[k] = a.src[k * a.stride + sb];
                        real dry, jy[3], Py[6];
                        moments3(hb, dry, jy, Py);
                        const real w1 = a.wq1[side], w2 = a.wq[side];
                        drb = w1 * dr - w2 * dry;
                        Pb1 = w1 * P[1] - w2 * Py[1];
                        Pb2 = w1 * P[2] - w2 * Py[2];
                        Pb5 = w1 * P[5] - w2 * Py[5];
                    }
                    real Ps[6];
                    Ps[0] = -(n * v[0]) - a.lm * drb;             // sigma*_xx = n t_x
                    Ps[1] = Pb1;                                  // tangential block
                    Ps[2] = Pb2;
                    Ps[3] = -(n * v[1]);                          // sigma*_xy = n t_y
                    Ps[4] = -(n * v[2]);                          // sigma*_xz = n t_z
                    Ps[5] = Pb5;
                    real e;
                    switch (i) {
#define SLBM3_GEQ(k) case k: e = geq3<k, real>(drb, jz, Ps); break;
                        SLBM3_GEQ(1) SLBM3_GEQ(2) SLBM3_GEQ(3) SLBM3_GEQ(4) SLBM3_GEQ(5) SLBM3_GEQ(6)
                        SLBM3_GEQ(7) SLBM3_GEQ(8) SLBM3_GEQ(9) SLBM3_GEQ(10) SLBM3_GEQ(11) SLBM3_GEQ(12)
                        SLBM3_GEQ(13) SLBM3_GEQ(14) SLBM3_GEQ(15) SLBM3_GEQ(16) SLBM3_GEQ(17) SLBM3_GEQ(18)
#undef SLBM3_GEQ
                        default: e = real(0);
                    }
                    val = -h[i] - kap * (hy + h[opp3(i)]) + bet * (real(2) * e);
                }
                g[opp3(i)] = val;
            }
        }
    }
}

// Density gradient of eq:sourceterm, isotropic D3Q19 stencil
// grad = 3 sum_i w_i c_i rho(x + c_i), from the delta-rho buffer; across a
// cut link the neighbour is 2 rho(x) - rho(x - c_i) (rho(x) if that is cut too).
template <typename real, bool PX, bool GEO = false>
__device__ __forceinline__ void grad3(const Step3Args<real>& a, const Site3& st, real dr, real grad[3],
                                      uint32_t fl = 0u)
{
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const real* d = a.dens;
    const int ym = wrap(st.y - 1, ny), yp = wrap(st.y + 1, ny);
    const int zm = wrap(st.z - 1, nz), zp = wrap(st.z + 1, nz);
    const bool cutm = !PX && st.x == 0, cutp = !PX && st.x == nx - 1;
    const int xm = PX ? wrap(st.x - 1, nx) : (cutm ? st.x : st.x - 1);
    const int xp = PX ? wrap(st.x + 1, nx) : (cutp ? st.x : st.x + 1);
    real nb[kQ];
#pragma unroll
    for (int i = 1; i < kQ; ++i) {
        const int xx = kCX[i] > 0 ? xp : (kCX[i] < 0 ? xm : st.x);
        const int yy = kCY[i] > 0 ? yp : (kCY[i] < 0 ? ym : st.y);
        const int zz = kCZ[i] > 0 ? zp : (kCZ[i] < 0 ? zm : st.z);
        nb[i] = d[sidx3(xx, yy, zz, nx, ny)];
    }
    if (cutm || cutp) {
        real sub[kQ];
#pragma unroll
        for (int i = 1; i < kQ; ++i) {
            const bool ci = (kCX[i] < 0 && cutm) || (kCX[i] > 0 && cutp);
            const bool co = (kCX[i] > 0 && cutm) || (kCX[i] < 0 && cutp);
            sub[i] = ci ? (co ? dr : real(2) * dr - nb[opp3(i)]) : nb[i];
        }
#pragma unroll
        for (int i = 1; i < kQ; ++i) nb[i] = sub[i];
    }
    if (GEO && (fl & kCutMask3) != 0u) {
        real sub[kQ];
#pragma unroll
        for (int i = 1; i < kQ; ++i) {
            const bool ci = (fl >> (i - 1)) & 1u, co = (fl >> (opp3(i) - 1)) & 1u;
            sub[i] = ci ? (co ? dr : real(2) * dr - nb[opp3(i)]) : nb[i];
        }
#pragma unroll
        for (int i = 1; i < kQ; ++i) nb[i] = sub[i];
    }
    // 3 w_i = 1/6 (axis), 1/12 (diagonals)
    grad[0] = real(1.0 / 6.0) * (nb[1] - nb[2]) +
              real(1.0 / 12.0) * ((nb[7] - nb[8]) + (nb[9] - nb[10]) + (nb[11] - nb[12]) + (nb[13] - nb[14]));
    grad[1] = real(1.0 / 6.0) * (nb[3] - nb[4]) +
              real(1.0 / 12.0) * ((nb[7] - nb[8]) - (nb[9] - nb[10]) + (nb[15] - nb[16]) + (nb[17] - nb[18]));
    grad[2] = real(1.0 / 6.0) * (nb[5] - nb[6]) +
              real(1.0 / 12.0) * ((nb[11] - nb[12]) - (nb[13] - nb[14]) + (nb[15] - nb[16]) - (nb[17] - nb[18]));
}

// Workgroups are dealt round-robin to the 8 XCDs.  Each XCD takes groups of
// kXcdGroup consecutive workgroups, and the groups of the 8 XCDs interleave:
// the chip streams through one region of the box at a time (one set of 19
// plane streams rather than one per XCD), while rows that share neighbours
// stay in one L2.  The grid size is a multiple of 8 groups, which makes the
// map a permutation of the workgroup indices.  Groups of 16 suit the plane
// walls; a general geometry runs best with groups of 64 (its flags, link
// records and rule values stay longer in one L2: 0.98 against 1.09 ms per
// step on the 256^3 porous solid, while the slab is the same within 0.2 %).
__host__ __device__ constexpr int xcd_group_size3(bool geo) { return geo ? 64 : 16; }
template <bool GEO>
__device__ __forceinline__ int xcd_group3(int b)
{
    constexpr int G = xcd_group_size3(GEO);
    const int x = b & 7, l = b >> 3;
    return ((l / G) * 8 + x) * G + l % G;
}

// delta-rho of the pulled state at every site.
template <typename real, bool PX, bool GEO = false>
__global__ __launch_bounds__(256) void k3_density(Step3Args<real> a)
{
    const int tile = xcd_group3<GEO>(blockIdx.x) * 4 + (threadIdx.x >> 6);
    if (tile >= a.ntiles) return;
    const Site3 st = site_of(tile, threadIdx.x & 63, a.nx, a.ny);
    real g[kQ];
    uint32_t fl;
    pull3<real, PX, GEO>(a, st, g, fl);
    real dr = real(0);
#pragma unroll
    for (int i = 0; i < kQ; ++i) dr += g[i];
    if (GEO && (fl & kVoid3)) dr = real(0);               // void: never read
    if (st.in) a.dens[sidx3(st.x, st.y, st.z, a.nx, a.ny)] = dr;
}

// 1/x: the hardware reciprocal in single precision, a division in double.
__device__ __forceinline__ float recip3(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double recip3(double x) { return 1.0 / x; }

// One time step at every site: pull (with the wall rules), moments, source
// term, eq:coll, U += j/rho, store.
template <typename real, bool PX, bool GEO = false>
__global__ __launch_bounds__(256) void k3_step(Step3Args<real> a)
{
    const int wg = xcd_group3<GEO>(blockIdx.x);
    int tile = wg * 4 + (threadIdx.x >> 6);
    if (wg * 4 >= a.ntiles) return;                     // uniform over the workgroup
    const bool tvalid = tile < a.ntiles;
    if (!tvalid) {
        if constexpr (!GEO) return;
        tile = a.ntiles - 1;                            // GEO: stays for the barrier, stores nothing
    }
    Site3 st = site_of(tile, threadIdx.x & 63, a.nx, a.ny);
    if (!tvalid) st.in = false;
    real g[kQ];
    uint32_t fl;
    pull3<real, PX, GEO>(a, st, g, fl);
    const bool live = st.in && !(GEO && (fl & kVoid3));  // void sites stay at rest
    real dr, j[3], P[6];
    moments3(g, dr, j, P);
    real grad[3];
    grad3<real, PX, GEO>(a, st, dr, grad, fl);
    const real rho = real(1) + dr;
    const real ir = recip3(rho);
    const real c = a.ml * ir;
    real S[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        S[k] = a.F[k] + c * grad[k];
        j[k] = j[k] + real(0.5) * S[k];
    }
    const unsigned s = sidx3(st.x, st.y, st.z, a.nx, a.ny);
    // eq:coll in ghost-moment form (exact conserved moments)
    real o[kQ];
    collide_ghost3(g, dr, j, P, S, a.omega, a.omega_h, o);
    const bool bad = !(fabs(dr) + fabs(j[0]) + fabs(j[1]) + fabs(j[2]) < real(kDivergeBound));
    // void sites store the rest state (zeros) rather than nothing: whole
    // lines reach HBM, where a partly written line costs a read-modify-write
    if (st.in) {
#pragma unroll
        for (int i = 0; i < kQ; ++i) a.dst[i * a.stride + s] = live ? o[i] : real(0);
#pragma unroll
        for (int k = 0; k < 3; ++k)
            a.U[k * a.stride + s] = live ? a.U[k * a.stride + s] + (double)(j[k] * ir) : 0.0;
    }
    if (__any(bad && live) && (threadIdx.x & 63) == 0 && *(volatile unsigned int*)a.diverged == 0u)
        atomicOr(a.diverged, 1u);
    if constexpr (GEO) {
        // A at the cut links of the workgroup's sites (a contiguous range of
        // at most 256 from the first site of its first tile), one thread per
        // record, from the post-collision populations staged in LDS
        const int r0 = a.wrec[wg], nrec = a.wrec[wg + 1] - r0;   // uniform over the workgroup
        if (nrec > 0) {
            __shared__ real lo[kQ][256];
            const Site3 b0 = site_of(wg * 4, 0, a.nx, a.ny);
            const unsigned base = sidx3(b0.x, b0.y, b0.z, a.nx, a.ny);
            if (live) {
#pragma unroll
                for (int i = 0; i < kQ; ++i) lo[i][s - base] = o[i];
            }
            __syncthreads();
            for (int r = threadIdx.x; r < nrec; r += 256) {
                const Link3<real> L = a.links[r0 + r];
                if ((L.meta >> 12) & 1u) continue;              // ext: k3_links_ext
                const int slot = (int)((unsigned)L.site - base);
                real h[kQ];
#pragma unroll
                for (int i = 0; i < kQ; ++i) h[i] = lo[i][slot];
                real hd, hj[3], hP[6];
                moments3(h, hd, hj, hP);
                const int k = (int)(L.meta & 31u), kb = (int)((L.meta >> 5) & 31u);
                a.lval[2 * (r0 + r)] =
                    link_part3(L, lo[k][slot], lo[kb][slot], hd, hd, hP, a.pf_next[(L.meta >> 19) & 15u]);
            }
        }
    }
}

// Outputs at every site (lattice units, double, planes of `out`): 0
// delta-rho, 1-3 j (with S/2), 4-9 P, 10-15 the Cauchy stress
// sigma = -P - (lambda - mu) drho I, 16-18 the displacement U + (j/rho)/2.
// Needs k3_density of the same state first.
template <typename real, bool PX, bool GEO = false>
__global__ __launch_bounds__(256) void k3_outputs(Step3Args<real> a, double* out)
{
    const int tile = xcd_group3<GEO>(blockIdx.x) * 4 + (threadIdx.x >> 6);
    if (tile >= a.ntiles) return;
    const Site3 st = site_of(tile, threadIdx.x & 63, a.nx, a.ny);
    real g[kQ];
    uint32_t fl;
    pull3<real, PX, GEO>(a, st, g, fl);
    real dr, j[3], P[6];
    moments3(g, dr, j, P);
    real grad[3];
    grad3<real, PX, GEO>(a, st, dr, grad, fl);
    const real rho = real(1) + dr;
    const real c = a.ml / rho;
    if (!st.in) return;
    const unsigned s = sidx3(st.x, st.y, st.z, a.nx, a.ny);
    const long long n = a.plane;
    if (GEO && (fl & kVoid3)) {                             // void sites report zeros (rho too)
        out[s] = -1.0;
        for (int k = 1; k < 19; ++k) out[k * n + s] = 0.0;
        return;
    }
    out[s] = (double)dr;
    for (int k = 0; k < 3; ++k) {
        const double jk = (double)j[k] + 0.5 * ((double)a.F[k] + (double)c * (double)grad[k]);
        out[(1 + k) * n + s] = jk;
        out[(16 + k) * n + s] = a.U[k * a.stride + s] + 0.5 * jk / (double)rho;
    }
    for (int k = 0; k < 6; ++k) {
        out[(4 + k) * n + s] = (double)P[k];
        out[(10 + k) * n + s] = -(double)P[k] - (k < 3 ? (double)a.lm * (double)dr : 0.0);
    }
}

// delta-rho of the initial fields into the density buffer (k3_init's stencil).
template <typename real>
__global__ __launch_bounds__(256) void k3_set_dens(Step3Args<real> a, const double* in)
{
    const long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (s < a.plane) a.dens[s] = (real)in[s];
}

// Initial state from fields (lattice units, double, planes of `in`): 0
// delta-rho, 1-3 j, 4-9 P, 10-12 u0; dens must hold delta-rho.  Populations
// g = g_eq(drho, j - S/2, P) at the sites themselves (the state is "local"),
// U = u0 - (j/rho)/2.
template <typename real, bool PX, bool GEO = false>
__global__ __launch_bounds__(256) void k3_init(Step3Args<real> a, const double* in)
{
    const int tile = xcd_group3<GEO>(blockIdx.x) * 4 + (threadIdx.x >> 6);
    if (tile >= a.ntiles) return;
    const Site3 st = site_of(tile, threadIdx.x & 63, a.nx, a.ny);
    const unsigned s = sidx3(st.x, st.y, st.z, a.nx, a.ny);
    const long long n = a.plane;
    const uint32_t fl = GEO ? a.flags[s] : 0u;
    if (GEO && (fl & kVoid3)) {                             // void: the rest state, no displacement
        if (st.in) {
            for (int k = 0; k < kQ; ++k) a.dst[k * a.stride + s] = real(0);
            for (int k = 0; k < 3; ++k) a.U[k * a.stride + s] = 0.0;
        }
        return;
    }
    const real dr = (real)in[s];
    real grad[3];
    grad3<real, PX, GEO>(a, st, dr, grad, fl);
    const double rho = 1.0 + in[s];
    const real c = a.ml / (real)rho;
    real j[3], P[6];
    for (int k = 0; k < 3; ++k) j[k] = (real)(in[(1 + k) * n + s] - 0.5 * ((double)a.F[k] + (double)(c * grad[k])));
    for (int k = 0; k < 6; ++k) P[k] = (real)in[(4 + k) * n + s];
    if (!st.in) return;
    real* d = a.dst;
#define SLBM3_INIT(k) d[k * a.stride + s] = geq3<k, real>(dr, j, P);
    SLBM3_INIT(0) SLBM3_INIT(1) SLBM3_INIT(2) SLBM3_INIT(3) SLBM3_INIT(4) SLBM3_INIT(5) SLBM3_INIT(6)
    SLBM3_INIT(7) SLBM3_INIT(8) SLBM3_INIT(9) SLBM3_INIT(10) SLBM3_INIT(11) SLBM3_INIT(12)
    SLBM3_INIT(13) SLBM3_INIT(14) SLBM3_INIT(15) SLBM3_INIT(16) SLBM3_INIT(17) SLBM3_INIT(18)
#undef SLBM3_INIT
    for (int k = 0; k < 3; ++k) a.U[k * a.stride + s] = in[(10 + k) * n + s] - 0.5 * in[(1 + k) * n + s] / rho;
}

}  // namespace slbm3_dev
