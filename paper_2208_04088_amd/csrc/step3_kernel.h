// Device code of the three-dimensional (D3Q19) solid lattice-Boltzmann step.
//
// The paper's method (sections 2-4) is two-dimensional; its rules are local
// to a link, and this is their D3Q19 form: the same moments (eq:moments),
// source term (eq:sourceterm), equilibrium with the populations' own second
// moment (eq:fieq) and forced BGK collision (eq:coll), with c_s^2 = 1/3 and
// weights 1/3, 1/18, 1/36.  Walls are lattice-conforming planes at
// x = -1/2 and x = nx - 1/2 (q = 1/2), y and z periodic; the Dirichlet rule
// is eq:bbcon, the Neumann rule eq:abbcon with the boundary stress
// sigma* = Pi sigma(x) Pi + n t* + t* n - (t*.n) n n (Pi = I - n n).
//
// State: shifted post-collision populations g = f - r (r the rest state),
// SoA planes g[i][z][y][x], site offset (z ny + y) nx + x.  One step is two
// launches: k3_density (delta-rho of the pulled state, needed by the
// gradient stencil of every neighbour) and k3_step (pull with the wall
// rules, moments, source term, collision, U, store).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace slbm3_dev {

// D3Q19: rest; +x -x +y -y +z -z; (1,1,0) (-1,-1,0) (1,-1,0) (-1,1,0);
// (1,0,1) (-1,0,-1) (1,0,-1) (-1,0,1); (0,1,1) (0,-1,-1) (0,1,-1) (0,-1,1).
// Opposite directions are adjacent: opp(i) = i + 1 for odd i.
constexpr int kQ = 19;
constexpr int kCX[kQ] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
constexpr int kCY[kQ] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
constexpr int kCZ[kQ] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
__host__ __device__ constexpr int opp3(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }
__host__ __device__ constexpr double w3(int i) { return i == 0 ? 1.0 / 3.0 : (i <= 6 ? 1.0 / 18.0 : 1.0 / 36.0); }
__host__ __device__ constexpr int c2_3(int i) { return kCX[i] * kCX[i] + kCY[i] * kCY[i] + kCZ[i] * kCZ[i]; }

enum { kWallNone = 0, kWallDirichlet = 1, kWallNeumann = 2 };

template <typename real>
struct Step3Args {
    const real* src;           // post-collision state (pulled), or the populations themselves (local)
    real* dst;
    double* U;                 // [3] planes
    real* dens;                // delta-rho of the pulled state (written by k3_density)
    unsigned int* diverged;
    long long plane;           // sites per plane
    int nx, ny, nz;
    int px;                    // periodic in x (else walls)
    int local;                 // src holds the populations at the sites themselves
    int ntiles;                // 64-site row chunks
    int wkind[2];              // walls at x = -1/2, x = nx - 1/2
    real wval[2][3];           // lattice units: wall velocity (Dirichlet) or traction (Neumann)
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
template <typename real, bool PX>
__device__ __forceinline__ void pull3(const Step3Args<real>& a, const Site3& st, real g[kQ])
{
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const unsigned s = sidx3(st.x, st.y, st.z, nx, ny);
    if (a.local) {
#pragma unroll
        for (int i = 0; i < kQ; ++i) g[i] = a.src[i * a.plane + s];
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
        g[i] = a.src[i * a.plane + sidx3(xx, yy, zz, nx, ny)];
    }
    if (!PX && (st.x == 0 || st.x == nx - 1)) {
        real h[kQ];
#pragma unroll
        for (int i = 0; i < kQ; ++i) h[i] = a.src[i * a.plane + s];
        real dr, j[3], P[6];
        moments3(h, dr, j, P);
        // both walls when nx == 1
#pragma unroll
        for (int side = 0; side < 2; ++side) {
            if (side == 0 ? st.x != 0 : st.x != nx - 1) continue;
            const int kind = a.wkind[side];
            const real n = side == 0 ? real(-1) : real(1);
            const real* v = a.wval[side];
            // Neumann: boundary Poisson stress P* = -sigma* - (lambda - mu) drho I
            // with sigma = -P - (lambda - mu) drho I at the site
            real Ps[6];
            Ps[0] = -(n * v[0]) - a.lm * dr;                  // sigma*_xx = n t_x
            Ps[1] = P[1];                                     // tangential block: sigma*_tt = sigma_tt
            Ps[2] = P[2];
            Ps[3] = -(n * v[1]);                              // sigma*_xy = n t_y
            Ps[4] = -(n * v[2]);                              // sigma*_xz = n t_z
            Ps[5] = P[5];
            const real rho = real(1) + dr;
            const real jz[3] = {real(0), real(0), real(0)};
#pragma unroll
            for (int i = 1; i < kQ; ++i) {
                // link i leaves through this wall; its opposite returns
                if (kCX[i] != (side == 0 ? -1 : 1)) continue;
                real val;
                if (kind == kWallDirichlet) {
                    // eq:bbcon, q = 1/2: f_ib = f_i - 6 w_i c_i.j*, j* = rho v*
                    const real cv = real(kCX[i]) * v[0] + real(kCY[i]) * v[1] + real(kCZ[i]) * v[2];
                    val = h[i] - real(6.0 * w3(i)) * rho * cv;
                } else {
                    // eq:abbcon, q = 1/2: f_ib = -f_i + 2 f_eq,i(rho, 0, P*);
                    // shifted: g_ib = -g_i + 2 g_eq,i
                    real e;
                    switch (i) {
#define SLBM3_GEQ(k) case k: e = geq3<k, real>(dr, jz, Ps); break;
                        SLBM3_GEQ(1) SLBM3_GEQ(2) SLBM3_GEQ(3) SLBM3_GEQ(4) SLBM3_GEQ(5) SLBM3_GEQ(6)
                        SLBM3_GEQ(7) SLBM3_GEQ(8) SLBM3_GEQ(9) SLBM3_GEQ(10) SLBM3_GEQ(11) SLBM3_GEQ(12)
                        SLBM3_GEQ(13) SLBM3_GEQ(14) SLBM3_GEQ(15) SLBM3_GEQ(16) SLBM3_GEQ(17) SLBM3_GEQ(18)
#undef SLBM3_GEQ
                        default: e = real(0);
                    }
                    val = -h[i] + real(2) * e;
                }
                g[opp3(i)] = val;
            }
        }
    }
}

// Density gradient of eq:sourceterm, isotropic D3Q19 stencil
// grad = 3 sum_i w_i c_i rho(x + c_i), from the delta-rho buffer; across a
// cut link the neighbour is 2 rho(x) - rho(x - c_i) (rho(x) if that is cut too).
template <typename real, bool PX>
__device__ __forceinline__ void grad3(const Step3Args<real>& a, const Site3& st, real dr, real grad[3])
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
    // 3 w_i = 1/6 (axis), 1/12 (diagonals)
    grad[0] = real(1.0 / 6.0) * (nb[1] - nb[2]) +
              real(1.0 / 12.0) * ((nb[7] - nb[8]) + (nb[9] - nb[10]) + (nb[11] - nb[12]) + (nb[13] - nb[14]));
    grad[1] = real(1.0 / 6.0) * (nb[3] - nb[4]) +
              real(1.0 / 12.0) * ((nb[7] - nb[8]) - (nb[9] - nb[10]) + (nb[15] - nb[16]) + (nb[17] - nb[18]));
    grad[2] = real(1.0 / 6.0) * (nb[5] - nb[6]) +
              real(1.0 / 12.0) * ((nb[11] - nb[12]) - (nb[13] - nb[14]) + (nb[15] - nb[16]) - (nb[17] - nb[18]));
}

// Workgroups are dealt round-robin to the 8 XCDs; each XCD gets a contiguous
// band of tiles (nb, the grid size, is a multiple of 8).
__device__ __forceinline__ int xcd_band3(int b, int nb) { return (b & 7) * (nb >> 3) + (b >> 3); }

// delta-rho of the pulled state at every site.
template <typename real, bool PX>
__global__ __launch_bounds__(256) void k3_density(Step3Args<real> a)
{
    const int tile = xcd_band3(blockIdx.x, gridDim.x) * 4 + (threadIdx.x >> 6);
    if (tile >= a.ntiles) return;
    const Site3 st = site_of(tile, threadIdx.x & 63, a.nx, a.ny);
    real g[kQ];
    pull3<real, PX>(a, st, g);
    real dr = real(0);
#pragma unroll
    for (int i = 0; i < kQ; ++i) dr += g[i];
    if (st.in) a.dens[sidx3(st.x, st.y, st.z, a.nx, a.ny)] = dr;
}

// 1/x: the hardware reciprocal in single precision, a division in double.
__device__ __forceinline__ float recip3(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double recip3(double x) { return 1.0 / x; }

// One time step at every site: pull (with the wall rules), moments, source
// term, eq:coll, U += j/rho, store.
template <typename real, bool PX>
__global__ __launch_bounds__(256) void k3_step(Step3Args<real> a)
{
    const int tile = xcd_band3(blockIdx.x, gridDim.x) * 4 + (threadIdx.x >> 6);
    if (tile >= a.ntiles) return;
    const Site3 st = site_of(tile, threadIdx.x & 63, a.nx, a.ny);
    real g[kQ];
    pull3<real, PX>(a, st, g);
    real dr, j[3], P[6];
    moments3(g, dr, j, P);
    real grad[3];
    grad3<real, PX>(a, st, dr, grad);
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
    real o[kQ];
#define SLBM3_COLL(k)                                                                             \
    {                                                                                             \
        const real psi = real(3.0 * w3(k)) * (real(kCX[k]) * S[0] + real(kCY[k]) * S[1] + real(kCZ[k]) * S[2]); \
        o[k] = g[k] - a.omega * (g[k] - geq3<k, real>(dr, j, P)) + a.omega_h * psi;              \
    }
    SLBM3_COLL(0) SLBM3_COLL(1) SLBM3_COLL(2) SLBM3_COLL(3) SLBM3_COLL(4) SLBM3_COLL(5) SLBM3_COLL(6)
    SLBM3_COLL(7) SLBM3_COLL(8) SLBM3_COLL(9) SLBM3_COLL(10) SLBM3_COLL(11) SLBM3_COLL(12)
    SLBM3_COLL(13) SLBM3_COLL(14) SLBM3_COLL(15) SLBM3_COLL(16) SLBM3_COLL(17) SLBM3_COLL(18)
#undef SLBM3_COLL
    const bool bad = !(fabs(dr) + fabs(j[0]) + fabs(j[1]) + fabs(j[2]) < real(1e30));
    if (st.in) {
#pragma unroll
        for (int i = 0; i < kQ; ++i) a.dst[i * a.plane + s] = o[i];
#pragma unroll
        for (int k = 0; k < 3; ++k) a.U[k * a.plane + s] = a.U[k * a.plane + s] + (double)(j[k] * ir);
    }
    if (__any(bad && st.in) && (threadIdx.x & 63) == 0 && *(volatile unsigned int*)a.diverged == 0u)
        atomicOr(a.diverged, 1u);
}

// Outputs at every site (lattice units, double, planes of `out`): 0
// delta-rho, 1-3 j (with S/2), 4-9 P, 10-15 the Cauchy stress
// sigma = -P - (lambda - mu) drho I, 16-18 the displacement U + (j/rho)/2.
// Needs k3_density of the same state first.
template <typename real, bool PX>
__global__ __launch_bounds__(256) void k3_outputs(Step3Args<real> a, double* out)
{
    const int tile = xcd_band3(blockIdx.x, gridDim.x) * 4 + (threadIdx.x >> 6);
    if (tile >= a.ntiles) return;
    const Site3 st = site_of(tile, threadIdx.x & 63, a.nx, a.ny);
    real g[kQ];
    pull3<real, PX>(a, st, g);
    real dr, j[3], P[6];
    moments3(g, dr, j, P);
    real grad[3];
    grad3<real, PX>(a, st, dr, grad);
    const real rho = real(1) + dr;
    const real c = a.ml / rho;
    if (!st.in) return;
    const unsigned s = sidx3(st.x, st.y, st.z, a.nx, a.ny);
    const long long n = a.plane;
    out[s] = (double)dr;
    for (int k = 0; k < 3; ++k) {
        const double jk = (double)j[k] + 0.5 * ((double)a.F[k] + (double)c * (double)grad[k]);
        out[(1 + k) * n + s] = jk;
        out[(16 + k) * n + s] = a.U[k * n + s] + 0.5 * jk / (double)rho;
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
template <typename real, bool PX>
__global__ __launch_bounds__(256) void k3_init(Step3Args<real> a, const double* in)
{
    const int tile = xcd_band3(blockIdx.x, gridDim.x) * 4 + (threadIdx.x >> 6);
    if (tile >= a.ntiles) return;
    const Site3 st = site_of(tile, threadIdx.x & 63, a.nx, a.ny);
    const unsigned s = sidx3(st.x, st.y, st.z, a.nx, a.ny);
    const long long n = a.plane;
    const real dr = (real)in[s];
    real grad[3];
    grad3<real, PX>(a, st, dr, grad);
    const double rho = 1.0 + in[s];
    const real c = a.ml / (real)rho;
    real j[3], P[6];
    for (int k = 0; k < 3; ++k) j[k] = (real)(in[(1 + k) * n + s] - 0.5 * ((double)a.F[k] + (double)(c * grad[k])));
    for (int k = 0; k < 6; ++k) P[k] = (real)in[(4 + k) * n + s];
    if (!st.in) return;
    real* d = a.dst;
#define SLBM3_INIT(k) d[k * n + s] = geq3<k, real>(dr, j, P);
    SLBM3_INIT(0) SLBM3_INIT(1) SLBM3_INIT(2) SLBM3_INIT(3) SLBM3_INIT(4) SLBM3_INIT(5) SLBM3_INIT(6)
    SLBM3_INIT(7) SLBM3_INIT(8) SLBM3_INIT(9) SLBM3_INIT(10) SLBM3_INIT(11) SLBM3_INIT(12)
    SLBM3_INIT(13) SLBM3_INIT(14) SLBM3_INIT(15) SLBM3_INIT(16) SLBM3_INIT(17) SLBM3_INIT(18)
#undef SLBM3_INIT
    for (int k = 0; k < 3; ++k) a.U[k * n + s] = in[(10 + k) * n + s] - 0.5 * in[(1 + k) * n + s] / rho;
}

}  // namespace slbm3_dev
