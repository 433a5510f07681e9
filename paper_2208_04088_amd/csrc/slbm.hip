// slbm.hip -- solid lattice-Boltzmann step for MI355X (gfx950) behind the C
// ABI declared in include/slbm.h.
//
// Method: Faust, Schlueter, H. Mueller, R. Mueller, "Dirichlet and Neumann
// boundary conditions in a Lattice Boltzmann Method for Elastodynamics"
// (2022), sections 2-4.  See include/slbm.h for the problem statement and
// conventions.
//
// Data layout in HBM (one plate):
//   populations  two buffers of [9][ny+2][ld] `real`, structure of arrays:
//                site (x, y) sits at row y+1, column x+64 of each plane, inside
//                a padding ring that no step writes (one row above and below,
//                64 columns left, at least one right), so that the pull
//                addresses of every in-grid site stay inside the allocation
//                and can be issued before the site's flags arrive, and so
//                that the 64 columns a wave owns start on a 256-byte
//                boundary.  The row pitch ld is a multiple of 64.  They hold shifted
//                populations g_i = f_i - r_i, r_i the rest equilibrium
//                (8/9, 1/18 x4, -1/36 x4), so that fp32 resolves the small
//                deviation from rest instead of the O(1) rest values.
//   U            [2][ny+2][ld] double, the running sum of j/rho.
//   flags        [ny+2][ld] uint8: 0 = material site with no cut link,
//                0xFF = no state (void or the ring), otherwise bit k-1 set
//                when the link toward x + c_k is cut.
//   bidx         [ny+2][ld] int32, index of the site's first cut-link record
//                (read only at boundary sites).
//   links        one record per cut link, sorted by (site, direction), with
//                the coefficients of its boundary rule precomputed.
//
// A buffer holds, after a step, the post-collision populations of that step
// at their own site.  The next step pulls g_i(x) from x - c_i and, for a cut
// link (x, k), evaluates the boundary rule of section 4 from the
// post-collision values at x and x - c_k -- the rule the paper applies right
// after streaming, moved to the start of the next step so that streaming,
// boundary rules, moments, collision and displacement update are one pass
// over HBM.  Density and Poisson stress at time t, which the Neumann rule
// needs, are sums of post-collision populations because the collision
// conserves both.  After slbm_create or slbm_init_fields a buffer holds the
// populations themselves ("local" state) and the first step reads them in
// place.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <climits>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "slbm.h"

namespace {

// ------------------------------------------------------------------ errors

thread_local std::string g_err;

int fail(int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

// Runs the body of a C entry point: no exception crosses the ABI (host
// allocation failure is SLBM_E_NOMEM).
template <class F>
int guarded(F&& body) noexcept
{
    try {
        return body();
    } catch (const std::bad_alloc&) {
        return fail(SLBM_E_NOMEM, "host allocation failed");
    } catch (...) {
        return fail(SLBM_E_DEVICE, "unexpected host error");
    }
}

#define HIP_TRY(expr)                                                              \
    do {                                                                           \
        hipError_t e_ = (expr);                                                    \
        if (e_ != hipSuccess)                                                      \
            return fail(SLBM_E_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

}  // namespace

#include "step_kernel.h"

namespace {

using namespace slbm_dev;

// ------------------------------------------------------ output kernels

// delta-rho of the current state at every site (0 where there is no state).
template <typename real, bool PER>
__global__ __launch_bounds__(256) void k_density(StepArgs<real> a, double* dr_out)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= a.plane) return;
    const int y = idx / a.ld - 1, x = idx % a.ld - kPadL;
    double v = 0.0;
    if (x >= 0 && x < a.nx && y >= 0 && y < a.ny) {
        real g[9];
        unsigned fl;
        if (fetch_site<real, PER>(a, x, y, g, fl)) {
            double s = 0.0;
            for (int i = 0; i < 9; ++i) s += (double)g[i];
            v = s;
        }
    }
    dr_out[idx] = v;
}

// Density-gradient stencil at a site from a delta-rho field (same closure as
// the step kernel).
template <bool PER>
__device__ void grad_rho(const double* dr, const uint8_t* flags, int x, int y, int nx, int ny, int ld,
                         int px, int py, double& gx, double& gy)
{
    const unsigned fl = flags[sidx(x, y, ld)];
    const double d0 = dr[sidx(x, y, ld)];
    double nb[9];
#pragma unroll
    for (int i = 1; i < 9; ++i) {
        const bool ci = (fl >> (i - 1)) & 1u;
        nb[i] = ci ? 0.0 : dr[wrap_off<PER>(x, y, CX(i), CY(i), nx, ny, ld, px, py)];
    }
    double rt[9];
#pragma unroll
    for (int i = 1; i < 9; ++i) {
        const bool ci = (fl >> (i - 1)) & 1u;
        const bool co = (fl >> (OPP(i) - 1)) & 1u;
        rt[i] = ci ? (co ? d0 : 2.0 * d0 - nb[OPP(i)]) : nb[i];
    }
    gx = (1.0 / 3.0) * (rt[1] - rt[3]) + (1.0 / 12.0) * (rt[5] - rt[6] - rt[7] + rt[8]);
    gy = (1.0 / 3.0) * (rt[2] - rt[4]) + (1.0 / 12.0) * (rt[5] + rt[6] - rt[7] - rt[8]);
}

// Lattice-unit moments and displacement of the material site (x, y) (padded
// offset idx) from the current state and the density field dr: o[11] = rho,
// jx, jy, Pxx, Pyy, Pxy, sxx, syy, sxy, ux, uy (eq:moments with the half-step
// source, eq:poissonstress with eq:approxdiv, the trapezoid displacement).
template <typename real, bool PER>
__device__ __forceinline__ void site_outputs(const StepArgs<real>& a, const double* dr, int x, int y, int idx,
                                             double o[11])
{
    real g[9];
    unsigned fl;
    fetch_site<real, PER>(a, x, y, g, fl);
    double gd[9];
    for (int i = 0; i < 9; ++i) gd[i] = (double)g[i];
    double d, jx, jy, pxx, pyy, pxy;
    moments9(gd, d, jx, jy, pxx, pyy, pxy);
    double gx, gy;
    grad_rho<PER>(dr, a.flags, x, y, a.nx, a.ny, a.ld, a.px, a.py, gx, gy);
    const double rho = 1.0 + d;
    const double c = (double)a.ml / rho;
    jx += 0.5 * ((double)a.Fx + c * gx);
    jy += 0.5 * ((double)a.Fy + c * gy);
    const double lm = (double)a.lm;
    o[0] = rho; o[1] = jx; o[2] = jy; o[3] = pxx; o[4] = pyy; o[5] = pxy;
    o[6] = -pxx - lm * d; o[7] = -pyy - lm * d; o[8] = -pxy;
    // trapezoid readout: U holds u0 - v0/2 + sum of earlier j/rho
    o[9] = a.U[idx] + 0.5 * jx / rho;
    o[10] = a.U[a.plane + idx] + 0.5 * jy / rho;
}

// Padded planes out[11] (site_outputs; zero where there is no state), or
// only ux, uy (ncomp 2).
template <typename real, bool PER>
__global__ __launch_bounds__(256) void k_outputs(StepArgs<real> a, const double* dr, double* out, int ncomp)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    const long long P = a.plane;
    if (idx >= P) return;
    const int y = idx / a.ld - 1, x = idx % a.ld - kPadL;
    double o[11] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    if (x >= 0 && x < a.nx && y >= 0 && y < a.ny && a.flags[idx] != kVoid) site_outputs<real, PER>(a, dr, x, y, idx, o);
    if (ncomp == 11) {
        for (int c = 0; c < 11; ++c) out[c * P + idx] = o[c];
    } else {
        out[idx] = o[9];
        out[P + idx] = o[10];
    }
}

// The displacement straight into an unpadded [2][ny][nx] array (zero where
// there is no state): the values k_outputs gives, without its padded planes.
template <typename real, bool PER>
__global__ __launch_bounds__(256) void k_displacement_out(StepArgs<real> a, const double* dr, double* u)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    const int n = a.nx * a.ny;
    if (idx >= n) return;
    const int y = idx / a.nx, x = idx - y * a.nx;
    const int s = sidx(x, y, a.ld);
    double o[11] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    if (a.flags[s] != kVoid) site_outputs<real, PER>(a, dr, x, y, s, o);
    u[idx] = o[9];
    u[n + idx] = o[10];
}

// One padded plane into an unpadded, contiguous [ny][nx] array.
__global__ __launch_bounds__(256) void k_unpad(const double* plane, int nx, int ny, int ld, double* dst)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= nx * ny) return;
    const int y = idx / nx, x = idx - y * nx;
    dst[idx] = plane[sidx(x, y, ld)];
}

// Displacement into a caller's unpadded [2][ny][nx] device array.
__global__ __launch_bounds__(256) void k_unpad_u(const double* out, int nx, int ny, int ld, double* u)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= nx * ny) return;
    const int y = idx / nx, x = idx - y * nx;
    const long long P = (long long)(ny + 2) * ld;
    u[idx] = out[sidx(x, y, ld)];
    u[(long long)nx * ny + idx] = out[P + sidx(x, y, ld)];
}

// One padded lattice-unit plane, times a unit scale, into a caller's
// unpadded [ny][nx] device array of doubles or floats.
template <typename T>
__global__ __launch_bounds__(256) void k_unpad_scaled(const double* plane, int nx, int ny, int ld, double scale,
                                                      T* dst)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= nx * ny) return;
    const int y = idx / nx, x = idx - y * nx;
    dst[idx] = (T)(plane[sidx(x, y, ld)] * scale);
}

// ------------------------------------------------------- initial state

// Equilibrium of given lattice-unit fields (drho, j, P) with j the physical
// momentum: the populations carry j - S/2 so that eq:moments returns j.
template <typename real, bool PER>
__global__ __launch_bounds__(256) void k_init(StepArgs<real> a, const double* dr, const double* jf,
                                              const double* Pf, const double* uf, real* g_out)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    const long long P = a.plane;
    if (idx >= P) return;
    const int y = idx / a.ld - 1, x = idx % a.ld - kPadL;
    double gi[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    double ux = 0, uy = 0;
    if (x >= 0 && x < a.nx && y >= 0 && y < a.ny && a.flags[idx] != kVoid) {
        double gx, gy;
        grad_rho<PER>(dr, a.flags, x, y, a.nx, a.ny, a.ld, a.px, a.py, gx, gy);
        const double d = dr[idx], rho = 1.0 + d;
        const double c = (double)a.ml / rho;
        const double Sx = (double)a.Fx + c * gx, Sy = (double)a.Fy + c * gy;
        const double jx = jf[idx], jy = jf[P + idx];
        const double rx = jx - 0.5 * Sx, ry = jy - 0.5 * Sy;
        const double pxx = Pf[idx], pyy = Pf[P + idx], pxy = Pf[2 * P + idx];
        gi[0] = geq<0>(d, rx, ry, pxx, pyy, pxy);
        gi[1] = geq<1>(d, rx, ry, pxx, pyy, pxy);
        gi[2] = geq<2>(d, rx, ry, pxx, pyy, pxy);
        gi[3] = geq<3>(d, rx, ry, pxx, pyy, pxy);
        gi[4] = geq<4>(d, rx, ry, pxx, pyy, pxy);
        gi[5] = geq<5>(d, rx, ry, pxx, pyy, pxy);
        gi[6] = geq<6>(d, rx, ry, pxx, pyy, pxy);
        gi[7] = geq<7>(d, rx, ry, pxx, pyy, pxy);
        gi[8] = geq<8>(d, rx, ry, pxx, pyy, pxy);
        ux = uf[idx] - 0.5 * jx / rho;
        uy = uf[P + idx] - 0.5 * jy / rho;
    }
    for (int i = 0; i < 9; ++i) g_out[i * P + idx] = (real)gi[i];
    a.U[idx] = ux;
    a.U[P + idx] = uy;
}

// Plain streaming copy (one 16-byte access per thread): the bandwidth
// reference the step is compared with, and the known-size kernel that
// calibrates the memory counters.
__global__ __launch_bounds__(256) void k_copy16(const float4* __restrict__ src, float4* __restrict__ dst, long long n)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

}  // namespace

// ======================================================= host side (C ABI)

namespace {

// Device memory of a batch: one allocation of the batch's budget, handed out
// first-fit in 256-byte aligned blocks.  A block released while queued work
// may still touch it becomes reusable once events recorded after that work
// have completed, so that nothing the serving loop calls while the GPU runs
// has to wait for the device (hipFree would).  Allocation fails, rather than
// exceed the budget, when no free block is large enough.
struct Arena {
    static constexpr size_t kAlign = 256;
    char* base = nullptr;
    size_t size = 0;
    std::map<size_t, size_t> free_;                   // offset -> length, coalesced
    std::map<size_t, size_t> used;                    // offset -> length
    size_t deferred_bytes = 0;
    struct Deferred {
        std::vector<hipEvent_t> events;               // all must complete
        std::vector<size_t> offs;
        std::vector<hipEvent_t> destroy;              // per-plate events retired with the blocks
    };
    std::deque<Deferred> deferred;

    hipError_t init(size_t n)
    {
        size = (n + kAlign - 1) / kAlign * kAlign;
        const hipError_t e = hipMalloc((void**)&base, size);
        if (e == hipSuccess) free_[0] = size;
        return e;
    }
    size_t live() const
    {
        size_t s = deferred_bytes;
        for (const auto& u : used) s += u.second;
        return s;
    }
    void give_back(size_t off)
    {
        auto it = used.find(off);
        if (it == used.end()) return;
        size_t o = off, len = it->second;
        used.erase(it);
        auto nx = free_.lower_bound(o);
        if (nx != free_.end() && nx->first == o + len) {
            len += nx->second;
            nx = free_.erase(nx);
        }
        if (nx != free_.begin()) {
            auto pv = std::prev(nx);
            if (pv->first + pv->second == o) {
                pv->second += len;
                return;
            }
        }
        free_[o] = len;
    }
    bool done(const Deferred& d) const
    {
        for (hipEvent_t e : d.events)
            if (hipEventQuery(e) != hipSuccess) return false;
        return true;
    }
    void retire(Deferred& d)
    {
        for (hipEvent_t e : d.events) (void)hipEventDestroy(e);
        for (hipEvent_t e : d.destroy) (void)hipEventDestroy(e);
        for (size_t o : d.offs) {
            deferred_bytes -= used_len(o);
            give_back(o);
        }
    }
    size_t used_len(size_t o) const
    {
        auto it = used.find(o);
        return it == used.end() ? 0 : it->second;
    }
    // Returns blocks whose events have completed to the free list; with wait,
    // waits for the oldest outstanding release first.
    void reclaim(bool wait)
    {
        if (wait && !deferred.empty())
            for (hipEvent_t e : deferred.front().events) (void)hipEventSynchronize(e);
        while (!deferred.empty() && done(deferred.front())) {
            retire(deferred.front());
            deferred.pop_front();
        }
    }
    void* try_alloc(size_t n)
    {
        n = (n + kAlign - 1) / kAlign * kAlign;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < n) continue;
            const size_t o = it->first, len = it->second;
            free_.erase(it);
            if (len > n) free_[o + n] = len - n;
            used[o] = n;
            return base + o;
        }
        return nullptr;
    }
    // nullptr when no block fits even after every outstanding release has completed
    void* alloc(size_t n)
    {
        if (n == 0) n = 1;
        reclaim(false);
        for (;;) {
            if (void* p = try_alloc(n)) return p;
            if (deferred.empty()) return nullptr;
            reclaim(true);
        }
    }
    void release(void* p)
    {
        if (p) give_back((size_t)((char*)p - base));
    }
    // Releases blocks once every event of evs (recorded after the last work
    // that may touch them) has completed; the events are the arena's now.
    void release_after(std::vector<hipEvent_t> evs, const std::vector<void*>& ptrs,
                       std::vector<hipEvent_t> destroy = {})
    {
        Deferred d;
        d.events = std::move(evs);
        d.destroy = std::move(destroy);
        for (void* p : ptrs) {
            if (!p) continue;
            const size_t o = (size_t)((char*)p - base);
            d.offs.push_back(o);
            deferred_bytes += used_len(o);
        }
        deferred.push_back(std::move(d));
    }
    void destroy_all()
    {
        for (Deferred& d : deferred) {
            for (hipEvent_t e : d.events) (void)hipEventSynchronize(e);
            retire(d);
        }
        deferred.clear();
        if (base) (void)hipFree(base);
        base = nullptr;
        used.clear();
        free_.clear();
    }
};

}  // namespace

struct slbm_batch_s;

struct slbm_s {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int nx = 0, ny = 0, ld = 0;
    long long plane = 0;
    int precision = SLBM_FP64;
    int px = 0, py = 0, norder = 1;
    double lamL = 0, muL = 1.0 / 3.0, tau = 0.55, FL[2] = {0, 0};
    double dt_user = 1, s_sigma = 1, s_v = 1, rho_user = 1;
    size_t esize = 8;
    void* buf[2] = {nullptr, nullptr};
    int cur = 0;
    double* U = nullptr;
    uint8_t* flags = nullptr;
    int32_t* bidx = nullptr;
    void* links = nullptr;
    GroupDev* groups = nullptr;
    unsigned int* diverged = nullptr;
    double* scratch = nullptr;       // outputs and initial fields, allocated on demand
    int scratch_planes = 0;
    // a plate owned by a batch: device memory from the batch's arena, the
    // divergence word and the readout scratch the batch's, readouts queued on
    // the batch's side stream after the event recorded behind the plate's
    // last batched launch; stepping and state changes go through the batch
    slbm_batch_s* batch = nullptr;
    Arena* arena = nullptr;
    bool ext_flag = false;
    hipEvent_t ready = nullptr;
    uint64_t batch_id = 0;
    int64_t n_material = 0;
    int n_links = 0;
    int64_t step = 0;
    bool local = true;
    int seg = 0;
    int wide = -1;                   // strip shape: 1 wide, 0 narrow, -1 library default
    int two = 0;                     // 1: two steps per launch (58-column strips, seg rows <= 10)
    int group = 0;                   // workgroups to XCDs: 0 contiguous bands, g > 0 interleaved groups of g
    std::vector<uint8_t> mask;
    // per-tile cut-link records of the two-step kernel (build_tile_records):
    // the link records as uploaded and each link's site, the lists on the
    // device for tiles of rec_seg rows, rec_fit when every tile's fits the
    // cooperative kernel
    std::vector<char> link_host;
    std::vector<int32_t> link_site;
    int ngroups = 0;
    int32_t* rec_start = nullptr;
    void* recs = nullptr;
    int rec_seg = 0;
    bool rec_fit = false;
    int64_t rec_bytes = 0;
    int64_t rec_count = 0;
    int32_t rec_max = 0;
};

namespace {

// XCD groups: 0 (contiguous bands) or a power of two up to 64; the kernels
// take log2 of the group, -1 for bands.
bool valid_group(int g) { return g == 0 || (g > 0 && g <= 64 && (g & (g - 1)) == 0); }
int group_shift(int g) { return g > 0 ? __builtin_ctz((unsigned)g) : -1; }

bool pick_wide(const slbm_s* h)
{
    return h->wide == 1;             // narrow strips unless asked: measured faster on every plate tried
}

// Rows per tile: short tiles give small plates enough workgroups to fill the
// machine, tall ones cut the halo-row overhead (2 rows per tile) on large
// plates; the autotuner refines this per plate.
int pick_seg(const slbm_s* h)
{
    const int mx = pick_wide(h) ? max_tile_rows<true>() : max_tile_rows<false>();
    if (h->seg > 0) return std::min(h->seg, mx);
    const long long n = (long long)h->nx * h->ny;
    const int r = n >= (1LL << 22) ? 14 : (n >= (1LL << 16) ? 6 : 2);
    return std::min(r, mx);
}

template <typename real>
StepArgs<real> make_args(const slbm_s* h, int src)
{
    StepArgs<real> a{};
    a.src = (const real*)h->buf[src];
    a.dst = (real*)h->buf[src ^ 1];
    a.U = h->U;
    a.flags = h->flags;
    a.bidx = h->bidx;
    a.links = (const LinkDev<real>*)h->links;
    a.groups = h->groups;
    a.ngroups = h->ngroups;
    a.diverged = h->diverged;
    a.plane = h->plane;
    a.t_prev = h->step - 1;
    a.nx = h->nx; a.ny = h->ny; a.ld = h->ld;
    a.seg = pick_seg(h);
    const int sw = pick_wide(h) ? 64 : 62;
    a.nstrips = (h->nx + sw - 1) / sw;
    a.ntiles = a.nstrips * ((h->ny + a.seg - 1) / a.seg);
    a.px = h->px; a.py = h->py;
    a.local = h->local ? 1 : 0;
    a.group_shift = group_shift(h->group);
    a.omega = (real)(1.0 / h->tau);
    a.lm = (real)(h->lamL - h->muL);
    a.ml = (real)(h->muL - h->lamL);
    a.Fx = (real)h->FL[0];
    a.Fy = (real)h->FL[1];
    return a;
}

// Workgroups of a single-plate launch: the tiles, rounded up to a whole
// number of XCD rounds (8 workgroups, or 8 groups with interleaved groups).
template <typename real>
int grid_for(const StepArgs<real>& a)
{
    const int unit = 8 << std::max(0, a.group_shift);
    return (a.ntiles + unit - 1) / unit * unit;
}

template <typename real>
void dispatch_step(const slbm_s* h, const StepArgs<real>& a)
{
    const int grid = grid_for(a);
    const bool per = h->px || h->py, wide = pick_wide(h);
    const dim3 blk(64 * (wide ? tile_waves<true>(a.seg) : tile_waves<false>(a.seg)));
    if (per && wide)
        hipLaunchKernelGGL((k_step<real, true, true>), dim3(grid), blk, 0, h->stream, a);
    else if (per)
        hipLaunchKernelGGL((k_step<real, true, false>), dim3(grid), blk, 0, h->stream, a);
    else if (wide)
        hipLaunchKernelGGL((k_step<real, false, true>), dim3(grid), blk, 0, h->stream, a);
    else
        hipLaunchKernelGGL((k_step<real, false, false>), dim3(grid), blk, 0, h->stream, a);
}

// One step from the current state into the other buffer with the given
// launch shape, without committing it (the caller decides).
template <typename real>
int launch_step_raw(slbm_s* h, int seg, int wide)
{
    const int keep = h->seg, keepw = h->wide;
    h->seg = seg;
    h->wide = wide;
    StepArgs<real> a = make_args<real>(h, h->cur);
    h->seg = keep;
    // always the pull path, whose memory traffic is that of a step (a state
    // just created or initialised would otherwise be read in place)
    a.local = 0;
    dispatch_step<real>(h, a);
    h->wide = keepw;
    HIP_TRY(hipGetLastError());
    return SLBM_OK;
}

// A batch plate's steps run on the batch's compute stream (defined with the
// batch code below); device memory of a plate (defined below).
hipStream_t batch_compute_stream(slbm_batch_s* b);
hipError_t dev_alloc(slbm_s* h, void** p, size_t n);

// Rows per tile of the two-step kernel for a requested number (0: default).
int seg2_rows(int seg) { return std::max(1, std::min(seg > 0 ? seg : 6, kMaxTileRows2)); }

// Frees a plate's tile lists: at once for a single plate (hipFree waits for
// the device), for a batch plate back to the batch's arena once the launches
// and readouts queued so far have completed.
void drop_tile_records(slbm_s* h)
{
    if (h->arena && (h->rec_start || h->recs)) {
        if (h->batch) {
            hipEvent_t ec = nullptr, es = nullptr;
            if (hipEventCreateWithFlags(&ec, hipEventDisableTiming) == hipSuccess &&
                hipEventCreateWithFlags(&es, hipEventDisableTiming) == hipSuccess &&
                hipEventRecord(ec, batch_compute_stream(h->batch)) == hipSuccess &&
                hipEventRecord(es, h->stream) == hipSuccess) {
                h->arena->release_after({ec, es}, {h->rec_start, h->recs});
            } else {
                if (ec) (void)hipEventDestroy(ec);
                if (es) (void)hipEventDestroy(es);
                (void)hipDeviceSynchronize();
                h->arena->release(h->rec_start);
                h->arena->release(h->recs);
            }
        } else {
            h->arena->release(h->rec_start);
            h->arena->release(h->recs);
        }
    } else {
        if (h->rec_start) (void)hipFree(h->rec_start);
        if (h->recs) (void)hipFree(h->recs);
    }
    h->rec_start = nullptr;
    h->recs = nullptr;
    h->rec_seg = 0;
    h->rec_fit = false;
    h->rec_bytes = 0;
    h->rec_count = 0;
    h->rec_max = 0;
}

// Coordinates c + m n (any m on a periodic axis, m = 0 otherwise) in [lo, hi]:
// where a site of that coordinate sits in the tiles' footprints, which on a
// periodic axis reach past the grid and wrap.
template <class F>
void axis_images(int c, int n, bool per, int lo, int hi, F&& f)
{
    if (!per) {
        if (c >= lo && c <= hi) f(c);
        return;
    }
    long long v = c - (long long)n * ((c - lo + n - 1) / n);   // the smallest image >= lo (c >= 0 > lo - n)
    if (v < lo) v += n;
    for (; v <= hi; v += n) f((int)v);
}

long long floor_div(long long a, long long b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }

// Where the cut links sit in the tiles of the two-step kernel (R rows,
// 58-column strips): a tile's reach is rows y0 - 3 .. y0 + R + 2 and columns
// xs - 3 .. xs + 60, wave w and lane l at y0 - 3 + w, xs - 3 + l, wrapping on
// periodic axes.  Every link (site y nx + x) appears in each tile whose reach
// holds its site, once per image of the site there.  start[t] .. start[t + 1]
// index tile t's records, each a link and a position (w << 8 | l); `most` is
// the largest count in one tile.  Host only.
struct TileLayout {
    std::vector<int32_t> start, link, pos;
    int32_t most = 0;
    long long ntiles = 0;
};

TileLayout tile_layout(int nx, int ny, bool px, bool py, int R, const int32_t* site, int n, int64_t cap)
{
    TileLayout out;
    const int nstrips = (nx + kStrip2 - 1) / kStrip2, ntr = (ny + R - 1) / R;
    out.ntiles = (long long)nstrips * ntr;
    auto each = [&](auto&& f) {
        for (int i = 0; i < n; ++i) {
            const int x = site[i] % nx, y = site[i] / nx;
            axis_images(y, ny, py, -3, ntr * R + 2, [&](int yh) {
                const long long tr0 = std::max<long long>(0, -floor_div(-(yh - R - 2), R));
                const long long tr1 = std::min<long long>(ntr - 1, floor_div(yh + 3, R));
                for (long long tr = tr0; tr <= tr1; ++tr) {
                    const int w = yh - (int)(tr * R - 3);
                    axis_images(x, nx, px, -3, nstrips * kStrip2 + 2, [&](int xh) {
                        const long long s0 = std::max<long long>(0, -floor_div(-(xh - 60), kStrip2));
                        const long long s1 = std::min<long long>(nstrips - 1, floor_div(xh + 3, kStrip2));
                        for (long long st = s0; st <= s1; ++st)
                            f(st + tr * nstrips, w, xh - (int)(st * kStrip2 - 3), i);
                    });
                }
            });
        }
    };
    out.start.assign((size_t)out.ntiles + 1, 0);
    each([&](long long t, int, int, int) { ++out.start[(size_t)t + 1]; });
    for (long long t = 0; t < out.ntiles; ++t) out.most = std::max(out.most, out.start[(size_t)t + 1]);
    int64_t total = 0;
    for (long long t = 0; t < out.ntiles; ++t) total += out.start[(size_t)t + 1];
    if (total > INT32_MAX) {                           // offsets are 32-bit: no lists
        out.most = INT32_MAX;
        out.start.clear();
        return out;
    }
    for (long long t = 0; t < out.ntiles; ++t) out.start[(size_t)t + 1] += out.start[(size_t)t];
    if (out.most > cap) return out;                    // counts only
    out.link.resize((size_t)total);
    out.pos.resize((size_t)total);
    std::vector<int32_t> fill(out.start.begin(), out.start.end() - 1);
    each([&](long long t, int w, int l, int i) {
        const int32_t k = fill[(size_t)t]++;
        out.link[(size_t)k] = i;
        out.pos[(size_t)k] = (w << 8) | l;
    });
    return out;
}

// The plate's tile lists on the device for tiles of seg rows: tile_layout's
// records, each with its link's coefficients (TileRec).  When a tile has more
// than the cooperative kernel takes (or the plate more groups than it
// tabulates), no lists are kept and the two-step kernel takes the rules site
// by site.
template <typename real>
int build_tile_records(slbm_s* h, int seg)
{
    seg = seg2_rows(seg);
    if (h->rec_seg == seg) return SLBM_OK;
    drop_tile_records(h);
    h->rec_seg = seg;
    if (h->n_links == 0 || h->ngroups > kTileGroupCap) return SLBM_OK;
    const int R = seg;
    // one record per thread of the tile's workgroup, and what its LDS holds
    const int cap = std::min(kTileRecCap, 64 * (R + 6));
    const TileLayout lay = tile_layout(h->nx, h->ny, h->px != 0, h->py != 0, R, h->link_site.data(), h->n_links, cap);
    if (lay.most > cap) return SLBM_OK;
    const std::vector<int32_t>& start = lay.start;
    const int32_t most = lay.most;
    const size_t total = lay.link.size();
    const LinkDev<real>* L = reinterpret_cast<const LinkDev<real>*>(h->link_host.data());
    std::vector<TileRec<real>> rec(total);
    for (size_t k = 0; k < total; ++k) {
        TileRec<real>& r = rec[k];
        const LinkDev<real>& d = L[lay.link[k]];
        r.kappa = d.kappa; r.wx = d.wx; r.wy = d.wy; r.D = d.D;
        for (int j = 0; j < 4; ++j) r.be[j] = d.be[j];
        for (int j = 0; j < 3; ++j) {
            r.K1[j] = d.K1[j];
            r.K2[j] = d.K2[j];
            r.E3[j] = d.E3[j];
        }
        r.meta = d.k | (d.kind << 4) | (d.behind << 6) | ((d.g1 + 1) << 8) | ((d.g2 + 1) << 16);
        r.pos = lay.pos[k];
    }
    hipError_t e = dev_alloc(h, (void**)&h->rec_start, start.size() * sizeof(int32_t));
    if (e == hipSuccess) e = dev_alloc(h, &h->recs, std::max<size_t>(1, total) * sizeof(TileRec<real>));
    if (e != hipSuccess) {
        drop_tile_records(h);
        h->rec_seg = seg;
        // a batch plate without room in the budget goes without lists
        if (e == hipErrorOutOfMemory && h->arena) return SLBM_OK;
        if (e == hipErrorOutOfMemory) return fail(SLBM_E_NOMEM, "no device memory for the tile record lists");
        HIP_TRY(e);
    }
    HIP_TRY(hipMemcpyAsync(h->rec_start, start.data(), start.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                           h->stream));
    if (total)
        HIP_TRY(hipMemcpyAsync(h->recs, rec.data(), total * sizeof(TileRec<real>), hipMemcpyHostToDevice, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    h->rec_fit = true;
    h->rec_bytes = (int64_t)(start.size() * sizeof(int32_t) + total * sizeof(TileRec<real>));
    h->rec_count = (int64_t)total;
    h->rec_max = most;
    return SLBM_OK;
}

int tile_records(slbm_s* h, int seg)
{
    return h->precision == SLBM_FP32 ? build_tile_records<float>(h, seg) : build_tile_records<double>(h, seg);
}

// Arguments of the two-steps-per-launch kernel: 58-column strips, at most
// kMaxTileRows2 rows per tile.
template <typename real>
StepArgs<real> make_args2(const slbm_s* h, int src, int seg)
{
    StepArgs<real> a = make_args<real>(h, src);
    a.seg = seg2_rows(seg);
    a.nstrips = (h->nx + kStrip2 - 1) / kStrip2;
    a.ntiles = a.nstrips * ((h->ny + a.seg - 1) / a.seg);
    if (h->rec_fit && h->rec_seg == a.seg) {
        a.rec_start = h->rec_start;
        a.recs = (const TileRec<real>*)h->recs;
    }
    return a;
}

template <typename real, bool PER, int W>
void dispatch_step2_w(const slbm_s* h, const StepArgs<real>& a, int grid, dim3 blk)
{
    if (a.rec_start)
        hipLaunchKernelGGL((k_step2<real, PER, W, true>), dim3(grid), blk, 0, h->stream, a);
    else
        hipLaunchKernelGGL((k_step2<real, PER, W, false>), dim3(grid), blk, 0, h->stream, a);
}

template <typename real>
void dispatch_step2(const slbm_s* h, const StepArgs<real>& a)
{
    const int grid = grid_for(a);
    const dim3 blk(64 * (a.seg + 6));
    constexpr int lo = k2_waves<real>(1), hi = k2_waves<real>(kMaxTileRows2);
    const bool per = h->px || h->py;
    if (k2_waves<real>(a.seg) == hi) {
        if (per)
            dispatch_step2_w<real, true, hi>(h, a, grid, blk);
        else
            dispatch_step2_w<real, false, hi>(h, a, grid, blk);
    } else {
        if (per)
            dispatch_step2_w<real, true, lo>(h, a, grid, blk);
        else
            dispatch_step2_w<real, false, lo>(h, a, grid, blk);
    }
}

// Two steps in one launch, not committed (autotuner trials; see launch_step_raw).
template <typename real>
int launch_step2_raw(slbm_s* h, int seg)
{
    StepArgs<real> a = make_args2<real>(h, h->cur, seg);
    a.local = 0;
    dispatch_step2<real>(h, a);
    HIP_TRY(hipGetLastError());
    return SLBM_OK;
}

template <typename real>
int launch_step2(slbm_s* h)
{
    StepArgs<real> a = make_args2<real>(h, h->cur, h->seg);
    dispatch_step2<real>(h, a);
    HIP_TRY(hipGetLastError());
    h->cur ^= 1;
    h->local = false;
    h->step += 2;
    return SLBM_OK;
}

template <typename real>
int launch_step(slbm_s* h)
{
    StepArgs<real> a = make_args<real>(h, h->cur);
    dispatch_step<real>(h, a);
    HIP_TRY(hipGetLastError());
    h->cur ^= 1;
    h->local = false;
    h->step += 1;
    return SLBM_OK;
}

// A batch plate's readouts use the batch's shared scratch (defined with the
// batch code below).
int batch_scratch(slbm_s* h, int planes);

int ensure_scratch(slbm_s* h, int planes)
{
    if (h->batch) return batch_scratch(h, planes);
    if (h->scratch && h->scratch_planes >= planes) return SLBM_OK;
    if (h->scratch) (void)hipFree(h->scratch);
    h->scratch = nullptr;
    h->scratch_planes = 0;
    HIP_TRY(hipMalloc((void**)&h->scratch, (size_t)planes * h->plane * sizeof(double)));
    h->scratch_planes = planes;
    return SLBM_OK;
}

// A batch plate forgets the batch's scratch after each readout (the batch
// may move it to a larger block later).
void release_transient_scratch(slbm_s* h)
{
    if (!h->batch) return;
    h->scratch = nullptr;
    h->scratch_planes = 0;
}

// Readouts of a batch plate are queued on its side stream behind the plate's
// last batched launch (queued on the batch's compute stream).
int wait_ready(slbm_s* h)
{
    if (h->ready) HIP_TRY(hipStreamWaitEvent(h->stream, h->ready, 0));
    return SLBM_OK;
}

// outputs in lattice units into scratch[1..11]; scratch[0] holds delta-rho
template <typename real>
int launch_outputs(slbm_s* h, bool full)
{
    int rc = ensure_scratch(h, full ? 12 : 3);
    if (rc) return rc;
    StepArgs<real> a = make_args<real>(h, h->cur);
    const int n = (int)h->plane;
    const int grid = (n + 255) / 256;
    double* dr = h->scratch;
    double* out = h->scratch + h->plane;
    const int ncomp = full ? 11 : 2;
    if (h->px || h->py) {
        hipLaunchKernelGGL((k_density<real, true>), dim3(grid), dim3(256), 0, h->stream, a, dr);
        hipLaunchKernelGGL((k_outputs<real, true>), dim3(grid), dim3(256), 0, h->stream, a, dr, out, ncomp);
    } else {
        hipLaunchKernelGGL((k_density<real, false>), dim3(grid), dim3(256), 0, h->stream, a, dr);
        hipLaunchKernelGGL((k_outputs<real, false>), dim3(grid), dim3(256), 0, h->stream, a, dr, out, ncomp);
    }
    HIP_TRY(hipGetLastError());
    return SLBM_OK;
}

// Readout kernels: full = all moments (11 planes), else the displacement only
// (2 planes, components 9 and 10 of the full set come first).
int outputs(slbm_s* h, bool full)
{
    return h->precision == SLBM_FP32 ? launch_outputs<float>(h, full) : launch_outputs<double>(h, full);
}

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int d)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != d) (void)hipSetDevice(d);
    }
    ~DeviceGuard()
    {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

// Device memory of a plate: from the batch's arena for batch plates, else
// hipMalloc.  An exhausted arena reports out-of-memory.
hipError_t dev_alloc(slbm_s* h, void** p, size_t n)
{
    if (!h->arena) return hipMalloc(p, n);
    *p = h->arena->alloc(n);
    return *p ? hipSuccess : hipErrorOutOfMemory;
}

// The plate's own device blocks (not the batch's divergence word or scratch).
std::vector<void*> plate_blocks(slbm_s* h)
{
    std::vector<void*> v = {h->buf[0], h->buf[1], h->U, h->flags, h->bidx, h->links, h->groups, h->rec_start,
                            h->recs};
    if (!h->ext_flag) v.push_back(h->diverged);
    if (!h->batch) v.push_back(h->scratch);
    return v;
}

// Frees at once: nothing queued may still use the plate.
void free_all(slbm_s* h)
{
    for (void* p : plate_blocks(h)) {
        if (!p) continue;
        if (h->arena)
            h->arena->release(p);
        else
            (void)hipFree(p);
    }
    h->buf[0] = h->buf[1] = nullptr;
    h->rec_start = nullptr;
    h->recs = nullptr;
    h->rec_fit = false;
    h->U = nullptr;
    h->scratch = nullptr;
    if (h->ready) (void)hipEventDestroy(h->ready);
    h->ready = nullptr;
    if (h->own_stream && h->stream) (void)hipStreamDestroy(h->stream);
}

template <typename real>
void fill_link(LinkDev<real>& d, const slbm_link& l, bool behind, const slbm_params* p, const slbm_s* h)
{
    // Coefficients of the section 4 rules for link (x, k), in lattice units.
    const int k = l.dir;
    const double q = l.q;
    const double cx = CX(k), cy = CY(k), w = WD(k);
    const double kappa = behind ? (1.0 - 2.0 * q) / (1.0 + 2.0 * q) : 0.0;
    const double beta = behind ? 2.0 / (1.0 + 2.0 * q) : 1.0;
    std::memset(&d, 0, sizeof d);
    d.k = k; d.dx = (int)cx; d.dy = (int)cy;
    d.behind = behind ? 1 : 0;
    d.kappa = (real)kappa;
    d.g2 = -1;
    const slbm_bc_group& G1 = p->groups[l.group];
    const slbm_bc_group* G2 = l.group2 >= 0 ? &p->groups[l.group2] : nullptr;
    int gd = -1;
    if (G1.kind == SLBM_DIRICHLET) gd = l.group;
    else if (G2 && G2->kind == SLBM_DIRICHLET) gd = l.group2;
    if (gd >= 0) {
        const slbm_bc_group& G = p->groups[gd];
        const double vx = G.value[0] / h->s_v, vy = G.value[1] / h->s_v;
        d.kind = SLBM_DIRICHLET;
        d.g1 = gd;
        d.D = (real)(-beta * 6.0 * w * (cx * vx + cy * vy));
        return;
    }
    d.kind = SLBM_NEUMANN;
    const bool extrap = behind && h->norder == 1;
    d.wx = (real)(extrap ? 1.0 + q : 1.0);
    d.wy = (real)(extrap ? -q : 0.0);
    // d(E_k - 2 r_k)/d(drho_bd, Pxx, Pyy, Pxy), E_k of eq:abbcon, times beta
    d.be[0] = (real)(beta * 2.0 * w * (2.0 - 1.5 * (cx * cx + cy * cy)));
    d.be[1] = (real)(beta * 9.0 * w * (cx * cx - 1.0 / 3.0));
    d.be[2] = (real)(beta * 9.0 * w * (cy * cy - 1.0 / 3.0));
    d.be[3] = (real)(beta * 18.0 * w * cx * cy);
    d.g1 = l.group;
    const double nx_ = l.normal[0], ny_ = l.normal[1];
    const double tx = G1.value[0] / h->s_sigma, ty = G1.value[1] / h->s_sigma;
    if (G2) {
        // two walls: sigma* = sym(t_A n_A + t_B n_B), nothing extrapolated
        const double ux = G2->value[0] / h->s_sigma, uy = G2->value[1] / h->s_sigma;
        const double mx = l.normal2[0], my = l.normal2[1];
        d.K1[0] = (real)(tx * nx_); d.K1[1] = (real)(ty * ny_); d.K1[2] = (real)(0.5 * (tx * ny_ + ty * nx_));
        d.K2[0] = (real)(ux * mx); d.K2[1] = (real)(uy * my); d.K2[2] = (real)(0.5 * (ux * my + uy * mx));
        d.g2 = l.group2;
        return;
    }
    // eq:trafocauchy: sigma* = t_n n n + t_t (n e + e n) + sigma_tt e e, e = (-n_y, n_x)
    const double ex = -ny_, ey = nx_;
    const double tn = tx * nx_ + ty * ny_, tt = tx * ex + ty * ey;
    d.K1[0] = (real)(tn * nx_ * nx_ + 2.0 * tt * nx_ * ex);
    d.K1[1] = (real)(tn * ny_ * ny_ + 2.0 * tt * ny_ * ey);
    d.K1[2] = (real)(tn * nx_ * ny_ + tt * (nx_ * ey + ex * ny_));
    d.E3[0] = (real)(ex * ex); d.E3[1] = (real)(ey * ey); d.E3[2] = (real)(ex * ey);
}

template <typename real>
int upload_links(slbm_s* h, const std::vector<slbm_link>& L, const std::vector<uint8_t>& cutmask,
                 const slbm_params* p)
{
    const int n = h->nx * h->ny;
    std::vector<LinkDev<real>> d(L.size());
    for (size_t i = 0; i < L.size(); ++i) {
        const slbm_link& l = L[i];
        const int k = l.dir;
        const bool behind = !((cutmask[l.site] >> (OPP(k) - 1)) & 1u);
        fill_link(d[i], l, behind, p, h);
    }
    (void)n;
    h->link_host.assign(reinterpret_cast<const char*>(d.data()), reinterpret_cast<const char*>(d.data() + d.size()));
    h->link_site.resize(L.size());
    for (size_t i = 0; i < L.size(); ++i) h->link_site[i] = L[i].site;
    if (!d.empty()) {
        const hipError_t e = dev_alloc(h, &h->links, d.size() * sizeof(LinkDev<real>));
        if (e == hipErrorOutOfMemory) return fail(SLBM_E_NOMEM, "no device memory for the link records");
        HIP_TRY(e);
        HIP_TRY(hipMemcpyAsync(h->links, d.data(), d.size() * sizeof(LinkDev<real>), hipMemcpyHostToDevice,
                               h->stream));
        HIP_TRY(hipStreamSynchronize(h->stream));
    }
    return SLBM_OK;
}

// A plate from its parameters.  With an arena (batch plates) its device
// memory comes from there and ext_flag, if given, is its divergence word.
int create_impl(const slbm_params* p, slbm_handle* out, Arena* arena = nullptr, unsigned int* ext_flag = nullptr)
{
    if (!p || !out) return fail(SLBM_E_INVAL, "null argument");
    *out = nullptr;
    if (p->nx < 1 || p->ny < 1) return fail(SLBM_E_INVAL, "grid must be at least 1x1");
    if ((long long)p->nx * p->ny > (1LL << 28)) return fail(SLBM_E_UNSUPPORTED, "grid larger than 2^28 sites");
    if (!(p->mu > 0) || !(p->rho > 0)) return fail(SLBM_E_INVAL, "mu and rho must be positive");
    if (!(p->tau > 0.5)) return fail(SLBM_E_INVAL, "tau must exceed 1/2");
    if (!std::isfinite(p->lambda)) return fail(SLBM_E_INVAL, "lambda must be finite");
    if (p->precision != SLBM_FP64 && p->precision != SLBM_FP32) return fail(SLBM_E_INVAL, "unknown precision");
    if (p->neumann_order != 0 && p->neumann_order != 1) return fail(SLBM_E_INVAL, "neumann_order must be 0 or 1");
    if (!p->mask) return fail(SLBM_E_INVAL, "mask is required");
    if (p->n_links < 0 || (p->n_links > 0 && !p->links)) return fail(SLBM_E_INVAL, "bad link list");
    if (p->n_groups < 0 || (p->n_groups > 0 && !p->groups)) return fail(SLBM_E_INVAL, "bad group list");
    for (int g = 0; g < p->n_groups; ++g) {
        const slbm_bc_group& G = p->groups[g];
        if (G.kind != SLBM_DIRICHLET && G.kind != SLBM_NEUMANN) return fail(SLBM_E_INVAL, "group %d: bad kind", g);
        if (G.profile != SLBM_PROFILE_STEP && G.profile != SLBM_PROFILE_RAMP) return fail(SLBM_E_INVAL, "group %d: bad profile", g);
        if (G.profile == SLBM_PROFILE_RAMP && !(G.ramp_time > 0)) return fail(SLBM_E_INVAL, "group %d: ramp time must be positive", g);
        if (!std::isfinite(G.value[0]) || !std::isfinite(G.value[1])) return fail(SLBM_E_INVAL, "group %d: value not finite", g);
    }
    const int nx = p->nx, ny = p->ny, n = nx * ny;
    std::vector<uint8_t> mat(n), cut(n, 0);
    for (int s = 0; s < n; ++s) mat[s] = p->mask[s] ? 1 : 0;
    std::vector<slbm_link> L(p->links, p->links + p->n_links);
    for (int i = 0; i < p->n_links; ++i) {
        const slbm_link& l = L[i];
        if (l.site < 0 || l.site >= n || !mat[l.site]) return fail(SLBM_E_INVAL, "link %d: site is not material", i);
        if (l.dir < 1 || l.dir > 8) return fail(SLBM_E_INVAL, "link %d: direction must be 1..8", i);
        if (!(l.q > 0 && l.q <= 1)) return fail(SLBM_E_INVAL, "link %d: q outside (0,1]", i);
        if (l.group < 0 || l.group >= p->n_groups) return fail(SLBM_E_INVAL, "link %d: bad group", i);
        if (l.group2 >= p->n_groups || l.group2 < -1) return fail(SLBM_E_INVAL, "link %d: bad second group", i);
        const double nn = l.normal[0] * l.normal[0] + l.normal[1] * l.normal[1];
        if (!(std::fabs(nn - 1.0) < 1e-9)) return fail(SLBM_E_INVAL, "link %d: normal is not a unit vector", i);
        if (l.group2 >= 0) {
            const double m2 = l.normal2[0] * l.normal2[0] + l.normal2[1] * l.normal2[1];
            if (!(std::fabs(m2 - 1.0) < 1e-9)) return fail(SLBM_E_INVAL, "link %d: second normal is not a unit vector", i);
        }
        const uint8_t bit = (uint8_t)(1u << (l.dir - 1));
        if (cut[l.site] & bit) return fail(SLBM_E_INVAL, "link %d: duplicate", i);
        cut[l.site] |= bit;
    }
    // every uncut link of a material site must end at a material site whose
    // opposite link is uncut too: checked in parallel over contiguous site
    // ranges (a large plate has hundreds of millions of links); the error
    // reported is the one at the lowest site, as a sequential scan finds it
    auto check_site = [&](int s, int& kbad) -> int {
        kbad = 0;
        if (!mat[s]) return 0;
        if (cut[s] == 0xFF) return 1;
        const int x = s % nx, y = s / nx;
        for (int k = 1; k <= 8; ++k) {
            if (cut[s] & (1u << (k - 1))) continue;
            int tx = x + CX(k), ty = y + CY(k);
            if (p->periodic_x) tx = (tx + nx) % nx;
            if (p->periodic_y) ty = (ty + ny) % ny;
            kbad = k;
            if (tx < 0 || tx >= nx || ty < 0 || ty >= ny || !mat[ty * nx + tx]) return 2;
            if (cut[ty * nx + tx] & (1u << (OPP(k) - 1))) return 3;
        }
        return 0;
    };
    {
        const int nthreads = (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
        const int parts = n >= (1 << 16) ? nthreads : 1;
        std::vector<int> first(parts, n);
        auto scan = [&](int part) {
            const int s0 = (int)((int64_t)n * part / parts), s1 = (int)((int64_t)n * (part + 1) / parts);
            int kb;
            for (int s = s0; s < s1; ++s)
                if (check_site(s, kb)) { first[part] = s; return; }
        };
        std::vector<std::thread> pool;
        for (int t = 1; t < parts; ++t) pool.emplace_back(scan, t);
        scan(0);
        for (std::thread& t : pool) t.join();
        const int s = *std::min_element(first.begin(), first.end());
        if (s < n) {
            int k = 0;
            const int why = check_site(s, k);
            if (why == 1) return fail(SLBM_E_INVAL, "site %d: every link is cut", s);
            if (why == 2) return fail(SLBM_E_INVAL, "site (%d,%d): uncut link %d leaves the material", s % nx, s / nx, k);
            return fail(SLBM_E_INVAL, "site (%d,%d): link %d is cut from one end only", s % nx, s / nx, k);
        }
    }
    std::sort(L.begin(), L.end(), [](const slbm_link& a, const slbm_link& b) {
        return a.site != b.site ? a.site < b.site : a.dir < b.dir;
    });

    slbm_s* h = new (std::nothrow) slbm_s();
    if (!h) return fail(SLBM_E_NOMEM, "out of host memory");
    h->device = p->device;
    h->nx = nx; h->ny = ny;
    h->ld = (kPadL + nx + 1 + 63) / 64 * 64;
    h->plane = (long long)h->ld * (ny + 2);
    if (h->plane * (long long)sizeof(double) >= (1LL << 32)) {
        delete h;
        return fail(SLBM_E_UNSUPPORTED, "padded plane exceeds 4 GiB (kernels address planes with 32-bit offsets)");
    }
    h->precision = p->precision;
    h->px = p->periodic_x ? 1 : 0;
    h->py = p->periodic_y ? 1 : 0;
    h->norder = p->neumann_order;
    // units (section 5.1): c_s = sqrt(mu/rho) = dx/(sqrt 3 dt)
    h->rho_user = p->rho;
    h->dt_user = std::sqrt(p->rho / (3.0 * p->mu));
    h->s_sigma = 3.0 * p->mu;
    h->s_v = 1.0 / h->dt_user;
    h->muL = 1.0 / 3.0;
    h->lamL = p->lambda / h->s_sigma;
    h->tau = p->tau;
    h->FL[0] = p->body_force[0] / h->s_sigma;
    h->FL[1] = p->body_force[1] / h->s_sigma;
    h->esize = p->precision == SLBM_FP32 ? 4 : 8;
    h->n_links = p->n_links;
    h->ngroups = p->n_groups;
    h->mask = mat;
    h->arena = arena;
    for (int s = 0; s < n; ++s) h->n_material += mat[s];

    int dev_count = 0;
    if (hipGetDeviceCount(&dev_count) != hipSuccess || dev_count < 1) {
        delete h;
        return fail(SLBM_E_DEVICE, "no HIP device");
    }
    if (p->device < 0 || p->device >= dev_count) {
        delete h;
        return fail(SLBM_E_INVAL, "device %d out of range", p->device);
    }
    DeviceGuard dg(h->device);
    auto bail = [&](int rc) { free_all(h); delete h; return rc; };
#define TRY_OR_BAIL(expr)                                                               \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess) {                                                         \
            int rc_ = (e_ == hipErrorOutOfMemory) ? SLBM_E_NOMEM : SLBM_E_DEVICE;       \
            fail(rc_, "%s failed: %s", #expr, hipGetErrorString(e_));                   \
            return bail(rc_);                                                           \
        }                                                                               \
    } while (0)
    if (p->stream) {
        h->stream = (hipStream_t)p->stream;
    } else {
        TRY_OR_BAIL(hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking));
        h->own_stream = true;
    }
    const size_t pop_bytes = (size_t)9 * h->plane * h->esize;
    TRY_OR_BAIL(dev_alloc(h, &h->buf[0], pop_bytes));
    TRY_OR_BAIL(dev_alloc(h, &h->buf[1], pop_bytes));
    TRY_OR_BAIL(dev_alloc(h, (void**)&h->U, (size_t)2 * h->plane * sizeof(double)));
    TRY_OR_BAIL(dev_alloc(h, (void**)&h->flags, (size_t)h->plane));
    TRY_OR_BAIL(dev_alloc(h, (void**)&h->bidx, (size_t)h->plane * sizeof(int32_t)));
    if (ext_flag) {
        h->diverged = ext_flag;
        h->ext_flag = true;
    } else {
        TRY_OR_BAIL(dev_alloc(h, (void**)&h->diverged, sizeof(unsigned int)));
    }
    {
        std::vector<uint8_t> fl((size_t)h->plane, (uint8_t)kVoid);
        std::vector<int32_t> bi((size_t)h->plane, -1);
        for (int s = 0; s < n; ++s) {
            if (!mat[s]) continue;
            const size_t d = (size_t)sidx(s % nx, s / nx, h->ld);
            fl[d] = cut[s];
        }
        for (size_t i = 0; i < L.size(); ++i) {
            const int s = L[i].site;
            const size_t d = (size_t)sidx(s % nx, s / nx, h->ld);
            if (bi[d] < 0) bi[d] = (int32_t)i;
        }
        // queued on the plate's stream (for batch plates the batch's side
        // stream, so that the upload does not wait for running steps)
        TRY_OR_BAIL(hipMemcpyAsync(h->flags, fl.data(), fl.size(), hipMemcpyHostToDevice, h->stream));
        TRY_OR_BAIL(hipMemcpyAsync(h->bidx, bi.data(), bi.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                                   h->stream));
        TRY_OR_BAIL(hipStreamSynchronize(h->stream));
    }
    {
        std::vector<GroupDev> gd(std::max(1, p->n_groups));
        for (int g = 0; g < p->n_groups; ++g) {
            gd[g].profile = p->groups[g].profile;
            gd[g].ramp_steps = p->groups[g].profile == SLBM_PROFILE_RAMP ? p->groups[g].ramp_time / h->dt_user : 1.0;
        }
        TRY_OR_BAIL(dev_alloc(h, (void**)&h->groups, gd.size() * sizeof(GroupDev)));
        TRY_OR_BAIL(hipMemcpyAsync(h->groups, gd.data(), gd.size() * sizeof(GroupDev), hipMemcpyHostToDevice,
                                   h->stream));
        TRY_OR_BAIL(hipStreamSynchronize(h->stream));
    }
    {
        int rc = h->precision == SLBM_FP32 ? upload_links<float>(h, L, cut, p) : upload_links<double>(h, L, cut, p);
        if (rc) return bail(rc);
    }
    // rest state: g = 0 (f = r), U = 0
    TRY_OR_BAIL(hipMemsetAsync(h->buf[0], 0, pop_bytes, h->stream));
    TRY_OR_BAIL(hipMemsetAsync(h->buf[1], 0, pop_bytes, h->stream));
    TRY_OR_BAIL(hipMemsetAsync(h->U, 0, (size_t)2 * h->plane * sizeof(double), h->stream));
    TRY_OR_BAIL(hipMemsetAsync(h->diverged, 0, sizeof(unsigned int), h->stream));
    TRY_OR_BAIL(hipStreamSynchronize(h->stream));
#undef TRY_OR_BAIL
    h->cur = 0;
    h->step = 0;
    h->local = true;
    *out = h;
    return SLBM_OK;
}

int copy_out(slbm_s* h, int comp, double scale, double offset, double* dst)
{
    // lattice field comp of scratch (after outputs()) -> unpadded host array:
    // unpadded on the device into scratch plane 0 (the density, no longer
    // needed once the output kernels ran), then one contiguous copy
    const int n = h->nx * h->ny;
    hipLaunchKernelGGL(k_unpad, dim3((n + 255) / 256), dim3(256), 0, h->stream,
                       (const double*)(h->scratch + (size_t)(1 + comp) * h->plane), h->nx, h->ny, h->ld,
                       h->scratch);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(dst, h->scratch, (size_t)n * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    for (int s = 0; s < n; ++s) dst[s] = h->mask[s] ? dst[s] * scale + offset : 0.0;
    return SLBM_OK;
}

}  // namespace

// ------------------------------------------------ readout without allocation

// The density plane slbm_displacement_device_noalloc reads the displacement
// through: a fixed array in the library's code object, so the call needs no
// device allocation.  Each device the library runs on holds its own copy
// (144 MiB) until the process ends; every call on a device shares it.
constexpr size_t kStaticScratchDoubles = (size_t)18874368;   // 144 MiB of fp64: a 4096 x 4096 plate's padded plane
static __device__ __align__(256) double scratch[kStaticScratchDoubles];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// The device address of `scratch` on the current device (the host-side name
// is only a stand-in, not a device address), looked up once per device.
int static_scratch(int device, double** out)
{
    if (device < 0 || device >= kMaxDevices) return fail(SLBM_E_UNSUPPORTED, "device %d beyond %d", device, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(SLBM_E_DEVICE, "address of the static readout scratch: %s", hipGetErrorString(e));
        g_scratch_ptr[device] = (double*)p;
    }
    *out = g_scratch_ptr[device];
    return SLBM_OK;
}

template <typename real, bool PER>
void launch_displacement_noalloc(slbm_s* h, double* dr, double* u)
{
    const StepArgs<real> a = make_args<real>(h, h->cur);
    const int n = h->nx * h->ny;
    hipLaunchKernelGGL((k_density<real, PER>), dim3((int)((h->plane + 255) / 256)), dim3(256), 0, h->stream, a, dr);
    hipLaunchKernelGGL((k_displacement_out<real, PER>), dim3((n + 255) / 256), dim3(256), 0, h->stream, a,
                       (const double*)dr, u);
}

}  // namespace

// ------------------------------------------------------------------ ABI

extern "C" {

int slbm_create(const slbm_params* params, slbm_handle* out)
{
    try {
        return create_impl(params, out);
    } catch (...) {
        return fail(SLBM_E_NOMEM, "host allocation failed");
    }
}

int slbm_destroy(slbm_handle h)
{
    return guarded([&]() -> int {
        if (!h) return SLBM_OK;
        if (h->batch) return fail(SLBM_E_INVAL, "the plate belongs to a batch: remove it with slbm_batch_remove");
        DeviceGuard dg(h->device);
        if (h->stream) (void)hipStreamSynchronize(h->stream);
        free_all(h);
        delete h;
        return SLBM_OK;
    });
}

int slbm_step(slbm_handle h, int64_t nsteps)
{
    return guarded([&]() -> int {
        if (!h) return fail(SLBM_E_INVAL, "null handle");
        if (h->batch) return fail(SLBM_E_INVAL, "the plate belongs to a batch (only readouts go through its handle)");
        if (nsteps < 0) return fail(SLBM_E_INVAL, "negative step count");
        DeviceGuard dg(h->device);
        int64_t i = 0;
        if (h->two) {
            for (; i + 2 <= nsteps; i += 2) {
                int rc = h->precision == SLBM_FP32 ? launch_step2<float>(h) : launch_step2<double>(h);
                if (rc) return rc;
            }
        }
        for (; i < nsteps; ++i) {
            int rc = h->precision == SLBM_FP32 ? launch_step<float>(h) : launch_step<double>(h);
            if (rc) return rc;
        }
        return SLBM_OK;
    });
}

int slbm_sync(slbm_handle h)
{
    return guarded([&]() -> int {
        if (!h) return fail(SLBM_E_INVAL, "null handle");
        DeviceGuard dg(h->device);
        if (int rw = wait_ready(h)) return rw;
        unsigned int flag = 0;
        HIP_TRY(hipMemcpyAsync(&flag, h->diverged, sizeof flag, hipMemcpyDeviceToHost, h->stream));
        HIP_TRY(hipStreamSynchronize(h->stream));
        if (flag)
            return fail(SLBM_E_DIVERGED, "the state diverged (a value not finite or beyond the rest density) by step %lld",
                        (long long)h->step);
        return SLBM_OK;
    });
}

int slbm_moments(slbm_handle h, double* rho, double* j, double* P, double* sigma)
{
    return guarded([&]() -> int {
        if (!h) return fail(SLBM_E_INVAL, "null handle");
        DeviceGuard dg(h->device);
        if (int rw = wait_ready(h)) return rw;
        int rc = outputs(h, true);
        if (rc) return rc;
        const size_t n = (size_t)h->nx * h->ny;
        const double sj = h->rho_user * h->s_v;
        if (rho && (rc = copy_out(h, 0, h->rho_user, 0.0, rho))) return rc;
        if (j && ((rc = copy_out(h, 1, sj, 0.0, j)) || (rc = copy_out(h, 2, sj, 0.0, j + n)))) return rc;
        if (P && ((rc = copy_out(h, 3, h->s_sigma, 0.0, P)) || (rc = copy_out(h, 4, h->s_sigma, 0.0, P + n)) ||
                  (rc = copy_out(h, 5, h->s_sigma, 0.0, P + 2 * n))))
            return rc;
        if (sigma && ((rc = copy_out(h, 6, h->s_sigma, 0.0, sigma)) || (rc = copy_out(h, 7, h->s_sigma, 0.0, sigma + n)) ||
                      (rc = copy_out(h, 8, h->s_sigma, 0.0, sigma + 2 * n))))
            return rc;
        release_transient_scratch(h);
        return SLBM_OK;
    });
}

int slbm_displacement(slbm_handle h, double* u)
{
    return guarded([&]() -> int {
        if (!h || !u) return fail(SLBM_E_INVAL, "null argument");
        DeviceGuard dg(h->device);
        if (int rw = wait_ready(h)) return rw;
        int rc = outputs(h, false);
        if (rc) return rc;
        const size_t n = (size_t)h->nx * h->ny;
        if ((rc = copy_out(h, 0, 1.0, 0.0, u)) || (rc = copy_out(h, 1, 1.0, 0.0, u + n))) return rc;
        release_transient_scratch(h);
        return SLBM_OK;
    });
}

int slbm_displacement_device(slbm_handle h, void* u_dev)
{
    return guarded([&]() -> int {
        if (!h || !u_dev) return fail(SLBM_E_INVAL, "null argument");
        DeviceGuard dg(h->device);
        if (int rw = wait_ready(h)) return rw;
        int rc = outputs(h, false);
        if (rc) return rc;
        const int n = h->nx * h->ny;
        hipLaunchKernelGGL(k_unpad_u, dim3((n + 255) / 256), dim3(256), 0, h->stream,
                           (const double*)(h->scratch + h->plane), h->nx, h->ny, h->ld, (double*)u_dev);
        HIP_TRY(hipGetLastError());
        release_transient_scratch(h);
        return SLBM_OK;
    });
}

int slbm_displacement_device_noalloc(slbm_handle h, void* u_dev)
{
    return guarded([&]() -> int {
        if (!h || !u_dev) return fail(SLBM_E_INVAL, "null argument");
        if ((size_t)h->plane > kStaticScratchDoubles)
            return fail(SLBM_E_INVAL, "padded plane of %lld sites exceeds the static readout scratch of %zu sites",
                        (long long)h->plane, kStaticScratchDoubles);
        DeviceGuard dg(h->device);
        if (int rw = wait_ready(h)) return rw;
        double* dr = nullptr;
        if (int rc = static_scratch(h->device, &dr)) return rc;
        const bool per = h->px || h->py;
        if (h->precision == SLBM_FP32)
            per ? launch_displacement_noalloc<float, true>(h, dr, (double*)u_dev)
                : launch_displacement_noalloc<float, false>(h, dr, (double*)u_dev);
        else
            per ? launch_displacement_noalloc<double, true>(h, dr, (double*)u_dev)
                : launch_displacement_noalloc<double, false>(h, dr, (double*)u_dev);
        HIP_TRY(hipGetLastError());
        return SLBM_OK;
    });
}

int slbm_moments_device(slbm_handle h, void* rho, void* j, void* P, void* sigma, int dtype)
{
    return guarded([&]() -> int {
        if (!h) return fail(SLBM_E_INVAL, "null handle");
        if (dtype != SLBM_FP64 && dtype != SLBM_FP32) return fail(SLBM_E_INVAL, "dtype must be SLBM_FP64 or SLBM_FP32");
        DeviceGuard dg(h->device);
        if (int rw = wait_ready(h)) return rw;
        int rc = outputs(h, true);
        if (rc) return rc;
        const int n = h->nx * h->ny;
        const double sj = h->rho_user * h->s_v;
        // output components (as in slbm_moments): 0 rho, 1-2 j, 3-5 P, 6-8 sigma
        const struct { void* dst; int first, count; double scale; } part[4] = {
            {rho, 0, 1, h->rho_user}, {j, 1, 2, sj}, {P, 3, 3, h->s_sigma}, {sigma, 6, 3, h->s_sigma}};
        for (const auto& pt : part) {
            if (!pt.dst) continue;
            for (int c = 0; c < pt.count; ++c) {
                const double* src = h->scratch + (size_t)(1 + pt.first + c) * h->plane;
                if (dtype == SLBM_FP64)
                    hipLaunchKernelGGL(k_unpad_scaled<double>, dim3((n + 255) / 256), dim3(256), 0, h->stream, src,
                                       h->nx, h->ny, h->ld, pt.scale, (double*)pt.dst + (size_t)c * n);
                else
                    hipLaunchKernelGGL(k_unpad_scaled<float>, dim3((n + 255) / 256), dim3(256), 0, h->stream, src,
                                       h->nx, h->ny, h->ld, pt.scale, (float*)pt.dst + (size_t)c * n);
            }
        }
        HIP_TRY(hipGetLastError());
        release_transient_scratch(h);
        return SLBM_OK;
    });
}

int slbm_init_fields(slbm_handle h, const double* rho, const double* vel, const double* sigma, const double* u)
{
    return guarded([&]() -> int {
        if (!h) return fail(SLBM_E_INVAL, "null handle");
        if (h->batch) return fail(SLBM_E_INVAL, "the plate belongs to a batch (only readouts go through its handle)");
        DeviceGuard dg(h->device);
        int rc = ensure_scratch(h, 8);
        if (rc) return rc;
        const int nx = h->nx, ny = h->ny, n = nx * ny;
        const size_t P = (size_t)h->plane;
        // lattice-unit fields on the host, padded layout: dr, jx, jy, pxx, pyy, pxy, ux, uy
        std::vector<double> f((size_t)8 * P, 0.0);
        const double lm = h->lamL - h->muL;
        for (int s = 0; s < n; ++s) {
            if (!h->mask[s]) continue;
            const size_t d = (size_t)sidx(s % nx, s / nx, h->ld);
            const double rL = rho ? rho[s] / h->rho_user : 1.0;
            if (!(rL > 0) || !std::isfinite(rL)) return fail(SLBM_E_INVAL, "density must be positive");
            const double vx = vel ? vel[s] / h->s_v : 0.0, vy = vel ? vel[n + s] / h->s_v : 0.0;
            const double sxx = sigma ? sigma[s] / h->s_sigma : 0.0, syy = sigma ? sigma[n + s] / h->s_sigma : 0.0;
            const double sxy = sigma ? sigma[2 * n + s] / h->s_sigma : 0.0;
            const double div = 1.0 - rL;   // eq:approxdiv
            f[d] = rL - 1.0;
            f[P + d] = rL * vx;
            f[2 * P + d] = rL * vy;
            f[3 * P + d] = -sxx + lm * div;   // eq:poissonstress
            f[4 * P + d] = -syy + lm * div;
            f[5 * P + d] = -sxy;
            f[6 * P + d] = u ? u[s] : 0.0;
            f[7 * P + d] = u ? u[n + s] : 0.0;
        }
        double* dev = h->scratch;   // 8 planes
        HIP_TRY(hipMemcpyAsync(dev, f.data(), f.size() * sizeof(double), hipMemcpyHostToDevice, h->stream));
        h->cur = 0;
        h->local = true;
        h->step = 0;
        const int grid = (int)((P + 255) / 256);
        if (h->precision == SLBM_FP32) {
            StepArgs<float> a = make_args<float>(h, 0);
            if (h->px || h->py)
                hipLaunchKernelGGL((k_init<float, true>), dim3(grid), dim3(256), 0, h->stream, a, dev, dev + P, dev + 3 * P, dev + 6 * P, (float*)h->buf[0]);
            else
                hipLaunchKernelGGL((k_init<float, false>), dim3(grid), dim3(256), 0, h->stream, a, dev, dev + P, dev + 3 * P, dev + 6 * P, (float*)h->buf[0]);
        } else {
            StepArgs<double> a = make_args<double>(h, 0);
            if (h->px || h->py)
                hipLaunchKernelGGL((k_init<double, true>), dim3(grid), dim3(256), 0, h->stream, a, dev, dev + P, dev + 3 * P, dev + 6 * P, (double*)h->buf[0]);
            else
                hipLaunchKernelGGL((k_init<double, false>), dim3(grid), dim3(256), 0, h->stream, a, dev, dev + P, dev + 3 * P, dev + 6 * P, (double*)h->buf[0]);
        }
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipMemsetAsync(h->diverged, 0, sizeof(unsigned int), h->stream));
        HIP_TRY(hipStreamSynchronize(h->stream));
        release_transient_scratch(h);
        return SLBM_OK;
    });
}

int slbm_time(slbm_handle h, int64_t* step, double* t_user)
{
    return guarded([&]() -> int {
        if (!h) return fail(SLBM_E_INVAL, "null handle");
        if (step) *step = h->step;
        if (t_user) *t_user = (double)h->step * h->dt_user;
        return SLBM_OK;
    });
}

int slbm_set_launch(slbm_handle h, int32_t seg_rows, int32_t strip)
{
    return guarded([&]() -> int {
        if (!h) return fail(SLBM_E_INVAL, "null handle");
        if (h->batch) return fail(SLBM_E_INVAL, "the plate belongs to a batch (only readouts go through its handle)");
        if (seg_rows < 0) return fail(SLBM_E_INVAL, "seg_rows must be >= 0");
        if (strip != 0 && strip != 62 && strip != 64 && strip != kStrip2)
            return fail(SLBM_E_INVAL, "strip must be 0, 58, 62 or 64");
        if (seg_rows > (strip == kStrip2 ? kMaxTileRows2 : kMaxTileRows))
            return fail(SLBM_E_INVAL, "rows per tile above the maximum (14; 10 with two steps per launch)");
        if (strip == kStrip2) {
            DeviceGuard dg(h->device);
            const int rc = tile_records(h, seg_rows);
            if (rc) return rc;
        }
        h->seg = seg_rows;
        h->two = strip == kStrip2 ? 1 : 0;
        h->wide = (strip == 0 || strip == kStrip2) ? -1 : (strip == 64 ? 1 : 0);
        return SLBM_OK;
    });
}

int slbm_set_xcd_group(slbm_handle h, int32_t group)
{
    return guarded([&]() -> int {
        if (!h) return fail(SLBM_E_INVAL, "null handle");
        if (h->batch) return fail(SLBM_E_INVAL, "the plate belongs to a batch (only readouts go through its handle)");
        if (!valid_group(group)) return fail(SLBM_E_INVAL, "xcd group must be 0 (bands) or a power of two up to 64");
        h->group = group;
        return SLBM_OK;
    });
}

int slbm_tile_list_layout(int32_t nx, int32_t ny, int32_t periodic_x, int32_t periodic_y, int32_t rows,
                          int32_t n_links, const int32_t* link_sites, int32_t* tile_start, int32_t* rec_link,
                          int32_t* rec_pos, int64_t capacity, int64_t* n_tiles, int64_t* n_records,
                          int32_t* max_per_tile)
{
    return guarded([&]() -> int {
        if (nx < 1 || ny < 1 || (long long)nx * ny > (1LL << 28)) return fail(SLBM_E_INVAL, "bad grid");
        if (rows < 1 || rows > kMaxTileRows2) return fail(SLBM_E_INVAL, "rows per tile must be in [1, 10]");
        if (n_links < 0 || (n_links > 0 && !link_sites)) return fail(SLBM_E_INVAL, "bad link list");
        for (int i = 0; i < n_links; ++i)
            if (link_sites[i] < 0 || (long long)link_sites[i] >= (long long)nx * ny)
                return fail(SLBM_E_INVAL, "link %d: site out of the grid", i);
        const TileLayout lay = tile_layout(nx, ny, periodic_x != 0, periodic_y != 0, rows, link_sites, n_links,
                                           INT64_MAX);
        if (lay.start.empty()) return fail(SLBM_E_UNSUPPORTED, "more than 2^31 - 1 tile records");
        const int64_t total = lay.start[(size_t)lay.ntiles];
        if (n_tiles) *n_tiles = lay.ntiles;
        if (n_records) *n_records = total;
        if (max_per_tile) *max_per_tile = lay.most;
        if (tile_start) std::memcpy(tile_start, lay.start.data(), lay.start.size() * sizeof(int32_t));
        if ((rec_link || rec_pos) && total > capacity) return fail(SLBM_E_INVAL, "capacity below the record count");
        if (rec_link) std::memcpy(rec_link, lay.link.data(), (size_t)total * sizeof(int32_t));
        if (rec_pos) std::memcpy(rec_pos, lay.pos.data(), (size_t)total * sizeof(int32_t));
        return SLBM_OK;
    });
}

int slbm_boundary_lists(slbm_handle h, int32_t* rows, int64_t* records, int32_t* max_per_tile)
{
    return guarded([&]() -> int {
        if (!h) return fail(SLBM_E_INVAL, "null handle");
        if (rows) *rows = h->rec_fit ? h->rec_seg : 0;
        if (records) *records = h->rec_fit ? h->rec_count : 0;
        if (max_per_tile) *max_per_tile = h->rec_fit ? h->rec_max : 0;
        return SLBM_OK;
    });
}

int slbm_get_launch(slbm_handle h, int32_t* seg_rows, int32_t* strip, int32_t* xcd_group)
{
    return guarded([&]() -> int {
        if (!h) return fail(SLBM_E_INVAL, "null handle");
        if (seg_rows) *seg_rows = h->seg;
        if (strip) *strip = h->two ? kStrip2 : (h->wide < 0 ? 0 : (h->wide ? 64 : 62));
        if (xcd_group) *xcd_group = h->group;
        return SLBM_OK;
    });
}

int slbm_autotune(slbm_handle h, int32_t* seg_out, int32_t* strip_out, double* us_out)
{
    return guarded([&]() -> int {
        if (!h) return fail(SLBM_E_INVAL, "null handle");
        if (h->batch) return fail(SLBM_E_INVAL, "the plate belongs to a batch (only readouts go through its handle)");
        DeviceGuard dg(h->device);
        int rc = ensure_scratch(h, 3);
        if (rc) return rc;
        // the trial steps write the other population buffer (free) and update U
        // in place: keep U and the divergence flag aside and restore them after
        // every trial, so the state is left exactly as it was
        const size_t ub = (size_t)2 * h->plane * sizeof(double);
        double* saved = h->scratch;
        unsigned int* flag_saved = (unsigned int*)(h->scratch + 2 * h->plane);
        HIP_TRY(hipMemcpyAsync(saved, h->U, ub, hipMemcpyDeviceToDevice, h->stream));
        HIP_TRY(hipMemcpyAsync(flag_saved, h->diverged, sizeof(unsigned int), hipMemcpyDeviceToDevice, h->stream));
        hipEvent_t e0, e1;
        HIP_TRY(hipEventCreate(&e0));
        HIP_TRY(hipEventCreate(&e1));
        // time per step of a shape (wv: 0 narrow, 1 wide, 2 two steps per
        // launch) with the current XCD map: the best of two bursts of
        // back-to-back launches after a warm one, as steps run; each launch
        // rereads the same state, and U is put back after every burst
        auto time_shape = [&](int c, int wv, double& us) -> int {
            const int burst = wv == 2 ? 3 : 6;
            if (wv == 2) {
                const int rc2 = tile_records(h, c);
                if (rc2) return rc2;
            }
            std::vector<float> t;
            for (int r = 0; r < 3; ++r) {
                HIP_TRY(hipEventRecord(e0, h->stream));
                for (int q = 0; q < burst; ++q) {
                    const int rc2 = wv == 2
                        ? (h->precision == SLBM_FP32 ? launch_step2_raw<float>(h, c) : launch_step2_raw<double>(h, c))
                        : (h->precision == SLBM_FP32 ? launch_step_raw<float>(h, c, wv) : launch_step_raw<double>(h, c, wv));
                    if (rc2) return rc2;
                }
                HIP_TRY(hipEventRecord(e1, h->stream));
                HIP_TRY(hipMemcpyAsync(h->U, saved, ub, hipMemcpyDeviceToDevice, h->stream));
                HIP_TRY(hipEventSynchronize(e1));
                float ms = 0;
                HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
                if (r > 0) t.push_back(ms / (wv == 2 ? 2 * burst : burst));
            }
            us = 1e3 * *std::min_element(t.begin(), t.end());
            return SLBM_OK;
        };
        const int keep_group = h->group;
        h->group = 0;
        const int cand[] = {2, 3, 4, 6, 8, 10, 12, 14};
        int best = 0, best_w = 0;
        double best_us = 1e30, us = 0;
        for (int wv = 0; wv < 2; ++wv)
        for (int c : cand) {
            if (c > (wv ? max_tile_rows<true>() : max_tile_rows<false>())) break;
            if (c > std::max(2, h->ny)) break;
            if ((rc = time_shape(c, wv, us))) { h->group = keep_group; return rc; }
            if (us < best_us) { best_us = us; best = c; best_w = wv; }
        }
        // two steps per launch
        const int cand2[] = {2, 3, 4, 5, 6, 7, 8, 9, 10};
        for (int c : cand2) {
            if (c > std::max(2, h->ny)) break;
            if ((rc = time_shape(c, 2, us))) { h->group = keep_group; return rc; }
            if (us < best_us) { best_us = us; best = c; best_w = 2; }
        }
        // the best shape with interleaved XCD groups of 8, kept when at least
        // 1 % faster (plates whose boundary tiles cluster)
        h->group = 8;
        if ((rc = time_shape(best, best_w, us))) { h->group = keep_group; return rc; }
        if (us < 0.99 * best_us)
            best_us = us;
        else
            h->group = 0;
        HIP_TRY(hipMemcpyAsync(h->diverged, flag_saved, sizeof(unsigned int), hipMemcpyDeviceToDevice, h->stream));
        HIP_TRY(hipStreamSynchronize(h->stream));
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        release_transient_scratch(h);
        if (best_w == 2 && (rc = tile_records(h, best))) return rc;
        h->seg = best;
        h->two = best_w == 2 ? 1 : 0;
        h->wide = best_w == 2 ? -1 : best_w;
        if (seg_out) *seg_out = best;
        if (strip_out) *strip_out = best_w == 2 ? kStrip2 : (best_w ? 64 : 62);
        if (us_out) *us_out = best_us;
        return SLBM_OK;
    });
}

int slbm_device_bytes(slbm_handle h, int64_t* bytes)
{
    return guarded([&]() -> int {
        if (!h || !bytes) return fail(SLBM_E_INVAL, "null argument");
        int64_t b = 2 * (int64_t)9 * h->plane * (int64_t)h->esize + 2 * h->plane * 8 + h->plane * 5;
        b += (int64_t)h->n_links * (h->esize == 4 ? (int64_t)sizeof(LinkDev<float>) : (int64_t)sizeof(LinkDev<double>));
        b += h->rec_bytes;
        if (h->scratch) b += (int64_t)h->scratch_planes * h->plane * 8;
        *bytes = b;
        return SLBM_OK;
    });
}

namespace {
struct SaveHeader {
    uint64_t magic;
    int32_t nx, ny, ld, precision;
    int64_t step;
    int32_t local, diverged;
};
constexpr uint64_t kMagic = 0x31304d424c53ULL;  // "SLBM01"
}  // namespace

int slbm_save(slbm_handle h, void* buf, size_t* bytes)
{
    return guarded([&]() -> int {
        if (!h || !bytes) return fail(SLBM_E_INVAL, "null argument");
        const size_t pop = (size_t)9 * h->plane * h->esize, ub = (size_t)2 * h->plane * sizeof(double);
        const size_t need = sizeof(SaveHeader) + pop + ub;
        if (!buf) { *bytes = need; return SLBM_OK; }
        if (*bytes < need) return fail(SLBM_E_INVAL, "buffer too small: %zu < %zu", *bytes, need);
        DeviceGuard dg(h->device);
        if (int rw = wait_ready(h)) return rw;
        SaveHeader hd{kMagic, h->nx, h->ny, h->ld, h->precision, h->step, h->local ? 1 : 0, 0};
        unsigned int flag = 0;
        char* p = (char*)buf;
        HIP_TRY(hipMemcpyAsync(&flag, h->diverged, sizeof flag, hipMemcpyDeviceToHost, h->stream));
        HIP_TRY(hipMemcpyAsync(p + sizeof hd, h->buf[h->cur], pop, hipMemcpyDeviceToHost, h->stream));
        HIP_TRY(hipMemcpyAsync(p + sizeof hd + pop, h->U, ub, hipMemcpyDeviceToHost, h->stream));
        HIP_TRY(hipStreamSynchronize(h->stream));
        hd.diverged = (int32_t)flag;
        std::memcpy(p, &hd, sizeof hd);
        *bytes = need;
        return SLBM_OK;
    });
}

int slbm_load(slbm_handle h, const void* buf, size_t bytes)
{
    return guarded([&]() -> int {
        if (!h || !buf) return fail(SLBM_E_INVAL, "null argument");
        if (h->batch) return fail(SLBM_E_INVAL, "the plate belongs to a batch (only readouts go through its handle)");
        const size_t pop = (size_t)9 * h->plane * h->esize, ub = (size_t)2 * h->plane * sizeof(double);
        SaveHeader hd;
        if (bytes < sizeof hd + pop + ub) return fail(SLBM_E_INVAL, "checkpoint too short");
        std::memcpy(&hd, buf, sizeof hd);
        if (hd.magic != kMagic || hd.nx != h->nx || hd.ny != h->ny || hd.ld != h->ld || hd.precision != h->precision)
            return fail(SLBM_E_INVAL, "checkpoint does not match this plate");
        DeviceGuard dg(h->device);
        const char* p = (const char*)buf;
        h->cur = 0;
        HIP_TRY(hipMemcpyAsync(h->buf[0], p + sizeof hd, pop, hipMemcpyHostToDevice, h->stream));
        HIP_TRY(hipMemcpyAsync(h->U, p + sizeof hd + pop, ub, hipMemcpyHostToDevice, h->stream));
        unsigned int flag = (unsigned int)hd.diverged;
        HIP_TRY(hipMemcpyAsync(h->diverged, &flag, sizeof flag, hipMemcpyHostToDevice, h->stream));
        HIP_TRY(hipStreamSynchronize(h->stream));
        h->step = hd.step;
        h->local = hd.local != 0;
        return SLBM_OK;
    });
}

int slbm_copy(void* dst, const void* src, size_t bytes, int32_t device, void* stream)
{
    return guarded([&]() -> int {
        if (!dst || !src) return fail(SLBM_E_INVAL, "null pointer");
        if (bytes % 16 != 0 || ((uintptr_t)dst | (uintptr_t)src) % 16 != 0)
            return fail(SLBM_E_INVAL, "bytes and both pointers must be multiples of 16");
        DeviceGuard dg(device);
        const long long n = (long long)(bytes / 16);
        if (n > (1LL << 31) * 256) return fail(SLBM_E_UNSUPPORTED, "copy larger than 2^39 x 16 bytes");
        const unsigned grid = (unsigned)((n + 255) / 256);
        if (n > 0)
            hipLaunchKernelGGL(k_copy16, dim3(grid), dim3(256), 0, (hipStream_t)stream,
                               (const float4*)src, (float4*)dst, n);
        HIP_TRY(hipGetLastError());
        return SLBM_OK;
    });
}

// ================================================================ batches

}  // extern "C"

#include "batch_api.h"

extern "C" {

const char* slbm_last_error(void) { return g_err.c_str(); }

}  // extern "C"

// ------------------------------------------------ three-dimensional step

#include "slbm3_api.h"
