// Host side of the three-dimensional step (slbm3_* in include/slbm3.h).
// Included at the end of slbm.hip: it shares that translation unit's error
// reporting (fail, HIP_TRY, slbm_last_error) and DeviceGuard.
#include "slbm3.h"
#include "step3_kernel.h"

struct slbm3_s {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int nx = 0, ny = 0, nz = 0;
    long long plane = 0;             // sites
    long long stride = 0;            // elements between planes of the population and U buffers
    int precision = SLBM_FP64;
    size_t esize = 8;
    int px = 1;
    int wkind[2] = {0, 0};
    double wval[2][3] = {{0, 0, 0}, {0, 0, 0}};   // lattice units
    double wq[2] = {0.5, 0.5};
    // time profiles: the walls' (RAMP: ramp length in steps, else 0) and the
    // general geometry's ramp slots (slot 0: constant)
    double wramp[2] = {0.0, 0.0};
    double slot_ramp[slbm3_dev::kProfileSlots3] = {};
    int norder = 0;
    double lamL = 0, muL = 1.0 / 3.0, tau = 0.55, FL[3] = {0, 0, 0};
    double dt_user = 1, s_sigma = 1, s_v = 1, rho_user = 1;
    void* buf[2] = {nullptr, nullptr};
    int cur = 0;
    bool local = true;
    double* U = nullptr;
    void* dens = nullptr;
    unsigned int* diverged = nullptr;
    double* scratch = nullptr;       // 19 planes of doubles, on demand (outputs, initial fields)
    int64_t step = 0;
    // general geometry: site flags, first link record of each site, records
    bool geo = false;
    uint32_t* flags = nullptr;
    int32_t* bidx = nullptr;
    void* links = nullptr;
    void* lval = nullptr;            // per link record: (A, s_kappa) of the rule (k3_step, k3_links_ext)
    int32_t* wrec = nullptr;         // per workgroup of k3_step: first record
    int32_t* elink = nullptr;        // the records whose Neumann data are extrapolated
    int64_t n_ext = 0;
    uint64_t geo_hash = 0;           // the geometry a checkpoint must match (mask and cut links, or the walls)
    int64_t n_links = 0;
    size_t link_bytes = 0;
};

namespace {

using namespace slbm3_dev;

template <typename real>
Step3Args<real> make_args3(const slbm3_s* h, int src)
{
    Step3Args<real> a{};
    a.src = (const real*)h->buf[src];
    a.dst = (real*)h->buf[src ^ 1];
    a.U = h->U;
    a.dens = (real*)h->dens;
    a.diverged = h->diverged;
    a.plane = h->plane;
    a.stride = h->stride;
    a.nx = h->nx; a.ny = h->ny; a.nz = h->nz;
    a.px = h->px;
    a.local = h->local ? 1 : 0;
    a.ntiles = ((h->nx + 63) / 64) * h->ny * h->nz;
    // time profiles at the step of the state the pulls read (the previous
    // step's post-collision state) and of the state this step produces
    const double n_pull = h->step >= 1 ? (double)(h->step - 1) : 0.0, n_next = (double)h->step;
    auto ramp = [](double n, double len) { return len > 0.0 ? std::min(n / len, 1.0) : 1.0; };
    for (int k = 0; k < kProfileSlots3; ++k) {
        a.pf_pull[k] = (real)ramp(n_pull, h->slot_ramp[k]);
        a.pf_next[k] = (real)ramp(n_next, h->slot_ramp[k]);
    }
    for (int s = 0; s < 2; ++s) {
        a.wkind[s] = h->wkind[s];
        for (int k = 0; k < 3; ++k) a.wval[s][k] = (real)(h->wval[s][k] * ramp(n_pull, h->wramp[s]));
        // section 4.2: a site behind x along the cut link exists unless nx = 1
        const bool behind = h->nx >= 2;
        const double q = h->wq[s];
        a.wkap[s] = (real)(behind ? (1.0 - 2.0 * q) / (1.0 + 2.0 * q) : 0.0);
        a.wbeta[s] = (real)(behind ? 2.0 / (1.0 + 2.0 * q) : 1.0);
        a.wq1[s] = (real)(1.0 + q);
        a.wq[s] = (real)q;
        a.wext[s] = behind && h->norder == 1 && h->wkind[s] == SLBM_NEUMANN ? 1 : 0;
    }
    a.omega = (real)(1.0 / h->tau);
    a.omega_h = (real)(1.0 - 0.5 / h->tau);
    a.ml = (real)(h->muL - h->lamL);
    a.lm = (real)(h->lamL - h->muL);
    for (int k = 0; k < 3; ++k) a.F[k] = (real)h->FL[k];
    a.flags = h->flags;
    a.bidx = h->bidx;
    a.links = (const Link3<real>*)h->links;
    a.lval = (real*)h->lval;
    a.wrec = h->wrec;
    return a;
}

// The cut links of a general geometry as the kernels read them: per-site
// flags (bit i - 1: link i cut; kVoid3: void), each cut site's first record,
// and the records sorted by site and direction, in lattice units.  Validates
// what slbm3_create documents; the host arrays are the caller's.
struct Geo3 {
    std::vector<int> gslot;          // per group: its time-profile slot
    std::vector<double> slot_ramp;   // per slot: ramp length in steps (0: constant)
    std::vector<uint32_t> flags;
    std::vector<int32_t> bidx;
    std::vector<Link3<double>> recs;
    std::vector<double> skap;        // per record: kappa (Dirichlet), -kappa (Neumann) or 0 (ext)
    std::vector<int32_t> elink;      // the ext records
    std::vector<int32_t> wrec;       // per workgroup of k3_step: its first record, then the count
    uint64_t hash = 0;               // FNV-1a of the mask and of each cut link's site, direction, q,
                                     // groups and normals, in record order
};

// 64-bit FNV-1a, fed value by value (no struct padding enters it).
struct Fnv64 {
    uint64_t h = 0xcbf29ce484222325ull;
    void bytes(const void* p, size_t n)
    {
        const unsigned char* c = (const unsigned char*)p;
        for (size_t i = 0; i < n; ++i) h = (h ^ c[i]) * 0x100000001b3ull;
    }
    template <typename T> void put(T v) { bytes(&v, sizeof v); }
};

int build_geo3(const slbm3_params* p, const slbm3_s* h, Geo3& g)
{
    const long long n = h->plane;
    const int nx = h->nx, ny = h->ny, nz = h->nz;
    if (p->n_links < 0 || (p->n_links > 0 && !p->links)) return fail(SLBM_E_INVAL, "links: null array");
    if (p->n_groups < 0 || (p->n_groups > 0 && !p->groups)) return fail(SLBM_E_INVAL, "groups: null array");
    if (p->n_links > 18LL * n) return fail(SLBM_E_INVAL, "more links than a box has");
    if (p->n_links > (int64_t)INT_MAX - 255)
        return fail(SLBM_E_UNSUPPORTED, "more than 2^31 - 256 cut links (records are indexed with 32 bits)");
    for (int k = 0; k < p->n_groups; ++k) {
        const slbm3_bc_group& gr = p->groups[k];
        if (gr.kind != SLBM_DIRICHLET && gr.kind != SLBM_NEUMANN)
            return fail(SLBM_E_INVAL, "group %d: kind must be SLBM_DIRICHLET or SLBM_NEUMANN", k);
        if (!std::isfinite(gr.value[0]) || !std::isfinite(gr.value[1]) || !std::isfinite(gr.value[2]) ||
            !std::isfinite(gr.pressure))
            return fail(SLBM_E_INVAL, "group %d: values must be finite", k);
        if (gr.profile != SLBM_PROFILE_STEP && gr.profile != SLBM_PROFILE_RAMP)
            return fail(SLBM_E_INVAL, "group %d: profile must be SLBM_PROFILE_STEP or SLBM_PROFILE_RAMP", k);
        if (gr.profile == SLBM_PROFILE_RAMP && !(gr.ramp_time > 0.0))
            return fail(SLBM_E_INVAL, "group %d: ramp time must be positive", k);
    }
    // each group's time-profile slot: 0 for STEP, one slot per distinct ramp time
    g.gslot.assign((size_t)p->n_groups, 0);
    g.slot_ramp.assign(kProfileSlots3, 0.0);
    {
        int nslots = 1;
        for (int k = 0; k < p->n_groups; ++k) {
            if (p->groups[k].profile != SLBM_PROFILE_RAMP) continue;
            const double len = p->groups[k].ramp_time / h->dt_user;
            int sl = 1;
            while (sl < nslots && g.slot_ramp[(size_t)sl] != len) ++sl;
            if (sl == nslots) {
                if (nslots == kProfileSlots3)
                    return fail(SLBM_E_UNSUPPORTED, "more than %d distinct ramp times", kProfileSlots3 - 1);
                g.slot_ramp[(size_t)nslots++] = len;
            }
            g.gslot[(size_t)k] = sl;
        }
    }
    g.flags.assign((size_t)n, 0u);
    for (long long s = 0; s < n; ++s)
        if (!p->mask[s]) g.flags[s] = kVoid3;
    auto far_site = [&](long long s, int i) {
        const long long x = s % nx, y = (s / nx) % ny, z = s / ((long long)nx * ny);
        const long long fx = (x + kCX[i] + nx) % nx, fy = (y + kCY[i] + ny) % ny, fz = (z + kCZ[i] + nz) % nz;
        return (fz * ny + fy) * nx + fx;
    };
    for (int64_t l = 0; l < p->n_links; ++l) {
        const slbm3_link& L = p->links[l];
        if (L.site < 0 || (long long)L.site >= n) return fail(SLBM_E_INVAL, "link %lld: site out of range", (long long)l);
        if (L.dir < 1 || L.dir > 18) return fail(SLBM_E_INVAL, "link %lld: direction must be in 1..18", (long long)l);
        if (!p->mask[L.site]) return fail(SLBM_E_INVAL, "link %lld: starts at a void site", (long long)l);
        if (!(L.q > 0.0 && L.q <= 1.0)) return fail(SLBM_E_INVAL, "link %lld: q must be in (0, 1]", (long long)l);
        if (L.group < 0 || L.group >= p->n_groups) return fail(SLBM_E_INVAL, "link %lld: group out of range", (long long)l);
        const double nn = std::sqrt(L.normal[0] * L.normal[0] + L.normal[1] * L.normal[1] + L.normal[2] * L.normal[2]);
        if (!(std::fabs(nn - 1.0) <= 1e-9)) return fail(SLBM_E_INVAL, "link %lld: normal is not a unit vector", (long long)l);
        if (L.group2 < -1 || L.group2 >= p->n_groups)
            return fail(SLBM_E_INVAL, "link %lld: second group out of range", (long long)l);
        if (L.group2 >= 0) {
            const double* m2 = L.normal2;
            const double n2 = std::sqrt(m2[0] * m2[0] + m2[1] * m2[1] + m2[2] * m2[2]);
            if (!(std::fabs(n2 - 1.0) <= 1e-9))
                return fail(SLBM_E_INVAL, "link %lld: second normal is not a unit vector", (long long)l);
            const double d = L.normal[0] * m2[0] + L.normal[1] * m2[1] + L.normal[2] * m2[2];
            if (!(std::fabs(d) <= 1e-9))
                return fail(SLBM_E_INVAL, "link %lld: the two faces' normals are not orthogonal", (long long)l);
            if (g.gslot[(size_t)L.group] != g.gslot[(size_t)L.group2])
                return fail(SLBM_E_INVAL, "link %lld: the two faces of an edge need the same time profile", (long long)l);
        }
        const uint32_t bit = 1u << (L.dir - 1);
        if (g.flags[L.site] & bit) return fail(SLBM_E_INVAL, "link %lld: listed twice", (long long)l);
        g.flags[L.site] |= bit;
    }
    // a link into the material crosses a crack: the link back is listed too
    for (int64_t l = 0; l < p->n_links; ++l) {
        const slbm3_link& L = p->links[l];
        const long long f = far_site(L.site, L.dir);
        if (p->mask[f] && !(g.flags[f] & (1u << (opp3(L.dir) - 1))))
            return fail(SLBM_E_INVAL, "link %lld: ends in the material but the link back (the crack's other face) "
                                      "is not listed", (long long)l);
    }
    // every link from the material into the void is listed: planes of z on
    // several host threads, each site's 18 neighbours through the 9 rows
    // around it; the first offending site (lowest index) is reported
    {
        const int nthreads = (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
        std::vector<long long> first((size_t)nthreads, -1);
        std::vector<int> first_dir((size_t)nthreads, 0);
        auto scan = [&](int t) {
            for (int z = t; z < nz; z += nthreads) {
                for (int y = 0; y < ny; ++y) {
                    const uint8_t* row[3][3];
                    for (int dz = -1; dz <= 1; ++dz)
                        for (int dy = -1; dy <= 1; ++dy)
                            row[dz + 1][dy + 1] = p->mask + (((long long)((z + dz + nz) % nz) * ny + (y + dy + ny) % ny) * nx);
                    const long long base = ((long long)z * ny + y) * nx;
                    for (int x = 0; x < nx; ++x) {
                        if (!p->mask[base + x]) continue;
                        const uint32_t fl = g.flags[base + x];
                        const int xm = x == 0 ? nx - 1 : x - 1, xp = x == nx - 1 ? 0 : x + 1;
                        for (int i = 1; i < kQ; ++i) {
                            const int fx = kCX[i] < 0 ? xm : (kCX[i] > 0 ? xp : x);
                            if (!row[kCZ[i] + 1][kCY[i] + 1][fx] && !(fl & (1u << (i - 1)))) {
                                if (first[t] < 0 || base + x < first[t]) {
                                    first[t] = base + x;
                                    first_dir[t] = i;
                                }
                                break;
                            }
                        }
                        if (first[t] >= 0) break;
                    }
                    if (first[t] >= 0) break;
                }
                if (first[t] >= 0) break;              // later planes of this thread have higher indices
            }
        };
        std::vector<std::thread> pool;
        for (int t = 1; t < nthreads; ++t) pool.emplace_back(scan, t);
        scan(0);
        for (std::thread& th : pool) th.join();
        long long bad = -1;
        int bad_dir = 0;
        for (int t = 0; t < nthreads; ++t)
            if (first[t] >= 0 && (bad < 0 || first[t] < bad)) {
                bad = first[t];
                bad_dir = first_dir[t];
            }
        if (bad >= 0) return fail(SLBM_E_INVAL, "site %lld: link %d into the void is not listed", bad, bad_dir);
    }
    // records sorted by site, then direction (the kernel walks a site's cut
    // bits upwards from its first record)
    std::vector<int64_t> order((size_t)p->n_links);
    for (int64_t l = 0; l < p->n_links; ++l) order[(size_t)l] = l;
    std::sort(order.begin(), order.end(), [&](int64_t u, int64_t v) {
        const slbm3_link &A = p->links[u], &B = p->links[v];
        return A.site != B.site ? A.site < B.site : A.dir < B.dir;
    });
    {
        Fnv64 f;
        for (long long i = 0; i < n; ++i) f.put((uint8_t)(p->mask[i] != 0));   // any nonzero is material
        for (int64_t l : order) {
            const slbm3_link& L = p->links[l];
            f.put(L.site); f.put(L.dir); f.put(L.q); f.put(L.group); f.put(L.group2);
            for (int k = 0; k < 3; ++k) { f.put(L.normal[k]); f.put(L.normal2[k]); }
        }
        g.hash = f.h;
    }
    g.bidx.assign((size_t)n, 0);
    g.recs.resize(order.size());
    g.skap.resize(order.size());
    for (size_t r = 0; r < order.size(); ++r) {
        const slbm3_link& L = p->links[order[r]];
        if (r == 0 || p->links[order[r - 1]].site != L.site) g.bidx[L.site] = (int32_t)r;
        // a link through the edge of two faces: the Dirichlet face wins
        const bool two = L.group2 >= 0;
        const bool d1 = p->groups[L.group].kind == SLBM_DIRICHLET;
        const bool d2 = two && p->groups[L.group2].kind == SLBM_DIRICHLET;
        const slbm3_bc_group& gr = p->groups[(!d1 && d2) ? L.group2 : L.group];
        const int i = L.dir, ib = opp3(i);
        // section 4.2: no site behind x when the opposite link is cut too
        const bool thin = (g.flags[L.site] >> (ib - 1)) & 1u;
        const double q = L.q;
        const double kap = thin ? 0.0 : (1.0 - 2.0 * q) / (1.0 + 2.0 * q);
        const double bet = thin ? 1.0 : 2.0 / (1.0 + 2.0 * q);
        const double w = w3(i);
        const double c[3] = {(double)kCX[i], (double)kCY[i], (double)kCZ[i]};
        const double c2 = c[0] * c[0] + c[1] * c[1] + c[2] * c[2];
        Link3<double>& R = g.recs[r];
        R.kap = kap;
        R.bet2 = 2.0 * bet;
        R.q1 = 1.0 + q;
        R.q = q;
        for (int k = 0; k < 6; ++k) R.B[k] = 0.0;
        R.K = 0.0;
        if (gr.kind == SLBM_DIRICHLET) {
            const double cv = (c[0] * gr.value[0] + c[1] * gr.value[1] + c[2] * gr.value[2]) / h->s_v;
            R.c0 = bet * 6.0 * w * cv;
        } else {
            // the constants of e = c0 drho_bd + B:P_b - K (the record's
            // comment): sigma* = Pi sigma_b Pi + N, with N fixed by the
            // traction(s).  One face: Pi = I - n n, N = n t + t n - (t.n) n n.
            // Two faces (an edge): Pi = e e with e = n_A x n_B, and N holds the
            // rows of n_A and n_B in the frame (n_A, n_B, e), their shear
            // averaged.
            const double* n = L.normal;
            double t[3], A[3][3], Pi[3][3], N[3][3], T[3][3], B0[3][3];
            for (int k = 0; k < 3; ++k) t[k] = (gr.value[k] - gr.pressure * n[k]) / h->s_sigma;
            for (int u = 0; u < 3; ++u)
                for (int v = 0; v < 3; ++v) A[u][v] = c[u] * c[v] - (u == v ? 1.0 / 3.0 : 0.0);
            if (!two) {
                const double tn = t[0] * n[0] + t[1] * n[1] + t[2] * n[2];
                for (int u = 0; u < 3; ++u)
                    for (int v = 0; v < 3; ++v) {
                        Pi[u][v] = (u == v ? 1.0 : 0.0) - n[u] * n[v];
                        N[u][v] = n[u] * t[v] + t[u] * n[v] - tn * n[u] * n[v];
                    }
            } else {
                const slbm3_bc_group& g2r = p->groups[L.group2];
                const double* nb = L.normal2;
                double tb[3];
                for (int k = 0; k < 3; ++k) tb[k] = (g2r.value[k] - g2r.pressure * nb[k]) / h->s_sigma;
                const double e[3] = {n[1] * nb[2] - n[2] * nb[1], n[2] * nb[0] - n[0] * nb[2], n[0] * nb[1] - n[1] * nb[0]};
                auto dot = [](const double* a_, const double* b_) { return a_[0] * b_[0] + a_[1] * b_[1] + a_[2] * b_[2]; };
                const double* u3[3] = {n, nb, e};
                double S[3][3] = {{dot(t, n), 0.5 * (dot(t, nb) + dot(tb, n)), dot(t, e)},
                                  {0.5 * (dot(t, nb) + dot(tb, n)), dot(tb, nb), dot(tb, e)},
                                  {dot(t, e), dot(tb, e), 0.0}};
                for (int u = 0; u < 3; ++u)
                    for (int v = 0; v < 3; ++v) {
                        Pi[u][v] = e[u] * e[v];
                        double acc = 0.0;
                        for (int X = 0; X < 3; ++X)
                            for (int Y = 0; Y < 3; ++Y) acc += S[X][Y] * u3[X][u] * u3[Y][v];
                        N[u][v] = acc;
                    }
            }
            for (int u = 0; u < 3; ++u)
                for (int v = 0; v < 3; ++v) T[u][v] = A[u][0] * Pi[0][v] + A[u][1] * Pi[1][v] + A[u][2] * Pi[2][v];
            for (int u = 0; u < 3; ++u)
                for (int v = 0; v < 3; ++v) B0[u][v] = Pi[u][0] * T[0][v] + Pi[u][1] * T[1][v] + Pi[u][2] * T[2][v];
            double NA = 0.0;
            for (int u = 0; u < 3; ++u)
                for (int v = 0; v < 3; ++v) NA += N[u][v] * A[u][v];
            const double trB = B0[0][0] + B0[1][1] + B0[2][2];
            const double lm = h->lamL - h->muL;
            R.c0 = w * (2.5 - 1.5 * c2) + 4.5 * w * lm * (trB - c2 + 1.0);
            R.B[0] = 4.5 * w * B0[0][0];
            R.B[1] = 4.5 * w * B0[1][1];
            R.B[2] = 4.5 * w * B0[2][2];
            R.B[3] = 9.0 * w * B0[0][1];
            R.B[4] = 9.0 * w * B0[0][2];
            R.B[5] = 9.0 * w * B0[1][2];
            R.K = 4.5 * w * NA;
        }
        const int ext = gr.kind == SLBM_NEUMANN && h->norder == 1 && !thin ? 1 : 0;
        R.meta = link3_meta(i, ib, gr.kind, ext, kCX[i], kCY[i], kCZ[i], g.gslot[(size_t)(&gr - p->groups)]);
        R.site = L.site;
        g.skap[r] = ext ? 0.0 : (gr.kind == SLBM_DIRICHLET ? kap : -kap);
        if (ext) g.elink.push_back((int32_t)r);
    }
    // k3_step's workgroups take four 64-site row chunks each, a contiguous
    // range of sites from the first site of their first chunk
    {
        const long long chunks = (nx + 63) / 64, ntiles = chunks * ny * nz, nwg = (ntiles + 3) / 4;
        g.wrec.resize((size_t)nwg + 1);
        size_t r = 0;
        for (long long w = 0; w < nwg; ++w) {
            const long long t = 4 * w, row = t / chunks;
            const long long first = row * nx + 64 * (t % chunks);
            while (r < g.recs.size() && g.recs[r].site < first) ++r;
            g.wrec[(size_t)w] = (int32_t)r;
        }
        g.wrec[(size_t)nwg] = (int32_t)g.recs.size();
    }
    return SLBM_OK;
}

// The records in the handle's precision.
template <typename real>
std::vector<Link3<real>> cast_links3(const std::vector<Link3<double>>& in)
{
    std::vector<Link3<real>> out(in.size());
    for (size_t r = 0; r < in.size(); ++r) {
        const Link3<double>& A = in[r];
        Link3<real>& B = out[r];
        B.kap = (real)A.kap; B.bet2 = (real)A.bet2; B.q1 = (real)A.q1; B.q = (real)A.q; B.c0 = (real)A.c0;
        for (int k = 0; k < 6; ++k) B.B[k] = (real)A.B[k];
        B.K = (real)A.K;
        B.meta = A.meta;
        B.site = A.site;
    }
    return out;
}

// Elements from one plane of a population or displacement buffer to the
// next: the plane rounded up to 4096 sites, then to an odd multiple of 4096,
// so that a power-of-two box does not start all its planes on one channel.
long long plane_stride(long long plane)
{
    long long q = (plane + 4095) / 4096;
    if ((q & 1) == 0) q += 1;
    return q * 4096;
}

int grid3(const slbm3_s* h)
{
    const long long tiles = (long long)((h->nx + 63) / 64) * h->ny * h->nz;
    const long long wg = (tiles + 3) / 4;
    const long long unit = 8LL * xcd_group_size3(h->geo);   // xcd_group3 permutes whole units
    return (int)((wg + unit - 1) / unit * unit);
}

// The extrapolating rules (general geometry, GEO, which implies PX; the other
// cut links' parts come from the previous k3_step), density pass, then
// `what` (0 step, 1 outputs into scratch, 2 init from scratch).
template <typename real, bool PX, bool GEO>
int launch3(slbm3_s* h, int what)
{
    Step3Args<real> a = make_args3<real>(h, h->cur);
    const dim3 grid(grid3(h)), blk(256);
    if (what == 2) {
        a.dst = (real*)h->buf[h->cur];
        hipLaunchKernelGGL((k3_set_dens<real>), dim3((unsigned)((h->plane + 255) / 256)), blk, 0, h->stream, a,
                           (const double*)h->scratch);
        hipLaunchKernelGGL((k3_init<real, PX, GEO>), grid, blk, 0, h->stream, a, (const double*)h->scratch);
        HIP_TRY(hipGetLastError());
        return SLBM_OK;
    }
    if (GEO && !h->local && h->n_ext > 0)            // the extrapolating rules, read by both pulls
        hipLaunchKernelGGL((k3_links_ext<real>), dim3((unsigned)((h->n_ext + 255) / 256)), blk, 0, h->stream, a,
                           (const int32_t*)h->elink, (int)h->n_ext);
    hipLaunchKernelGGL((k3_density<real, PX, GEO>), grid, blk, 0, h->stream, a);
    if (what == 0)
        hipLaunchKernelGGL((k3_step<real, PX, GEO>), grid, blk, 0, h->stream, a);
    else
        hipLaunchKernelGGL((k3_outputs<real, PX, GEO>), grid, blk, 0, h->stream, a, h->scratch);
    HIP_TRY(hipGetLastError());
    return SLBM_OK;
}

int launch3_any(slbm3_s* h, int what)
{
    if (h->precision == SLBM_FP32) {
        if (h->geo) return launch3<float, true, true>(h, what);
        return h->px ? launch3<float, true, false>(h, what) : launch3<float, false, false>(h, what);
    }
    if (h->geo) return launch3<double, true, true>(h, what);
    return h->px ? launch3<double, true, false>(h, what) : launch3<double, false, false>(h, what);
}

int ensure_scratch3(slbm3_s* h)
{
    if (h->scratch) return SLBM_OK;
    HIP_TRY(hipMalloc((void**)&h->scratch, (size_t)19 * h->plane * sizeof(double)));
    return SLBM_OK;
}

void free3(slbm3_s* h)
{
    for (void* p : {h->buf[0], h->buf[1], (void*)h->U, h->dens, (void*)h->diverged, (void*)h->scratch,
                    (void*)h->flags, (void*)h->bidx, h->links, h->lval, (void*)h->wrec, (void*)h->elink})
        if (p) (void)hipFree(p);
    if (h->own_stream && h->stream) (void)hipStreamDestroy(h->stream);
}

// count consecutive output planes, x -> (x + add) * scale (lattice to user
// units, as copy_planes3), into caller device memory of doubles or floats
// (the planes are contiguous in both).
template <typename T>
__global__ __launch_bounds__(256) void k3_scale_out(const double* src, long long n, double add, double scale, T* dst)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = (T)((src[i] + add) * scale);
}

int device_planes3(slbm3_handle h, int first, int count, double add, double scale, void* dst, int dtype)
{
    const long long n = (long long)count * h->plane;
    const double* src = h->scratch + (size_t)first * (size_t)h->plane;
    const dim3 grid((unsigned)((n + 255) / 256)), blk(256);
    if (dtype == SLBM_FP64)
        hipLaunchKernelGGL(k3_scale_out<double>, grid, blk, 0, h->stream, src, n, add, scale, (double*)dst);
    else
        hipLaunchKernelGGL(k3_scale_out<float>, grid, blk, 0, h->stream, src, n, add, scale, (float*)dst);
    HIP_TRY(hipGetLastError());
    return SLBM_OK;
}

}  // namespace

extern "C" {

int slbm3_create(const slbm3_params* p, slbm3_handle* out)
{
    return guarded([&]() -> int {
        if (!p || !out) return fail(SLBM_E_INVAL, "null argument");
        *out = nullptr;
        if (p->nx < 1 || p->ny < 1 || p->nz < 1) return fail(SLBM_E_INVAL, "box sizes must be positive");
        if (!(p->mu > 0) || !(p->rho > 0)) return fail(SLBM_E_INVAL, "mu and rho must be positive");
        if (!(p->tau_bar > 0.5)) return fail(SLBM_E_INVAL, "tau_bar must exceed 1/2");
        if (!(p->lambda > -p->mu)) return fail(SLBM_E_INVAL, "lambda must exceed -mu");
        if (p->precision != SLBM_FP32 && p->precision != SLBM_FP64) return fail(SLBM_E_INVAL, "bad precision");
        const long long plane = (long long)p->nx * p->ny * p->nz;
        if (plane > (1LL << 29))
            return fail(SLBM_E_UNSUPPORTED, "box exceeds 2^29 sites (kernels index a plane's sites with 32-bit offsets)");
        if (p->neumann_order != 0 && p->neumann_order != 1) return fail(SLBM_E_INVAL, "neumann_order must be 0 or 1");
        if (p->mask && !p->periodic_x)
            return fail(SLBM_E_INVAL, "a box with a material mask is periodic on every axis (periodic_x = 1)");
        if (!p->mask && (p->n_links != 0 || p->n_groups != 0))
            return fail(SLBM_E_INVAL, "links and groups need a material mask");
        if (!p->periodic_x) {
            for (int s = 0; s < 2; ++s) {
                if (p->walls[s].kind != SLBM_DIRICHLET && p->walls[s].kind != SLBM_NEUMANN)
                    return fail(SLBM_E_INVAL, "wall %d: kind must be SLBM_DIRICHLET or SLBM_NEUMANN", s);
                if (!(p->walls[s].q > 0.0 && p->walls[s].q <= 1.0))
                    return fail(SLBM_E_INVAL, "wall %d: q must be in (0, 1]", s);
                if (p->walls[s].profile != SLBM_PROFILE_STEP && p->walls[s].profile != SLBM_PROFILE_RAMP)
                    return fail(SLBM_E_INVAL, "wall %d: profile must be SLBM_PROFILE_STEP or SLBM_PROFILE_RAMP", s);
                if (p->walls[s].profile == SLBM_PROFILE_RAMP && !(p->walls[s].ramp_time > 0.0))
                    return fail(SLBM_E_INVAL, "wall %d: ramp time must be positive", s);
            }
        }
        slbm3_s* h = new (std::nothrow) slbm3_s();
        if (!h) return fail(SLBM_E_NOMEM, "out of host memory");
        h->device = p->device;
        h->nx = p->nx; h->ny = p->ny; h->nz = p->nz;
        h->plane = plane;
        h->stride = plane_stride(plane);
        h->precision = p->precision;
        h->esize = p->precision == SLBM_FP32 ? 4 : 8;
        h->px = p->periodic_x ? 1 : 0;
        // units (section 5.1): c_s = sqrt(mu/rho) = dx/(sqrt 3 dt)
        h->rho_user = p->rho;
        h->dt_user = std::sqrt(p->rho / (3.0 * p->mu));
        h->s_sigma = 3.0 * p->mu;
        h->s_v = 1.0 / h->dt_user;
        h->lamL = p->lambda / h->s_sigma;
        h->muL = p->mu / h->s_sigma;
        h->tau = p->tau_bar;
        for (int k = 0; k < 3; ++k) h->FL[k] = p->body_force[k] / h->s_sigma;
        if (!h->px) {
            for (int s = 0; s < 2; ++s) {
                h->wkind[s] = p->walls[s].kind;
                const double scale = p->walls[s].kind == SLBM_DIRICHLET ? h->s_v : h->s_sigma;
                for (int k = 0; k < 3; ++k) h->wval[s][k] = p->walls[s].value[k] / scale;
                h->wq[s] = p->walls[s].q;
                h->wramp[s] = p->walls[s].profile == SLBM_PROFILE_RAMP ? p->walls[s].ramp_time / h->dt_user : 0.0;
            }
        }
        h->norder = p->neumann_order;
        {
            // the geometry without cut links: periodic in x, or the two walls' kinds and q
            Fnv64 f;
            f.put(h->px);
            for (int s = 0; s < 2 && !h->px; ++s) { f.put(h->wkind[s]); f.put(h->wq[s]); }
            h->geo_hash = f.h;
        }
        Geo3 geo;
        if (p->mask) {
            const int rc = build_geo3(p, h, geo);
            if (rc) { delete h; return rc; }
            h->geo = true;
            h->geo_hash = geo.hash;
            for (int k = 0; k < kProfileSlots3; ++k) h->slot_ramp[k] = geo.slot_ramp[(size_t)k];
            h->n_links = (int64_t)geo.recs.size();
            h->n_ext = (int64_t)geo.elink.size();
        }
        DeviceGuard dg(h->device);
    #define TRY_OR_BAIL(expr)                                \
        do {                                                 \
            int rc_ = [&]() -> int { HIP_TRY(expr); return SLBM_OK; }(); \
            if (rc_) { free3(h); delete h; return rc_; }     \
        } while (0)
        if (p->stream) {
            h->stream = (hipStream_t)p->stream;
        } else {
            TRY_OR_BAIL(hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking));
            h->own_stream = true;
        }
        const size_t pop = (size_t)19 * h->stride * h->esize;
        TRY_OR_BAIL(hipMalloc(&h->buf[0], pop));
        TRY_OR_BAIL(hipMalloc(&h->buf[1], pop));
        TRY_OR_BAIL(hipMalloc((void**)&h->U, (size_t)3 * h->stride * sizeof(double)));
        TRY_OR_BAIL(hipMalloc(&h->dens, (size_t)plane * h->esize));
        TRY_OR_BAIL(hipMalloc((void**)&h->diverged, sizeof(unsigned int)));
        // rest state: g = 0 (f = r), U = 0
        TRY_OR_BAIL(hipMemsetAsync(h->buf[0], 0, pop, h->stream));
        TRY_OR_BAIL(hipMemsetAsync(h->buf[1], 0, pop, h->stream));
        TRY_OR_BAIL(hipMemsetAsync(h->U, 0, (size_t)3 * h->stride * sizeof(double), h->stream));
        TRY_OR_BAIL(hipMemsetAsync(h->diverged, 0, sizeof(unsigned int), h->stream));
        if (h->geo) {
            TRY_OR_BAIL(hipMalloc((void**)&h->flags, (size_t)plane * sizeof(uint32_t)));
            TRY_OR_BAIL(hipMalloc((void**)&h->bidx, (size_t)plane * sizeof(int32_t)));
            TRY_OR_BAIL(hipMemcpyAsync(h->flags, geo.flags.data(), (size_t)plane * sizeof(uint32_t),
                                       hipMemcpyHostToDevice, h->stream));
            TRY_OR_BAIL(hipMemcpyAsync(h->bidx, geo.bidx.data(), (size_t)plane * sizeof(int32_t),
                                       hipMemcpyHostToDevice, h->stream));
            TRY_OR_BAIL(hipMalloc((void**)&h->wrec, geo.wrec.size() * sizeof(int32_t)));
            TRY_OR_BAIL(hipMemcpyAsync(h->wrec, geo.wrec.data(), geo.wrec.size() * sizeof(int32_t),
                                       hipMemcpyHostToDevice, h->stream));
            if (!geo.recs.empty()) {
                if (h->precision == SLBM_FP32) {
                    const std::vector<Link3<float>> r = cast_links3<float>(geo.recs);
                    h->link_bytes = r.size() * sizeof(Link3<float>);
                    TRY_OR_BAIL(hipMalloc(&h->links, h->link_bytes));
                    TRY_OR_BAIL(hipMemcpyAsync(h->links, r.data(), h->link_bytes, hipMemcpyHostToDevice, h->stream));
                    TRY_OR_BAIL(hipStreamSynchronize(h->stream));
                } else {
                    h->link_bytes = geo.recs.size() * sizeof(Link3<double>);
                    TRY_OR_BAIL(hipMalloc(&h->links, h->link_bytes));
                    TRY_OR_BAIL(hipMemcpyAsync(h->links, geo.recs.data(), h->link_bytes, hipMemcpyHostToDevice,
                                               h->stream));
                }
                // (A, s_kappa) per record: the parts come from the steps, s_kappa from here
                std::vector<double> lv(2 * geo.recs.size(), 0.0);
                for (size_t r = 0; r < geo.recs.size(); ++r) lv[2 * r + 1] = geo.skap[r];
                TRY_OR_BAIL(hipMalloc(&h->lval, lv.size() * h->esize));
                if (h->precision == SLBM_FP32) {
                    const std::vector<float> lf(lv.begin(), lv.end());
                    TRY_OR_BAIL(hipMemcpyAsync(h->lval, lf.data(), lf.size() * sizeof(float), hipMemcpyHostToDevice,
                                               h->stream));
                    TRY_OR_BAIL(hipStreamSynchronize(h->stream));
                } else {
                    TRY_OR_BAIL(hipMemcpyAsync(h->lval, lv.data(), lv.size() * sizeof(double), hipMemcpyHostToDevice,
                                               h->stream));
                    TRY_OR_BAIL(hipStreamSynchronize(h->stream));
                }
                if (h->n_ext > 0) {
                    TRY_OR_BAIL(hipMalloc((void**)&h->elink, geo.elink.size() * sizeof(int32_t)));
                    TRY_OR_BAIL(hipMemcpyAsync(h->elink, geo.elink.data(), geo.elink.size() * sizeof(int32_t),
                                               hipMemcpyHostToDevice, h->stream));
                }
            }
        }
        TRY_OR_BAIL(hipStreamSynchronize(h->stream));
    #undef TRY_OR_BAIL
        *out = h;
        return SLBM_OK;
    });
}

int slbm3_destroy(slbm3_handle h)
{
    return guarded([&]() -> int {
        if (!h) return SLBM_OK;
        DeviceGuard dg(h->device);
        if (h->stream) (void)hipStreamSynchronize(h->stream);
        free3(h);
        delete h;
        return SLBM_OK;
    });
}

int slbm3_init_fields(slbm3_handle h, const double* rho, const double* vel, const double* sigma, const double* u)
{
    return guarded([&]() -> int {
        if (!h) return fail(SLBM_E_INVAL, "null handle");
        DeviceGuard dg(h->device);
        int rc = ensure_scratch3(h);
        if (rc) return rc;
        const long long n = h->plane;
        // lattice units on the host: delta-rho, j = rho v, P = -sigma - (lambda - mu) drho I, u0
        std::vector<double> in((size_t)13 * n, 0.0);
        for (long long s = 0; s < n; ++s) {
            const double r = rho ? rho[s] / h->rho_user : 1.0;
            if (!(r > 0)) return fail(SLBM_E_INVAL, "density must be positive");
            in[s] = r - 1.0;
            for (int k = 0; k < 3; ++k) {
                in[(1 + k) * n + s] = vel ? r * vel[k * n + s] / h->s_v : 0.0;
                in[(10 + k) * n + s] = u ? u[k * n + s] : 0.0;
            }
            for (int k = 0; k < 6; ++k) {
                const double sg = sigma ? sigma[k * n + s] / h->s_sigma : 0.0;
                in[(4 + k) * n + s] = -sg - (k < 3 ? (h->lamL - h->muL) * (r - 1.0) : 0.0);
            }
        }
        HIP_TRY(hipMemcpyAsync(h->scratch, in.data(), in.size() * sizeof(double), hipMemcpyHostToDevice, h->stream));
        rc = launch3_any(h, 2);
        if (rc) return rc;
        HIP_TRY(hipMemsetAsync(h->diverged, 0, sizeof(unsigned int), h->stream));
        HIP_TRY(hipStreamSynchronize(h->stream));
        h->local = true;
        h->step = 0;
        return SLBM_OK;
    });
}

int slbm3_step(slbm3_handle h, int64_t nsteps)
{
    return guarded([&]() -> int {
        if (!h) return fail(SLBM_E_INVAL, "null handle");
        if (nsteps < 0) return fail(SLBM_E_INVAL, "negative step count");
        DeviceGuard dg(h->device);
        for (int64_t k = 0; k < nsteps; ++k) {
            int rc = launch3_any(h, 0);
            if (rc) return rc;
            h->cur ^= 1;
            h->local = false;
            h->step += 1;
        }
        return SLBM_OK;
    });
}

int slbm3_sync(slbm3_handle h)
{
    return guarded([&]() -> int {
        if (!h) return fail(SLBM_E_INVAL, "null handle");
        DeviceGuard dg(h->device);
        HIP_TRY(hipStreamSynchronize(h->stream));
        unsigned int flag = 0;
        HIP_TRY(hipMemcpy(&flag, h->diverged, sizeof flag, hipMemcpyDeviceToHost));
        if (flag) return fail(SLBM_E_DIVERGED, "non-finite state (diverged)");
        return SLBM_OK;
    });
}

// Outputs of the current state (lattice units) into the device scratch
// planes, laid out as k3_outputs writes them.
static int outputs3(slbm3_handle h)
{
    int rc = ensure_scratch3(h);
    if (rc) return rc;
    return launch3_any(h, 1);
}

// Planes [first, first + count) of the output scratch into a host array (x
// fastest), then x -> (x + add) * scale (lattice to user units).
static int copy_planes3(slbm3_handle h, int first, int count, double add, double scale, double* dst)
{
    const size_t n = (size_t)count * (size_t)h->plane;
    HIP_TRY(hipMemcpyAsync(dst, h->scratch + (size_t)first * (size_t)h->plane, n * sizeof(double),
                           hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    if (add != 0.0 || scale != 1.0)
        for (size_t s = 0; s < n; ++s) dst[s] = (dst[s] + add) * scale;
    return SLBM_OK;
}

int slbm3_moments(slbm3_handle h, double* rho, double* j, double* P, double* sigma)
{
    return guarded([&]() -> int {
        if (!h) return fail(SLBM_E_INVAL, "null handle");
        DeviceGuard dg(h->device);
        int rc = outputs3(h);
        if (rc) return rc;
        if (rho && (rc = copy_planes3(h, 0, 1, 1.0, h->rho_user, rho))) return rc;
        if (j && (rc = copy_planes3(h, 1, 3, 0.0, h->rho_user * h->s_v, j))) return rc;
        if (P && (rc = copy_planes3(h, 4, 6, 0.0, h->s_sigma, P))) return rc;
        if (sigma && (rc = copy_planes3(h, 10, 6, 0.0, h->s_sigma, sigma))) return rc;
        return SLBM_OK;
    });
}

int slbm3_displacement(slbm3_handle h, double* u)
{
    return guarded([&]() -> int {
        if (!h || !u) return fail(SLBM_E_INVAL, "null argument");
        DeviceGuard dg(h->device);
        int rc = outputs3(h);
        if (rc) return rc;
        return copy_planes3(h, 16, 3, 0.0, 1.0, u);
    });
}

int slbm3_displacement_device(slbm3_handle h, void* u_dev)
{
    return guarded([&]() -> int {
        if (!h || !u_dev) return fail(SLBM_E_INVAL, "null argument");
        DeviceGuard dg(h->device);
        int rc = outputs3(h);
        if (rc) return rc;
        return device_planes3(h, 16, 3, 0.0, 1.0, u_dev, SLBM_FP64);
    });
}

int slbm3_moments_device(slbm3_handle h, void* rho, void* j, void* P, void* sigma, int dtype)
{
    return guarded([&]() -> int {
        if (!h) return fail(SLBM_E_INVAL, "null handle");
        if (dtype != SLBM_FP64 && dtype != SLBM_FP32) return fail(SLBM_E_INVAL, "dtype must be SLBM_FP64 or SLBM_FP32");
        DeviceGuard dg(h->device);
        int rc = outputs3(h);
        if (rc) return rc;
        if (rho && (rc = device_planes3(h, 0, 1, 1.0, h->rho_user, rho, dtype))) return rc;
        if (j && (rc = device_planes3(h, 1, 3, 0.0, h->rho_user * h->s_v, j, dtype))) return rc;
        if (P && (rc = device_planes3(h, 4, 6, 0.0, h->s_sigma, P, dtype))) return rc;
        if (sigma && (rc = device_planes3(h, 10, 6, 0.0, h->s_sigma, sigma, dtype))) return rc;
        return SLBM_OK;
    });
}

int slbm3_time(slbm3_handle h, int64_t* step, double* t_user)
{
    return guarded([&]() -> int {
        if (!h) return fail(SLBM_E_INVAL, "null handle");
        if (step) *step = h->step;
        if (t_user) *t_user = (double)h->step * h->dt_user;
        return SLBM_OK;
    });
}

int slbm3_device_bytes(slbm3_handle h, int64_t* bytes)
{
    return guarded([&]() -> int {
        if (!h || !bytes) return fail(SLBM_E_INVAL, "null argument");
        int64_t b = 2 * (int64_t)19 * h->stride * (int64_t)h->esize + 3 * h->stride * 8 + h->plane * (int64_t)h->esize;
        if (h->scratch) b += (int64_t)19 * h->plane * 8;
        if (h->geo) {
            const long long nwg = (((long long)(h->nx + 63) / 64) * h->ny * h->nz + 3) / 4;
            b += h->plane * 8 + (int64_t)h->link_bytes + 2 * h->n_links * (int64_t)h->esize + (nwg + 1) * 4 +
                 h->n_ext * 4;
        }
        *bytes = b;
        return SLBM_OK;
    });
}

namespace {
struct Save3Header {
    uint64_t magic;
    int32_t nx, ny, nz, precision;
    int64_t step, n_links, stride;
    int32_t local, diverged;
    uint64_t geo_hash;
};
constexpr uint64_t kMagic3 = 0x3464335f6d626c73ull;    // "slbm_3d4"

size_t save3_bytes(const slbm3_s* h)
{
    return sizeof(Save3Header) + (size_t)19 * h->stride * h->esize + (size_t)3 * h->stride * sizeof(double) +
           (size_t)2 * h->n_links * h->esize;
}
}  // namespace

int slbm3_save(slbm3_handle h, void* buf, size_t* bytes)
{
    return guarded([&]() -> int {
        if (!h || !bytes) return fail(SLBM_E_INVAL, "null argument");
        const size_t need = save3_bytes(h);
        if (!buf) { *bytes = need; return SLBM_OK; }
        if (*bytes < need) return fail(SLBM_E_INVAL, "buffer too small: %zu < %zu", *bytes, need);
        DeviceGuard dg(h->device);
        const size_t pop = (size_t)19 * h->stride * h->esize, ub = (size_t)3 * h->stride * sizeof(double);
        Save3Header hd{kMagic3, h->nx, h->ny, h->nz, h->precision, h->step, h->n_links, h->stride,
                       h->local ? 1 : 0, 0, h->geo_hash};
        unsigned int flag = 0;
        char* p = (char*)buf;
        HIP_TRY(hipMemcpyAsync(&flag, h->diverged, sizeof flag, hipMemcpyDeviceToHost, h->stream));
        HIP_TRY(hipMemcpyAsync(p + sizeof hd, h->buf[h->cur], pop, hipMemcpyDeviceToHost, h->stream));
        HIP_TRY(hipMemcpyAsync(p + sizeof hd + pop, h->U, ub, hipMemcpyDeviceToHost, h->stream));
        if (h->n_links > 0)
            HIP_TRY(hipMemcpyAsync(p + sizeof hd + pop + ub, h->lval, (size_t)2 * h->n_links * h->esize,
                                   hipMemcpyDeviceToHost, h->stream));
        HIP_TRY(hipStreamSynchronize(h->stream));
        hd.diverged = (int32_t)flag;
        std::memcpy(p, &hd, sizeof hd);
        *bytes = need;
        return SLBM_OK;
    });
}

int slbm3_load(slbm3_handle h, const void* buf, size_t bytes)
{
    return guarded([&]() -> int {
        if (!h || !buf) return fail(SLBM_E_INVAL, "null argument");
        Save3Header hd;
        if (bytes < save3_bytes(h)) return fail(SLBM_E_INVAL, "checkpoint too short");
        std::memcpy(&hd, buf, sizeof hd);
        if (hd.magic != kMagic3 || hd.nx != h->nx || hd.ny != h->ny || hd.nz != h->nz ||
            hd.precision != h->precision || hd.n_links != h->n_links || hd.stride != h->stride)
            return fail(SLBM_E_INVAL, "checkpoint does not match this box");
        if (hd.geo_hash != h->geo_hash) return fail(SLBM_E_INVAL, "checkpoint of another geometry");
        DeviceGuard dg(h->device);
        const size_t pop = (size_t)19 * h->stride * h->esize, ub = (size_t)3 * h->stride * sizeof(double);
        const char* p = (const char*)buf;
        // the other buffer, which the next step writes, keeps the rest state
        // at void sites from creation
        h->cur = 0;
        HIP_TRY(hipMemcpyAsync(h->buf[0], p + sizeof hd, pop, hipMemcpyHostToDevice, h->stream));
        HIP_TRY(hipMemcpyAsync(h->U, p + sizeof hd + pop, ub, hipMemcpyHostToDevice, h->stream));
        if (h->n_links > 0)
            HIP_TRY(hipMemcpyAsync(h->lval, p + sizeof hd + pop + ub, (size_t)2 * h->n_links * h->esize,
                                   hipMemcpyHostToDevice, h->stream));
        unsigned int flag = (unsigned int)hd.diverged;
        HIP_TRY(hipMemcpyAsync(h->diverged, &flag, sizeof flag, hipMemcpyHostToDevice, h->stream));
        HIP_TRY(hipStreamSynchronize(h->stream));
        h->step = hd.step;
        h->local = hd.local != 0;
        return SLBM_OK;
    });
}

}  // extern "C"
