// batch_api.h -- host side of the batched path (slbm_batch_* in
// include/slbm.h): many plates advanced by shared launches, continuous
// batching under an HBM budget.  Included by slbm.hip after the single-plate
// API, whose helpers it uses.
//
// Layout and ordering:
//   * every plate's device memory, and the readout scratch the plates share,
//     come from one arena of the batch's budget (no allocation or free on
//     the device while steps run);
//   * steps are queued on the compute stream; plates are created (uploads)
//     and read out on a second, side stream, a readout behind an event
//     recorded after the plate's last batched launch, so admission and
//     readout of some plates overlap the steps of the others;
//   * the per-plate descriptors and the tile map live in device tables
//     uploaded, stream-ordered, from pinned host staging when plates join or
//     leave; the step kernels advance each plate's descriptor themselves
//     (two copies, one per launch parity), so a captured graph of launches
//     replays with no bookkeeping kernels;
//   * the plates' divergence words sit in one device array; the step kernels
//     stop computing a plate whose word is set (its steps are still counted),
//     and every call that queues steps also queues a copy of the words and
//     an event, so that a later call retires every plate found diverged (its
//     countdown set to zero) and slbm_batch_wait can bound the calls in
//     flight.
#pragma once

struct slbm_batch_s {
    int device = 0;
    hipStream_t stream = nullptr;    // steps
    bool own_stream = false;
    hipStream_t side = nullptr;      // plate creation and readouts
    Arena arena;
    int precision = -1;
    std::vector<slbm_s*> slot;       // nullptr: free
    std::vector<int64_t> remaining;  // host mirror of the device countdown
    uint64_t next_id = 1;
    int wide = 0;                    // strip shape of the batched launch
    int rows = 6;                    // rows per tile for every plate
    int two = 0;                     // 1: two steps per launch (58-column strips)
    int group = 0;                   // workgroups to XCDs: 0 contiguous bands, g > 0 interleaved groups of g
    // divergence words by slot
    unsigned int* d_flags = nullptr;
    int flags_cap = 0;
    // every call that queued steps: an event behind its launches and a copy
    // of the divergence words taken then (pinned), oldest first
    struct Call {
        hipEvent_t ev = nullptr;
        unsigned int* flags = nullptr;
        int cap = 0;
        std::vector<uint64_t> ids;   // plate of each slot when the copy was queued
    };
    std::deque<Call> calls;
    std::vector<Call> spare;
    // device tables: descriptors (two copies of plates_cap), tile -> plate, first tile of each plate
    void* d_plates = nullptr;
    int plates_cap = 0;
    int* d_tile_plate = nullptr;
    int* d_tile_start = nullptr;
    int tiles_cap = 0;
    char* h_stage = nullptr;         // pinned staging of the tables
    size_t stage_cap = 0;
    hipEvent_t stage_ev = nullptr;
    std::vector<void*> retired;      // outgrown tables and flag arrays, freed with the batch
    std::vector<int> live;           // slot of each device plate entry
    int ntiles = 0;
    bool coop = false;               // every running plate has tile lists for the launch shape
    bool dirty = true;
    int parity = 0;                  // descriptor copy the next launch reads
    hipGraphExec_t graph[2] = {nullptr, nullptr};   // kChunk steps from either parity
    std::vector<std::pair<hipEvent_t, hipGraphExec_t>> dead_graphs;
    // readout scratch shared by the plates (in the arena)
    double* scratch = nullptr;
    size_t scratch_bytes = 0;
};

namespace {

constexpr int kChunk = 32;           // steps per captured graph

void batch_drop_graphs(slbm_batch_s* b)
{
    // the graphs may still be running: destroyed once an event queued behind them completes
    hipEvent_t ev = nullptr;
    for (hipGraphExec_t& g : b->graph) {
        if (!g) continue;
        if (!ev && hipEventCreateWithFlags(&ev, hipEventDisableTiming) == hipSuccess)
            (void)hipEventRecord(ev, b->stream);
        b->dead_graphs.push_back({ev, g});
        ev = nullptr;
        g = nullptr;
    }
    for (size_t i = 0; i < b->dead_graphs.size();) {
        auto& d = b->dead_graphs[i];
        if (!d.first || hipEventQuery(d.first) == hipSuccess) {
            if (d.first) (void)hipEventDestroy(d.first);
            (void)hipGraphExecDestroy(d.second);
            b->dead_graphs.erase(b->dead_graphs.begin() + i);
        } else {
            ++i;
        }
    }
}

// Grows the slot-indexed divergence words to hold n slots; existing plates
// are repointed (their words copied in stream order).
int batch_reserve_flags(slbm_batch_s* b, int n)
{
    if (n <= b->flags_cap) return SLBM_OK;
    const int cap = std::max(n, std::max(64, 2 * b->flags_cap));
    unsigned int* d = nullptr;
    HIP_TRY(hipMalloc((void**)&d, (size_t)cap * sizeof(unsigned int)));
    HIP_TRY(hipMemsetAsync(d, 0, (size_t)cap * sizeof(unsigned int), b->stream));
    if (b->d_flags) {
        HIP_TRY(hipMemcpyAsync(d, b->d_flags, (size_t)b->flags_cap * sizeof(unsigned int), hipMemcpyDeviceToDevice,
                               b->stream));
        HIP_TRY(hipStreamSynchronize(b->stream));     // rare: capacity doubles
        b->retired.push_back(b->d_flags);
    }
    b->d_flags = d;
    b->flags_cap = cap;
    for (size_t k = 0; k < b->slot.size(); ++k)
        if (b->slot[k]) b->slot[k]->diverged = d + k;
    b->dirty = true;
    return SLBM_OK;
}

// Takes finished step calls off the queue, oldest first, and retires the
// plates their copies of the divergence words found diverged; waits until at
// most `keep` calls remain (keep < 0: takes only what has finished).
void batch_harvest(slbm_batch_s* b, int keep)
{
    while (!b->calls.empty()) {
        slbm_batch_s::Call& c = b->calls.front();
        if (keep >= 0 && (int)b->calls.size() > keep)
            (void)hipEventSynchronize(c.ev);
        else if (hipEventQuery(c.ev) != hipSuccess)
            break;
        for (size_t k = 0; k < c.ids.size() && k < b->slot.size(); ++k) {
            slbm_s* h = b->slot[k];
            if (!h || h->batch_id != c.ids[k] || !c.flags[k] || b->remaining[k] <= 0) continue;
            b->remaining[k] = 0;      // halted on the device already; not stepped again
            b->dirty = true;
        }
        b->spare.push_back(std::move(c));
        b->calls.pop_front();
    }
}

// Records a step call: an event behind its launches and a copy of the
// divergence words.
int batch_record_call(slbm_batch_s* b)
{
    slbm_batch_s::Call c;
    if (!b->spare.empty()) {
        c = std::move(b->spare.back());
        b->spare.pop_back();
    } else {
        HIP_TRY(hipEventCreateWithFlags(&c.ev, hipEventDisableTiming));
    }
    const int n = (int)b->slot.size();
    if (c.cap < n) {
        if (c.flags) (void)hipHostFree(c.flags);
        c.flags = nullptr;
        c.cap = std::max(n, b->flags_cap);
        const hipError_t e = hipHostMalloc((void**)&c.flags, (size_t)c.cap * sizeof(unsigned int), hipHostMallocDefault);
        if (e != hipSuccess) {
            c.cap = 0;
            b->spare.push_back(std::move(c));
            return fail(SLBM_E_DEVICE, "pinned buffer: %s", hipGetErrorString(e));
        }
    }
    c.ids.assign(n, 0);
    for (int k = 0; k < n; ++k)
        if (b->slot[k]) c.ids[k] = b->slot[k]->batch_id;
    if (n > 0) HIP_TRY(hipMemcpyAsync(c.flags, b->d_flags, (size_t)n * sizeof(unsigned int), hipMemcpyDeviceToHost,
                                      b->stream));
    HIP_TRY(hipEventRecord(c.ev, b->stream));
    b->calls.push_back(std::move(c));
    return SLBM_OK;
}

// Device tables of the plates still running, uploaded in stream order on
// the compute stream (queued launches keep reading the old contents until
// the copy runs).  Plates that are done get no tiles.
template <typename real>
int batch_build(slbm_batch_s* b)
{
    batch_drop_graphs(b);
    b->live.clear();
    bool all_lists = b->two != 0;
    std::vector<BatchPlate<real>> bp;
    std::vector<int> tile_plate, tile_start;
    for (size_t k = 0; k < b->slot.size(); ++k) {
        slbm_s* h = b->slot[k];
        if (!h || b->remaining[k] <= 0) continue;
        const int keep_seg = h->seg, keep_w = h->wide;
        h->seg = b->rows;
        h->wide = b->wide;
        BatchPlate<real> e{};
        e.args = b->two ? make_args2<real>(h, h->cur, b->rows) : make_args<real>(h, h->cur);
        h->seg = keep_seg;
        h->wide = keep_w;
        e.remaining = b->remaining[k];
        e.active = 1;
        if (!e.args.rec_start) all_lists = false;
        const int p = (int)bp.size();
        tile_start.push_back((int)tile_plate.size());
        for (int t = 0; t < e.args.ntiles; ++t) tile_plate.push_back(p);
        bp.push_back(e);
        b->live.push_back((int)k);
    }
    b->ntiles = (int)tile_plate.size();
    b->coop = all_lists;
    b->dirty = false;
    b->parity = 0;
    if (bp.empty()) return SLBM_OK;
    const int np = (int)bp.size();
    if (np > b->plates_cap || b->ntiles > b->tiles_cap) {
        // capacity with headroom; outgrown tables stay allocated (queued
        // launches may still read them) until the batch is destroyed
        if (b->d_plates) b->retired.push_back(b->d_plates);
        if (b->d_tile_plate) b->retired.push_back(b->d_tile_plate);
        if (b->d_tile_start) b->retired.push_back(b->d_tile_start);
        b->plates_cap = std::max(np, std::max(64, 2 * b->plates_cap));
        b->tiles_cap = std::max(b->ntiles, std::max(1 << 16, 2 * b->tiles_cap));
        HIP_TRY(hipMalloc(&b->d_plates, (size_t)2 * b->plates_cap * sizeof(BatchPlate<real>)));
        HIP_TRY(hipMalloc((void**)&b->d_tile_plate, (size_t)b->tiles_cap * sizeof(int)));
        HIP_TRY(hipMalloc((void**)&b->d_tile_start, (size_t)b->plates_cap * sizeof(int)));
    }
    const size_t pb = (size_t)np * sizeof(BatchPlate<real>), tb = tile_plate.size() * sizeof(int),
                 sb = tile_start.size() * sizeof(int);
    const size_t need = pb + tb + sb;
    // the staging may still feed the previous upload
    if (b->h_stage) HIP_TRY(hipEventSynchronize(b->stage_ev));
    if (need > b->stage_cap) {
        if (b->h_stage) (void)hipHostFree(b->h_stage);
        b->stage_cap = std::max(need, 2 * b->stage_cap);
        HIP_TRY(hipHostMalloc((void**)&b->h_stage, b->stage_cap, hipHostMallocDefault));
    }
    std::memcpy(b->h_stage, bp.data(), pb);
    std::memcpy(b->h_stage + pb, tile_plate.data(), tb);
    std::memcpy(b->h_stage + pb + tb, tile_start.data(), sb);
    HIP_TRY(hipMemcpyAsync(b->d_plates, b->h_stage, pb, hipMemcpyHostToDevice, b->stream));
    HIP_TRY(hipMemcpyAsync(b->d_tile_plate, b->h_stage + pb, tb, hipMemcpyHostToDevice, b->stream));
    HIP_TRY(hipMemcpyAsync(b->d_tile_start, b->h_stage + pb + tb, sb, hipMemcpyHostToDevice, b->stream));
    HIP_TRY(hipEventRecord(b->stage_ev, b->stream));
    return SLBM_OK;
}

int batch_grid(const slbm_batch_s* b)
{
    // one workgroup per tile: the batched kernels assume at least ntiles
    // workgroups, a whole number of XCD rounds (8 workgroups, or 8 groups)
    const int unit = 8 << std::max(0, group_shift(b->group));
    return (b->ntiles + unit - 1) / unit * unit;
}

// Queues one batched launch of up to maxk steps (2 only in two-step mode)
// reading descriptor copy `parity`.
template <typename real>
void batch_launch(slbm_batch_s* b, int parity, int maxk)
{
    const int grid = batch_grid(b);
    BatchPlate<real>* plates = (BatchPlate<real>*)b->d_plates;
    const int cap = b->plates_cap;
    if (b->two) {
        const dim3 blk(64 * (b->rows + 6));
        constexpr int lo = k2_waves<real>(1), hi = k2_waves<real>(kMaxTileRows2);
        const int gs = group_shift(b->group);
        if (k2_waves<real>(b->rows) == hi) {
            if (b->coop)
                hipLaunchKernelGGL((k_step2_batch<real, hi, true>), dim3(grid), blk, 0, b->stream, plates, cap, parity,
                                   b->d_tile_plate, b->d_tile_start, b->ntiles, maxk, gs);
            else
                hipLaunchKernelGGL((k_step2_batch<real, hi, false>), dim3(grid), blk, 0, b->stream, plates, cap,
                                   parity, b->d_tile_plate, b->d_tile_start, b->ntiles, maxk, gs);
        } else {
            if (b->coop)
                hipLaunchKernelGGL((k_step2_batch<real, lo, true>), dim3(grid), blk, 0, b->stream, plates, cap, parity,
                                   b->d_tile_plate, b->d_tile_start, b->ntiles, maxk, gs);
            else
                hipLaunchKernelGGL((k_step2_batch<real, lo, false>), dim3(grid), blk, 0, b->stream, plates, cap,
                                   parity, b->d_tile_plate, b->d_tile_start, b->ntiles, maxk, gs);
        }
    } else {
        const dim3 blk(64 * (b->wide ? tile_waves<true>(b->rows) : tile_waves<false>(b->rows)));
        if (b->wide)
            hipLaunchKernelGGL((k_step_batch<real, true>), dim3(grid), blk, 0, b->stream, plates, cap, parity,
                               b->d_tile_plate, b->d_tile_start, b->ntiles, group_shift(b->group));
        else
            hipLaunchKernelGGL((k_step_batch<real, false>), dim3(grid), blk, 0, b->stream, plates, cap, parity,
                               b->d_tile_plate, b->d_tile_start, b->ntiles, group_shift(b->group));
    }
}

template <typename real>
int batch_run(slbm_batch_s* b, int64_t k)
{
    batch_harvest(b, -1);
    if (b->dirty) {
        int rc = batch_build<real>(b);
        if (rc) return rc;
    }
    if (b->ntiles == 0 || k <= 0) return SLBM_OK;
    // launches of up to `per` steps; in two-step mode an odd step count ends
    // with a launch of one step.  Each launch flips the descriptor copy.
    const int per = b->two ? 2 : 1;
    int64_t left = k / per;                       // launches of `per` steps
    const int64_t chunk = kChunk / per;           // launches per captured graph (an even number)
    while (left >= chunk) {
        hipGraphExec_t& g = b->graph[b->parity];
        if (!g) {
            hipGraph_t gr = nullptr;
            HIP_TRY(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
            for (int64_t i = 0; i < chunk; ++i) batch_launch<real>(b, (int)((b->parity + i) & 1), per);
            hipError_t e = hipStreamEndCapture(b->stream, &gr);
            if (e != hipSuccess) return fail(SLBM_E_DEVICE, "graph capture failed: %s", hipGetErrorString(e));
            e = hipGraphInstantiate(&g, gr, nullptr, nullptr, 0);
            (void)hipGraphDestroy(gr);
            if (e != hipSuccess) {
                g = nullptr;
                return fail(SLBM_E_DEVICE, "graph instantiation failed: %s", hipGetErrorString(e));
            }
        }
        HIP_TRY(hipGraphLaunch(g, b->stream));
        left -= chunk;
    }
    for (int64_t i = 0; i < left; ++i) {
        batch_launch<real>(b, b->parity, per);
        b->parity ^= 1;
    }
    const bool odd = b->two && (k & 1);
    if (odd) {
        batch_launch<real>(b, b->parity, 1);
        b->parity ^= 1;
    }
    HIP_TRY(hipGetLastError());
    // host mirror of what the kernels do to the descriptors: each launch in
    // which a plate is active swaps its buffers once and takes min(steps of
    // the launch, remaining); readouts of the plate wait for these launches
    const int64_t full = k / per;
    for (int k2 : b->live) {
        slbm_s* h = b->slot[k2];
        const int64_t rem = b->remaining[k2];
        if (!h || rem <= 0) continue;
        int64_t launches = std::min(full, (rem + per - 1) / per);
        int64_t done = std::min(rem, full * per);
        if (odd && done < rem) {
            launches += 1;
            done += 1;
        }
        h->cur ^= (int)(launches & 1);
        h->step += done;
        h->local = false;
        b->remaining[k2] -= done;
        HIP_TRY(hipEventRecord(h->ready, b->stream));
    }
    return batch_record_call(b);
}

int batch_run_any(slbm_batch_s* b, int64_t k)
{
    if (b->precision < 0) return SLBM_OK;
    return b->precision == SLBM_FP32 ? batch_run<float>(b, k) : batch_run<double>(b, k);
}

hipStream_t batch_compute_stream(slbm_batch_s* b) { return b->stream; }

// Tile lists of every plate for the batch's launch shape (two steps per
// launch only; a plate without room for its lists in the budget goes
// without, and the batch then takes the boundary rules site by site).
int batch_lists(slbm_batch_s* b)
{
    if (!b->two) return SLBM_OK;
    for (slbm_s* h : b->slot) {
        if (!h) continue;
        const int rc = tile_records(h, b->rows);
        if (rc) return rc;
    }
    return SLBM_OK;
}

// Bytes of the readout scratch a plate needs (its padded planes, fp64).
size_t scratch_need(const slbm_s* h, int planes) { return (size_t)planes * h->plane * sizeof(double); }

// Grows the batch's shared readout scratch (in the arena) to `bytes`.
int batch_grow_scratch(slbm_batch_s* b, size_t bytes)
{
    if (bytes <= b->scratch_bytes) return SLBM_OK;
    void* p = b->arena.alloc(bytes);
    if (!p) return fail(SLBM_E_BUDGET, "readout scratch of %zu bytes does not fit the batch's budget", bytes);
    if (b->scratch) {
        // earlier readouts on the side stream may still use the old block
        hipEvent_t ev = nullptr;
        HIP_TRY(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        HIP_TRY(hipEventRecord(ev, b->side));
        b->arena.release_after({ev}, {b->scratch});
    }
    b->scratch = (double*)p;
    b->scratch_bytes = bytes;
    return SLBM_OK;
}

// Readouts of a batch plate share the batch's scratch (declared with the
// single-plate readouts above).
int batch_scratch(slbm_s* h, int planes)
{
    int rc = batch_grow_scratch(h->batch, scratch_need(h, planes));
    if (rc) return rc;
    h->scratch = h->batch->scratch;
    h->scratch_planes = planes;
    return SLBM_OK;
}

// Queues the release of a plate's memory behind the work already queued on
// both streams, and frees its host state.
int batch_drop_plate(slbm_batch_s* b, int slot)
{
    slbm_s* h = b->slot[slot];
    hipEvent_t ec = nullptr, es = nullptr;
    HIP_TRY(hipEventCreateWithFlags(&ec, hipEventDisableTiming));
    HIP_TRY(hipEventCreateWithFlags(&es, hipEventDisableTiming));
    HIP_TRY(hipEventRecord(ec, b->stream));
    HIP_TRY(hipEventRecord(es, b->side));
    std::vector<hipEvent_t> destroy;
    if (h->ready) destroy.push_back(h->ready);
    h->ready = nullptr;
    b->arena.release_after({ec, es}, plate_blocks(h), destroy);
    h->arena = nullptr;
    h->batch = nullptr;
    delete h;
    b->slot[slot] = nullptr;
    b->remaining[slot] = 0;
    b->dirty = true;
    if (b->scratch && std::none_of(b->slot.begin(), b->slot.end(), [](slbm_s* q) { return q != nullptr; })) {
        // an empty batch holds nothing in its budget
        hipEvent_t ev = nullptr;
        HIP_TRY(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        HIP_TRY(hipEventRecord(ev, b->side));
        b->arena.release_after({ev}, {b->scratch});
        b->scratch = nullptr;
        b->scratch_bytes = 0;
    }
    return SLBM_OK;
}

}  // namespace

extern "C" {

int slbm_batch_create(int64_t hbm_budget_bytes, int32_t device, void* stream, slbm_batch* out)
{
    return guarded([&]() -> int {
        if (!out) return fail(SLBM_E_INVAL, "null argument");
        *out = nullptr;
        if (hbm_budget_bytes <= 0) return fail(SLBM_E_INVAL, "budget must be positive");
        int n = 0;
        if (hipGetDeviceCount(&n) != hipSuccess || n < 1) return fail(SLBM_E_DEVICE, "no HIP device");
        if (device < 0 || device >= n) return fail(SLBM_E_INVAL, "device %d out of range", device);
        slbm_batch_s* b = new (std::nothrow) slbm_batch_s();
        if (!b) return fail(SLBM_E_NOMEM, "out of host memory");
        b->device = device;
        DeviceGuard dg(device);
        auto bail = [&](int rc) {
            if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
            if (b->side) (void)hipStreamDestroy(b->side);
            if (b->stage_ev) (void)hipEventDestroy(b->stage_ev);
            b->arena.destroy_all();
            delete b;
            return rc;
        };
        hipError_t e = hipSuccess;
        if (stream) {
            b->stream = (hipStream_t)stream;
        } else {
            e = hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking);
            if (e != hipSuccess) return bail(fail(SLBM_E_DEVICE, "stream: %s", hipGetErrorString(e)));
            b->own_stream = true;
        }
        if ((e = hipStreamCreateWithFlags(&b->side, hipStreamNonBlocking)) != hipSuccess ||
            (e = hipEventCreateWithFlags(&b->stage_ev, hipEventDisableTiming)) != hipSuccess)
            return bail(fail(SLBM_E_DEVICE, "stream or event: %s", hipGetErrorString(e)));
        e = b->arena.init((size_t)hbm_budget_bytes);
        if (e != hipSuccess)
            return bail(fail(e == hipErrorOutOfMemory ? SLBM_E_NOMEM : SLBM_E_DEVICE,
                             "budget of %lld bytes could not be reserved: %s", (long long)hbm_budget_bytes,
                             hipGetErrorString(e)));
        if (int rc = batch_reserve_flags(b, 64)) return bail(rc);
        *out = b;
        return SLBM_OK;
    });
}

int slbm_batch_add(slbm_batch b, const slbm_params* params, int64_t nsteps, int32_t* slot)
{
    return guarded([&]() -> int {
        if (!b || !params || !slot) return fail(SLBM_E_INVAL, "null argument");
        if (nsteps < 0) return fail(SLBM_E_INVAL, "negative step count");
        if (params->periodic_x || params->periodic_y) return fail(SLBM_E_UNSUPPORTED, "periodic plates are not batched");
        if (b->precision >= 0 && params->precision != b->precision)
            return fail(SLBM_E_INVAL, "every plate of a batch has the batch's precision");
        DeviceGuard dg(b->device);
        int k = -1;
        for (size_t i = 0; i < b->slot.size(); ++i)
            if (!b->slot[i]) { k = (int)i; break; }
        if (k < 0) k = (int)b->slot.size();
        if (int rc = batch_reserve_flags(b, k + 1)) return rc;
        slbm_params p = *params;
        p.device = b->device;
        p.stream = b->side;
        slbm_handle h = nullptr;
        int rc = create_impl(&p, &h, &b->arena, b->d_flags + k);
        if (rc == SLBM_E_NOMEM)
            return fail(SLBM_E_BUDGET, "the plate does not fit the batch's budget (%lld of %lld bytes in use)",
                        (long long)b->arena.live(), (long long)b->arena.size);
        if (rc) return rc;
        h->batch = b;
        h->batch_id = b->next_id++;
        // the displacement readout's scratch must fit the budget as well
        rc = batch_grow_scratch(b, scratch_need(h, 3));
        if (rc) {
            h->batch = nullptr;
            free_all(h);
            delete h;
            return rc;
        }
        const hipError_t e = hipEventCreateWithFlags(&h->ready, hipEventDisableTiming);
        if (e != hipSuccess) {
            h->batch = nullptr;
            free_all(h);
            delete h;
            return fail(SLBM_E_DEVICE, "event: %s", hipGetErrorString(e));
        }
        if (b->two && (rc = tile_records(h, b->rows))) {
            h->batch = nullptr;
            free_all(h);
            delete h;
            return rc;
        }
        b->precision = params->precision;
        if (k == (int)b->slot.size()) {
            b->slot.push_back(nullptr);
            b->remaining.push_back(0);
        }
        b->slot[k] = h;
        b->remaining[k] = nsteps;
        b->dirty = true;
        *slot = k;
        return SLBM_OK;
    });
}

int slbm_batch_step(slbm_batch b, int64_t k)
{
    return guarded([&]() -> int {
        if (!b) return fail(SLBM_E_INVAL, "null batch");
        if (k < 0) return fail(SLBM_E_INVAL, "negative step count");
        DeviceGuard dg(b->device);
        return batch_run_any(b, k);
    });
}

int slbm_batch_poll(slbm_batch b, int32_t* done_slots, int32_t capacity, int32_t* n_done)
{
    return guarded([&]() -> int {
        if (!b || !n_done) return fail(SLBM_E_INVAL, "null argument");
        batch_harvest(b, -1);
        int n = 0;
        for (size_t k = 0; k < b->slot.size(); ++k) {
            if (!b->slot[k] || b->remaining[k] > 0) continue;
            if (done_slots && n < capacity) done_slots[n] = (int32_t)k;
            ++n;
        }
        *n_done = n;
        return SLBM_OK;
    });
}

int slbm_batch_handle(slbm_batch b, int32_t slot, slbm_handle* h)
{
    return guarded([&]() -> int {
        if (!b || !h) return fail(SLBM_E_INVAL, "null argument");
        if (slot < 0 || slot >= (int)b->slot.size() || !b->slot[slot]) return fail(SLBM_E_INVAL, "no plate in slot %d", slot);
        *h = b->slot[slot];
        return SLBM_OK;
    });
}

int slbm_batch_displacement(slbm_batch b, int32_t slot, double* u)
{
    return guarded([&]() -> int {
        if (!b || !u) return fail(SLBM_E_INVAL, "null argument");
        if (slot < 0 || slot >= (int)b->slot.size() || !b->slot[slot]) return fail(SLBM_E_INVAL, "no plate in slot %d", slot);
        return slbm_displacement(b->slot[slot], u);
    });
}

int slbm_batch_remaining(slbm_batch b, int32_t slot, int64_t* steps)
{
    return guarded([&]() -> int {
        if (!b || !steps) return fail(SLBM_E_INVAL, "null argument");
        if (slot < 0 || slot >= (int)b->slot.size() || !b->slot[slot]) return fail(SLBM_E_INVAL, "no plate in slot %d", slot);
        *steps = b->remaining[slot];
        return SLBM_OK;
    });
}

int slbm_batch_remove(slbm_batch b, int32_t slot)
{
    return guarded([&]() -> int {
        if (!b) return fail(SLBM_E_INVAL, "null batch");
        if (slot < 0 || slot >= (int)b->slot.size() || !b->slot[slot]) return fail(SLBM_E_INVAL, "no plate in slot %d", slot);
        DeviceGuard dg(b->device);
        return batch_drop_plate(b, slot);
    });
}

int slbm_batch_set_launch(slbm_batch b, int32_t rows, int32_t strip)
{
    return guarded([&]() -> int {
        if (!b) return fail(SLBM_E_INVAL, "null batch");
        if (strip != 62 && strip != 64 && strip != kStrip2) return fail(SLBM_E_INVAL, "strip must be 58, 62 or 64");
        if (rows < 1 || rows > (strip == kStrip2 ? kMaxTileRows2 : kMaxTileRows))
            return fail(SLBM_E_INVAL, "rows per tile must be in [1, 14] ([1, 10] with strip 58)");
        DeviceGuard dg(b->device);
        b->rows = rows;
        b->wide = strip == 64 ? 1 : 0;
        b->two = strip == kStrip2 ? 1 : 0;
        b->dirty = true;
        return batch_lists(b);
    });
}

int slbm_batch_set_xcd_group(slbm_batch b, int32_t group)
{
    return guarded([&]() -> int {
        if (!b) return fail(SLBM_E_INVAL, "null batch");
        if (!valid_group(group)) return fail(SLBM_E_INVAL, "xcd group must be 0 (bands) or a power of two up to 64");
        b->group = group;
        b->dirty = true;
        return SLBM_OK;
    });
}

int slbm_batch_get_launch(slbm_batch b, int32_t* rows, int32_t* strip, int32_t* xcd_group)
{
    return guarded([&]() -> int {
        if (!b) return fail(SLBM_E_INVAL, "null batch");
        if (rows) *rows = b->rows;
        if (strip) *strip = b->two ? kStrip2 : (b->wide ? 64 : 62);
        if (xcd_group) *xcd_group = b->group;
        return SLBM_OK;
    });
}

int slbm_batch_autotune(slbm_batch b, int64_t max_steps, int32_t* rows_out, int32_t* strip_out, int32_t* group_out,
                        double* us_out)
{
    return guarded([&]() -> int {
        if (!b) return fail(SLBM_E_INVAL, "null batch");
        if (max_steps < 0) return fail(SLBM_E_INVAL, "negative step budget");
        DeviceGuard dg(b->device);
        // every trial takes real steps: results do not depend on the launch
        // shape, so the plates simply advance (each by at most its remaining
        // steps) while the shapes are timed
        struct Shape { int rows, strip, group; };
        const Shape cand[] = {{6, 58, 0}, {10, 58, 0}, {4, 58, 0}, {8, 58, 0}, {6, 62, 0}, {10, 62, 0}, {14, 62, 0}};
        const int64_t per_trial = 2 * kChunk;         // a chunk to rebuild and capture, a chunk timed
        hipEvent_t e0, e1;
        HIP_TRY(hipEventCreate(&e0));
        HIP_TRY(hipEventCreate(&e1));
        int64_t spent = 0;
        Shape best{b->rows, b->two ? kStrip2 : (b->wide ? 64 : 62), b->group};
        double best_us = 0;
        // shapes are compared by time per material-site update of the plates
        // running in the timed chunk: plates retired during the trials
        // (diverged, or done) would otherwise favour the later candidates
        auto trial = [&](const Shape& s, double& us, double& per_site) -> int {
            b->rows = s.rows;
            b->two = s.strip == kStrip2 ? 1 : 0;
            b->wide = s.strip == 64 ? 1 : 0;
            b->group = s.group;
            b->dirty = true;
            int rc = batch_lists(b);
            if (rc) return rc;
            if ((rc = batch_run_any(b, kChunk))) return rc;
            batch_harvest(b, 0);
            double sites = 0;
            for (size_t k = 0; k < b->slot.size(); ++k)
                if (b->slot[k] && b->remaining[k] >= kChunk) sites += (double)b->slot[k]->n_material;
            HIP_TRY(hipEventRecord(e0, b->stream));
            if ((rc = batch_run_any(b, kChunk))) return rc;
            HIP_TRY(hipEventRecord(e1, b->stream));
            HIP_TRY(hipEventSynchronize(e1));
            float ms = 0;
            HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
            spent += per_trial;
            us = 1e3 * ms / kChunk;
            per_site = sites > 0 ? us / sites : us;
            return SLBM_OK;
        };
        auto running = [&]() {
            for (size_t k = 0; k < b->slot.size(); ++k)
                if (b->slot[k] && b->remaining[k] > 0) return true;
            return false;
        };
        int rc = SLBM_OK;
        bool any = false;
        double best_site = 0;
        for (const Shape& s : cand) {
            if (spent + per_trial > max_steps || !running()) break;
            double us = 0, site = 0;
            if ((rc = trial(s, us, site))) break;
            if (!any || site < best_site) { best = s; best_us = us; best_site = site; any = true; }
        }
        // the best shape with interleaved XCD groups of 8, kept when at least 1 % faster
        if (!rc && any && spent + per_trial <= max_steps && running()) {
            double us = 0, site = 0;
            Shape g = best;
            g.group = 8;
            if (!(rc = trial(g, us, site)) && site < 0.99 * best_site) {
                best = g;
                best_us = us;
            }
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        if (rc) return rc;
        b->rows = best.rows;
        b->two = best.strip == kStrip2 ? 1 : 0;
        b->wide = best.strip == 64 ? 1 : 0;
        b->group = best.group;
        b->dirty = true;
        if ((rc = batch_lists(b))) return rc;
        if (rows_out) *rows_out = best.rows;
        if (strip_out) *strip_out = best.strip;
        if (group_out) *group_out = best.group;
        if (us_out) *us_out = any ? best_us : 0.0;
        return SLBM_OK;
    });
}

int slbm_batch_sync(slbm_batch b)
{
    return guarded([&]() -> int {
        if (!b) return fail(SLBM_E_INVAL, "null batch");
        DeviceGuard dg(b->device);
        HIP_TRY(hipStreamSynchronize(b->stream));
        HIP_TRY(hipStreamSynchronize(b->side));
        batch_harvest(b, 0);
        b->arena.reclaim(false);
        return SLBM_OK;
    });
}

int slbm_batch_wait(slbm_batch b, int32_t in_flight)
{
    return guarded([&]() -> int {
        if (!b) return fail(SLBM_E_INVAL, "null batch");
        if (in_flight < 0) return fail(SLBM_E_INVAL, "in_flight must be >= 0");
        DeviceGuard dg(b->device);
        batch_harvest(b, in_flight);
        return SLBM_OK;
    });
}

int slbm_batch_bytes(slbm_batch b, int64_t* used, int64_t* budget)
{
    return guarded([&]() -> int {
        if (!b) return fail(SLBM_E_INVAL, "null batch");
        b->arena.reclaim(false);
        if (used) *used = (int64_t)b->arena.live();
        if (budget) *budget = (int64_t)b->arena.size;
        return SLBM_OK;
    });
}

int slbm_batch_destroy(slbm_batch b)
{
    return guarded([&]() -> int {
        if (!b) return SLBM_OK;
        DeviceGuard dg(b->device);
        (void)hipStreamSynchronize(b->stream);
        (void)hipStreamSynchronize(b->side);
        for (slbm_s*& h : b->slot) {
            if (!h) continue;
            h->batch = nullptr;
            free_all(h);
            delete h;
            h = nullptr;
        }
        for (hipGraphExec_t g : b->graph)
            if (g) (void)hipGraphExecDestroy(g);
        for (auto& d : b->dead_graphs) {
            if (d.first) (void)hipEventDestroy(d.first);
            (void)hipGraphExecDestroy(d.second);
        }
        for (void* p : b->retired) (void)hipFree(p);
        if (b->d_plates) (void)hipFree(b->d_plates);
        if (b->d_tile_plate) (void)hipFree(b->d_tile_plate);
        if (b->d_tile_start) (void)hipFree(b->d_tile_start);
        if (b->d_flags) (void)hipFree(b->d_flags);
        for (auto& c : b->calls) {
            if (c.ev) (void)hipEventDestroy(c.ev);
            if (c.flags) (void)hipHostFree(c.flags);
        }
        for (auto& c : b->spare) {
            if (c.ev) (void)hipEventDestroy(c.ev);
            if (c.flags) (void)hipHostFree(c.flags);
        }
        if (b->h_stage) (void)hipHostFree(b->h_stage);
        if (b->stage_ev) (void)hipEventDestroy(b->stage_ev);
        b->arena.destroy_all();
        if (b->side) (void)hipStreamDestroy(b->side);
        if (b->own_stream) (void)hipStreamDestroy(b->stream);
        delete b;
        return SLBM_OK;
    });
}

}  // extern "C"
