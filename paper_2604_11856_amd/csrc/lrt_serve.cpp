// Serving loop of liblrt: continuous batching of line-of-sight requests.
//
// Clients submit requests (cell states along a line of sight and a spectral
// window on the resident grid); one scheduler thread owns every HIP call:
//   - admission: FIFO with skip-ahead, by free slot and by HBM budget (one
//     arena allocated at start, first-fit, so nothing is allocated or freed
//     on the device while kernels run); admitted requests get their cell data
//     uploaded and their per-cell constants, candidate ranges and scales
//     computed on the admission stream (the scale from the binned bound of
//     the line peaks, over the bins whose lines can reach the window);
//   - epochs: items (request, tile, cell chunk) of every admitted request are
//     handed out round-robin into bounded epochs, each one launch of the
//     serving kernel (one workgroup per item) on one of two epoch streams, so
//     new work joins while earlier epochs run, and workgroups retire all
//     through an epoch, leaving slots for the admission kernels and copies;
//   - completion: the workgroup that finishes a tile's last chunk composes
//     the tile, the one that finishes the last tile writes the integral into
//     the request's slot of pinned host memory; once every item of a request
//     is done the scheduler reads it (and optionally copies the spectrum back)
//     and releases the slot and memory.
// A request's decomposition depends only on the request itself, so its result
// is bitwise the same alone and in a mix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "lrt_ctx.h"
#include "lrt_internal.h"

using namespace lrt;

namespace {

using Clock = std::chrono::steady_clock;

constexpr size_t kAlign = 256;
constexpr int kEpochStreams = 2;
constexpr int32_t kChunkCells = 32;
constexpr int kEpochCap = 32768;            // items per epoch at most
constexpr int64_t kEpochUnits = 512ll << 20; // cell x point units per epoch (target)
constexpr int kItemsPerTurn = 64;          // round-robin share per request

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// First-fit allocator over one device block.
struct Arena {
    char *base = nullptr;
    size_t size = 0, used = 0;
    std::map<size_t, size_t> free_;   // offset -> length
    bool alloc(size_t bytes, size_t &off)
    {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                off = it->first;
                const size_t rest = it->second - bytes;
                free_.erase(it);
                if (rest) free_[off + bytes] = rest;
                used += bytes;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes)
    {
        used -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
};

enum State { ST_PENDING, ST_ADMITTED, ST_DONE };

struct Req {
    uint64_t ticket = 0;
    State state = ST_PENDING;
    lrt_status status = LRT_OK;
    std::string err;
    // inputs (host copies)
    int64_t n_cells = 0;
    std::vector<double> T_tr, T_v, N, n_e, ds;
    std::vector<char> packed;   // the five arrays in their arena layout, one upload
    int32_t k_first = 0, n_window = 0;
    uint64_t mask = 0;
    bool keep = false;
    double T_far = 0.0;   // solid far boundary (0: free)
    int scheme = 0;       // LRT_MARCH_CELL or LRT_MARCH_LINEAR_J
    // layout
    int32_t n_tiles = 0, n_chunks = 0;
    size_t bytes = 0, off = 0;
    int slot = -1;
    int64_t items_total = 0, items_issued = 0, items_done = 0;
    hipEvent_t prep_ev = nullptr;
    ServeReq dev{};
    // timing and results
    Clock::time_point t_submit, t_admit, t_done;
    double I_int = 0.0;
    std::vector<double> spectrum;
};

struct Epoch {
    bool busy = false;
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    ServeItem *h_items = nullptr;   // pinned
    DBuf d_items;
    std::vector<std::pair<uint64_t, int64_t>> credit;   // ticket -> items
};

// Device bytes of one request (inputs, per-cell constants, ranges, chunk
// transmittance / source, outputs), each sub-buffer 256-byte aligned.
size_t request_bytes(int64_t nc, int S, int32_t n_window, int32_t n_thr, int32_t cr_row, int32_t &n_tiles,
                     int32_t &n_chunks)
{
    n_tiles = (n_window + kTilePoints - 1) / kTilePoints;
    n_chunks = (int32_t)((nc + kChunkCells - 1) / kChunkCells);
    const size_t nb = (size_t)(n_window + 255) / 256;
    size_t b = 0;
    b += 4 * align_up(nc * 8);                              // T_tr, T_v, n_e, ds
    b += align_up((size_t)nc * S * 8);                      // N
    b += align_up(nc * sizeof(CellConst));
    b += align_up((size_t)nc * S * sizeof(CellSpecies));
    b += align_up(nc * 2 * sizeof(int32_t));                // escale
    b += align_up((size_t)nc * n_tiles * sizeof(int2));     // ranges
    b += align_up((size_t)n_tiles * n_chunks * 2 * kTilePoints * 8);   // T, S
    b += align_up((size_t)n_window * 8);                    // I
    b += align_up((size_t)(n_tiles + 1) * 4);               // done counters
    b += align_up((size_t)n_tiles * 8) + align_up(8);       // tile sums, I_int
    if (n_thr >= 0)                                         // continuum: cum, ff, lnb
        b += align_up((size_t)nc * 2 * (n_thr + 1) * 8) + 2 * align_up((size_t)nc * 2 * 8);
    if (cr_row > 0)                                         // QSS-CR: populations, departures
        b += 2 * align_up((size_t)nc * cr_row * 8);
    return b;
}

double ms_between(Clock::time_point a, Clock::time_point b)
{
    return std::chrono::duration<double, std::milli>(b - a).count();
}

}  // namespace

struct lrt_server {
    lrt_ctx *ctx = nullptr;
    size_t budget = 0;
    int max_slots = 0;
    Arena arena;
    DBuf d_arena, d_reqs;
    std::vector<int> free_slots;
    hipStream_t admit_stream = nullptr;
    double *h_I_int = nullptr;   // pinned, one per slot: the integral written by the serving kernel
    Epoch epochs[kEpochStreams];

    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::thread th;
    bool stopping = false;
    std::string fatal;
    uint64_t next_ticket = 1;
    std::map<uint64_t, std::unique_ptr<Req>> reqs;
    std::deque<uint64_t> pending;
    std::vector<uint64_t> admitted;
    size_t rr = 0;
    int64_t n_completed = 0, n_epochs = 0;

    void run();
    bool admit(Req &r);
    bool launch_epoch(Epoch &e);
    void fail_request(Req &r, lrt_status s, const std::string &msg);
    void release(Req &r);
};

void lrt_server::fail_request(Req &r, lrt_status s, const std::string &msg)
{
    r.status = s;
    r.err = msg;
    r.state = ST_DONE;
    r.t_done = Clock::now();
    cv_done.notify_all();
}

void lrt_server::release(Req &r)
{
    if (r.slot >= 0) {
        free_slots.push_back(r.slot);
        r.slot = -1;
    }
    if (r.bytes) {
        arena.release(r.off, r.bytes);
        r.bytes = 0;
    }
    if (r.prep_ev) (void)hipEventDestroy(r.prep_ev);
    r.prep_ev = nullptr;
}

bool lrt_server::admit(Req &r)
{
    const int S = ctx->n_species;
    const int32_t n_thr = ctx->n_cont_rec > 0 ? ctx->n_cont_thr : -1;
    const int32_t cr_row = ctx->n_cr > 0 ? ctx->n_cr * ctx->cr_LS : 0;
    const size_t bytes = request_bytes(r.n_cells, S, r.n_window, n_thr, cr_row, r.n_tiles, r.n_chunks);
    if (free_slots.empty()) return false;
    size_t off;
    if (!arena.alloc(bytes, off)) return false;
    r.off = off;
    r.bytes = bytes;
    r.slot = free_slots.back();
    free_slots.pop_back();
    r.t_admit = Clock::now();
    const int64_t nc = r.n_cells;
    char *p = arena.base + off;
    auto take = [&](size_t b) {
        char *q = p;
        p += align_up(b);
        return (void *)q;
    };
    double *T_tr = (double *)take(nc * 8), *T_v = (double *)take(nc * 8);
    double *n_e = (double *)take(nc * 8), *ds = (double *)take(nc * 8);
    double *N = (double *)take((size_t)nc * S * 8);
    CellConst *cc = (CellConst *)take(nc * sizeof(CellConst));
    CellSpecies *cs = (CellSpecies *)take((size_t)nc * S * sizeof(CellSpecies));
    int32_t *escale = (int32_t *)take(nc * 2 * sizeof(int32_t));
    int2 *ranges = (int2 *)take((size_t)nc * r.n_tiles * sizeof(int2));
    double *TS = (double *)take((size_t)r.n_tiles * r.n_chunks * 2 * kTilePoints * 8);
    double *I_out = (double *)take((size_t)r.n_window * 8);
    int32_t *done = (int32_t *)take((size_t)(r.n_tiles + 1) * 4);
    double *tile_part = (double *)take((size_t)r.n_tiles * 8);
    double *I_int = (double *)take(8);
    double *cum = nullptr, *ff = nullptr, *lnb = nullptr;
    if (n_thr >= 0) {
        cum = (double *)take((size_t)nc * 2 * (n_thr + 1) * 8);
        ff = (double *)take((size_t)nc * 2 * 8);
        lnb = (double *)take((size_t)nc * 2 * 8);
    }
    // QSS-CR rows of the request's cells (the context's rate data and records)
    DevCR crq = dev_cr(ctx);
    if (cr_row > 0) {
        crq.pop = (double *)take((size_t)nc * cr_row * 8);
        crq.lnd = (double *)take((size_t)nc * cr_row * 8);
    }
    hipStream_t st = admit_stream;
    auto ok = [&](hipError_t e, const char *what) {
        if (e != hipSuccess) {
            fail_request(r, LRT_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
            release(r);
            return false;
        }
        return true;
    };
    // T_tr, T_v, n_e, ds and N are consecutive in the arena: pack them host-side
    // in that layout (padding zeroed) and upload once.  Small copies run as blit
    // kernels beside the persistent serve kernel, each costing admission latency.
    const size_t span = (size_t)((char *)(N + (size_t)nc * S) - (char *)T_tr);
    r.packed.assign(span, 0);
    const std::pair<const double *, const std::vector<double> *> parts[] = {
        {T_tr, &r.T_tr}, {T_v, &r.T_v}, {n_e, &r.n_e}, {ds, &r.ds}, {N, &r.N}};
    for (const auto &pt : parts)
        std::memcpy(r.packed.data() + ((const char *)pt.first - (const char *)T_tr), pt.second->data(),
                    pt.second->size() * sizeof(double));
    if (!ok(hipMemcpyAsync(T_tr, r.packed.data(), span, hipMemcpyHostToDevice, st), "upload"))
        return true;   // failed and released; counts as handled
    // lines tied to QSS-CR levels read the request's departure rows
    DevLines L = dev_lines(ctx);
    const bool cr_lines = cr_row > 0 && ctx->line_lev_ready;
    L.lev = cr_lines ? ctx->d_line_lev.as<int32_t>() : nullptr;
    L.lnd = cr_lines ? crq.lnd : nullptr;
    L.lnd_stride = cr_lines ? cr_row : 0;
    const DevGrid g = dev_grid(ctx);
    const DevCells cells{(int32_t)nc, S, T_tr, T_v, N, n_e};
    int32_t max_lev = 0;
    for (int32_t v : ctx->h_cr_nlev) max_lev = std::max(max_lev, v);
    if (!ok(launch_thermo(ctx->sp, cells, dev_widths(ctx), ctx->M_min, r.mask, cc, cs, st), "thermo") ||
        (cr_row > 0 && !ok(launch_cr(ctx->sp, cells, crq, ctx->cr_max_l, max_lev, cs, st), "QSS-CR")) ||
        !ok(launch_ranges(L, g, cc, (int32_t)nc, r.k_first, r.n_window, kTilePoints, ranges, st), "ranges"))
        return true;
    // the atomic continuum of the species the request lets radiate, over its window
    DevCont ct{-1, nullptr, nullptr, nullptr, nullptr};
    if (n_thr >= 0) {
        const double w_lo = ctx->nu_min + (double)r.k_first * ctx->h;
        const double w_hi = ctx->nu_min + (double)(r.k_first + r.n_window - 1) * ctx->h;
        if (!ok(launch_cont_cells(ctx->d_cont_thr.as<ContThr>(), n_thr, ctx->d_cont_rec.as<ContRec>(),
                                  ctx->n_cont_rec, cells, cs, cr_row > 0 ? crq : DevCR{}, r.mask, w_lo, w_hi,
                                  cum, ff, lnb, st),
                "continuum"))
            return true;
        ct = DevCont{n_thr, ctx->d_cont_thr.as<ContThr>(), cum, ff, T_v};
    }
    // per-cell power-of-two scale: the upper bound of the line peaks over the
    // level-energy bins whose lines can reach the window (and the continuum's
    // own bound), as the batch path bounds every line
    {
        DevBins B{(int32_t)ctx->n_bins, ctx->d_bin_sp.as<int32_t>(), ctx->d_bin_Ev.as<double>(),
                  ctx->d_bin_Er.as<double>(), ctx->d_bin_aeta.as<double>(), ctx->d_bin_akap.as<double>()};
        if (cr_lines) {
            B.lev_off = ctx->d_bin_lev_off.as<int32_t>();
            B.lev = ctx->d_bin_lev.as<int32_t>();
            B.lnd = crq.lnd;
            B.lnd_stride = cr_row;
        }
        B.nu_lo = ctx->d_bin_nlo.as<double>();
        B.nu_hi = ctx->d_bin_nhi.as<double>();
        B.win_a = ctx->nu_min + (double)r.k_first * ctx->h - ctx->h;
        B.win_b = ctx->nu_min + (double)(r.k_first + r.n_window - 1) * ctx->h + ctx->h;
        if (!ok(launch_scale_bound(B, cc, cs, lnb, (int32_t)nc, S, escale, st), "scale"))
            return true;
    }
    if (!ok(launch_fill_i32(done, 0, (int64_t)r.n_tiles + 1, st), "counters")) return true;
    r.dev = ServeReq{(int32_t)nc, r.k_first, r.n_window, r.n_tiles, r.n_chunks, kChunkCells,
                     cc, cs, escale, ds, ranges, TS, I_out, done, tile_part, I_int, h_I_int + r.slot, ct, r.T_far,
                     r.scheme == LRT_MARCH_LINEAR_J ? 1 : 0, L.lnd_stride, L.lnd};
    if (!ok(hipMemcpyAsync(d_reqs.as<ServeReq>() + r.slot, &r.dev, sizeof(ServeReq),
                           hipMemcpyHostToDevice, st), "upload") ||
        !ok(hipEventCreateWithFlags(&r.prep_ev, hipEventDisableTiming), "event") ||
        !ok(hipEventRecord(r.prep_ev, st), "event"))
        return true;
    r.items_total = (int64_t)r.n_tiles * r.n_chunks;
    r.state = ST_ADMITTED;
    admitted.push_back(r.ticket);
    return true;
}

bool lrt_server::launch_epoch(Epoch &e)
{
    // round-robin over admitted requests with items left
    std::vector<Req *> live;
    for (uint64_t t : admitted) {
        Req &r = *reqs[t];
        if (r.state == ST_ADMITTED && r.items_issued < r.items_total) live.push_back(&r);
    }
    if (live.empty()) return false;
    int n = 0;
    int64_t units = 0;
    e.credit.clear();
    std::map<uint64_t, int64_t> credit;
    bool progress = true;
    size_t start = rr % live.size();
    while (progress && n < kEpochCap && units < kEpochUnits) {
        progress = false;
        for (size_t q = 0; q < live.size() && n < kEpochCap && units < kEpochUnits; ++q) {
            Req &r = *live[(start + q) % live.size()];
            for (int k = 0; k < kItemsPerTurn && r.items_issued < r.items_total && n < kEpochCap &&
                            units < kEpochUnits; ++k) {
                const int64_t it = r.items_issued++;
                const int32_t tile = (int32_t)(it / r.n_chunks), chunk = (int32_t)(it % r.n_chunks);
                e.h_items[n++] = ServeItem{r.slot, tile, chunk};
                const int64_t cells = std::min<int64_t>(kChunkCells, r.n_cells - (int64_t)chunk * kChunkCells);
                units += cells * kTilePoints;
                credit[r.ticket] += 1;
                progress = true;
            }
        }
    }
    rr = (start + 1) % std::max<size_t>(1, live.size());
    for (auto &kv : credit) {
        e.credit.push_back(kv);
        Req &r = *reqs[kv.first];
        if (hipStreamWaitEvent(e.stream, r.prep_ev, 0) != hipSuccess) {
            fatal = "hipStreamWaitEvent failed";
            return false;
        }
    }
    // level offsets of the lines tied to QSS-CR levels; each request brings its
    // own departure rows
    DevLines L = dev_lines(ctx);
    const bool cr_lines = ctx->n_cr > 0 && ctx->line_lev_ready;
    L.lev = cr_lines ? ctx->d_line_lev.as<int32_t>() : nullptr;
    L.lnd = nullptr;
    L.lnd_stride = 0;
    const DevGrid g = dev_grid(ctx);
    hipError_t err = hipMemcpyAsync(e.d_items.p, e.h_items, (size_t)n * sizeof(ServeItem),
                                    hipMemcpyHostToDevice, e.stream);
    if (err == hipSuccess)
        err = launch_serve(L, g, d_reqs.as<ServeReq>(), e.d_items.as<ServeItem>(), n, ctx->n_species, e.stream);
    if (err == hipSuccess) err = hipEventRecord(e.done, e.stream);
    if (err != hipSuccess) {
        fatal = std::string("epoch launch: ") + hipGetErrorString(err);
        return false;
    }
    e.busy = true;
    ++n_epochs;
    return true;
}

void lrt_server::run()
{
    (void)hipSetDevice(ctx->device);
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
        bool progress = false;
        // 1) finished epochs credit their requests
        for (auto &e : epochs) {
            if (!e.busy) continue;
            const hipError_t q = hipEventQuery(e.done);
            if (q == hipErrorNotReady) continue;
            if (q != hipSuccess) {
                fatal = std::string("epoch: ") + hipGetErrorString(q);
                break;
            }
            for (auto &kv : e.credit) reqs[kv.first]->items_done += kv.second;
            e.credit.clear();
            e.busy = false;
            progress = true;
        }
        if (!fatal.empty()) break;
        // 2) requests with every item done: the serving kernel has composed
        //    them and written the integral to the slot's pinned host word
        for (size_t a = 0; a < admitted.size();) {
            Req &r = *reqs[admitted[a]];
            if (r.state != ST_ADMITTED || r.items_done < r.items_total) {
                ++a;
                continue;
            }
            r.I_int = h_I_int[r.slot];
            if (r.keep) {
                r.spectrum.resize(r.n_window);
                const hipError_t err = hipMemcpy(r.spectrum.data(), r.dev.I_out, (size_t)r.n_window * 8,
                                                 hipMemcpyDeviceToHost);
                if (err != hipSuccess) {
                    fatal = std::string("result copy: ") + hipGetErrorString(err);
                    break;
                }
            }
            r.state = ST_DONE;
            r.t_done = Clock::now();
            release(r);
            ++n_completed;
            admitted.erase(admitted.begin() + a);
            progress = true;
            cv_done.notify_all();
        }
        if (!fatal.empty()) break;
        // 3) admission: FIFO with skip-ahead
        for (auto it = pending.begin(); it != pending.end();) {
            Req &r = *reqs[*it];
            if (admit(r)) {
                it = pending.erase(it);
                progress = true;
            } else {
                ++it;
            }
            if (free_slots.empty()) break;
        }
        // 4) keep the epoch streams fed
        for (auto &e : epochs) {
            if (!e.busy && launch_epoch(e)) progress = true;
            if (!fatal.empty()) break;
        }
        if (!fatal.empty()) break;
        const bool in_flight = !admitted.empty() || epochs[0].busy || epochs[1].busy;
        if (stopping && pending.empty() && !in_flight) break;
        if (!progress) {
            if (in_flight) cv_work.wait_for(lk, std::chrono::microseconds(100));
            else cv_work.wait_for(lk, std::chrono::milliseconds(20));
        }
    }
    if (!fatal.empty()) {
        // the device is in an unknown state: fail everything still open
        for (auto &kv : reqs)
            if (kv.second->state != ST_DONE) fail_request(*kv.second, LRT_E_DEVICE, fatal);
        pending.clear();
        admitted.clear();
    }
    cv_done.notify_all();
}

extern "C" {

lrt_status lrt_server_start(lrt_ctx *ctx, size_t budget, int max_slots, lrt_server **out)
{
    if (!ctx || !out) return LRT_E_ARG;
    ctx->err.clear();
    *out = nullptr;
    if (max_slots < 1 || budget < ((size_t)1 << 20))
        return fail(ctx, LRT_E_ARG, "server needs max_slots >= 1 and a budget >= 1 MiB");
    lrt_status st;
    if ((st = prepare_lines(ctx))) return st;   // lines on the grid; ctx cells are not used
    std::unique_ptr<lrt_server> s(new (std::nothrow) lrt_server());
    if (!s) return fail(ctx, LRT_E_OOM, "server allocation failed");
    s->ctx = ctx;
    s->budget = budget;
    s->max_slots = max_slots;
    if ((st = upload(ctx, s->d_arena, nullptr, budget))) return st;
    s->arena.base = s->d_arena.as<char>();
    s->arena.size = budget;
    s->arena.free_[0] = budget;
    if ((st = upload(ctx, s->d_reqs, nullptr, (size_t)max_slots * sizeof(ServeReq)))) return st;
    for (int i = max_slots - 1; i >= 0; --i) s->free_slots.push_back(i);
    LRT_HIP(ctx, hipStreamCreateWithFlags(&s->admit_stream, hipStreamNonBlocking));
    LRT_HIP(ctx, hipHostMalloc((void **)&s->h_I_int, (size_t)max_slots * 8, hipHostMallocDefault));
    for (auto &e : s->epochs) {
        LRT_HIP(ctx, hipStreamCreateWithFlags(&e.stream, hipStreamNonBlocking));
        LRT_HIP(ctx, hipEventCreateWithFlags(&e.done, hipEventDisableTiming));
        LRT_HIP(ctx, hipHostMalloc((void **)&e.h_items, kEpochCap * sizeof(ServeItem), hipHostMallocDefault));
        if ((st = upload(ctx, e.d_items, nullptr, kEpochCap * sizeof(ServeItem)))) return st;
    }
    lrt_server *raw = s.release();
    raw->th = std::thread([raw] { raw->run(); });
    *out = raw;
    return LRT_OK;
}

lrt_status lrt_submit(lrt_server *s, const lrt_los_request *q, uint64_t *ticket)
{
    if (!s || !q || !ticket) return LRT_E_ARG;
    lrt_ctx *ctx = s->ctx;
    const int S = ctx->n_species;
    if (q->n_cells < 1 || q->n_cells >= INT_MAX || q->n_species != S || !q->T_tr || !q->T_v || !q->N ||
        !q->n_e || !q->ds)
        return fail(nullptr, LRT_E_ARG, "request: cells, species count or arrays invalid");
    if (q->n_window < 1 || q->k_first < 0 || q->k_first + q->n_window > ctx->n_points)
        return fail(nullptr, LRT_E_ARG, "request: window outside the grid");
    for (int64_t c = 0; c < q->n_cells; ++c) {
        if (!(q->T_tr[c] > 0.0) || !(q->T_v[c] > 0.0) || !std::isfinite(q->T_tr[c]) || !std::isfinite(q->T_v[c]) ||
            !(q->n_e[c] >= 0.0) || !std::isfinite(q->n_e[c]) || !(q->ds[c] > 0.0) || !std::isfinite(q->ds[c]))
            return fail(nullptr, LRT_E_ARG, "request: cell %lld has an invalid state", (long long)c);
        for (int sp = 0; sp < S; ++sp)
            if (!(q->N[c * S + sp] >= 0.0) || !std::isfinite(q->N[c * S + sp]))
                return fail(nullptr, LRT_E_ARG, "request: cell %lld density %d invalid", (long long)c, sp);
    }
    if (!(q->T_far >= 0.0) || !std::isfinite(q->T_far))
        return fail(nullptr, LRT_E_ARG, "request: far-boundary temperature %g invalid", q->T_far);
    if (q->scheme != LRT_MARCH_CELL && q->scheme != LRT_MARCH_LINEAR_J)
        return fail(nullptr, LRT_E_ARG, "request: unknown segment scheme %d", q->scheme);
    int32_t nt, nch;
    const int32_t n_thr = ctx->n_cont_rec > 0 ? ctx->n_cont_thr : -1;
    const int32_t cr_row = ctx->n_cr > 0 ? ctx->n_cr * ctx->cr_LS : 0;
    const size_t bytes = request_bytes(q->n_cells, S, (int32_t)q->n_window, n_thr, cr_row, nt, nch);
    if (bytes > s->budget)
        return fail(nullptr, LRT_E_BUDGET, "request needs %zu bytes, budget is %zu", bytes, s->budget);
    std::unique_ptr<Req> r(new (std::nothrow) Req());
    if (!r) return fail(nullptr, LRT_E_OOM, "request allocation failed");
    const int64_t nc = q->n_cells;
    r->n_cells = nc;
    r->T_tr.assign(q->T_tr, q->T_tr + nc);
    r->T_v.assign(q->T_v, q->T_v + nc);
    r->n_e.assign(q->n_e, q->n_e + nc);
    r->ds.assign(q->ds, q->ds + nc);
    r->N.assign(q->N, q->N + nc * S);
    r->k_first = (int32_t)q->k_first;
    r->n_window = (int32_t)q->n_window;
    r->mask = q->species_mask;
    r->keep = q->keep_spectrum != 0;
    r->T_far = q->T_far;
    r->scheme = q->scheme;
    r->t_submit = Clock::now();
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stopping) return fail(nullptr, LRT_E_STATE, "server is stopping");
    if (!s->fatal.empty()) return fail(nullptr, LRT_E_DEVICE, "server failed: %s", s->fatal.c_str());
    r->ticket = s->next_ticket++;
    *ticket = r->ticket;
    s->pending.push_back(r->ticket);
    s->reqs[r->ticket] = std::move(r);
    s->cv_work.notify_one();
    return LRT_OK;
}

static lrt_status take_result(lrt_server *s, uint64_t ticket, lrt_los_result *out, double *spectrum)
{
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return fail(nullptr, LRT_E_ARG, "unknown ticket %llu", (unsigned long long)ticket);
    Req &r = *it->second;
    if (r.state != ST_DONE) return LRT_E_NOT_READY;
    if (out) {
        out->status = r.status;
        out->I_int = r.I_int;
        out->n_window = r.n_window;
        out->queue_ms = r.t_admit.time_since_epoch().count() ? ms_between(r.t_submit, r.t_admit) : -1.0;
        out->latency_ms = ms_between(r.t_submit, r.t_done);
    }
    if (spectrum && r.status == LRT_OK && !r.spectrum.empty())
        std::memcpy(spectrum, r.spectrum.data(), r.spectrum.size() * 8);
    const lrt_status st = r.status;
    if (st != LRT_OK) fail(nullptr, st, "%s", r.err.c_str());
    s->reqs.erase(it);
    return LRT_OK;
}

lrt_status lrt_poll(lrt_server *s, uint64_t ticket, lrt_los_result *out, double *spectrum)
{
    if (!s) return LRT_E_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    return take_result(s, ticket, out, spectrum);
}

lrt_status lrt_wait(lrt_server *s, uint64_t ticket, double timeout_ms, lrt_los_result *out, double *spectrum)
{
    if (!s) return LRT_E_ARG;
    std::unique_lock<std::mutex> lk(s->mu);
    const auto deadline = Clock::now() + std::chrono::duration<double, std::milli>(timeout_ms);
    for (;;) {
        const lrt_status st = take_result(s, ticket, out, spectrum);
        if (st != LRT_E_NOT_READY) return st;
        if (timeout_ms >= 0 && Clock::now() >= deadline) return LRT_E_NOT_READY;
        s->cv_done.wait_until(lk, timeout_ms >= 0 ? deadline : Clock::now() + std::chrono::milliseconds(50));
    }
}

lrt_status lrt_cancel(lrt_server *s, uint64_t ticket)
{
    if (!s) return LRT_E_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return fail(nullptr, LRT_E_ARG, "unknown ticket %llu", (unsigned long long)ticket);
    Req &r = *it->second;
    if (r.state != ST_PENDING) return fail(nullptr, LRT_E_STATE, "request already admitted");
    s->pending.erase(std::find(s->pending.begin(), s->pending.end(), ticket));
    s->fail_request(r, LRT_E_STATE, "cancelled");
    return LRT_OK;
}

lrt_status lrt_server_info(lrt_server *s, int64_t *pending, int64_t *admitted, int64_t *completed,
                           int64_t *epochs, size_t *bytes_in_use)
{
    if (!s) return LRT_E_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    if (pending) *pending = (int64_t)s->pending.size();
    if (admitted) *admitted = (int64_t)s->admitted.size();
    if (completed) *completed = s->n_completed;
    if (epochs) *epochs = s->n_epochs;
    if (bytes_in_use) *bytes_in_use = s->arena.used;
    return LRT_OK;
}

lrt_status lrt_server_stop(lrt_server *s)
{
    if (!s) return LRT_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stopping = true;
        s->cv_work.notify_all();
    }
    if (s->th.joinable()) s->th.join();
    const bool ok = s->fatal.empty();
    (void)hipDeviceSynchronize();
    for (auto &kv : s->reqs) s->release(*kv.second);
    for (auto &e : s->epochs) {
        if (e.h_items) (void)hipHostFree(e.h_items);
        if (e.done) (void)hipEventDestroy(e.done);
        if (e.stream) (void)hipStreamDestroy(e.stream);
    }
    if (s->admit_stream) (void)hipStreamDestroy(s->admit_stream);
    if (s->h_I_int) (void)hipHostFree(s->h_I_int);
    const std::string msg = s->fatal;
    delete s;
    if (!ok) return fail(nullptr, LRT_E_DEVICE, "server failed: %s", msg.c_str());
    return LRT_OK;
}

}  // extern "C"
