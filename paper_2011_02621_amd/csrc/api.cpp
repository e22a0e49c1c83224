// extern "C" boundary: argument checks, error capture, contexts, plans and
// the serving loop.  No C++ exception crosses into the caller.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <functional>
#include <list>
#include <new>
#include <thread>

#include "internal.h"

namespace tns {

static thread_local std::string g_last_error;

void set_last_error(const std::string &msg) { g_last_error = msg; }

[[noreturn]] void fail(tns_status code, const std::string &msg) { throw Error(code, msg); }

template <typename F>
static tns_status guard(F &&f) {
    try {
        f();
        return TNS_OK;
    } catch (const Error &e) {
        set_last_error(e.what());
        return e.code;
    } catch (const std::bad_alloc &) {
        set_last_error("host allocation failed");
        return TNS_E_OUT_OF_MEMORY;
    } catch (const std::exception &e) {
        set_last_error(std::string("internal error: ") + e.what());
        return TNS_E_DEVICE;
    } catch (...) {
        set_last_error("unknown internal error");
        return TNS_E_DEVICE;
    }
}

static void hip_check(hipError_t e, const char *what) {
    if (e != hipSuccess) fail(TNS_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

// ----------------------------------------------------------------------------
// serving.  A request is cut into work items, each a range of bitstrings
// times a range of slices, i.e. a block of (bitstring, slice) units.  Worker
// threads (one HIP stream and workspace each) take items from
// the active requests, so a request that arrives while others run starts as
// soon as a worker and the memory for one of its items are free, and its
// items overlap with theirs on the device.  A free worker takes the next item
// of the request with the least planned work left (shortest remaining work
// first).
//
// Memory: the workers share a pool, the context's budget less the share kept
// for synchronous calls.  A worker holds a reservation for the workspace it
// caches; an item starts only when its workspace fits the pool beside the
// other workers' reservations, and while items wait for memory, idle
// workers give their cached workspace back.
//
// An item's shape is fixed when the request is submitted, so its partial
// sums -- added per bitstring in slice-range order -- do not depend on how
// the request's items interleave with other work.

using clk = std::chrono::steady_clock;

struct Request {
    const Plan *plan = nullptr;
    int64_t n = 0;
    const uint8_t *bits = nullptr;
    double *amps = nullptr;
    int64_t nb_chunk = 1, ns_chunk = 1;   // bitstrings and slices per item
    int64_t n_schunks = 1;               // slice ranges per bitstring range
    int64_t n_items = 0, next_item = 0, finished_items = 0;
    uint64_t item_bytes = 0;             // workspace of one item
    double item_flops = 0;               // planned contraction flops of one item
    std::vector<double> part;            // [n][n_schunks][opu][2] when n_schunks > 1
    int running = 0;                     // items in flight
    std::atomic<int> cancel{0};          // set by tns_cancel, read by the worker mid-item
    tns_status status = TNS_OK;          // written with both the server's lock and m held
    bool done = false;
    std::string error;
    clk::time_point t_submit, t_start, t_end;
    bool started = false;
    std::mutex m;
    std::condition_variable cv;
};

struct Item {
    Request *r = nullptr;
    int64_t b0 = 0, b1 = 0, s0 = 0, s1 = 0, si = 0;
    bool release_first = false;
    uint64_t release_bytes = 0;   // reservation of the cache freed before the item runs
    uint64_t budget = 0;
};

struct Server {
    Ctx *ctx = nullptr;
    std::vector<std::thread> workers;
    std::vector<void *> streams;
    std::vector<Workspace> ws;
    std::vector<uint64_t> held;          // per worker: reserved workspace bytes
    std::vector<const Plan *> held_plan; // per worker: plan its workspace was sized for
    std::mutex m;
    std::condition_variable cv;
    std::list<Request *> active;
    bool stop = false;
    bool pressure = false;               // an item waits for memory
    uint64_t pool = 0;                   // bytes the workers share
    uint64_t reserved = 0;               // sum of held
    uint64_t sync_budget = 0;            // workspace of synchronous calls

    void start(Ctx *c, int n_workers) {
        ctx = c;
        sync_budget = ctx->budget / 4;
        pool = ctx->budget - sync_budget;
        streams.resize(n_workers);
        ws.resize(n_workers);
        held.assign(n_workers, 0);
        held_plan.assign(n_workers, nullptr);
        for (int i = 0; i < n_workers; ++i) {
            hipStream_t s;
            hip_check(hipSetDevice(ctx->device), "hipSetDevice");
            hip_check(hipStreamCreate(&s), "hipStreamCreate");
            streams[i] = s;
        }
        for (int i = 0; i < n_workers; ++i) workers.emplace_back([this, i] { loop(i); });
    }

    void shutdown() {
        {
            std::lock_guard<std::mutex> lk(m);
            stop = true;
        }
        cv.notify_all();
        for (auto &t : workers) t.join();
        // requests left without workers end as cancelled (their plans are
        // destroyed first, so normally none is left)
        {
            std::lock_guard<std::mutex> lk_server(m);
            for (Request *r : active) {
                r->plan->serving_in_flight--;
                std::lock_guard<std::mutex> lk(r->m);
                if (r->status == TNS_OK) {
                    r->status = TNS_E_CANCELLED;
                    r->error = "context finalized";
                }
                r->t_end = clk::now();
                r->done = true;
                r->cv.notify_all();
            }
            active.clear();
        }
        for (size_t i = 0; i < streams.size(); ++i) {
            ws[i].release(ctx, streams[i]);
            (void)hipStreamDestroy((hipStream_t)streams[i]);
        }
    }

    // called with m held (lock order: the server's m, then r->m), so that
    // pick() and complete_if_done() may read r->status under m alone
    void finish(Request *r, tns_status st, const std::string &err) {
        std::lock_guard<std::mutex> lk(r->m);
        if (st != TNS_OK && r->status == TNS_OK) {
            r->status = st;
            r->error = err;
        }
    }

    // called with m held: the next item a worker may run now, if any.
    // Sets `newly_blocked` when this call is the one that raised `pressure`.
    bool pick(int w, Item &it, bool &newly_blocked) {
        newly_blocked = false;
        if (active.empty()) return false;
        // shortest remaining work first: the request with the fewest planned
        // flops left whose next item fits the memory pool (ties: the earlier
        // request), so short requests are not held behind long ones
        bool blocked = false;
        Request *best = nullptr;
        double best_left = 0;
        for (Request *r : active) {
            if (r->next_item >= r->n_items || r->status != TNS_OK || r->cancel) continue;
            // a worker that switches plans frees its cache only after the
            // pick, so until then the old reservation counts beside the new
            const bool reuse = held_plan[w] == r->plan && held[w] >= r->item_bytes;
            if (!reuse && reserved + r->item_bytes > pool) {
                blocked = true;
                continue;
            }
            const double left = (double)(r->n_items - r->next_item) * r->item_flops;
            if (!best || left < best_left) {
                best = r;
                best_left = left;
            }
        }
        if (best) {
            Request *r = best;
            const bool reuse = held_plan[w] == r->plan && held[w] >= r->item_bytes;
            const uint64_t mine = reuse ? held[w] : r->item_bytes;
            it = Item{};
            it.r = r;
            it.release_first = !reuse && held[w] > 0;
            it.release_bytes = reuse ? 0 : held[w];
            if (!reuse) reserved += mine;
            held[w] = mine;
            held_plan[w] = r->plan;
            it.budget = mine;
            const int64_t i = r->next_item++;
            it.si = i % r->n_schunks;
            it.b0 = (i / r->n_schunks) * r->nb_chunk;
            it.b1 = std::min(r->n, it.b0 + r->nb_chunk);
            it.s0 = it.si * r->ns_chunk;
            it.s1 = std::min(r->plan->n_slices, it.s0 + r->ns_chunk);
            r->running++;
            if (!r->started) {
                r->started = true;
                r->t_start = clk::now();
            }
            return true;
        }
        if (blocked && !pressure) {
            pressure = true;
            newly_blocked = true;
        }
        return false;
    }

    void complete_if_done(Request *r) {
        // called with m held
        const bool over = r->running == 0 &&
                          (r->finished_items >= r->n_items || r->status != TNS_OK || r->cancel);
        if (!over) return;
        auto it = std::find(active.begin(), active.end(), r);
        if (it == active.end()) return;   // already completed
        active.erase(it);
        r->plan->serving_in_flight--;
        cv.notify_all();   // a tns_plan_destroy may wait for this plan's requests
        // notify under r->m: a waiter that sees done may free r at once
        std::lock_guard<std::mutex> lk(r->m);
        if (r->cancel && r->status == TNS_OK && r->finished_items < r->n_items) {
            r->status = TNS_E_CANCELLED;
            r->error = "request cancelled";
        }
        if (r->status == TNS_OK && r->n_schunks > 1) {
            // partial sums of each bitstring, added in slice-range order
            const int64_t opu = r->plan->out_per_unit, S = r->n_schunks;
            for (int64_t b = 0; b < r->n; ++b)
                for (int64_t j = 0; j < opu; ++j) {
                    double re = 0, im = 0;
                    for (int64_t k = 0; k < S; ++k) {
                        const double *v = &r->part[((b * S + k) * opu + j) * 2];
                        re += v[0];
                        im += v[1];
                    }
                    r->amps[2 * (b * opu + j)] = re;
                    r->amps[2 * (b * opu + j) + 1] = im;
                }
        }
        r->t_end = clk::now();
        r->done = true;
        r->cv.notify_all();
    }

    void loop(int wi) {
        (void)hipSetDevice(ctx->device);
        std::vector<double> tmp;
        for (;;) {
            Item it;
            bool give_back = false;
            {
                std::unique_lock<std::mutex> lk(m);
                for (;;) {
                    if (stop) return;
                    bool newly = false;
                    if (pick(wi, it, newly)) break;
                    if (pressure && held[wi] > 0) {
                        give_back = true;
                        break;
                    }
                    // wake the idle workers that hold memory (once per rise of pressure)
                    if (newly) cv.notify_all();
                    cv.wait(lk);
                }
            }
            if (give_back) {
                // another item waits for memory: return this worker's cache
                ws[wi].release(ctx, streams[wi]);
                {
                    std::lock_guard<std::mutex> lk(m);
                    reserved -= held[wi];
                    held[wi] = 0;
                    held_plan[wi] = nullptr;
                    pressure = false;
                }
                cv.notify_all();
                continue;
            }
            Request *r = it.r;
            tns_status st = TNS_OK;
            std::string err;
            RunStats rs;
            try {
                if (it.release_first) {
                    ws[wi].release(ctx, streams[wi]);
                    {
                        std::lock_guard<std::mutex> lk(m);
                        reserved -= it.release_bytes;
                    }
                    cv.notify_all();
                }
                const Plan &p = *r->plan;
                const int64_t nb = it.b1 - it.b0, opu = p.out_per_unit;
                double *out = r->amps + 2 * it.b0 * opu;
                if (r->n_schunks > 1) {
                    tmp.resize((size_t)(nb * opu * 2));
                    out = tmp.data();
                }
                run_amplitudes(ctx, p, nb, r->bits + it.b0 * p.circ.n, out, streams[wi], ws[wi], rs,
                               &r->cancel, it.budget, it.s0, it.s1);
                if (r->n_schunks > 1)
                    for (int64_t b = 0; b < nb; ++b)
                        std::memcpy(&r->part[(((it.b0 + b) * r->n_schunks + it.si) * opu) * 2],
                                    &tmp[b * opu * 2], sizeof(double) * 2 * opu);
            } catch (const Error &e) {
                st = e.code;
                err = e.what();
            } catch (const std::exception &e) {
                st = TNS_E_DEVICE;
                err = e.what();
            }
            {
                std::lock_guard<std::mutex> lk(m);
                if (st != TNS_OK) finish(r, st, err);
                // the workspace may have grown within this worker's reservation
                r->running--;
                if (st == TNS_OK) r->finished_items++;
                complete_if_done(r);
            }
            cv.notify_all();
        }
    }

    void submit(Request *r) {
        {
            std::lock_guard<std::mutex> lk(m);
            r->plan->serving_in_flight++;
            active.push_back(r);
        }
        cv.notify_all();
    }

    void cancel(Request *r) {
        std::lock_guard<std::mutex> lk(m);
        r->cancel = 1;
        complete_if_done(r);
    }
};

// Item shape of a request: about kItemFlops of contraction per item (a few
// tenths of a second on the device), at most 1024 bitstrings (light circuits
// take whole requests, so the fixed cost of a call -- the bra evolution's
// launches, the host round trip -- is paid once), and a workspace that fits
// the pool.
constexpr double kItemFlops = 4e13;

static void shape_items(Request *r, const Server &sv, double item_flops) {
    const double kItemFlops = item_flops > 0 ? item_flops : tns::kItemFlops;
    const Plan &p = *r->plan;
    const double per_slice = p.flops_per_amp / (double)p.n_slices;
    int64_t nb = (int64_t)std::floor(kItemFlops / std::max(p.flops_per_amp, 1.0));
    nb = std::max<int64_t>(1, std::min<int64_t>({nb, 1024, r->n}));
    int64_t ns = p.n_slices;
    if (nb == 1) ns = std::max<int64_t>(1, std::min<int64_t>(p.n_slices, (int64_t)(kItemFlops / std::max(per_slice, 1.0))));
    while (call_workspace_bytes(p, nb, ns, sv.pool) > sv.pool && (nb > 1 || ns > 1)) {
        if (nb > 1) nb = (nb + 1) / 2;
        else ns = (ns + 1) / 2;
    }
    r->nb_chunk = nb;
    r->ns_chunk = ns;
    r->n_schunks = (p.n_slices + ns - 1) / ns;
    r->n_items = ((r->n + nb - 1) / nb) * r->n_schunks;
    r->item_bytes = call_workspace_bytes(p, nb, ns, sv.pool);
    r->item_flops = p.flops_per_amp / (double)p.n_slices * (double)nb * (double)ns;
}

}  // namespace tns

using namespace tns;

struct tns_ctx : public Ctx {};
struct tns_plan : public Plan {};
struct tns_request : public Request {};

extern "C" {

const char *tns_last_error(void) { return g_last_error.c_str(); }
const char *tns_version(void) { return "tns-amp 0.1 (gfx950)"; }

tns_status tns_init(int device, uint64_t hbm_budget_bytes, tns_ctx **out) {
    return guard([&] {
        if (!out) fail(TNS_E_INVALID_ARG, "out is NULL");
        *out = nullptr;
        if (device < -1) fail(TNS_E_INVALID_ARG, "device must be >= -1");
        std::unique_ptr<tns_ctx> c(new tns_ctx());
        c->device = device;
        if (device >= 0) {
            int count = 0;
            hip_check(hipGetDeviceCount(&count), "hipGetDeviceCount");
            if (device >= count) fail(TNS_E_INVALID_ARG, "no such device");
            hip_check(hipSetDevice(device), "hipSetDevice");
            scratch_setup(device);   // tns_amplitudes_noalloc's workspace on this device
            hipStream_t s;
            hip_check(hipStreamCreate(&s), "hipStreamCreate");
            c->stream = s;
            size_t free_b = 0, total_b = 0;
            hip_check(hipMemGetInfo(&free_b, &total_b), "hipMemGetInfo");
            c->budget = hbm_budget_bytes ? hbm_budget_bytes : (uint64_t)(0.9 * (double)free_b);
        } else {
            c->budget = hbm_budget_bytes;
        }
        *out = c.release();
    });
}

tns_status tns_set_allocator(tns_ctx *ctx, void *(*alloc)(size_t, void *, void *),
                             void (*free_)(void *, void *, void *), void *user) {
    return guard([&] {
        if (!ctx) fail(TNS_E_INVALID_ARG, "ctx is NULL");
        if ((alloc == nullptr) != (free_ == nullptr))
            fail(TNS_E_INVALID_ARG, "alloc and free must both be set or both be NULL");
        std::lock_guard<std::mutex> lk(ctx->mu);
        if (!ctx->ws.bufs.empty() || ctx->server)
            fail(TNS_E_INVALID_ARG, "allocator must be installed before any device memory is used");
        ctx->alloc_fn = alloc;
        ctx->free_fn = free_;
        ctx->alloc_user = user;
    });
}

tns_status tns_finalize(tns_ctx *ctx) {
    return guard([&] {
        if (!ctx) return;
        // a plan keeps device memory of its context: the context outlives it
        if (ctx->live_plans > 0)
            fail(TNS_E_INVALID_ARG, std::to_string(ctx->live_plans.load()) +
                                        " plan(s) created on this context are alive; destroy them first");
        if (ctx->device >= 0) (void)hipSetDevice(ctx->device);
        if (ctx->server) {
            ctx->server->shutdown();
            delete ctx->server;
            ctx->server = nullptr;
        }
        if (ctx->device >= 0) {
            ctx->ws.release(ctx, ctx->stream);
            (void)hipStreamDestroy((hipStream_t)ctx->stream);
        }
        delete ctx;
    });
}

void tns_plan_opts_default(tns_plan_opts *o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->split_cycle = -1;
    o->path = nullptr;
    o->path_mode = TNS_PATH_ALGORITHM1;
    o->max_rank = 0;
    o->path_assumptions = 1;
    o->n_cuts = -1;
    o->cut_edges = nullptr;
    o->max_intermediate_elems = 1ULL << 32;
    o->svd_rel_cutoff = 1e-12;
    o->max_search_states = 0;
    o->precision = TNS_C128;
    o->n_open = 0;
    o->open_qubits = nullptr;
    o->path_branches = 1;
}

tns_status tns_plan_create(tns_ctx *ctx, const tns_circuit_desc *desc, const tns_plan_opts *opts,
                           tns_plan **out) {
    return guard([&] {
        if (!ctx || !out) fail(TNS_E_INVALID_ARG, "ctx or out is NULL");
        *out = nullptr;
        tns_plan_opts o;
        if (opts) o = *opts; else tns_plan_opts_default(&o);
        if (o.path_mode != TNS_PATH_GREEDY && o.path_mode != TNS_PATH_ALGORITHM1)
            fail(TNS_E_INVALID_ARG, "unknown path_mode");
        if (o.max_rank < 0 || o.max_search_states < 0) fail(TNS_E_INVALID_ARG, "negative search limit");
        if (o.svd_rel_cutoff < 0) fail(TNS_E_INVALID_ARG, "negative svd_rel_cutoff");
        if (o.n_cuts < -1) fail(TNS_E_INVALID_ARG, "n_cuts must be >= -1");
        Circuit c;
        validate_and_build(desc, c);
        add_open_legs(c, o);
        if (o.split_cycle > c.max_cycle + 1) fail(TNS_E_INVALID_ARG, "split_cycle beyond the last cycle");
        std::unique_ptr<tns_plan> p(new tns_plan());
        plan_host(c, o, *p);
        if (ctx->device >= 0) {
            std::lock_guard<std::mutex> lk(ctx->mu);
            hip_check(hipSetDevice(ctx->device), "hipSetDevice");
            const uint64_t need = p->bytes_per_bitstring + p->bytes_per_unit;
            if (ctx->budget && need > ctx->budget)
                fail(TNS_E_OUT_OF_MEMORY, "one bitstring needs " + std::to_string(need) +
                                              " bytes of workspace, budget is " + std::to_string(ctx->budget));
            plan_device_setup(ctx, *p);
            ctx->live_plans++;
        }
        *out = p.release();
    });
}

tns_status tns_plan_info_get(const tns_plan *p, tns_plan_info *o) {
    return guard([&] {
        if (!p || !o) fail(TNS_E_INVALID_ARG, "NULL argument");
        std::memset(o, 0, sizeof(*o));
        o->n_qubits = p->circ.n;
        o->n_edges = (int32_t)p->circ.g.edges.size();
        o->split_cycle = p->split;
        o->n_steps = (int32_t)p->info_m.size();
        o->path = p->info_path.data();
        o->step_m = p->info_m.data();
        o->step_k = p->info_k.data();
        o->step_n = p->info_n.data();
        o->step_kernel = p->info_kernel.data();
        o->step_permute = p->info_permute.data();
        o->bond_ket = p->ket.bond.data();
        o->bond_bra = p->bra.bond.data();
        o->bond_overlap = p->bond_overlap.data();
        o->n_cuts = (int32_t)p->cuts.size();
        o->cut_edges = p->cuts.data();
        o->n_slices = p->n_slices;
        o->flops_per_amp = p->flops_per_amp;
        o->gemm_bytes_per_amp = p->gemm_bytes_per_amp;
        o->permute_bytes_per_amp = p->permute_bytes_per_amp;
        o->path_score = p->path_score;
        o->peak_elems = p->peak_elems;
        o->device_bytes_resident = p->resident_bytes;
        o->device_bytes_per_unit = p->bytes_per_unit;
        o->n_fused_ket = p->n_fused_ket;
        o->n_fused_bra = p->n_fused_bra;
        o->search_complete = p->search_complete ? 1 : 0;
        o->search_states = p->search_states;
        o->max_rank_used = p->path.max_rank;
        o->fidelity = p->fidelity;
        o->n_samples = p->n_samples;
        o->precision = (tns_precision)p->precision;
        o->n_open = p->circ.n_open;
        o->open_qubits = p->circ.open_qubits.data();
        o->n_branches = (int32_t)p->branches.size();
        o->branch_windows = p->info_branch_windows.data();
        o->step_chain = p->info_chain.data();
        o->linear_score = p->linear_score;
        int32_t np = 0;
        for (int m = 0; m < p->prefix_steps; ++m) np += p->steps[m].start ? 0 : 1;
        o->n_prefix_steps = np;
        o->prefix_flops_per_amp = p->prefix_flops;
    });
}

tns_status tns_plan_destroy(tns_plan *p) {
    return guard([&] {
        if (!p) return;
        Ctx *owner = p->on_device ? p->ctx : nullptr;
        if (owner && owner->server) {
            // requests on this plan are still being served: wait for them
            Server *sv = owner->server;
            std::unique_lock<std::mutex> lk(sv->m);
            sv->cv.wait(lk, [&] { return p->serving_in_flight.load() == 0; });
        }
        if (owner && owner->device >= 0) (void)hipSetDevice(owner->device);
        plan_device_release(*p);
        if (owner) owner->live_plans--;
        delete p;
    });
}

static tns_status amplitudes_impl(tns_ctx *ctx, const tns_plan *plan, int64_t n, const uint8_t *bits,
                                  int64_t slice_begin, int64_t slice_end, double *amps,
                                  void *hip_stream, tns_stats *stats,
                                  const FrugalAccept *frugal = nullptr) {
    return guard([&] {
        auto t0 = clk::now();
        if (!ctx || !plan) fail(TNS_E_INVALID_ARG, "ctx or plan is NULL");
        if (n < 0) fail(TNS_E_INVALID_ARG, "n must be >= 0");
        if (n > 0 && (!bits || !amps)) fail(TNS_E_INVALID_ARG, "bits or amps is NULL");
        if (ctx->device < 0) fail(TNS_E_NO_DEVICE, "planning-only context cannot compute amplitudes");
        if (!plan->on_device || plan->ctx != ctx) fail(TNS_E_INVALID_ARG, "plan was not created on this context");
        if (slice_end < 0) slice_end = plan->n_slices;
        if (slice_begin < 0 || slice_begin >= slice_end || slice_end > plan->n_slices)
            fail(TNS_E_INVALID_ARG, "slice range must satisfy 0 <= begin < end <= n_slices");
        for (int64_t i = 0; i < n * plan->circ.n; ++i)
            if (bits[i] > 1) fail(TNS_E_INVALID_ARG, "bits must be 0 or 1");
        RunStats rs;
        rs.profile = stats != nullptr;
        if (n > 0) {
            std::lock_guard<std::mutex> lk(ctx->mu);
            hip_check(hipSetDevice(ctx->device), "hipSetDevice");
            void *st = hip_stream ? hip_stream : ctx->stream;
            // once serving workers exist, synchronous calls take one slot's
            // share of the budget, like each worker
            const uint64_t budget = ctx->server ? ctx->server->sync_budget : ctx->budget;
            run_amplitudes(ctx, *plan, n, bits, amps, st, ctx->ws, rs, nullptr, budget, slice_begin,
                           slice_end, frugal);
        }
        if (stats) {
            std::memset(stats, 0, sizeof(*stats));
            stats->ms_total = std::chrono::duration<double, std::milli>(clk::now() - t0).count();
            stats->ms_bra = rs.ms_bra;
            stats->ms_merge = rs.ms_merge;
            stats->ms_contract = rs.ms_contract;
            stats->flops = rs.flops;
            stats->units = rs.units;
            stats->launches = rs.launches;
            stats->peak_device_bytes = ctx->peak_bytes;
            stats->ms_gemm = rs.ms_gemm;
            stats->gemm_launches = rs.gemm_launches;
            stats->gemm_flops = rs.gemm_flops;
            stats->gemm_bytes = rs.gemm_bytes;
            stats->ms_permute = rs.ms_permute;
            stats->permute_bytes = rs.permute_bytes;
            stats->ms_small = rs.ms_small;
            stats->gemm_mfma_flops = rs.gemm_mfma_flops;
            stats->ms_gemm3m = rs.ms_gemm3m;
            stats->gemm3m_launches = rs.gemm3m_launches;
            stats->gemm3m_flops = rs.gemm3m_flops;
            stats->gemm3m_mfma_flops = rs.gemm3m_mfma_flops;
            stats->gemm3m_bytes = rs.gemm3m_bytes;
        }
    });
}

tns_status tns_amplitudes(tns_ctx *ctx, const tns_plan *plan, int64_t n, const uint8_t *bits,
                          double *amps, void *hip_stream, tns_stats *stats) {
    return amplitudes_impl(ctx, plan, n, bits, 0, -1, amps, hip_stream, stats);
}

tns_status tns_amplitudes_sliced(tns_ctx *ctx, const tns_plan *plan, int64_t n, const uint8_t *bits,
                                 int64_t slice_begin, int64_t slice_end, double *amps,
                                 void *hip_stream, tns_stats *stats) {
    if (slice_end < 0) {
        set_last_error("slice_end must be >= 0");
        return TNS_E_INVALID_ARG;
    }
    return amplitudes_impl(ctx, plan, n, bits, slice_begin, slice_end, amps, hip_stream, stats);
}

tns_status tns_amplitudes_noalloc(tns_ctx *ctx, const tns_plan *plan, int64_t n,
                                  const uint8_t *bits_dev, double *amps_dev, void *hip_stream) {
    return guard([&] {
        if (!ctx || !plan) fail(TNS_E_INVALID_ARG, "ctx or plan is NULL");
        if (n < 0) fail(TNS_E_INVALID_ARG, "n must be >= 0");
        if (n > 0 && (!bits_dev || !amps_dev)) fail(TNS_E_INVALID_ARG, "bits_dev or amps_dev is NULL");
        if (ctx->device < 0) fail(TNS_E_NO_DEVICE, "planning-only context cannot compute amplitudes");
        if (!plan->on_device || plan->ctx != ctx) fail(TNS_E_INVALID_ARG, "plan was not created on this context");
        if (n == 0) return;
        std::lock_guard<std::mutex> lk(ctx->mu);
        hip_check(hipSetDevice(ctx->device), "hipSetDevice");
        char *base = (char *)scratch_device_ptr(ctx->device);
        if (!base) fail(TNS_E_DEVICE, "static workspace not set up on this device");
        Workspace arena;
        arena.arena = base;
        arena.arena_cap = kNoAllocScratchBytes;
        RunStats rs;
        void *st = hip_stream ? hip_stream : ctx->stream;
        run_amplitudes(ctx, *plan, n, nullptr, nullptr, st, arena, rs, nullptr, kNoAllocScratchBytes,
                       0, -1, nullptr, bits_dev, amps_dev);
    });
}

tns_status tns_sample_frugal(tns_ctx *ctx, const tns_plan *plan, int64_t n_batches,
                             const uint8_t *fixed_bits, const double *uniforms, double m_bound,
                             uint8_t *accepted, double *amps, void *hip_stream, tns_stats *stats) {
    {
        const tns_status st = guard([&] {
            if (!plan) fail(TNS_E_INVALID_ARG, "plan is NULL");
            if (n_batches > 0 && (!uniforms || !accepted || !amps))
                fail(TNS_E_INVALID_ARG, "uniforms, accepted or amps is NULL");
            if (!(m_bound > 0.0)) fail(TNS_E_INVALID_ARG, "m_bound must be positive");
            if (plan->circ.n > 1000) fail(TNS_E_UNSUPPORTED, "2^N overflows");
        });
        if (st != TNS_OK) return st;
    }
    FrugalAccept fa;
    fa.uniforms = uniforms;
    fa.scale = std::ldexp(1.0, plan->circ.n) / m_bound;
    fa.flags = accepted;
    return amplitudes_impl(ctx, plan, n_batches, fixed_bits, 0, -1, amps, hip_stream, stats, &fa);
}

tns_status tns_submit(tns_ctx *ctx, const tns_plan *plan, int64_t n, const uint8_t *bits,
                      double *amps, tns_request **out) {
    return guard([&] {
        if (!ctx || !plan || !out) fail(TNS_E_INVALID_ARG, "NULL argument");
        *out = nullptr;
        if (n < 0) fail(TNS_E_INVALID_ARG, "n must be >= 0");
        if (n > 0 && (!bits || !amps)) fail(TNS_E_INVALID_ARG, "bits or amps is NULL");
        if (ctx->device < 0) fail(TNS_E_NO_DEVICE, "planning-only context cannot serve");
        if (!plan->on_device || plan->ctx != ctx) fail(TNS_E_INVALID_ARG, "plan was not created on this context");
        for (int64_t i = 0; i < n * plan->circ.n; ++i)
            if (bits[i] > 1) fail(TNS_E_INVALID_ARG, "bits must be 0 or 1");
        {
            std::lock_guard<std::mutex> lk(ctx->mu);
            if (!ctx->server) {
                ctx->server = new Server();
                ctx->server->start(ctx, ctx->serving_workers > 0 ? ctx->serving_workers : 3);
                // the synchronous workspace may have grown to the whole budget;
                // from now on it keeps a quarter and the workers share the rest
                if ((uint64_t)ctx->ws.bytes > ctx->server->sync_budget) {
                    hip_check(hipSetDevice(ctx->device), "hipSetDevice");
                    ctx->ws.release(ctx, ctx->stream);
                }
            }
        }
        Server *sv = ctx->server;
        // admission: one (bitstring, slice) unit must fit the workers' pool
        const uint64_t need = call_workspace_bytes(*plan, 1, 1, sv->pool);
        if (need > sv->pool)
            fail(TNS_E_ADMISSION, "one work unit needs " + std::to_string(need) +
                                      " bytes, the serving pool has " + std::to_string(sv->pool));
        std::unique_ptr<tns_request> r(new tns_request());
        r->plan = plan;
        r->n = n;
        r->bits = bits;
        r->amps = amps;
        r->t_submit = clk::now();
        if (n == 0) {
            r->done = true;
            r->t_start = r->t_end = r->t_submit;
            *out = r.release();
            return;
        }
        shape_items(r.get(), *sv, ctx->serving_item_flops);
        if (r->n_schunks > 1)
            r->part.assign((size_t)(n * r->n_schunks * plan->out_per_unit * 2), 0.0);
        tns_request *raw = r.release();
        sv->submit(raw);
        *out = raw;
    });
}

tns_status tns_serving_configure(tns_ctx *ctx, int32_t n_workers, double item_flops) {
    return guard([&] {
        if (!ctx) fail(TNS_E_INVALID_ARG, "ctx is NULL");
        if (n_workers < 0 || n_workers > 16) fail(TNS_E_INVALID_ARG, "n_workers must be 0..16");
        if (!(item_flops >= 0)) fail(TNS_E_INVALID_ARG, "item_flops must be >= 0");
        std::lock_guard<std::mutex> lk(ctx->mu);
        if (ctx->server) fail(TNS_E_INVALID_ARG, "serving already started on this context");
        ctx->serving_workers = n_workers;
        ctx->serving_item_flops = item_flops;
    });
}

tns_status tns_poll(tns_request *r, int *done) {
    return guard([&] {
        if (!r || !done) fail(TNS_E_INVALID_ARG, "NULL argument");
        std::lock_guard<std::mutex> lk(r->m);
        *done = r->done ? 1 : 0;
    });
}

tns_status tns_wait(tns_request *r) {
    if (!r) {
        set_last_error("request is NULL");
        return TNS_E_INVALID_ARG;
    }
    std::unique_lock<std::mutex> lk(r->m);
    r->cv.wait(lk, [&] { return r->done; });
    if (r->status != TNS_OK) set_last_error(r->error);
    return r->status;
}

tns_status tns_cancel(tns_request *r) {
    return guard([&] {
        if (!r) fail(TNS_E_INVALID_ARG, "request is NULL");
        if (r->plan && r->plan->ctx && r->plan->ctx->server) r->plan->ctx->server->cancel(r);
        else r->cancel = 1;
    });
}

tns_status tns_request_free(tns_request *r) {
    if (!r) return TNS_OK;
    (void)tns_wait(r);
    delete r;
    return TNS_OK;
}

tns_status tns_request_latency(const tns_request *r, double *ms_total, double *ms_run) {
    return guard([&] {
        if (!r) fail(TNS_E_INVALID_ARG, "request is NULL");
        auto *rr = const_cast<tns_request *>(r);
        std::lock_guard<std::mutex> lk(rr->m);
        if (!r->done) fail(TNS_E_INVALID_ARG, "request not finished");
        if (ms_total) *ms_total = std::chrono::duration<double, std::milli>(r->t_end - r->t_submit).count();
        if (ms_run) *ms_run = std::chrono::duration<double, std::milli>(r->t_end - r->t_start).count();
    });
}

tns_status tns_path_search(int32_t n, int32_t n_edges, const int32_t *edges, const double *dims,
                           int32_t mode, int32_t max_rank, int32_t assumptions, int64_t max_states,
                           double max_intermediate, int32_t *path_out, double *score_out) {
    return guard([&] {
        if (n < 1 || n > TNS_MAX_QUBITS) fail(TNS_E_INVALID_ARG, "n out of range");
        if (n_edges < 0 || (n_edges > 0 && (!edges || !dims)) || !path_out)
            fail(TNS_E_INVALID_ARG, "NULL argument");
        std::vector<std::pair<int, int>> E;
        std::vector<double> D;
        for (int e = 0; e < n_edges; ++e) {
            int a = edges[2 * e], b = edges[2 * e + 1];
            if (a < 0 || b < 0 || a >= n || b >= n || a == b) fail(TNS_E_INVALID_ARG, "bad edge");
            if (!(dims[e] >= 1.0)) fail(TNS_E_INVALID_ARG, "bond dimensions must be >= 1");
            E.push_back({a, b});
            D.push_back(dims[e]);
        }
        if (mode != TNS_PATH_GREEDY && mode != TNS_PATH_ALGORITHM1) fail(TNS_E_INVALID_ARG, "unknown mode");
        if (!(max_intermediate >= 0)) fail(TNS_E_INVALID_ARG, "max_intermediate must be >= 0");
        PathResult r = path_search(n, E, D, mode, max_rank, assumptions != 0, max_states, max_intermediate);
        if (max_intermediate > 0 && mode == TNS_PATH_ALGORITHM1 && r.peak > max_intermediate * (1 + 1e-12))
            fail(TNS_E_BAD_PATH, "no path found with every intermediate within max_intermediate");
        for (int i = 0; i < n; ++i) path_out[i] = r.order[i];
        if (score_out) *score_out = r.score;
    });
}

}  // extern "C"
