// Request server for streams of Stokes solves (ensembles, inversion sweeps):
// requests of different mesh levels and viscosity fields arrive over time,
// are admitted into solver slots while memory allows, and run concurrently
// on the device.
//
// * Every configured level keeps its mesh hierarchy resident.
// * A slot is a solver instance (multigrid hierarchy, Krylov basis, scratch)
//   with its own context, HIP stream and host worker thread; slots of a level
//   are reused for later requests of that level.
// * Admission is FIFO per level: a queued request starts as soon as its level
//   has an idle slot, or a new slot fits in the HBM budget.  The memory model
//   of a level is measured once, when the server is created, by building one
//   slot and counting the device bytes allocated for it.
// * Requests of all slots overlap on the device through their streams; a
//   finished slot takes the next queued request of its level immediately.
// Each request solves the Stokes problem with eta = exp(-ln(contrast) T) and
// the buoyancy right-hand side Ra T rhat in mixed precision.
#include <atomic>
#include <climits>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>

#include "mg.hpp"

using Clock = std::chrono::steady_clock;

struct ServerReq {
    long long ticket;
    int level;
    const double* T;
    double contrast_log10;
    double Ra;
    double* u[3];
    double* p;
    Clock::time_point t_submit, t_start, t_done;
    int rc = TNG_OK;
    tng_solve_info info{};
    bool done = false;
};

struct ServerSlot;

struct ServerLevel {
    int mt, nr;
    tng_mesh* mesh = nullptr;
    std::vector<std::unique_ptr<ServerSlot>> slots;
    std::deque<ServerReq*> queue;
    long long bytes_per_slot = -1;      // measured at server creation
};

struct ServerSlot {
    tng_server* srv = nullptr;
    int level = 0;
    const tng_mesh* mesh = nullptr;
    tng_ctx* ctx = nullptr;
    hipStream_t stream = nullptr;
    tng_solver* solver = nullptr;
    tng::DevBuf<double> eta, f;
    std::thread th;
    ServerReq* job = nullptr;           // guarded by srv->mu
    bool stop = false;
    bool retire = false;                // free the slot's memory for another level
    bool dead = false;
};

struct tng_server {
    tng_ctx* ctx = nullptr;
    tng_solver_opts opts{};
    size_t budget = 0;
    int max_slots = 0;
    std::deque<ServerLevel> levels;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::map<long long, std::unique_ptr<ServerReq>> reqs;
    long long next_ticket = 1;
    long long bytes_in_use = 0;
    int busy = 0;
    std::string last_error;
};

namespace tng {
namespace {

void dispatch(tng_server* srv);

void run_request(ServerSlot* s, ServerReq* r) {
    const tng::Level& L = s->mesh->lv[0];
    const long long ns = L.node_slots();
    const double E = std::log(10.0) * r->contrast_log10;
    launch_eta_from_T(s->ctx, L, TNG_F64, r->T, s->eta.p, E, 0.0);
    double* f[3] = {s->f.p, s->f.p + ns, s->f.p + 2 * ns};
    energy_buoyancy(s->ctx, L, r->T, r->Ra, f);
    const double* fc[3] = {f[0], f[1], f[2]};
    r->rc = tng_stokes_solve(s->solver, s->eta.p, fc, nullptr, r->u, r->p, &r->info);
}

void worker(ServerSlot* s) {
    tng_server* srv = s->srv;
    (void)hipSetDevice(s->ctx->device);
    std::unique_lock<std::mutex> lk(srv->mu);
    for (;;) {
        srv->cv_work.wait(lk, [&] { return s->stop || s->retire || s->job != nullptr; });
        if (s->job == nullptr && s->retire) {
            // give the memory back and let the dispatcher admit other levels
            tng_solver* sv = s->solver;
            s->solver = nullptr;
            lk.unlock();
            tng_stokes_solver_destroy(sv);
            s->eta.release();
            s->f.release();
            (void)hipStreamSynchronize(s->stream);
            lk.lock();
            s->dead = true;
            srv->bytes_in_use -= srv->levels[s->level].bytes_per_slot;
            tng::dispatch(srv);
            srv->cv_done.notify_all();
            return;
        }
        if (s->job == nullptr && s->stop) return;
        ServerReq* r = s->job;
        lk.unlock();
        r->t_start = Clock::now();
        try {
            run_request(s, r);
        } catch (const tng::Error& e) {
            r->rc = e.code;
        } catch (...) {
            r->rc = TNG_E_INVAL;
        }
        r->t_done = Clock::now();
        lk.lock();
        r->done = true;
        s->job = nullptr;
        srv->busy -= 1;
        // take the next queued request of this level right away
        ServerLevel& lv = srv->levels[s->level];
        if (!lv.queue.empty() && !s->stop && !s->retire) {
            s->job = lv.queue.front();
            lv.queue.pop_front();
            srv->busy += 1;
        }
        srv->cv_done.notify_all();
        srv->cv_work.notify_all();
    }
}

// Creates a slot for level li (called with the lock held).
ServerSlot* make_slot(tng_server* srv, int li) {
    ServerLevel& lv = srv->levels[li];
    auto slot = std::make_unique<ServerSlot>();
    slot->srv = srv;
    slot->level = li;
    slot->mesh = lv.mesh;
    TNG_HIP(hipStreamCreate(&slot->stream));   // default priority
    if (tng_ctx_create(srv->ctx->device, slot->stream, &slot->ctx) != TNG_OK)
        throw Error(TNG_E_HIP, "slot context creation failed");
    const int rc = tng_stokes_solver_create(slot->ctx, lv.mesh, &srv->opts, &slot->solver);
    if (rc != TNG_OK) throw Error(rc, std::string("slot solver creation failed: ") + tng_last_error());
    const tng::Level& L = lv.mesh->lv[0];
    slot->eta.alloc(2 * L.cells());
    slot->f.alloc(3 * L.node_slots());
    srv->bytes_in_use += lv.bytes_per_slot;
    ServerSlot* raw = slot.get();
    lv.slots.push_back(std::move(slot));
    raw->th = std::thread(worker, raw);
    return raw;
}

// Device bytes of one slot of level li: a slot is built and released once,
// counting what this thread allocates for it.  A level whose slot cannot be
// allocated at all is given an unbounded cost and refuses every request.
long long measure_slot_bytes(tng_server* srv, ServerLevel& lv) {
    const long long before = tl_device_bytes;
    long long cost = LLONG_MAX;
    tng_solver* sv = nullptr;
    if (tng_stokes_solver_create(srv->ctx, lv.mesh, &srv->opts, &sv) == TNG_OK) {
        try {
            const tng::Level& L = lv.mesh->lv[0];
            DevBuf<double> eta(2 * L.cells()), f(3 * L.node_slots());
            cost = std::max(tl_device_bytes - before, 1LL);
        } catch (const Error&) {
        }
        tng_stokes_solver_destroy(sv);
    }
    return cost;
}

// Admits queued requests (lock held).
void dispatch(tng_server* srv) {
    for (size_t li = 0; li < srv->levels.size(); ++li) {
        ServerLevel& lv = srv->levels[li];
        while (!lv.queue.empty()) {
            ServerSlot* idle = nullptr;
            int live = 0;
            for (auto& sl : lv.slots) {
                if (sl->dead || sl->retire) continue;
                ++live;
                if (!idle && sl->job == nullptr) idle = sl.get();
            }
            if (!idle) {
                if (live >= srv->max_slots) break;
                if (lv.bytes_per_slot > (long long)srv->budget - srv->bytes_in_use) {
                    // an idle slot of another level may be retired to make room
                    if (live == 0) {
                        for (auto& other : srv->levels) {
                            if (&other == &lv) continue;
                            for (auto& sl : other.slots)
                                if (!sl->dead && !sl->retire && sl->job == nullptr && other.queue.empty()) {
                                    sl->retire = true;
                                    srv->cv_work.notify_all();
                                    return;   // the retiring worker calls dispatch again
                                }
                        }
                    }
                    break;
                }
                idle = make_slot(srv, (int)li);
            }
            idle->job = lv.queue.front();
            lv.queue.pop_front();
            srv->busy += 1;
        }
    }
    srv->cv_work.notify_all();
}

}  // namespace
}  // namespace tng

using tng::Error;

extern "C" {

int tng_server_create(tng_ctx* ctx, const int* levels, int nlevels, size_t hbm_budget_bytes, int max_slots,
                      const tng_solver_opts* opts, tng_server** out) {
    TNG_API_BEGIN
    TNG_REQUIRE(ctx && levels && opts && out && nlevels >= 1, "NULL argument or no levels");
    TNG_REQUIRE(max_slots >= 1, "max_slots must be >= 1");
    auto srv = std::make_unique<tng_server>();
    srv->ctx = ctx;
    srv->opts = *opts;
    srv->budget = hbm_budget_bytes;
    srv->max_slots = max_slots;
    srv->levels.resize(nlevels);
    for (int i = 0; i < nlevels; ++i) {
        ServerLevel& lv = srv->levels[i];
        lv.mt = levels[2 * i];
        lv.nr = levels[2 * i + 1];
        int nl = 1;
        while ((lv.mt >> nl) >= 2 && (lv.nr >> nl) >= 2 && ((lv.nr >> nl) << nl) == lv.nr) ++nl;
        const int rc = tng_mesh_create(ctx, lv.mt, lv.nr, 0.55, 1.0, nl, &lv.mesh);
        if (rc != TNG_OK) {
            for (int k = 0; k < i; ++k) tng_mesh_destroy(srv->levels[k].mesh);
            throw Error(rc, std::string("server level mesh: ") + tng_last_error());
        }
        lv.bytes_per_slot = tng::measure_slot_bytes(srv.get(), lv);
    }
    *out = srv.release();
    TNG_API_END
}

int tng_server_submit(tng_server* srv, int level_idx, const double* T, double log10_contrast, double Ra,
                      double* const u_out[3], double* p_out, long long* ticket) {
    TNG_API_BEGIN
    TNG_REQUIRE(srv && T && u_out && u_out[0] && u_out[1] && u_out[2] && p_out && ticket, "NULL argument");
    TNG_REQUIRE(level_idx >= 0 && level_idx < (int)srv->levels.size(), "level_idx out of range");
    std::lock_guard<std::mutex> lk(srv->mu);
    ServerLevel& lv = srv->levels[level_idx];
    if (lv.slots.empty() && lv.bytes_per_slot > (long long)srv->budget)
        throw Error(TNG_E_BUDGET, "request does not fit the HBM budget (a slot of this level needs " +
                                      std::to_string(lv.bytes_per_slot) + " bytes, budget " +
                                      std::to_string(srv->budget) + ")");
    auto r = std::make_unique<ServerReq>();
    r->ticket = srv->next_ticket++;
    r->level = level_idx;
    r->T = T;
    r->contrast_log10 = log10_contrast;
    r->Ra = Ra;
    for (int c = 0; c < 3; ++c) r->u[c] = u_out[c];
    r->p = p_out;
    r->t_submit = Clock::now();
    lv.queue.push_back(r.get());
    *ticket = r->ticket;
    srv->reqs.emplace(r->ticket, std::move(r));
    tng::dispatch(srv);
    TNG_API_END
}

int tng_server_poll(tng_server* srv, long long ticket, int* done, tng_solve_info* info, double* latency_s,
                    double* queue_s) {
    TNG_API_BEGIN
    TNG_REQUIRE(srv && done, "NULL argument");
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->reqs.find(ticket);
    TNG_REQUIRE(it != srv->reqs.end(), "unknown ticket");
    ServerReq* r = it->second.get();
    *done = r->done ? 1 : 0;
    if (r->done) {
        if (info) *info = r->info;
        if (latency_s) *latency_s = std::chrono::duration<double>(r->t_done - r->t_submit).count();
        if (queue_s) *queue_s = std::chrono::duration<double>(r->t_start - r->t_submit).count();
        if (r->rc != TNG_OK) {
            tng::set_last_error("request failed");
            return r->rc;
        }
    }
    TNG_API_END
}

int tng_server_wait(tng_server* srv, long long ticket) {
    TNG_API_BEGIN
    TNG_REQUIRE(srv, "NULL server");
    std::unique_lock<std::mutex> lk(srv->mu);
    if (ticket <= 0) {
        srv->cv_done.wait(lk, [&] {
            if (srv->busy != 0) return false;
            for (auto& lv : srv->levels)
                if (!lv.queue.empty()) return false;
            return true;
        });
    } else {
        auto it = srv->reqs.find(ticket);
        TNG_REQUIRE(it != srv->reqs.end(), "unknown ticket");
        ServerReq* r = it->second.get();
        srv->cv_done.wait(lk, [&] { return r->done; });
    }
    TNG_API_END
}

int tng_server_stats(tng_server* srv, long long* bytes_in_use, int* slots, int* busy, int* queued) {
    TNG_API_BEGIN
    TNG_REQUIRE(srv, "NULL server");
    std::lock_guard<std::mutex> lk(srv->mu);
    int ns = 0, nq = 0;
    for (auto& lv : srv->levels) {
        ns += (int)lv.slots.size();
        nq += (int)lv.queue.size();
    }
    if (bytes_in_use) *bytes_in_use = srv->bytes_in_use;
    if (slots) *slots = ns;
    if (busy) *busy = srv->busy;
    if (queued) *queued = nq;
    TNG_API_END
}

int tng_server_destroy(tng_server* srv) {
    TNG_API_BEGIN
    if (!srv) return TNG_OK;
    {
        std::unique_lock<std::mutex> lk(srv->mu);
        srv->cv_done.wait(lk, [&] { return srv->busy == 0; });
        for (auto& lv : srv->levels) {
            lv.queue.clear();
            for (auto& sl : lv.slots) sl->stop = true;
        }
        srv->cv_work.notify_all();
    }
    for (auto& lv : srv->levels) {
        for (auto& sl : lv.slots) {
            if (sl->th.joinable()) sl->th.join();
            if (sl->solver) tng_stokes_solver_destroy(sl->solver);
            sl->eta.release();
            sl->f.release();
            tng_ctx_destroy(sl->ctx);
            if (sl->stream) (void)hipStreamDestroy(sl->stream);
        }
        lv.slots.clear();
        tng_mesh_destroy(lv.mesh);
    }
    delete srv;
    TNG_API_END
}

}  // extern "C"
