// Request server for streams of Stokes solves (ensembles, inversion sweeps):
// requests of different mesh levels and viscosity fields arrive over time,
// are admitted into solver slots while memory allows, and advance together.
//
// * Every configured level keeps its mesh hierarchy resident and owns one
//   lockstep batch of solver slots (SolverBatch), one HIP stream and one host
//   driver thread: each step of the driver runs one FGMRES iteration of every
//   running slot of the level, every kernel launched once for all of them
//   (grid x slots), and levels overlap on the device through their streams.
// * A slot is one arena of device memory holding a whole solver (multigrid
//   hierarchy, Krylov basis, scratch); its size is measured once, when the
//   server is created, by building one slot.
// * Admission is FIFO per level at step boundaries: a queued request starts
//   in an idle slot of its level, or in a new slot while the budget allows;
//   a level with no slot at all may have an idle slot of another level (with
//   an empty queue) released to make room.  Finished slots take the next
//   queued request at the next step boundary.
// Each request solves the Stokes problem with eta = exp(-ln(contrast) T) and
// the buoyancy right-hand side Ra T rhat in the solver options' precision.
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>

#include "batch.hpp"
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

struct ServerLevel {
    int mt = 0, nr = 0;
    tng_mesh* mesh = nullptr;
    hipStream_t stream = nullptr;
    tng_ctx* ctx = nullptr;
    std::unique_ptr<tng::SolverBatch> batch;   // touched only by the driver thread (after creation)
    std::vector<ServerReq*> job;               // request of every slot (nullptr: idle); guarded by srv->mu
    std::deque<ServerReq*> queue;
    long long bytes_per_slot = -1;
    int cap_slots = 0;                         // max_slots, lowered if the device refuses a slot
    int release_wanted = 0;                    // idle slots another level asked this one to free
    bool room_asked = false;                   // this level has asked the others for room since
                                               // the slots last changed (no repeated asking)
    int failed = TNG_OK;                       // the level's stream failed: no further requests
    std::thread driver;
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
    bool stop = false;
};

namespace tng {
namespace {

int live_slots(const ServerLevel& lv) { return (int)lv.job.size(); }

int idle_index(const ServerLevel& lv) {
    for (size_t i = 0; i < lv.job.size(); ++i)
        if (lv.job[i] == nullptr) return (int)i;
    return -1;
}

// A queued request of lv could start now (lock held).
bool admissible(const tng_server* srv, const ServerLevel& lv) {
    if (lv.queue.empty()) return false;
    if (idle_index(lv) >= 0) return true;
    return live_slots(lv) < lv.cap_slots && lv.bytes_per_slot <= (long long)srv->budget - srv->bytes_in_use;
}

// lv has queued work but no slot and no room for one, and has not asked the
// other levels for room since the slots last changed (lock held).
bool wants_room(const tng_server* srv, const ServerLevel& lv) {
    return !lv.queue.empty() && lv.failed == TNG_OK && live_slots(lv) == 0 && lv.cap_slots > 0 && !lv.room_asked &&
           lv.bytes_per_slot > (long long)srv->budget - srv->bytes_in_use;
}

// Slots changed (some became idle or were freed): levels waiting for room may ask again.
void slots_changed(tng_server* srv) {
    for (auto& other : srv->levels) other.room_asked = false;
    srv->cv_work.notify_all();
}

// Asks another level to free an idle slot for lv, which has none (lock held).
void request_room(tng_server* srv, ServerLevel& lv) {
    lv.room_asked = true;
    if (live_slots(lv) != 0) return;
    for (auto& other : srv->levels) {
        if (&other == &lv || !other.queue.empty() || other.release_wanted > 0 || other.failed != TNG_OK) continue;
        if (idle_index(other) >= 0) {
            other.release_wanted += 1;
            srv->cv_work.notify_all();
            return;
        }
    }
}

void complete(tng_server* srv, ServerReq* r, int rc, const tng_solve_info& info) {
    r->rc = rc;
    r->info = info;
    r->t_done = Clock::now();
    r->done = true;
    srv->busy -= 1;
}

void driver(tng_server* srv, ServerLevel* lv) {
    (void)hipSetDevice(lv->ctx->device);
    SolverBatch& B = *lv->batch;
    std::unique_lock<std::mutex> lk(srv->mu);
    for (;;) {
        srv->cv_work.wait(lk, [&] {
            return srv->stop || B.running() > 0 || lv->release_wanted > 0 || admissible(srv, *lv) ||
                   wants_room(srv, *lv);
        });
        if (srv->stop && B.running() == 0) return;
        // a level without slots whose request cannot fit asks the others to release an idle one
        if (wants_room(srv, *lv)) request_room(srv, *lv);
        // free idle slots another level is waiting for
        while (lv->release_wanted > 0) {
            lv->release_wanted -= 1;
            const int i = idle_index(*lv);
            if (i < 0) break;
            lk.unlock();
            bool freed = true;
            try {
                B.remove_slot(i);
            } catch (const Error&) {
                freed = false;
            }
            lk.lock();
            if (freed) {
                lv->job.erase(lv->job.begin() + i);
                srv->bytes_in_use -= lv->bytes_per_slot;
            }
            slots_changed(srv);
        }
        // admit queued requests at this step boundary
        while (!srv->stop && !lv->queue.empty()) {
            int i = idle_index(*lv);
            if (i < 0) {
                if (live_slots(*lv) >= lv->cap_slots) break;
                if (lv->bytes_per_slot > (long long)srv->budget - srv->bytes_in_use) {
                    request_room(srv, *lv);
                    break;
                }
                srv->bytes_in_use += lv->bytes_per_slot;
                lk.unlock();
                int added = -1;
                try {
                    added = B.add_slot();
                } catch (const Error&) {
                    added = -1;
                }
                lk.lock();
                if (added < 0) {
                    // the device has no room for another slot: this level keeps the slots it has
                    srv->bytes_in_use -= lv->bytes_per_slot;
                    lv->cap_slots = live_slots(*lv);
                    if (lv->cap_slots == 0) {
                        while (!lv->queue.empty()) {
                            ServerReq* r = lv->queue.front();
                            lv->queue.pop_front();
                            r->t_start = Clock::now();
                            tng_solve_info info{};
                            info.status = TNG_E_NOMEM;
                            complete(srv, r, TNG_E_NOMEM, info);
                        }
                        srv->cv_done.notify_all();
                    }
                    break;
                }
                lv->job.push_back(nullptr);
                i = added;
            }
            ServerReq* r = lv->queue.front();
            lv->queue.pop_front();
            lv->job[i] = r;
            lk.unlock();
            r->t_start = Clock::now();
            const double E = std::log(10.0) * r->contrast_log10;
            bool running = false;
            try {
                running = B.start(i, r->T, E, r->Ra, r->u, r->p);
            } catch (const Error&) {
                running = false;
            }
            lk.lock();
            if (!running) {
                complete(srv, r, B.rc(i), B.info(i));
                lv->job[i] = nullptr;
                srv->cv_done.notify_all();
            }
        }
        if (B.running() == 0) continue;
        lk.unlock();
        std::vector<int> fin;
        int err = TNG_OK;
        try {
            fin = B.step();
        } catch (const Error& e) {
            err = e.code;
        }
        lk.lock();
        if (err != TNG_OK) {
            // the stream itself failed: end every running and queued request of the level,
            // and refuse later ones
            tng_solve_info info{};
            info.status = err;
            for (size_t i = 0; i < lv->job.size(); ++i)
                if (lv->job[i]) {
                    complete(srv, lv->job[i], err, info);
                    lv->job[i] = nullptr;
                }
            while (!lv->queue.empty()) {
                ServerReq* r = lv->queue.front();
                lv->queue.pop_front();
                r->t_start = Clock::now();
                complete(srv, r, err, info);
            }
            lv->failed = err;
            srv->cv_done.notify_all();
            srv->cv_work.notify_all();
            return;
        }
        for (int i : fin) {
            complete(srv, lv->job[i], B.rc(i), B.info(i));
            lv->job[i] = nullptr;
        }
        if (!fin.empty()) {
            srv->cv_done.notify_all();
            slots_changed(srv);   // idle slots: a level waiting for room may ask again
        }
    }
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
    auto cleanup = [&](int upto) {
        for (int k = 0; k < upto; ++k) {
            ServerLevel& lv = srv->levels[k];
            lv.batch.reset();
            if (lv.ctx) tng_ctx_destroy(lv.ctx);
            if (lv.stream) (void)hipStreamDestroy(lv.stream);
            if (lv.mesh) tng_mesh_destroy(lv.mesh);
        }
    };
    for (int i = 0; i < nlevels; ++i) {
        ServerLevel& lv = srv->levels[i];
        lv.mt = levels[2 * i];
        lv.nr = levels[2 * i + 1];
        try {
            int nl = 1;
            while ((lv.mt >> nl) >= 2 && (lv.nr >> nl) >= 2 && ((lv.nr >> nl) << nl) == lv.nr) ++nl;
            if (tng_mesh_create(ctx, lv.mt, lv.nr, 0.55, 1.0, nl, &lv.mesh) != TNG_OK)
                throw Error(TNG_E_INVAL, std::string("server level mesh: ") + tng_last_error());
            TNG_HIP(hipStreamCreate(&lv.stream));   // default priority
            if (tng_ctx_create(ctx->device, lv.stream, &lv.ctx) != TNG_OK)
                throw Error(TNG_E_HIP, "level context creation failed");
            lv.ctx->profile = ctx->profile;
            lv.batch = std::make_unique<tng::SolverBatch>(lv.ctx, lv.mesh, *opts);
            lv.bytes_per_slot = lv.batch->slot_bytes();
            lv.cap_slots = max_slots;
        } catch (...) {
            cleanup(i + 1);
            throw;
        }
    }
    for (auto& lv : srv->levels) lv.driver = std::thread(tng::driver, srv.get(), &lv);
    *out = srv.release();
    TNG_API_END
}

int tng_server_submit(tng_server* srv, int level_idx, const double* T, double log10_contrast, double Ra,
                      double* const u_out[3], double* p_out, long long* ticket) {
    TNG_API_BEGIN
    TNG_REQUIRE(srv && T && u_out && u_out[0] && u_out[1] && u_out[2] && p_out && ticket, "NULL argument");
    TNG_REQUIRE(level_idx >= 0 && level_idx < (int)srv->levels.size(), "level_idx out of range");
    {
        const tng::Level& L = srv->levels[level_idx].mesh->lv[0];
        const tng::Level& Lp = srv->levels[level_idx].mesh->lv[1];
        const size_t nsb = (size_t)L.node_slots() * sizeof(double);
        tng::require_device(srv->ctx, T, nsb, "T");
        for (int c = 0; c < 3; ++c) tng::require_device(srv->ctx, u_out[c], nsb, "u_out");
        tng::require_device(srv->ctx, p_out, (size_t)Lp.node_slots() * sizeof(double), "p_out");
    }
    std::lock_guard<std::mutex> lk(srv->mu);
    ServerLevel& lv = srv->levels[level_idx];
    if (lv.failed != TNG_OK) throw Error(lv.failed, "this level's device stream failed; it takes no requests");
    if (lv.bytes_per_slot > (long long)srv->budget)
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
    srv->busy += 1;
    *ticket = r->ticket;
    srv->reqs.emplace(r->ticket, std::move(r));
    srv->cv_work.notify_all();
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
        srv->cv_done.wait(lk, [&] { return srv->busy == 0; });
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
    int ns = 0, nq = 0, running = 0;
    for (auto& lv : srv->levels) {
        ns += (int)lv.job.size();
        nq += (int)lv.queue.size();
        for (auto* j : lv.job) running += j ? 1 : 0;
    }
    if (bytes_in_use) *bytes_in_use = srv->bytes_in_use;
    if (slots) *slots = ns;
    if (busy) *busy = running;
    if (queued) *queued = nq;
    TNG_API_END
}

int tng_server_destroy(tng_server* srv) {
    TNG_API_BEGIN
    if (!srv) return TNG_OK;
    {
        std::unique_lock<std::mutex> lk(srv->mu);
        // queued requests are dropped; running ones finish
        for (auto& lv : srv->levels) {
            srv->busy -= (int)lv.queue.size();
            lv.queue.clear();
        }
        srv->stop = true;
        srv->cv_work.notify_all();
    }
    for (auto& lv : srv->levels)
        if (lv.driver.joinable()) lv.driver.join();
    for (auto& lv : srv->levels) {
        lv.batch.reset();
        tng_ctx_destroy(lv.ctx);
        if (lv.stream) (void)hipStreamDestroy(lv.stream);
        tng_mesh_destroy(lv.mesh);
    }
    delete srv;
    TNG_API_END
}

}  // extern "C"
