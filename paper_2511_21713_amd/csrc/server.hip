// Continuous-batching server for Poisson-Boltzmann solves.
//
// Requests (problems with mesh, charges and parameters set) are queued by
// pbfb_server_submit.  An admission step moves them into the running set when
// a slot is free and their estimated device footprint fits in the HBM budget.
// A setup worker (own thread, own stream) assembles each admitted instance
// while the running set keeps iterating on the solve stream, so setup and the
// batched Krylov iterations of other requests overlap on the device.  Ready
// instances join the running set at the next Newton-step boundary; every
// round advances each running instance to its next linear solve and then runs
// one batched GMRES over all of them.  Finished requests release their slot
// and budget.  The per-instance arithmetic (work lists, reduction orders) does
// not depend on the other members of the batch, so a request's result is the
// same bit for bit alone or in any mix.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>

#include "pbfb_internal.hpp"

namespace pbfb {

int64_t bem_ld(int64_t nv);

// Device bytes an instance holds while solving, and the assembly workspace it
// needs while its dense operators are assembled (the mirrored double layer of
// a square-tile assembly, nv x nv in the storage precision, vertex
// coordinates and touching-pair blocks).
void footprint_estimate(const Problem &p, int restart, size_t *steady, size_t *setup_extra)
{
    const size_t elem = p.precision == PBFB_MIXED ? 4 : 8;
    size_t dense = 0, tmp = 0;
    for (int w = 0; w < 2 && p.bem_mf; ++w) {
        // matrix-free: touching-pair blocks, the apply's strength buffers and
        // the near-field rows of the preconditioner (~40 per vertex)
        const SurfaceTopo &T = p.topo[w];
        dense += T.tp_sig.size() * 18 * 8 + size_t(T.nt) * 15 * 8 + size_t(T.nv) * 40 * 16;
        tmp = std::max(tmp, size_t(T.nv) * 3 * 8);
    }
    for (int w = 0; w < NSURF && !p.bem_mf; ++w) {
        if (w == 2 && p.gm() != 2) continue; // the independent Gamma_m mesh: only when it is used
        const SurfaceTopo &T = p.topo[w];
        dense += size_t(T.nv) * bem_ld(T.nv) * elem;
        dense += size_t(sym_partials_doubles(T.nv)) * 8 + size_t(T.nv) * 20 * 12; // symmetric use: partials, Delta
        dense += size_t(T.nt) * 18 * 8 * 2 + size_t(T.nv) * (8 * 8 + 16 * 4);  // Morton copies, block tables, rings
        tmp = std::max(tmp, (size_t(T.nv) * T.nv * elem + 255) / 256 * 256 + size_t(T.nv) * 3 * 8 +
                                T.tp_sig.size() * 18 * 8 + 64);
    }
    const size_t n = size_t(p.n());
    const size_t nnz_est = size_t(p.ntet) * 3 + size_t(p.nn) * 4; // generous: ~14 per row
    const size_t csr = nnz_est * (4 + 8 + 8 + (p.precision == PBFB_MIXED ? 4 : 0)) + size_t(p.nn) * 8;
    const size_t fem = size_t(p.ntet) * (16 * 8 + 16 + 16 * 4) + size_t(p.nn) * 12;
    const size_t vec = n * 8 * (size_t(restart) + 1 + 16);
    *steady = dense + csr + fem + vec + (size_t(64) << 20);
    *setup_extra = tmp;
}

struct Request {
    uint64_t ticket;
    Problem *p;
    pbfb_solve_opts o;
    pbfb_result res{};
    size_t steady = 0, extra = 0;
    NewtonRun *run = nullptr;
    bool done = false;
    std::string message;
    std::chrono::steady_clock::time_point t_submit, t_admit;
};

struct Server {
    Ctx *ctx = nullptr;
    // used: steady footprints of the admitted, unfinished requests; ws_need: the
    // largest assembly workspace any admitted request needs (the context's
    // workspace grows to it and is kept, so it is charged once, never released)
    size_t budget = 0, used = 0, ws_need = 0;
    int max_slots = 1;
    hipStream_t s_solve = nullptr, s_setup = nullptr;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<Request *> pending;           // submitted, not admitted
    std::deque<Request *> to_setup;          // admitted, waiting for the setup worker
    std::deque<Request *> ready;             // set up, waiting to join the running set
    std::vector<Request *> running;
    std::map<uint64_t, Request *> all;
    uint64_t next_ticket = 1;
    int in_flight = 0; // admitted and not finished
    bool stop = false;
    std::thread solve_thread, setup_thread;
    std::string error;

    // device bytes charged for the shared assembly workspace if r were admitted
    size_t ws_with(const Request *r) const
    {
        return std::max(std::max(ws_need, r->extra), ctx->ws_held());
    }

    void admit_locked()
    {
        while (!pending.empty() && in_flight < max_slots) {
            Request *r = pending.front();
            if (used + r->steady + ws_with(r) > budget && in_flight > 0) break; // wait for memory
            pending.pop_front();
            ws_need = ws_with(r);
            used += r->steady;
            ++in_flight;
            r->t_admit = std::chrono::steady_clock::now();
            r->res.t_wait_s = std::chrono::duration<double>(r->t_admit - r->t_submit).count();
            to_setup.push_back(r);
        }
    }

    void setup_loop()
    {
        PB_HIP(hipSetDevice(ctx->device));
        for (;;) {
            Request *r = nullptr;
            {
                std::unique_lock<std::mutex> lk(mu);
                cv.wait(lk, [&] { return !to_setup.empty() || (stop && pending.empty()); });
                if (to_setup.empty()) return; // stopping and nothing left to admit
                r = to_setup.front();
                to_setup.pop_front();
            }
            const double wait = r->res.t_wait_s;
            r->run = new NewtonRun(r->p, r->o, &r->res, nullptr);
            r->res.t_wait_s = wait;
            // the setup part of the state machine: assembly, linear-solve request
            try {
                ensure_all(*r->p, s_setup);
                PB_HIP(hipStreamSynchronize(s_setup));
            } catch (const Error &e) {
                r->run->status = e.code;
                r->message = e.msg;
            }
            std::lock_guard<std::mutex> lk(mu);
            ready.push_back(r);
            cv.notify_all();
        }
    }

    void complete_locked(Request *r)
    {
        r->done = true;
        // every device allocation of the request (operators, mesh, Krylov and
        // work buffers) is freed before its budget is handed to the next one
        try {
            PB_HIP(hipStreamSynchronize(s_solve));
        } catch (const Error &) {
        }
        release_device_state(*r->p);
        used -= std::min(used, r->steady);
        --in_flight;
        admit_locked();
        cv.notify_all();
    }

    void solve_loop()
    {
        PB_HIP(hipSetDevice(ctx->device));
        std::vector<GmresJob *> jobs;
        for (;;) {
            {
                std::unique_lock<std::mutex> lk(mu);
                cv.wait(lk, [&] {
                    return !ready.empty() || !running.empty() || (stop && pending.empty() && in_flight == 0);
                });
                if (ready.empty() && running.empty()) return; // stopping and drained
                while (!ready.empty()) {
                    Request *r = ready.front();
                    ready.pop_front();
                    if (r->run->status != 0) {
                        r->res.status = pbfb_status(r->run->status);
                        delete r->run;
                        r->run = nullptr;
                        complete_locked(r);
                    } else {
                        running.push_back(r);
                    }
                }
            }
            if (running.empty()) continue;
            jobs.clear();
            std::vector<Request *> finished;
            {
                std::vector<NewtonRun *> runs, done;
                for (Request *r : running) runs.push_back(r->run);
                advance_all(runs, jobs, &done, s_solve);
                for (Request *r : running)
                    if (std::find(done.begin(), done.end(), r->run) != done.end()) finished.push_back(r);
            }
            if (!jobs.empty()) {
                try {
                    batched_gmres(jobs, s_solve);
                } catch (const Error &e) {
                    for (auto *J : jobs) J->status = e.code;
                    error = e.msg;
                }
            }
            if (!finished.empty()) {
                std::lock_guard<std::mutex> lk(mu);
                for (Request *r : finished) {
                    running.erase(std::find(running.begin(), running.end(), r));
                    if (!r->run->message.empty()) r->message = r->run->message;
                    delete r->run;
                    r->run = nullptr;
                    complete_locked(r);
                }
            }
        }
    }
};

} // namespace pbfb

struct pbfb_server {
    pbfb::Server s;
};

using namespace pbfb;

extern "C" {

pbfb_status pbfb_server_create(pbfb_ctx *ctx, size_t hbm_budget_bytes, int max_slots, pbfb_server **out)
{
    try {
        PB_CHECK(ctx && out && max_slots >= 1 && hbm_budget_bytes > 0, PBFB_EINVAL, "bad server arguments");
        PB_HIP(hipSetDevice(ctx->c.device));
        auto *sv = new pbfb_server;
        Server &S = sv->s;
        S.ctx = &ctx->c;
        S.budget = hbm_budget_bytes;
        S.max_slots = max_slots;
        PB_HIP(hipStreamCreateWithFlags(&S.s_solve, hipStreamNonBlocking));
        PB_HIP(hipStreamCreateWithFlags(&S.s_setup, hipStreamNonBlocking));
        S.solve_thread = std::thread([&S] {
            try {
                S.solve_loop();
            } catch (const Error &e) {
                S.error = e.msg;
            }
        });
        S.setup_thread = std::thread([&S] {
            try {
                S.setup_loop();
            } catch (const Error &e) {
                S.error = e.msg;
            }
        });
        *out = sv;
        return PBFB_OK;
    } catch (const Error &e) {
        set_error(e.msg);
        return e.code;
    }
}

pbfb_status pbfb_server_submit(pbfb_server *sv, pbfb_problem *pp, const pbfb_solve_opts *o, uint64_t *ticket)
{
    try {
        PB_CHECK(sv && pp && ticket, PBFB_EINVAL, "null argument");
        Problem &p = pp->p;
        PB_CHECK(p.ctx, PBFB_ESTATE, "the problem's context was destroyed");
        PB_CHECK(p.have_mesh && p.have_charges && p.have_params, PBFB_ESTATE, "problem not fully specified");
        PB_CHECK(p.ctx == sv->s.ctx, PBFB_EINVAL, "problem belongs to another context");
        pbfb_solve_opts O;
        if (o) O = *o;
        else pbfb_solve_opts_default(&O);
        check_opts(O);
        size_t steady = 0, extra = 0;
        footprint_estimate(p, O.gmres_restart, &steady, &extra);
        PB_CHECK(steady + extra <= sv->s.budget, PBFB_ENOMEM, "request exceeds the server's HBM budget");
        auto *r = new Request;
        r->o = O;
        r->p = &p;
        r->steady = steady;
        r->extra = extra;
        r->t_submit = std::chrono::steady_clock::now();
        std::lock_guard<std::mutex> lk(sv->s.mu);
        r->ticket = sv->s.next_ticket++;
        sv->s.all[r->ticket] = r;
        sv->s.pending.push_back(r);
        sv->s.admit_locked();
        sv->s.cv.notify_all();
        *ticket = r->ticket;
        return PBFB_OK;
    } catch (const Error &e) {
        set_error(e.msg);
        return e.code;
    }
}

pbfb_status pbfb_request_footprint(const pbfb_problem *pp, const pbfb_solve_opts *o, size_t *steady_bytes,
                                   size_t *setup_bytes)
{
    try {
        PB_CHECK(pp && steady_bytes && setup_bytes, PBFB_EINVAL, "null argument");
        const Problem &p = pp->p;
        PB_CHECK(p.have_mesh, PBFB_ESTATE, "set_mesh must precede the footprint estimate");
        pbfb_solve_opts O;
        if (o) O = *o;
        else pbfb_solve_opts_default(&O);
        check_opts(O);
        footprint_estimate(p, O.gmres_restart, steady_bytes, setup_bytes);
        return PBFB_OK;
    } catch (const Error &e) {
        set_error(e.msg);
        return e.code;
    }
}

pbfb_status pbfb_server_poll(pbfb_server *sv, uint64_t ticket, int *done, pbfb_result *res)
{
    if (!sv || !done) {
        set_error("null argument");
        return PBFB_EINVAL;
    }
    std::lock_guard<std::mutex> lk(sv->s.mu);
    auto it = sv->s.all.find(ticket);
    if (it == sv->s.all.end()) {
        set_error("unknown ticket");
        return PBFB_EINVAL;
    }
    Request *r = it->second;
    *done = r->done ? 1 : 0;
    if (r->done) {
        if (res) *res = r->res;
        if (!r->message.empty()) set_error(r->message);
    }
    return PBFB_OK;
}

pbfb_status pbfb_server_destroy(pbfb_server *sv)
{
    if (!sv) return PBFB_OK;
    Server &S = sv->s;
    {
        std::lock_guard<std::mutex> lk(S.mu);
        S.stop = true;
        S.cv.notify_all();
    }
    if (S.setup_thread.joinable()) S.setup_thread.join();
    if (S.solve_thread.joinable()) S.solve_thread.join();
    (void)hipStreamDestroy(S.s_solve);
    (void)hipStreamDestroy(S.s_setup);
    for (auto &kv : S.all) delete kv.second;
    const std::string err = S.error;
    delete sv;
    if (!err.empty()) {
        set_error(err);
        return PBFB_EDEVICE;
    }
    return PBFB_OK;
}

} // extern "C"
