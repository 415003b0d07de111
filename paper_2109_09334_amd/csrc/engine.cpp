// Serving engine (see engine.hpp) and its C ABI entry points.
#include "engine.hpp"

#include <chrono>
#include <cstdlib>

namespace sfft {

int read_plan_flag(Plan& pl, int* flag);

Engine::Engine(sfft_ctx* ctx, int slots)
    : ctx_(ctx), slots_(slots > 0 ? slots : 4), graphs_(getenv("SFFT_ENGINE_DIRECT") == nullptr) {
    (void)hipSetDevice(ctx_->device);
    for (auto& s : slots_) {
        (void)hipStreamCreateWithFlags(&s.st, hipStreamNonBlocking);
        (void)hipEventCreateWithFlags(&s.ev, hipEventDisableTiming);
    }
    th_ = std::thread([this] { loop(); });
}

Engine::~Engine() {
    {
        std::lock_guard<std::mutex> lk(mu_);
        stop_ = true;
    }
    cv_.notify_all();
    th_.join();
    (void)hipSetDevice(ctx_->device);
    std::lock_guard<std::mutex> lk(ctx_->mu);
    for (auto& s : slots_) {
        if (s.st) (void)hipStreamSynchronize(s.st);
        destroy_plan(ctx_, s.plan);
        if (s.ev) (void)hipEventDestroy(s.ev);
        if (s.st) (void)hipStreamDestroy(s.st);
    }
    for (auto& kv : idle_) destroy_plan(ctx_, kv.second);
    for (auto ev : events_) (void)hipEventDestroy(ev);
}

hipEvent_t Engine::take_event() {
    if (!events_.empty()) {
        hipEvent_t e = events_.back();
        events_.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
    return e;
}

int Engine::submit(const sfft_request& req, uint64_t* ticket) {
    int rc = check_params(&req.p);
    if (rc) return rc;
    if (!req.r_fit || !req.s_fit || !req.r || !req.s || !req.d) return SFFT_E_INVAL;
    const size_t bytes = workspace_bytes(&req.p);
    if (ctx_->budget && bytes > ctx_->budget) return SFFT_E_NOMEM;
    std::lock_guard<std::mutex> lk(mu_);
    // The request runs on a slot stream of its own; it starts after the work
    // enqueued on the caller's stream up to this call (which produced the
    // inputs and, e.g., initialised the outputs).
    (void)hipSetDevice(ctx_->device);
    hipEvent_t ev = take_event();
    if (!ev) return SFFT_E_HIP;
    if (hipEventRecord(ev, (hipStream_t)req.stream) != hipSuccess) {
        events_.push_back(ev);
        return SFFT_E_HIP;
    }
    const uint64_t t = next_++;
    queue_.push_back(Job{t, req, bytes, ev});
    status_[t] = SFFT_PENDING;
    *ticket = t;
    cv_.notify_all();
    return SFFT_OK;
}

int Engine::poll(uint64_t ticket) {
    std::lock_guard<std::mutex> lk(mu_);
    auto it = status_.find(ticket);
    if (it == status_.end()) return SFFT_E_NOTFOUND;
    const int s = it->second;
    if (s != SFFT_PENDING) status_.erase(it);
    return s;
}

int Engine::wait(uint64_t ticket) {
    std::unique_lock<std::mutex> lk(mu_);
    auto it = status_.find(ticket);
    if (it == status_.end()) return SFFT_E_NOTFOUND;
    done_cv_.wait(lk, [&] { return status_[ticket] != SFFT_PENDING; });
    const int s = status_[ticket];
    status_.erase(ticket);
    return s;
}

// Workspace for geometry p: an idle one of the same geometry, else a new
// one within the budget (evicting idle workspaces of other geometries).
// Caller holds mu_.
int Engine::acquire(const sfft_params& p, std::unique_ptr<Plan>& out, bool* wait_for_memory) {
    *wait_for_memory = false;
    auto key = key_of(&p);
    auto it = idle_.find(key);
    if (it != idle_.end()) {
        out = std::move(it->second);
        idle_.erase(it);
        return SFFT_OK;
    }
    std::lock_guard<std::mutex> ck(ctx_->mu);
    const size_t need = workspace_bytes(&p);
    while (ctx_->budget && ctx_->used + need > ctx_->budget && !idle_.empty()) {
        auto victim = idle_.begin();
        destroy_plan(ctx_, victim->second);
        idle_.erase(victim);
    }
    if (ctx_->budget && ctx_->used + need > ctx_->budget) {
        *wait_for_memory = true;
        return SFFT_E_NOMEM;
    }
    return create_plan(ctx_, &p, out);
}

void Engine::loop() {
    (void)hipSetDevice(ctx_->device);
    std::unique_lock<std::mutex> lk(mu_);
    for (;;) {
        bool running = false;
        // completions
        for (auto& s : slots_) {
            if (!s.busy) continue;
            if (hipEventQuery(s.ev) == hipSuccess) {
                int f = 0;
                int rc = read_plan_flag(*s.plan, &f);
                status_[s.ticket] = rc ? rc : flag_status(f);
                auto key = key_of(&s.plan->p);
                idle_.emplace(key, std::move(s.plan));
                s.busy = false;
                done_cv_.notify_all();
            } else {
                running = true;
            }
        }
        // admissions, in arrival order
        while (!queue_.empty()) {
            Slot* free_slot = nullptr;
            for (auto& s : slots_)
                if (!s.busy) { free_slot = &s; break; }
            if (!free_slot) break;
            Job& j = queue_.front();
            std::unique_ptr<Plan> pl;
            bool wait_mem = false;
            int rc = acquire(j.req.p, pl, &wait_mem);
            if (rc && wait_mem && running) break;       // memory frees as requests finish
            if (rc) {
                status_[j.ticket] = rc;
                events_.push_back(j.ready);
                queue_.pop_front();
                done_cv_.notify_all();
                continue;
            }
            pl->p.dtype = j.req.p.dtype;
            rc = hipStreamWaitEvent(free_slot->st, j.ready, 0) == hipSuccess ? SFFT_OK : SFFT_E_HIP;
            events_.push_back(j.ready);   // the wait holds the recorded state
            if (!rc)
                rc = graphs_ ? plan_run_graph(*pl, j.req.r_fit, j.req.s_fit, j.req.r, j.req.s,
                                          j.req.coef, j.req.d, free_slot->st)
                         : plan_run(*pl, j.req.r_fit, j.req.s_fit, j.req.r, j.req.s, j.req.coef,
                                    j.req.d, free_slot->st);
            if (!rc && hipEventRecord(free_slot->ev, free_slot->st) != hipSuccess) rc = SFFT_E_HIP;
            if (rc) {
                status_[j.ticket] = rc;
                idle_.emplace(key_of(&pl->p), std::move(pl));
                done_cv_.notify_all();
            } else {
                free_slot->plan = std::move(pl);
                free_slot->busy = true;
                free_slot->ticket = j.ticket;
                running = true;
            }
            queue_.pop_front();
        }
        if (stop_ && !running) {
            for (auto& j : queue_) {
                status_[j.ticket] = SFFT_E_INVAL;
                events_.push_back(j.ready);
            }
            queue_.clear();
            done_cv_.notify_all();
            return;
        }
        if (!running && queue_.empty()) {
            cv_.wait(lk);
        } else {
            lk.unlock();
            std::this_thread::sleep_for(std::chrono::microseconds(20));
            lk.lock();
        }
    }
}

int read_plan_flag(Plan& pl, int* flag) {
    if (hipMemcpy(flag, pl.ws.flag, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess) return SFFT_E_HIP;
    return SFFT_OK;
}

}  // namespace sfft

using sfft::Engine;

extern "C" {

int sfft_engine_config(sfft_ctx* ctx, int slots) {
    if (!ctx || slots < 0 || slots > 64) return SFFT_E_INVAL;
    if (ctx->engine) return ctx->engine->slots() == (slots ? slots : 4) ? SFFT_OK : SFFT_E_INVAL;
    ctx->engine = std::make_unique<Engine>(ctx, slots);
    return SFFT_OK;
}

int sfft_submit(sfft_ctx* ctx, const sfft_request* req, uint64_t* ticket) {
    if (!ctx || !req || !ticket) return SFFT_E_INVAL;
    if (!ctx->engine) ctx->engine = std::make_unique<Engine>(ctx, 4);
    return ctx->engine->submit(*req, ticket);
}

int sfft_poll(sfft_ctx* ctx, uint64_t ticket) {
    if (!ctx) return SFFT_E_INVAL;
    if (!ctx->engine) return SFFT_E_NOTFOUND;
    return ctx->engine->poll(ticket);
}

int sfft_wait(sfft_ctx* ctx, uint64_t ticket) {
    if (!ctx) return SFFT_E_INVAL;
    if (!ctx->engine) return SFFT_E_NOTFOUND;
    return ctx->engine->wait(ticket);
}

}  // extern "C"
