// Serving engine (see engine.hpp) and its C ABI entry points.
#include "engine.hpp"

#include <algorithm>
#include <chrono>
#include <cstdlib>

namespace sfft {

Engine::Engine(sfft_ctx* ctx, int slots, int max_batch)
    : ctx_(ctx),
      slots_(slots > 0 ? slots : 4),
      max_batch_(max_batch > 0 ? (max_batch < kMaxBatch ? max_batch : kMaxBatch) : 4),
      graphs_(getenv("SFFT_ENGINE_DIRECT") == nullptr) {
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

// Batch key: requests that can share one launch per stage.
static bool same_variant(const sfft_request& a, const sfft_request& b) {
    const bool sa = a.r == a.r_fit && a.s == a.s_fit, sb = b.r == b.r_fit && b.s == b.s_fit;
    return key_of(&a.p) == key_of(&b.p) && a.p.dtype == b.p.dtype && sa == sb;
}

static int pow2_at_least(int n) {
    int c = 1;
    while (c < n) c *= 2;
    return c;
}

void Engine::make_idle(std::unique_ptr<Plan> pl) {
    pl->idle_since = ++idle_tick_;
    auto key = key_of(&pl->p);
    idle_.emplace(key, std::move(pl));
}

std::multimap<PlanKey, std::unique_ptr<Plan>>::iterator Engine::eviction_victim() {
    auto v = idle_.begin();
    for (auto it = idle_.begin(); it != idle_.end(); ++it)
        if (it->second->idle_since < v->second->idle_since) v = it;
    return v;
}

// Workspace for `pairs` requests of geometry p: the idle one of that
// geometry with the least room that holds them, else a new one (room for
// the next power of two, at most max_batch) within the budget, evicting
// the idle workspaces that have been idle longest (a mix of geometries keeps
// its frequent ones; each eviction is a device-wide synchronising free and
// each new workspace an allocation and fresh graphs). Caller holds mu_.
int Engine::acquire(const sfft_params& p, int pairs, hipStream_t st, std::unique_ptr<Plan>& out,
                    bool* wait_for_memory) {
    *wait_for_memory = false;
    auto key = key_of(&p);
    auto range = idle_.equal_range(key);
    auto best = idle_.end();
    for (auto it = range.first; it != range.second; ++it)
        if (it->second->cap >= pairs && (best == idle_.end() || it->second->cap < best->second->cap))
            best = it;
    if (best != idle_.end()) {
        out = std::move(best->second);
        idle_.erase(best);
        return SFFT_OK;
    }
    std::lock_guard<std::mutex> ck(ctx_->mu);
    const int cap = std::min(pow2_at_least(pairs), max_batch_);
    const size_t need = ((workspace_bytes(&p) + 255) & ~size_t(255)) * cap;
    // an idle workspace of this geometry with less room is taken (the batch
    // shrinks to it) rather than evicting others to make a bigger one
    if (ctx_->budget && ctx_->used + need > ctx_->budget) {
        auto big = idle_.end();
        for (auto it = range.first; it != range.second; ++it)
            if (big == idle_.end() || it->second->cap > big->second->cap) big = it;
        if (big != idle_.end()) {
            out = std::move(big->second);
            idle_.erase(big);
            return SFFT_OK;
        }
    }
    while (ctx_->budget && ctx_->used + need > ctx_->budget && !idle_.empty()) {
        auto victim = eviction_victim();
        destroy_plan(ctx_, victim->second);
        idle_.erase(victim);
    }
    if (ctx_->budget && ctx_->used + need > ctx_->budget) {
        *wait_for_memory = true;
        return SFFT_E_NOMEM;
    }
    int rc = create_plan(ctx_, &p, out, cap, st);
    // the device itself out of memory: free idle workspaces, then wait for
    // running requests to return theirs
    while (rc == SFFT_E_NOMEM && !idle_.empty()) {
        auto victim = eviction_victim();
        destroy_plan(ctx_, victim->second);
        idle_.erase(victim);
        rc = create_plan(ctx_, &p, out, cap, st);
    }
    if (rc == SFFT_E_NOMEM) *wait_for_memory = true;
    return rc;
}

void Engine::loop() {
    (void)hipSetDevice(ctx_->device);
    std::unique_lock<std::mutex> lk(mu_);
    for (;;) {
        bool running = false;
        // completions: every pair of the slot's batch
        for (auto& s : slots_) {
            if (!s.busy) continue;
            if (hipEventQuery(s.ev) == hipSuccess) {
                for (size_t z = 0; z < s.tickets.size(); ++z) {
                    int f = 0;
                    const int rc = read_pair_flag(*s.plan, (int)z, &f);
                    status_[s.tickets[z]] = rc ? rc : flag_status(f);
                }
                s.tickets.clear();
                make_idle(std::move(s.plan));
                s.busy = false;
                done_cv_.notify_all();
            } else {
                running = true;
            }
        }
        // admissions, in arrival order: the head of the queue and the later
        // requests of its variant, up to max_batch
        while (!queue_.empty()) {
            Slot* free_slot = nullptr;
            for (auto& s : slots_)
                if (!s.busy) { free_slot = &s; break; }
            if (!free_slot) break;
            std::vector<size_t> pick{0};
            for (size_t i = 1; i < queue_.size() && (int)pick.size() < max_batch_; ++i)
                if (same_variant(queue_[i].req, queue_[0].req)) pick.push_back(i);
            std::unique_ptr<Plan> pl;
            bool wait_mem = false;
            int rc = acquire(queue_[0].req.p, (int)pick.size(), free_slot->st, pl, &wait_mem);
            if (rc && wait_mem && pick.size() > 1) {   // the head alone may still fit
                pick.resize(1);
                rc = acquire(queue_[0].req.p, 1, free_slot->st, pl, &wait_mem);
            }
            if (rc && wait_mem && running) break;       // memory frees as requests finish
            if (rc) {
                Job& j = queue_.front();
                status_[j.ticket] = rc;
                events_.push_back(j.ready);
                queue_.pop_front();
                done_cv_.notify_all();
                continue;
            }
            if ((int)pick.size() > pl->cap) pick.resize(pl->cap);
            const sfft_request& head = queue_[0].req;
            pl->p.dtype = head.p.dtype;
            const bool same_pair = head.r == head.r_fit && head.s == head.s_fit;
            IoBatch io{};
            io.n = (int)pick.size();
            rc = SFFT_OK;
            for (size_t z = 0; z < pick.size(); ++z) {
                Job& j = queue_[pick[z]];
                if (!rc && hipStreamWaitEvent(free_slot->st, j.ready, 0) != hipSuccess) rc = SFFT_E_HIP;
                events_.push_back(j.ready);   // the wait holds the recorded state
                const void* ptrs[kIoUsed] = {j.req.r_fit, j.req.s_fit, j.req.r, j.req.s, j.req.coef, j.req.d};
                for (int k = 0; k < kIoUsed; ++k) io.p[z][k] = ptrs[k];
            }
            if (!rc) rc = plan_run_batch(*pl, io, same_pair, graphs_, free_slot->st);
            if (!rc && hipEventRecord(free_slot->ev, free_slot->st) != hipSuccess) rc = SFFT_E_HIP;
            std::vector<uint64_t> tickets;
            for (size_t z = 0; z < pick.size(); ++z) tickets.push_back(queue_[pick[z]].ticket);
            // remove the batch from the queue (later indices first)
            for (size_t z = pick.size(); z-- > 0;) queue_.erase(queue_.begin() + (long)pick[z]);
            if (rc) {
                for (uint64_t t : tickets) status_[t] = rc;
                make_idle(std::move(pl));
                done_cv_.notify_all();
            } else {
                free_slot->plan = std::move(pl);
                free_slot->busy = true;
                free_slot->tickets = std::move(tickets);
                running = true;
            }
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

}  // namespace sfft

using sfft::Engine;

extern "C" {

int sfft_engine_config(sfft_ctx* ctx, int slots, int max_batch) {
    if (!ctx || slots < 0 || slots > 64 || max_batch < 0 || max_batch > sfft::kMaxBatch)
        return SFFT_E_INVAL;
    if (ctx->engine)
        return ctx->engine->slots() == (slots ? slots : 4) &&
                       ctx->engine->max_batch() == (max_batch ? max_batch : 4)
                   ? SFFT_OK
                   : SFFT_E_INVAL;
    ctx->engine = std::make_unique<Engine>(ctx, slots, max_batch);
    return SFFT_OK;
}

int sfft_submit(sfft_ctx* ctx, const sfft_request* req, uint64_t* ticket) {
    if (!ctx || !req || !ticket) return SFFT_E_INVAL;
    if (!ctx->engine) ctx->engine = std::make_unique<Engine>(ctx, 4, 4);
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
