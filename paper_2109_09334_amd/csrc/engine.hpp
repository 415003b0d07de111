// Serving engine: continuous batching of independent image pairs.
//
// Requests are queued in arrival order. A worker thread admits the head of
// the queue as soon as a slot (a HIP stream) is free and a workspace for
// its geometry fits the context's HBM budget -- reusing an idle workspace of
// the same geometry, or evicting idle workspaces of other geometries -- and
// enqueues the whole hot path on the slot's stream: the path is captured
// once per workspace into a HIP graph that reads the request's buffers from
// a device table, so a request costs a table write and a graph launch
// instead of some seventy kernel launches. Admitted requests run
// concurrently on the device; completion is detected with an event per
// slot. Each request's arithmetic is independent of the others (no shared
// buffers, no atomics across requests), so its result is the same alone or
// in any mix.
#pragma once
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "runtime.hpp"

namespace sfft {

class Engine {
public:
    Engine(sfft_ctx* ctx, int slots);
    ~Engine();
    int submit(const sfft_request& req, uint64_t* ticket);
    int poll(uint64_t ticket);
    int wait(uint64_t ticket);
    int slots() const { return (int)slots_.size(); }

private:
    struct Job {
        uint64_t ticket;
        sfft_request req;
        size_t bytes;
        hipEvent_t ready;   // recorded on req.stream at submit: the inputs are written
    };
    struct Slot {
        hipStream_t st = nullptr;
        hipEvent_t ev = nullptr;
        bool busy = false;
        uint64_t ticket = 0;
        std::unique_ptr<Plan> plan;
    };
    void loop();
    int acquire(const sfft_params& p, std::unique_ptr<Plan>& out, bool* wait_for_memory);
    hipEvent_t take_event();   // caller holds mu_

    sfft_ctx* ctx_;
    std::vector<Slot> slots_;
    bool graphs_;   // replay each workspace's captured graph (SFFT_ENGINE_DIRECT: launch directly)
    std::deque<Job> queue_;
    std::map<uint64_t, int> status_;
    std::multimap<PlanKey, std::unique_ptr<Plan>> idle_;
    std::vector<hipEvent_t> events_;   // free submit events
    std::mutex mu_;
    std::condition_variable cv_, done_cv_;
    bool stop_ = false;
    uint64_t next_ = 1;
    std::thread th_;
};

}  // namespace sfft
