// Serving engine: continuous batching of independent image pairs.
//
// Requests are queued in arrival order. A worker thread admits the head of
// the queue as soon as a slot (a HIP stream) is free, together with up to
// max_batch - 1 later queued requests of the same variant (geometry,
// precision, image type, apply pair = fit pair or not): the batch runs as
// one launch per stage, blockIdx.z selecting the pair, on a workspace that
// holds every pair's buffers -- an idle one of that geometry with room for
// the batch, or a new one within the context's HBM budget (evicting idle
// workspaces of other geometries). The whole hot path of a batch is
// captured once per workspace and batch size into a HIP graph that reads
// each pair's buffers from a device table, so a batch costs a table write
// and a graph launch. Batches on different slots run concurrently on the
// device; completion is detected with an event per slot. Each pair's
// arithmetic is independent of the others (no shared buffers, no atomics
// across pairs, every reduction in a fixed order), so its result is the same
// alone, in a batch, or in any mix.
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
    Engine(sfft_ctx* ctx, int slots, int max_batch);
    ~Engine();
    int submit(const sfft_request& req, uint64_t* ticket);
    int poll(uint64_t ticket);
    int wait(uint64_t ticket);
    int slots() const { return (int)slots_.size(); }
    int max_batch() const { return max_batch_; }

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
        std::vector<uint64_t> tickets;   // the batch in flight, pair z = tickets[z]
        std::unique_ptr<Plan> plan;
    };
    void loop();
    int acquire(const sfft_params& p, int pairs, hipStream_t st, std::unique_ptr<Plan>& out,
                bool* wait_for_memory);
    hipEvent_t take_event();   // caller holds mu_

    sfft_ctx* ctx_;
    std::vector<Slot> slots_;
    int max_batch_;
    bool graphs_;   // replay each workspace's captured graph (SFFT_ENGINE_DIRECT: launch directly)
    std::deque<Job> queue_;
    std::map<uint64_t, int> status_;
    std::multimap<PlanKey, std::unique_ptr<Plan>> idle_;
    uint64_t idle_tick_ = 0;   // orders the idle workspaces by when they went idle
    void make_idle(std::unique_ptr<Plan> pl);
    // the idle workspace that has been idle longest
    std::multimap<PlanKey, std::unique_ptr<Plan>>::iterator eviction_victim();
    std::vector<hipEvent_t> events_;   // free submit events
    std::mutex mu_;
    std::condition_variable cv_, done_cv_;
    bool stop_ = false;
    uint64_t next_ = 1;
    std::thread th_;
};

}  // namespace sfft
