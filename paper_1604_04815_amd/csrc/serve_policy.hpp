// serve_policy.hpp -- admission and batching policy of the scan server.
//
// Pure C++17 (no HIP): the server drives it from its scheduler thread, and
// the CPU tests drive it directly.  Requests move
//     pending (submitted) -> launched (in a batch, bytes reserved) -> done.
// Rules:
//   * a request whose bytes exceed the whole budget is refused at submit
//     (no-memory); a full queue refuses with try-again;
//   * batches are formed when a stream slot is free.  The oldest pending
//     request fixes the batch key (dtype, operator, flags); then every
//     pending request with that key is taken in submit order while the
//     reserved bytes stay within the budget, up to max_batch requests.  A
//     request of that key that does not fit ends the batch, and if the oldest
//     request itself does not fit, nothing is launched until bytes are
//     released, so a large request is never overtaken by later requests of
//     its own key and never starves;
//   * requests of other keys may be launched ahead of older ones only by
//     forming their own batch when they become the oldest;
//   * a request of at least solo_bytes is never grouped: when it is the
//     oldest it forms a batch of its own, marked solo, which the server runs
//     alone with the whole device (so the largest requests, which set the
//     tail latency, get the full-device kernel); smaller requests of its key
//     may still form batches while it waits behind older requests.
#pragma once

#include <cstdint>
#include <deque>
#include <unordered_map>
#include <vector>

namespace lscan {
namespace serve {

enum class Admit : int { kOk = 0, kTooLarge = 1, kQueueFull = 2 };

struct PendingRequest {
    uint64_t ticket;
    uint64_t key;       // dtype | op << 8 | flags << 16
    uint64_t bytes;     // HBM bytes the request holds while in flight
    uint64_t t_submit;  // steady-clock ns
};

struct Batch {
    uint64_t key = 0;
    uint64_t bytes = 0;
    bool solo = false;
    std::vector<uint64_t> tickets;
};

class Policy {
public:
    Policy(uint64_t budget_bytes, size_t max_queue, size_t max_batch, uint64_t solo_bytes = UINT64_MAX)
        : budget_(budget_bytes), max_queue_(max_queue), max_batch_(max_batch), solo_(solo_bytes)
    {
    }

    // The oldest pending request would run alone.
    bool head_is_solo() const { return !pending_.empty() && pending_.front().bytes >= solo_; }

    Admit submit(const PendingRequest& r)
    {
        if (r.bytes > budget_) return Admit::kTooLarge;
        if (pending_.size() >= max_queue_) return Admit::kQueueFull;
        pending_.push_back(r);
        return Admit::kOk;
    }

    // Form the next batch (empty if nothing can be launched now).
    Batch next_batch()
    {
        Batch b;
        if (pending_.empty()) return b;
        const uint64_t key = pending_.front().key;
        if (in_flight_ + pending_.front().bytes > budget_) return b;  // oldest first
        if (pending_.front().bytes >= solo_) {
            b.key = key;
            b.bytes = pending_.front().bytes;
            b.solo = true;
            b.tickets.push_back(pending_.front().ticket);
            pending_.pop_front();
            in_flight_ += b.bytes;
            if (in_flight_ > peak_) peak_ = in_flight_;
            return b;
        }
        std::deque<PendingRequest> keep;
        bool closed = false;
        while (!pending_.empty()) {
            PendingRequest r = pending_.front();
            pending_.pop_front();
            if (!closed && r.key == key && r.bytes < solo_) {
                if (b.tickets.size() < max_batch_ && in_flight_ + b.bytes + r.bytes <= budget_) {
                    b.tickets.push_back(r.ticket);
                    b.bytes += r.bytes;
                    continue;
                }
                closed = true;  // keep submit order within the key
            }
            keep.push_back(r);
        }
        pending_.swap(keep);
        b.key = key;
        in_flight_ += b.bytes;
        if (in_flight_ > peak_) peak_ = in_flight_;
        return b;
    }

    void release(uint64_t bytes) { in_flight_ = (bytes > in_flight_) ? 0 : in_flight_ - bytes; }

    size_t pending() const { return pending_.size(); }
    uint64_t in_flight_bytes() const { return in_flight_; }
    uint64_t peak_bytes() const { return peak_; }
    uint64_t budget() const { return budget_; }

private:
    uint64_t budget_;
    size_t max_queue_;
    size_t max_batch_;
    uint64_t solo_;
    uint64_t in_flight_ = 0;
    uint64_t peak_ = 0;
    std::deque<PendingRequest> pending_;
};

}  // namespace serve
}  // namespace lscan
