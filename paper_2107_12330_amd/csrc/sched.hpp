// sched.hpp -- the request scheduling of the survey server, as plain C++
// (no device calls), so that its policy can be exercised on the host alone.
//
// Served mode keeps graphs resident and answers survey requests against
// them.  Requests on one graph share passes over its tiles (continuous
// batching): a pass is cut into n_seg segments, a graph runs one segment per
// step for all requests that hold one of its slots, and a request admitted
// between two steps joins at the next segment.  It is complete after n_seg
// steps, having seen every segment once (wrapping around the end of the
// pass).  Admission takes a free slot of the graph and the request's device
// memory from the server's budget; requests wait in arrival order, but one
// that cannot be admitted does not hold back requests on other graphs.
#pragma once

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <deque>
#include <vector>

namespace tp {
namespace sched {

// Device memory a server may hold.
class Budget {
public:
    explicit Budget(uint64_t cap = 0) : cap_(cap) {}
    uint64_t cap() const { return cap_; }
    uint64_t used() const { return used_; }
    bool take(uint64_t b)
    {
        if (b > cap_ - used_) return false;
        used_ += b;
        return true;
    }
    void give(uint64_t b) { used_ = b > used_ ? 0 : used_ - b; }

private:
    uint64_t cap_ = 0, used_ = 0;
};

// The slots and segment cursor of one resident graph.
class Engine {
public:
    struct Slot {
        bool used = false;
        uint64_t ticket = 0;
        uint32_t steps = 0;  // segments seen so far
    };

    Engine(uint32_t n_slots = 1, uint32_t n_seg = 1) : n_seg_(n_seg ? n_seg : 1), slots_(n_slots) {}

    uint32_t n_seg() const { return n_seg_; }
    uint32_t cursor() const { return cur_; }
    bool in_flight() const { return in_flight_; }
    const Slot &slot(uint32_t i) const { return slots_[i]; }
    uint32_t n_slots() const { return (uint32_t)slots_.size(); }

    uint32_t active() const
    {
        uint32_t a = 0;
        for (const Slot &s : slots_) a += s.used ? 1u : 0u;
        return a;
    }

    // 1 + the highest slot in use (the slots a step must cover)
    uint32_t high_water() const
    {
        for (uint32_t i = (uint32_t)slots_.size(); i > 0; --i)
            if (slots_[i - 1].used) return i;
        return 0;
    }

    // Take the lowest free slot for `ticket`; -1 if none is free.
    int admit(uint64_t ticket)
    {
        for (uint32_t i = 0; i < slots_.size(); ++i) {
            if (!slots_[i].used) {
                slots_[i] = Slot{true, ticket, 0};
                fresh_.push_back(i);
                return (int)i;
            }
        }
        return -1;
    }

    // Slots admitted since the last step began (their counters must be
    // cleared before it runs); the list is handed over once.
    std::vector<uint32_t> take_fresh()
    {
        std::vector<uint32_t> f;
        f.swap(fresh_);
        return f;
    }

    // Begin a step over the current segment: the slots taking part, and
    // those among them that this step completes.  False if no slot is used
    // or a step is already in flight.
    bool begin_step(std::vector<uint32_t> &part, std::vector<uint32_t> &finishing)
    {
        part.clear();
        finishing.clear();
        if (in_flight_) return false;
        for (uint32_t i = 0; i < slots_.size(); ++i) {
            if (!slots_[i].used) continue;
            part.push_back(i);
            if (slots_[i].steps + 1 == n_seg_) finishing.push_back(i);
        }
        if (part.empty()) return false;
        in_flight_ = true;
        step_part_ = part;
        return true;
    }

    // The step has run: advance the cursor and the slots that took part;
    // the completed requests' tickets are appended to `done` and their
    // slots freed.
    void end_step(std::vector<uint64_t> &done)
    {
        if (!in_flight_) return;
        in_flight_ = false;
        cur_ = (cur_ + 1) % n_seg_;
        for (uint32_t i : step_part_) {
            Slot &s = slots_[i];
            if (++s.steps == n_seg_) {
                done.push_back(s.ticket);
                s = Slot{};
            }
        }
        step_part_.clear();
    }

private:
    uint32_t n_seg_ = 1, cur_ = 0;
    bool in_flight_ = false;
    std::vector<Slot> slots_;
    std::vector<uint32_t> fresh_, step_part_;
};

// Requests waiting for admission, in arrival order.
class Queue {
public:
    explicit Queue(size_t cap = 4096) : cap_(cap) {}
    bool push(uint64_t ticket)
    {
        if (q_.size() >= cap_) return false;
        q_.push_back(ticket);
        return true;
    }
    size_t size() const { return q_.size(); }

    // Offer every waiting request, oldest first, to `try_admit(ticket)`;
    // admitted ones leave the queue, the others keep their order.
    template <class F>
    size_t admit(F &&try_admit)
    {
        size_t n = 0;
        for (auto it = q_.begin(); it != q_.end();) {
            if (try_admit(*it)) {
                it = q_.erase(it);
                ++n;
            } else {
                ++it;
            }
        }
        return n;
    }

private:
    size_t cap_;
    std::deque<uint64_t> q_;
};

// Nearest-rank percentile (q in [0, 1]) of `v`, which it sorts; 0 if empty.
inline double percentile(std::vector<double> &v, double q)
{
    if (v.empty()) return 0.0;
    std::sort(v.begin(), v.end());
    size_t k = (size_t)std::ceil(q * (double)v.size());
    if (k < 1) k = 1;
    if (k > v.size()) k = v.size();
    return v[k - 1];
}

}  // namespace sched
}  // namespace tp
