// Host-only checks of the survey server's scheduling policy (sched.hpp).
// Prints one line per check: "ok <name>" or "FAIL <name>: <detail>".
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <map>
#include <mutex>
#include <set>
#include <string>
#include <thread>
#include <vector>

#include "sched.hpp"

using namespace tp::sched;

static int failures = 0;
static void check(bool c, const std::string &name, const std::string &detail = "")
{
    std::printf("%s %s%s%s\n", c ? "ok" : "FAIL", name.c_str(), c ? "" : ": ", c ? "" : detail.c_str());
    if (!c) ++failures;
}

// Drive an engine step by step; requests arrive at given steps.  Returns the
// segments each request saw, in order.
static std::vector<std::vector<uint32_t>> simulate(uint32_t slots, uint32_t n_seg,
                                                   const std::vector<uint32_t> &arrive_step, uint32_t max_steps,
                                                   std::vector<uint32_t> &done_step)
{
    Engine e(slots, n_seg);
    Queue q(1000);
    std::vector<std::vector<uint32_t>> seen(arrive_step.size());
    done_step.assign(arrive_step.size(), ~0u);
    std::vector<uint32_t> part, fin;
    for (uint32_t step = 0; step < max_steps; ++step) {
        for (uint32_t i = 0; i < arrive_step.size(); ++i)
            if (arrive_step[i] == step) q.push(i);
        q.admit([&](uint64_t t) { return e.admit(t) >= 0; });
        (void)e.take_fresh();
        if (!e.begin_step(part, fin)) continue;
        const uint32_t seg = e.cursor();
        for (uint32_t s : part) seen[e.slot(s).ticket].push_back(seg);
        std::set<uint64_t> fin_t;
        for (uint32_t s : fin) fin_t.insert(e.slot(s).ticket);
        std::vector<uint64_t> done;
        e.end_step(done);
        std::set<uint64_t> done_t(done.begin(), done.end());
        if (fin_t != done_t) check(false, "finishing list matches completions", "step " + std::to_string(step));
        for (uint64_t t : done) done_step[t] = step;
    }
    return seen;
}

// The server's threading discipline on the host alone: client threads
// submit under one mutex and wait on a condition variable; one worker thread
// admits (slot and budget), begins a step, runs the "device" part without
// the lock, then ends the step and wakes the clients -- as the server does
// around its device calls.  Built under ThreadSanitizer this checks that the
// policy objects are only ever touched under the lock.
static void threaded_serving()
{
    const uint32_t n_seg = 5, clients = 6, per_client = 40;
    std::mutex mu;
    std::condition_variable cv;
    Engine eng(3, n_seg);
    Queue queue(8);
    Budget budget(3 * 100);
    std::map<uint64_t, std::vector<uint32_t>> seen;  // ticket -> segments
    std::set<uint64_t> done;
    uint64_t next_ticket = 0, rejected = 0;
    bool stop = false;
    std::thread worker([&] {
        std::vector<uint32_t> part, fin;
        std::unique_lock<std::mutex> lk(mu);
        for (;;) {
            queue.admit([&](uint64_t t) {
                if (!budget.take(100)) return false;
                if (eng.admit(t) < 0) {
                    budget.give(100);
                    return false;
                }
                return true;
            });
            (void)eng.take_fresh();
            if (!eng.begin_step(part, fin)) {
                if (stop) break;
                // nothing runs: sleep until a request arrives or the clients
                // are done (an untimed wait: ThreadSanitizer of this toolchain
                // does not see the timed wait's unlock)
                cv.wait(lk, [&] { return stop || queue.size() > 0; });
                continue;
            }
            const uint32_t seg = eng.cursor();
            std::vector<uint64_t> tickets;
            for (uint32_t s : part) tickets.push_back(eng.slot(s).ticket);
            lk.unlock();
            std::this_thread::sleep_for(std::chrono::microseconds(50));  // the device step
            lk.lock();
            for (uint64_t t : tickets) seen[t].push_back(seg);
            std::vector<uint64_t> finished;
            eng.end_step(finished);
            for (uint64_t t : finished) {
                done.insert(t);
                budget.give(100);
            }
            if (!finished.empty()) cv.notify_all();
        }
    });
    std::vector<std::thread> cl;
    for (uint32_t c = 0; c < clients; ++c)
        cl.emplace_back([&] {
            for (uint32_t i = 0; i < per_client; ++i) {
                std::unique_lock<std::mutex> lk(mu);
                const uint64_t t = next_ticket++;
                if (!queue.push(t)) {  // queue full: counted, not kept
                    ++rejected;
                    continue;
                }
                cv.notify_all();
                cv.wait(lk, [&] { return done.count(t) != 0; });
            }
        });
    for (auto &t : cl) t.join();
    {
        std::lock_guard<std::mutex> lk(mu);
        stop = true;
    }
    cv.notify_all();
    worker.join();
    bool ok = done.size() + rejected == (size_t)clients * per_client && budget.used() == 0;
    for (uint64_t t : done) {
        const auto &v = seen[t];
        std::set<uint32_t> u(v.begin(), v.end());
        ok = ok && v.size() == n_seg && u.size() == n_seg;
    }
    check(ok, "threaded clients and worker: every admitted request sees each segment once",
          std::to_string(done.size()) + " done, " + std::to_string(rejected) + " rejected");
}

int main()
{
    threaded_serving();
    // every request sees every segment exactly once, whenever it arrives
    {
        std::vector<uint32_t> arrive = {0, 0, 3, 5, 5, 5, 9, 14, 14, 20};
        std::vector<uint32_t> done;
        auto seen = simulate(4, 7, arrive, 200, done);
        bool all = true;
        std::string why;
        for (size_t i = 0; i < seen.size(); ++i) {
            std::set<uint32_t> s(seen[i].begin(), seen[i].end());
            if (seen[i].size() != 7 || s.size() != 7 || done[i] == ~0u) {
                all = false;
                why = "request " + std::to_string(i) + " saw " + std::to_string(seen[i].size());
            }
            // consecutive segments, wrapping
            for (size_t k = 1; k < seen[i].size(); ++k)
                if (seen[i][k] != (seen[i][k - 1] + 1) % 7) {
                    all = false;
                    why = "request " + std::to_string(i) + " skipped a segment";
                }
        }
        check(all, "each request covers all segments once, in cursor order", why);
    }
    // with 4 slots no more than 4 requests run at once, and the 5th waits
    {
        std::vector<uint32_t> arrive = {0, 0, 0, 0, 0};
        std::vector<uint32_t> done;
        auto seen = simulate(4, 3, arrive, 50, done);
        check(done[0] == 2 && done[3] == 2, "first four finish after n_seg steps",
              std::to_string(done[0]) + "," + std::to_string(done[3]));
        check(done[4] == 5, "fifth request runs once a slot frees", std::to_string(done[4]));
    }
    // one segment: a request completes in the step it joins
    {
        std::vector<uint32_t> arrive = {0, 1, 1};
        std::vector<uint32_t> done;
        simulate(2, 1, arrive, 10, done);
        check(done[0] == 0 && done[1] == 1 && done[2] == 1, "single-segment graphs answer in one step");
    }
    // slots: lowest free first, high water shrinks when the top frees
    {
        Engine e(4, 2);
        check(e.admit(10) == 0 && e.admit(11) == 1 && e.admit(12) == 2, "admit takes the lowest free slots");
        check(e.high_water() == 3, "high water covers used slots");
        std::vector<uint32_t> part, fin;
        std::vector<uint64_t> done;
        check(e.begin_step(part, fin) && part.size() == 3 && fin.empty(), "step over three slots");
        check(!e.begin_step(part, fin), "one step in flight at a time");
        e.end_step(done);
        check(done.empty() && e.cursor() == 1, "cursor advances");
        check(e.admit(13) == 3, "a request admitted mid-pass takes slot 3");
        check(e.take_fresh().size() == 4, "fresh slots are reported once");
        check(e.take_fresh().empty(), "fresh list is cleared");
        e.begin_step(part, fin);
        check(fin.size() == 3, "three slots finish with their second step");
        e.end_step(done);
        check(done.size() == 3 && e.active() == 1 && e.high_water() == 4, "slot 3 keeps running");
        check(e.admit(14) == 0, "a freed slot is reused");
    }
    // budget
    {
        Budget b(100);
        check(b.take(60) && !b.take(41) && b.take(40) && b.used() == 100, "budget admits up to its cap");
        b.give(30);
        check(b.used() == 70 && b.take(30), "released memory is admitted again");
        b.give(1000);
        check(b.used() == 0, "over-release clamps at zero");
    }
    // queue: capacity, order, and no head-of-line blocking
    {
        Queue q(3);
        check(q.push(1) && q.push(2) && q.push(3) && !q.push(4), "queue refuses past its capacity");
        std::vector<uint64_t> order;
        q.admit([&](uint64_t t) {
            order.push_back(t);
            return t != 1;  // request 1 cannot be admitted yet
        });
        check(order == std::vector<uint64_t>({1, 2, 3}), "requests are offered oldest first");
        check(q.size() == 1, "the blocked request keeps waiting while later ones pass");
        check(q.push(5) && q.push(6) && !q.push(7), "admitted requests free queue room");
    }
    // percentiles (nearest rank)
    {
        std::vector<double> v;
        for (int i = 100; i >= 1; --i) v.push_back(i);
        check(percentile(v, 0.5) == 50 && percentile(v, 0.99) == 99 && percentile(v, 1.0) == 100,
              "nearest-rank percentiles");
        std::vector<double> one = {7};
        std::vector<double> none;
        check(percentile(one, 0.99) == 7 && percentile(none, 0.5) == 0, "percentiles of small samples");
    }
    std::printf("%s\n", failures ? "FAILED" : "PASSED");
    return failures ? 1 : 0;
}
