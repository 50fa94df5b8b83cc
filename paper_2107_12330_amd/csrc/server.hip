// server.hip -- served mode: resident graphs, a request queue and a worker
// thread that runs multi-request passes (continuous batching).
//
// The scheduling policy lives in sched.hpp; this file binds it to the
// device: per resident graph a slot table on the device, a result block per
// slot, pinned host staging, and one event per step in flight.  Large graphs
// step on one stream and small ones (a single segment) on another, so their
// work overlaps; while small graphs are resident the persistent grids of the
// large graphs' steps leave an eighth of the device to them.
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "graph.hpp"
#include "multi.hpp"
#include "sched.hpp"

using namespace tp;

namespace {

double now_us()
{
    using namespace std::chrono;
    return (double)duration_cast<nanoseconds>(steady_clock::now().time_since_epoch()).count() * 1e-3;
}

// Pinned host array.
template <class T>
struct HostArray {
    T *p = nullptr;
    explicit HostArray(size_t n)
    {
        if (n) TP_HIP(hipHostMalloc((void **)&p, n * sizeof(T), hipHostMallocDefault));
    }
    HostArray(const HostArray &) = delete;
    HostArray &operator=(const HostArray &) = delete;
    ~HostArray()
    {
        if (p) (void)hipHostFree(p);
    }
};

struct Resident {
    uint32_t id = 0;
    tp_graph *g = nullptr;
    uint64_t bytes = 0;       // taken from the budget
    bool small = false;       // one segment: runs on the second stream
    sched::Engine eng;
    hipStream_t stream = nullptr;
    DArray<SlotSpec> dslots;
    DArray<unsigned long long> dout;  // slots * words, then the claim counters
    std::unique_ptr<HostArray<SlotSpec>> hstage;   // slot table for the next step
    std::unique_ptr<HostArray<unsigned long long>> hres;  // result blocks of finishing slots
    std::vector<SlotSpec> spec;       // slot table as admitted
    hipEvent_t ev = nullptr;
    std::vector<uint32_t> part, finishing;
    uint32_t queued = 0;      // requests waiting or running on this graph
    ~Resident()
    {
        if (ev) (void)hipEventDestroy(ev);
        if (g) tripoll_graph_free(g);
    }
};

struct Request {
    uint64_t ticket = 0;
    uint32_t graph = 0, tag = 0;
    tp_survey_spec spec{};
    SlotSpec slot{};
    uint64_t mem = 0;
    int slot_idx = -1;
    int state = 0;  // 0 waiting, 1 running, 2 done, 3 failed
    uint32_t steps = 0;
    double t_arrive = 0, t_admit = 0, t_done = 0;
    tp_survey_result res{};
    std::string error;
    // Requests whose counters do not fit the shared pass (OPEN_CLOSE,
    // MAX_EDGE, DEGREE_TABLE, DIRECTED) keep their slot for the segment
    // bookkeeping but run the single-request kernels over each segment, into
    // result words of their own.
    bool solo = false;
    DArray<unsigned long long> dres;                       // TP_RESULT_WORDS on the device
    std::unique_ptr<HostArray<unsigned long long>> hres;  // the counters, copied back at completion
};

constexpr uint32_t kSoloOutputs = TP_OUT_OPEN_CLOSE | TP_OUT_MAX_EDGE | TP_OUT_DEGREE_TABLE | TP_OUT_DIRECTED;

}  // namespace

struct tp_server {
    tp_server_config cfg{};
    int device = 0;
    uint32_t words = 0;  // result block of a slot
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::thread worker;
    bool stop = false;
    std::string fatal;  // set when the worker met a device error
    sched::Budget budget;
    sched::Queue queue;
    hipStream_t big = nullptr, small = nullptr;
    std::map<uint32_t, std::unique_ptr<Resident>> graphs;
    uint32_t next_graph = 1;
    std::unordered_map<uint64_t, Request> reqs;
    uint64_t next_ticket = 1;
    // statistics
    uint64_t submitted = 0, completed = 0, rejected = 0, steps = 0, triangles = 0;
    double t_first = -1, t_last = 0;
    std::vector<double> lat_ms[TP_SERVER_TAGS];

    ~tp_server()
    {
        graphs.clear();
        if (big) (void)hipStreamDestroy(big);
        if (small) (void)hipStreamDestroy(small);
    }

    bool any_small() const
    {
        for (auto &kv : graphs)
            if (kv.second->small) return true;
        return false;
    }

    void complete(Request &r, const unsigned long long *blk, const Resident &G)
    {
        r.state = 2;
        r.t_done = now_us();
        std::memset(&r.res, 0, sizeof(r.res));
        if (r.solo) {
            // the result words of tripoll_survey's layout
            const unsigned long long *h = r.hres->p;
            r.res.triangles = h[TP_RW_TRIANGLES];
            r.res.spread_count = h[TP_RW_SPREAD];
            for (int i = 0; i < 32; ++i) r.res.close_hist[i] = h[TP_RW_HIST + i];
            for (uint32_t i = 0; i < TP_TABLE_MAX; ++i) r.res.label_table[i] = h[TP_RW_TABLE + i];
            for (int i = 0; i < 1024; ++i) r.res.open_close[i] = h[TP_RW_OPEN_CLOSE + i];
            for (uint32_t i = 0; i < TP_MAX_EDGE_BINS; ++i) r.res.max_edge[i] = h[TP_RW_MAX_EDGE + i];
            for (uint32_t i = 0; i < TP_DEGREE_MAX; ++i) r.res.degree_table[i] = h[TP_RW_DEGREE + i];
            for (int i = 0; i < 7; ++i) r.res.directed[i] = h[TP_RW_DIRECTED + i];
            r.dres.release();
            r.hres.reset();
        } else {
            r.res.triangles = blk[TP_BW_TRIANGLES];
            r.res.spread_count = blk[TP_BW_SPREAD];
            for (int i = 0; i < 32; ++i) r.res.close_hist[i] = blk[TP_BW_HIST + i];
            if (r.spec.outputs & TP_OUT_LABEL_TABLE) {
                const uint32_t ts = words - TP_BW_TABLE;
                for (uint32_t i = 0; i < ts && i < TP_TABLE_MAX; ++i) r.res.label_table[i] = blk[TP_BW_TABLE + i];
            }
        }
        r.res.probes = G.g->stats.probes;
        r.res.total_ms = (float)((r.t_done - r.t_admit) * 1e-3);
        budget.give(r.mem);
        ++completed;
        triangles += r.res.triangles;
        t_last = r.t_done;
        lat_ms[r.tag].push_back((r.t_done - r.t_arrive) * 1e-3);
    }

    void fail_all(const std::string &msg)
    {
        fatal = msg;
        for (auto &kv : reqs) {
            if (kv.second.state < 2) {
                kv.second.state = 3;
                kv.second.error = msg;
            }
        }
        cv_done.notify_all();
    }

    // Admit waiting requests; returns true if any was admitted.
    bool admit_locked()
    {
        const size_t n = queue.admit([&](uint64_t t) {
            Request &r = reqs.at(t);
            Resident &G = *graphs.at(r.graph);
            if (!budget.take(r.mem)) return false;
            const int s = G.eng.admit(t);
            if (s < 0) {
                budget.give(r.mem);
                return false;
            }
            r.slot_idx = s;
            r.state = 1;
            r.t_admit = now_us();
            G.spec[s] = r.slot;
            if (r.solo) {
                // the shared pass skips the slot; the request's own words
                // are cleared on the graph's stream before its first step
                G.spec[s].off = 1;
                r.dres.reset(TP_RESULT_WORDS, G.stream);
                zero_words(r.dres.get(), TP_RESULT_WORDS, G.stream);
                r.hres = std::make_unique<HostArray<unsigned long long>>(TP_RW_SCRATCH);
            }
            return true;
        });
        return n > 0;
    }

    // Finish the steps whose events have fired; returns true if any is
    // still in flight.
    bool reap_locked()
    {
        bool pending = false;
        for (auto &kv : graphs) {
            Resident &G = *kv.second;
            if (!G.eng.in_flight()) continue;
            const hipError_t q = hipEventQuery(G.ev);
            if (q == hipErrorNotReady) {
                pending = true;
                continue;
            }
            if (q != hipSuccess) {
                (void)hipGetLastError();
                throw Error{TP_ERR_DEVICE, std::string("survey step failed: ") + hipGetErrorString(q)};
            }
            std::vector<uint64_t> done;
            for (uint32_t i : G.part) ++reqs.at(G.eng.slot(i).ticket).steps;
            G.eng.end_step(done);
            for (uint64_t t : done) {
                Request &r = reqs.at(t);
                complete(r, G.hres->p + (size_t)r.slot_idx * words, G);
                G.spec[r.slot_idx].off = 1;
                --G.queued;
            }
            if (!done.empty()) cv_done.notify_all();
        }
        return pending;
    }

    // Issue a step on every graph with requests and no step in flight;
    // returns true if any was issued.
    bool issue_locked()
    {
        bool issued = false;
        const uint32_t eighths = any_small() ? 7u : 8u;
        for (auto &kv : graphs) {
            Resident &G = *kv.second;
            if (G.eng.in_flight() || G.eng.active() == 0) continue;
            const std::vector<uint32_t> fresh = G.eng.take_fresh();
            if (!G.eng.begin_step(G.part, G.finishing)) continue;
            const uint32_t hw = G.eng.high_water();
            for (uint32_t i = 0; i < hw; ++i) {
                G.hstage->p[i] = G.spec[i];
                if (!G.eng.slot(i).used) G.hstage->p[i].off = 1;
            }
            TP_HIP(hipMemcpyAsync(G.dslots.get(), G.hstage->p, hw * sizeof(SlotSpec), hipMemcpyHostToDevice,
                                  G.stream));
            for (uint32_t i : fresh) zero_words(G.dout.get() + (size_t)i * words, words, G.stream);
            const bool labels = true;
            bool shared = false;
            for (uint32_t i : G.part) shared = shared || !reqs.at(G.eng.slot(i).ticket).solo;
            if (shared)
                multi_segment_enqueue(G.g, G.dslots.get(), hw, cfg.n_labels, labels, G.dout.get(),
                                      G.dout.get() + (size_t)cfg.max_slots * words, G.eng.cursor(), G.eng.n_seg(),
                                      G.small ? 8u : eighths, G.stream);
            for (uint32_t i : G.part) {
                Request &r = reqs.at(G.eng.slot(i).ticket);
                if (r.solo)
                    solo_segment_enqueue(G.g, &r.spec, r.dres.get(), G.eng.cursor(), G.eng.n_seg(),
                                         G.small ? 8u : eighths, G.stream);
            }
            for (uint32_t i : G.finishing) {
                Request &r = reqs.at(G.eng.slot(i).ticket);
                if (r.solo)
                    TP_HIP(hipMemcpyAsync(r.hres->p, r.dres.get(), TP_RW_SCRATCH * 8, hipMemcpyDeviceToHost,
                                          G.stream));
                else
                    TP_HIP(hipMemcpyAsync(G.hres->p + (size_t)i * words, G.dout.get() + (size_t)i * words,
                                          words * 8, hipMemcpyDeviceToHost, G.stream));
            }
            TP_HIP(hipEventRecord(G.ev, G.stream));
            ++steps;
            issued = true;
        }
        return issued;
    }

    void run()
    {
        std::unique_lock<std::mutex> lk(mu);
        try {
            TP_HIP(hipSetDevice(device));
            while (!stop) {
                admit_locked();
                bool busy = reap_locked();
                if (admit_locked()) busy = true;
                if (issue_locked()) busy = true;
                busy = busy || reap_locked();
                if (busy) {
                    // steps are in flight: poll their events
                    lk.unlock();
                    std::this_thread::sleep_for(std::chrono::microseconds(50));
                    lk.lock();
                } else {
                    cv_work.wait(lk);
                }
            }
        } catch (const Error &e) {
            fail_all(e.msg);
        } catch (const std::exception &e) {
            fail_all(e.what());
        }
    }
};

namespace {

void check_served_spec(tp_server *srv, const tp_graph *g, const tp_survey_spec *sp)
{
    if (!sp) fail(TP_ERR_INVALID, "tripoll_server_submit: NULL spec");
    const uint32_t known = TP_OUT_COUNT | TP_OUT_CLOSE_HIST | TP_OUT_LABEL_TABLE | TP_OUT_SPREAD_COUNT |
                           TP_OUT_OPEN_CLOSE | TP_OUT_MAX_EDGE | TP_OUT_DEGREE_TABLE | TP_OUT_DIRECTED;
    if (sp->outputs & ~known) fail(TP_ERR_INVALID, "tripoll_server_submit: unknown output bits");
    if ((sp->outputs & TP_OUT_MAX_EDGE) && sp->max_edge_shift > 31)
        fail(TP_ERR_INVALID, "tripoll_server_submit: max_edge_shift must be in 0..31");
    if ((sp->outputs & TP_OUT_DIRECTED) && !g->directed)
        fail(TP_ERR_INVALID, "tripoll_server_submit: the directed census needs a graph built with TP_EDGES_DIRECTED");
    if (sp->reserved != 0) fail(TP_ERR_INVALID, "tripoll_server_submit: reserved field must be 0");
    if (sp->filters & ~(TP_FILT_WINDOW | TP_FILT_LABEL_MASK))
        fail(TP_ERR_INVALID, "tripoll_server_submit: unknown filter bits");
    if (sp->strategy > TP_STRAT_TABLE_STRESS) fail(TP_ERR_INVALID, "tripoll_server_submit: unknown strategy");
    const bool labels = (sp->outputs & TP_OUT_LABEL_TABLE) || (sp->filters & TP_FILT_LABEL_MASK);
    if (labels) {
        if (sp->n_labels != srv->cfg.n_labels)
            fail(TP_ERR_INVALID, "tripoll_server_submit: n_labels must be the server's (" +
                                     std::to_string(srv->cfg.n_labels) + ")");
        if (g->stats.max_label >= sp->n_labels)
            fail(TP_ERR_INVALID, "tripoll_server_submit: graph has label " + std::to_string(g->stats.max_label) +
                                     " >= n_labels");
    }
    if ((sp->filters & TP_FILT_WINDOW) && sp->t_lo > sp->t_hi)
        fail(TP_ERR_INVALID, "tripoll_server_submit: t_lo > t_hi");
}

void check_alive(tp_server *srv)
{
    if (!srv->fatal.empty()) fail(TP_ERR_DEVICE, "server stopped after a device error: " + srv->fatal);
}

}  // namespace

extern "C" tp_status tripoll_server_create(const tp_server_config *cfg, tp_server **out)
{
    return guard([&] {
        if (!out) fail(TP_ERR_INVALID, "tripoll_server_create: NULL argument");
        tp_server_config c = cfg ? *cfg : tp_server_config{};
        if (c.max_slots == 0) c.max_slots = 8;
        if (c.n_labels == 0) c.n_labels = 8;
        if (c.step_wedges == 0) c.step_wedges = 1ull << 34;
        if (c.max_queue == 0) c.max_queue = 4096;
        if (c.max_slots > kMaxSlots) fail(TP_ERR_INVALID, "tripoll_server_create: max_slots must be 1..16");
        if (c.n_labels > TP_MAX_LABELS) fail(TP_ERR_INVALID, "tripoll_server_create: n_labels must be 1..16");
        auto srv = std::make_unique<tp_server>();
        TP_HIP(hipGetDevice(&srv->device));
        if (c.hbm_budget == 0) {
            size_t free_b = 0, total_b = 0;
            TP_HIP(hipMemGetInfo(&free_b, &total_b));
            c.hbm_budget = (uint64_t)(free_b * 0.9);
        }
        srv->cfg = c;
        srv->words = slot_words(c.n_labels);
        srv->budget = sched::Budget(c.hbm_budget);
        srv->queue = sched::Queue(c.max_queue);
        TP_HIP(hipStreamCreateWithFlags(&srv->big, hipStreamNonBlocking));
        TP_HIP(hipStreamCreateWithFlags(&srv->small, hipStreamNonBlocking));
        tp_server *p = srv.get();
        srv->worker = std::thread([p] { p->run(); });
        *out = srv.release();
    });
}

extern "C" tp_status tripoll_server_destroy(tp_server *srv)
{
    return guard([&] {
        if (!srv) return;
        {
            std::lock_guard<std::mutex> lk(srv->mu);
            srv->stop = true;
        }
        srv->cv_work.notify_all();
        if (srv->worker.joinable()) srv->worker.join();
        (void)hipStreamSynchronize(srv->big);
        (void)hipStreamSynchronize(srv->small);
        delete srv;
    });
}

extern "C" tp_status tripoll_server_add_graph(tp_server *srv, const tp_edge_list *edges, uint32_t *graph_id)
{
    return guard([&] {
        if (!srv || !edges || !graph_id) fail(TP_ERR_INVALID, "tripoll_server_add_graph: NULL argument");
        {
            std::lock_guard<std::mutex> lk(srv->mu);
            check_alive(srv);
        }
        // build on the large-graph stream (the graph's arrays remember it)
        tp_graph *g = nullptr;
        const tp_status st = tripoll_build(edges, srv->big, &g);
        if (st != TP_OK) throw Error{st, tripoll_last_error()};
        auto R = std::make_unique<Resident>();
        R->g = g;
        const uint64_t probes = g->stats.probes;
        const uint64_t nseg = std::max<uint64_t>(1, (probes + srv->cfg.step_wedges - 1) / srv->cfg.step_wedges);
        R->small = nseg == 1;
        R->eng = sched::Engine(srv->cfg.max_slots, (uint32_t)std::min<uint64_t>(nseg, 4096));
        R->stream = R->small ? srv->small : srv->big;
        R->dslots.reset(kMaxSlots, srv->big);
        R->dout.reset((size_t)srv->cfg.max_slots * srv->words + kClaimWords, srv->big);
        R->hstage = std::make_unique<HostArray<SlotSpec>>(kMaxSlots);
        R->hres = std::make_unique<HostArray<unsigned long long>>((size_t)srv->cfg.max_slots * srv->words);
        R->spec.assign(srv->cfg.max_slots, SlotSpec{});
        for (auto &s : R->spec) s.off = 1;
        TP_HIP(hipEventCreateWithFlags(&R->ev, hipEventDisableTiming));
        R->bytes = g->stats.device_bytes + R->dslots.bytes() + R->dout.bytes();
        std::lock_guard<std::mutex> lk(srv->mu);
        check_alive(srv);
        if (!srv->budget.take(R->bytes))
            fail(TP_ERR_OOM, "tripoll_server_add_graph: " + std::to_string(R->bytes) +
                                 " bytes exceed the server's remaining budget of " +
                                 std::to_string(srv->budget.cap() - srv->budget.used()));
        R->id = srv->next_graph++;
        *graph_id = R->id;
        srv->graphs[R->id] = std::move(R);
    });
}

extern "C" tp_status tripoll_server_remove_graph(tp_server *srv, uint32_t graph_id)
{
    return guard([&] {
        if (!srv) fail(TP_ERR_INVALID, "tripoll_server_remove_graph: NULL server");
        std::unique_ptr<Resident> R;
        {
            std::lock_guard<std::mutex> lk(srv->mu);
            auto it = srv->graphs.find(graph_id);
            if (it == srv->graphs.end()) fail(TP_ERR_NOT_FOUND, "tripoll_server_remove_graph: unknown graph");
            if (it->second->queued || it->second->eng.in_flight())
                fail(TP_ERR_BUSY, "tripoll_server_remove_graph: requests on the graph are not complete");
            srv->budget.give(it->second->bytes);
            R = std::move(it->second);
            srv->graphs.erase(it);
        }
        R.reset();  // releases the graph outside the lock
    });
}

extern "C" tp_status tripoll_server_graph_stats(tp_server *srv, uint32_t graph_id, tp_graph_stats *out)
{
    return guard([&] {
        if (!srv || !out) fail(TP_ERR_INVALID, "tripoll_server_graph_stats: NULL argument");
        std::lock_guard<std::mutex> lk(srv->mu);
        auto it = srv->graphs.find(graph_id);
        if (it == srv->graphs.end()) fail(TP_ERR_NOT_FOUND, "tripoll_server_graph_stats: unknown graph");
        *out = it->second->g->stats;
    });
}

extern "C" tp_status tripoll_server_graph(tp_server *srv, uint32_t graph_id, const tp_graph **out)
{
    return guard([&] {
        if (!srv || !out) fail(TP_ERR_INVALID, "tripoll_server_graph: NULL argument");
        std::lock_guard<std::mutex> lk(srv->mu);
        auto it = srv->graphs.find(graph_id);
        if (it == srv->graphs.end()) fail(TP_ERR_NOT_FOUND, "tripoll_server_graph: unknown graph");
        *out = it->second->g;
    });
}

extern "C" tp_status tripoll_server_submit(tp_server *srv, uint32_t graph_id, const tp_survey_spec *spec,
                                           uint32_t tag, uint64_t *ticket)
{
    return guard([&] {
        if (!srv || !ticket) fail(TP_ERR_INVALID, "tripoll_server_submit: NULL argument");
        if (tag >= TP_SERVER_TAGS) fail(TP_ERR_INVALID, "tripoll_server_submit: tag must be 0..7");
        std::lock_guard<std::mutex> lk(srv->mu);
        check_alive(srv);
        auto it = srv->graphs.find(graph_id);
        if (it == srv->graphs.end()) fail(TP_ERR_NOT_FOUND, "tripoll_server_submit: unknown graph");
        check_served_spec(srv, it->second->g, spec);
        Request r;
        r.ticket = srv->next_ticket;
        r.graph = graph_id;
        r.tag = tag;
        r.spec = *spec;
        r.slot = make_slot(*spec);
        r.solo = (spec->outputs & kSoloOutputs) != 0;
        r.mem = r.solo ? (uint64_t)TP_RESULT_WORDS * 8 : (uint64_t)srv->words * 8 + sizeof(SlotSpec);
        r.t_arrive = now_us();
        if (!srv->queue.push(r.ticket)) {
            ++srv->rejected;
            fail(TP_ERR_BUSY, "tripoll_server_submit: request queue is full");
        }
        ++srv->next_ticket;
        ++srv->submitted;
        ++it->second->queued;
        if (srv->t_first < 0) srv->t_first = r.t_arrive;
        *ticket = r.ticket;
        srv->reqs.emplace(r.ticket, std::move(r));
        srv->cv_work.notify_all();
    });
}

extern "C" tp_status tripoll_server_wait(tp_server *srv, uint64_t ticket, int64_t timeout_us, tp_survey_result *out,
                                         tp_request_info *info)
{
    return guard([&] {
        if (!srv || !out) fail(TP_ERR_INVALID, "tripoll_server_wait: NULL argument");
        std::unique_lock<std::mutex> lk(srv->mu);
        if (srv->reqs.find(ticket) == srv->reqs.end()) fail(TP_ERR_NOT_FOUND, "tripoll_server_wait: unknown ticket");
        // submissions may rehash the table while this thread waits: look the
        // ticket up afresh every time
        auto ready = [&] {
            auto j = srv->reqs.find(ticket);
            return j == srv->reqs.end() || j->second.state >= 2;
        };
        if (timeout_us < 0) {
            srv->cv_done.wait(lk, ready);
        } else if (!srv->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), ready)) {
            fail(TP_ERR_BUSY, "tripoll_server_wait: request not complete");
        }
        auto it = srv->reqs.find(ticket);
        if (it == srv->reqs.end()) fail(TP_ERR_NOT_FOUND, "tripoll_server_wait: ticket taken by another caller");
        Request r = std::move(it->second);
        srv->reqs.erase(it);
        if (r.state == 3) fail(TP_ERR_DEVICE, "tripoll_server_wait: " + r.error);
        *out = r.res;
        if (info) {
            info->tag = r.tag;
            info->steps = r.steps;
            info->arrival_us = r.t_arrive;
            info->admit_us = r.t_admit;
            info->done_us = r.t_done;
        }
    });
}

extern "C" tp_status tripoll_server_stats(tp_server *srv, tp_server_stats *out)
{
    return guard([&] {
        if (!srv || !out) fail(TP_ERR_INVALID, "tripoll_server_stats: NULL argument");
        std::lock_guard<std::mutex> lk(srv->mu);
        std::memset(out, 0, sizeof(*out));
        out->submitted = srv->submitted;
        out->completed = srv->completed;
        out->rejected = srv->rejected;
        for (auto &kv : srv->reqs) {
            if (kv.second.state == 0) ++out->waiting;
            if (kv.second.state == 1) ++out->running;
        }
        out->steps = srv->steps;
        out->triangles = srv->triangles;
        out->hbm_used = srv->budget.used();
        out->hbm_budget = srv->budget.cap();
        out->elapsed_s = srv->t_first >= 0 && srv->t_last > srv->t_first ? (srv->t_last - srv->t_first) * 1e-6 : 0.0;
        for (uint32_t t = 0; t < TP_SERVER_TAGS; ++t) {
            std::vector<double> v = srv->lat_ms[t];
            out->count[t] = v.size();
            out->p50_ms[t] = sched::percentile(v, 0.50);
            out->p99_ms[t] = sched::percentile(v, 0.99);
        }
    });
}
