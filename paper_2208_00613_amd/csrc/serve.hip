// serve.hip -- the serving loop: IMM queries against one device-resident graph with
// continuous batching under a budget for RR stores.
//
// Two worker threads own the device work, each on a stream of its own, so sampling and
// selection of different queries overlap.  The sampler admits queued queries while slots
// and store memory allow, then runs one sampling block for every admitted query short of
// its target, all in shared launches; a query that reaches its target passes to the
// selector, which runs one batched greedy selection over every query handed to it and
// passes each back (next round) or finishes it.  A query that arrives while others run
// joins at the sampler's next step; a finished query frees its slot and store at once.
//
// Budget: the sum of the admitted queries' store bytes (index + payload + bitmap rows, as
// reported in hbm_store_stats) stays within the budget.  A sampling block is bounded by
// the room left, priced at the query's own bytes per set so far (or the running mean of
// finished queries).  When no admitted query can move and none is ready to select, the
// youngest one is preempted: its store is dropped and it goes back to the head of the
// queue, to be recomputed later with the same result (RR sets are pure functions of their
// index).  A query alone that still does not fit fails with HBM_EBUDGET.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>

#include "hbm_imm.h"

namespace hbm {
namespace {

struct Ticket {
    int64_t id = 0;
    hbm_query q{};
    double t_submit = 0;
    int32_t preemptions = 0;
};

struct Result {
    bool done = false;
    hbm_status status = HBM_OK;
    std::string error;
    std::vector<int32_t> seeds;
    std::vector<uint64_t> gains;
    hbm_imm_stats st{};
    double t_submit = 0, t_admit = -1, t_done = 0;
    int32_t preemptions = 0;
};

struct Slot {
    std::unique_ptr<Ctx> c;
    ImmJob job;
    Ticket t;
    double t_admit = 0;
    int64_t order = 0;  // admission sequence number
    bool busy = false;
    bool selecting = false;  // owned by the selector thread (else by the sampler)
};

// The store buffers of a finished query go back to the device; its sampling arena stays
// with the slot for the next query.
void release_store(Ctx &c) {
    Store &s = c.s;
    for (Buf *b : {&s.hist, &s.warm, &s.hot, &s.hot_rank, &s.bitmap, &s.raw_off, &s.raw_mem, &s.lens, &s.codes,
                   &s.symtab, &s.cbtab, &s.lut, &s.bitoff, &s.payload, &s.ckb, &s.mtmp, &s.ar_hot, &s.ar_rank,
                   &s.ar_off, &s.ar_low, &s.ar_tmp, &s.ar_keys, &s.ar_sort, &s.enc8})
        buf_free(c, *b);
    store_reset(c);
}

}  // namespace
}  // namespace hbm

using hbm::Ctx;

struct hbm_server {
    Ctx root;   // the sampler's stream, launch descriptors and scan space
    Ctx rootL;  // the selector's
    int64_t budget = 0;
    int32_t max_active = 1;
    int enc = HBM_ENC_NONE;
    double warmup_frac = 0.1, hot_frac = 0.01, hot_min_density = 0.0;
    bool implicit_roots = false, containers = false;
    hbm::DGraph graph;  // borrowed from the graph context
    std::chrono::steady_clock::time_point t0;

    std::mutex mu;
    std::condition_variable cv;       // sampler: an event (arrival, hand-back, completion) or stop
    std::condition_variable cvL;      // selector: a query handed over, or stop
    uint64_t events = 0;              // counts the sampler's wake-up events
    std::condition_variable cv_done;  // a query finished
    std::deque<hbm::Ticket> queue;
    std::map<int64_t, hbm::Result> results;
    int64_t next_id = 1;
    int64_t next_order = 0;
    bool stop = false;
    bool broken = false;
    std::string error;
    hbm_server_stats stats{};

    std::vector<std::unique_ptr<hbm::Slot>> slots;  // touched by the worker only
    int32_t active = 0;                             // busy slots (written under mu)
    double bps_mean = 0;                            // store bytes per set of finished queries
    int64_t bps_n = 0;
    bool hold = false;  // no admissions between a preemption and the next completion
    std::thread worker, worker_sel;

    double now_ms() const {
        return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
    double est_bps(const hbm::Slot &s) const {
        const Ctx &c = *s.c;
        if (c.s.nsets >= 1024) return (double)hbm::store_bytes(c) / (double)c.s.nsets;
        return bps_n ? bps_mean : 64.0;
    }
    void loop();
    void loop_select();
    void admit_locked();
    bool step(std::vector<hbm::Slot *> live);
    void finish_locked(hbm::Slot &s);
    void preempt_locked(hbm::Slot &s);
    void fail_all_locked(hbm_status st, const std::string &msg);
};

void hbm_server::finish_locked(hbm::Slot &s) {
    hbm::ImmJob &J = s.job;
    hbm::Result &R = results[s.t.id];
    R.done = true;
    R.status = J.phase == hbm::ImmJob::DONE ? HBM_OK : J.status;
    R.error = J.error;
    R.seeds = J.seeds;
    R.gains = J.gains;
    R.st = J.st;
    R.t_submit = s.t.t_submit;
    R.t_admit = s.t_admit;
    R.t_done = now_ms();
    R.preemptions = s.t.preemptions;
    if (R.status == HBM_OK) {
        stats.completed++;
        const double b = (double)J.st.store.store_bytes / (double)std::max<int64_t>(J.st.nsets_final, 1);
        bps_mean = (bps_mean * (double)bps_n + b) / (double)(bps_n + 1);
        bps_n++;
    } else {
        stats.failed++;
    }
    hbm::release_store(*s.c);
    s.busy = false;
    s.selecting = false;
    active--;
    hold = false;
    events++;
    cv.notify_all();
    cv_done.notify_all();
}

void hbm_server::fail_all_locked(hbm_status st, const std::string &msg) {
    broken = true;
    stop = true;
    error = msg;
    for (auto &sp : slots)
        if (sp->busy) {
            sp->job.phase = hbm::ImmJob::FAILED;
            sp->job.status = st;
            sp->job.error = msg;
            hbm::Result &R = results[sp->t.id];
            R.done = true;
            R.status = st;
            R.error = msg;
            R.t_submit = sp->t.t_submit;
            R.t_done = now_ms();
            sp->busy = false;
            stats.failed++;
        }
    active = 0;
    for (const hbm::Ticket &t : queue) {
        hbm::Result &R = results[t.id];
        R.done = true;
        R.status = st;
        R.error = msg;
        R.t_submit = t.t_submit;
        R.t_done = now_ms();
        stats.failed++;
    }
    queue.clear();
    cv.notify_all();
    cvL.notify_all();
    cv_done.notify_all();
}

// Admit queued queries in arrival order while a slot is free and the budget has room for
// their first estimation round (priced at the running bytes-per-set estimate).
void hbm_server::admit_locked() {
    double used = 0;
    for (auto &sp : slots)
        if (sp->busy) {
            const hbm::Ctx &c = *sp->c;
            // a query still short of its first round holds a reservation for it
            const double have = (double)hbm::store_bytes(c);
            // (the selector's queries are not read: their job state is the selector's)
            const double need =
                !sp->selecting && sp->job.st.rounds == 0 ? (double)sp->job.target * est_bps(*sp) : 0.0;
            used += std::max(have, need);
        }
    while (!queue.empty() && active < max_active && !(hold && active > 0)) {
        const hbm::Ticket t = queue.front();
        double reserve = 0;
        if (t.q.k >= 1 && t.q.k <= graph.n && t.q.eps > 0 && t.q.l > 0 && graph.n >= 2) {
            const hbm::ImmParams P = hbm::imm_params(graph.n, t.q.k, t.q.eps, t.q.l);
            reserve = std::ceil(P.lambda_prime / ((double)graph.n / 2.0)) * (bps_n ? bps_mean : 64.0);
        }
        if (active > 0 && used + reserve > (double)budget) break;
        queue.pop_front();
        hbm::Slot *s = nullptr;
        for (auto &sp : slots)
            if (!sp->busy) {
                s = sp.get();
                break;
            }
        if (!s) {
            slots.push_back(std::make_unique<hbm::Slot>());
            s = slots.back().get();
            s->c = std::make_unique<Ctx>();
            Ctx &c = *s->c;
            c.device = root.device;
            c.stream = root.stream;
            c.num_cus = root.num_cus;
            c.ic_tier1 = root.ic_tier1;
            c.ic_t1_budget = root.ic_t1_budget;
            c.block_sets = root.block_sets;
            c.lt_lw = root.lt_lw;
            c.t2_queue = root.t2_queue;
            c.t2_per_cu = root.t2_per_cu;
            c.t2_cap = int64_t(1) << 30;  // many queries share the device: fewer big-set slots each
            c.g = graph;
        }
        Ctx &c = *s->c;
        c.budget = budget;
        c.s.enc_req = c.s.enc = enc;
        c.s.implicit_roots = implicit_roots;
        c.s.containers = containers;
        c.s.warmup_frac = warmup_frac;
        c.s.hot_frac = hot_frac;
        c.s.hot_min_density = hot_min_density;
        s->t = t;
        s->t_admit = now_ms();
        s->order = next_order++;
        s->busy = true;
        s->selecting = false;
        c.stream = root.stream;
        active++;
        stats.admitted++;
        hbm::ImmJob &J = s->job;
        J = hbm::ImmJob{};
        J.c = &c;
        J.k = t.q.k;
        J.eps = t.q.eps;
        J.l = t.q.l;
        J.seed = t.q.seed;
        hbm::imm_start(J);
        if (J.phase == hbm::ImmJob::FAILED) {
            finish_locked(*s);
            continue;
        }
        used += reserve;
        stats.peak_active = std::max<int64_t>(stats.peak_active, active);
    }
}

// One sampling step over the sampler's queries (oldest first).  Returns whether anything
// moved; if nothing could, the caller waits for the selector or a completion.
bool hbm_server::step(std::vector<hbm::Slot *> live) {
    std::sort(live.begin(), live.end(), [](const hbm::Slot *a, const hbm::Slot *b) { return a->order < b->order; });
    std::vector<int64_t> cap(live.size(), -1);
    {
        std::lock_guard<std::mutex> lk(mu);
        // sampling caps from the room the budget leaves over every admitted store
        double used = 0;
        bool selector_busy = false;
        for (auto &sp : slots)
            if (sp->busy) {
                used += (double)hbm::store_bytes(*sp->c);
                selector_busy |= sp->selecting;
            }
        double room = (double)budget - used;
        bool moves = false;
        for (size_t i = 0; i < live.size(); i++) {
            hbm::ImmJob &J = live[i]->job;
            const Ctx &c = *live[i]->c;
            if (!hbm::imm_sampling(J) || c.s.nsets >= J.target) {
                moves = true;  // ready to select
                continue;
            }
            const int64_t want = std::min<int64_t>(J.target - c.s.nsets, root.block_sets);
            const double bps = est_bps(*live[i]);
            const int64_t allow = room > 0 ? (int64_t)std::min(room / bps, 9.0e18) : 0;
            int64_t cp = std::min(want, allow);
            if (c.s.enc != HBM_ENC_NONE && !c.s.model_ready) {
                // a warm-up block runs whatever the room; its sets are stored (after the model
                // is built from the first W of them) only when the cap covers the warm-up
                if (c.s.wcur > 0 || cp < c.s.W) cp = 0;
                cap[i] = cp;
                room -= (double)cp * bps;
                moves = true;
                continue;
            }
            if (cp < std::min<int64_t>(want, 4096)) cp = 0;  // wait for room rather than crawl
            cap[i] = cp;
            room -= (double)cp * bps;
            moves |= cp > 0;
        }
        if (!moves) {
            if (selector_busy) return false;  // its queries will finish or hand back room
            if (live.size() > 1) {
                preempt_locked(*live.back());  // the youngest restarts later with the same result
                return true;
            }
            cap[0] = -1;  // alone: the context budget decides (HBM_EBUDGET if it cannot fit)
        }
    }
    std::vector<hbm::ImmJob *> jobs;
    for (hbm::Slot *s : live) jobs.push_back(&s->job);
    hbm::imm_sample_step(root, jobs, cap);
    std::lock_guard<std::mutex> lk(mu);
    stats.steps++;
    for (hbm::Slot *s : live) {
        if (s->job.phase == hbm::ImmJob::FAILED) {
            finish_locked(*s);
        } else if (hbm::imm_selecting(s->job)) {
            s->selecting = true;  // hand over: the selector runs on its own stream
            s->c->stream = rootL.stream;
            cvL.notify_all();
        }
    }
    // a block priced too low may overshoot: the youngest sampling queries give their room back
    int64_t bytes = 0;
    for (auto &sp : slots)
        if (sp->busy) bytes += hbm::store_bytes(*sp->c);
    for (size_t i = live.size(); i-- > 0 && bytes > budget;) {
        if (!live[i]->busy || live[i]->selecting || active <= 1) continue;
        bytes -= hbm::store_bytes(*live[i]->c);
        preempt_locked(*live[i]);
    }
    stats.peak_store_bytes = std::max<int64_t>(stats.peak_store_bytes, bytes);
    return true;
}

void hbm_server::preempt_locked(hbm::Slot &y) {
    hbm::Ticket t = y.t;
    t.preemptions++;
    queue.push_front(t);
    hbm::release_store(*y.c);
    y.busy = false;
    active--;
    hold = true;
    stats.preemptions++;
    events++;
}

void hbm_server::loop() {
    (void)hipSetDevice(root.device);
    uint64_t seen = ~0ull;
    bool progressed = true;
    for (;;) {
        std::vector<hbm::Slot *> live;
        {
            std::unique_lock<std::mutex> lk(mu);
            cv.wait(lk, [&] {
                if (stop || events != seen) return true;
                if (!progressed) return false;
                for (auto &sp : slots)
                    if (sp->busy && !sp->selecting) return true;
                return false;
            });
            if (stop) break;
            seen = events;
            admit_locked();
            for (auto &sp : slots)
                if (sp->busy && !sp->selecting) live.push_back(sp.get());
        }
        if (live.empty()) {
            progressed = false;
            continue;
        }
        try {
            progressed = step(live);
        } catch (const hbm::Error &e) {
            std::lock_guard<std::mutex> lk(mu);
            fail_all_locked(e.st, e.msg);
            break;
        } catch (const std::exception &e) {
            std::lock_guard<std::mutex> lk(mu);
            fail_all_locked(HBM_EDEVICE, e.what());
            break;
        }
    }
}

void hbm_server::loop_select() {
    (void)hipSetDevice(rootL.device);
    for (;;) {
        std::vector<hbm::Slot *> live;
        {
            std::unique_lock<std::mutex> lk(mu);
            cvL.wait(lk, [&] {
                if (stop) return true;
                for (auto &sp : slots)
                    if (sp->busy && sp->selecting) return true;
                return false;
            });
            if (stop) break;
            for (auto &sp : slots)
                if (sp->busy && sp->selecting) live.push_back(sp.get());
        }
        try {
            std::vector<hbm::ImmJob *> jobs;
            for (hbm::Slot *s : live) jobs.push_back(&s->job);
            hbm::imm_select_step(rootL, jobs);
        } catch (const hbm::Error &e) {
            std::lock_guard<std::mutex> lk(mu);
            fail_all_locked(e.st, e.msg);
            break;
        } catch (const std::exception &e) {
            std::lock_guard<std::mutex> lk(mu);
            fail_all_locked(HBM_EDEVICE, e.what());
            break;
        }
        std::lock_guard<std::mutex> lk(mu);
        stats.steps++;
        for (hbm::Slot *s : live) {
            if (s->job.phase == hbm::ImmJob::DONE || s->job.phase == hbm::ImmJob::FAILED) {
                finish_locked(*s);
            } else {
                s->selecting = false;  // hand back to the sampler for the next round
                s->c->stream = root.stream;
            }
        }
        events++;
        cv.notify_all();
    }
}

extern "C" {

hbm_status hbm_server_create(hbm_server **out, hbm_ctx *graph, int64_t store_budget, int32_t max_active) {
    if (!out || !graph || store_budget <= 0 || max_active < 1) return HBM_EINVAL;
    *out = nullptr;
    Ctx &g = graph->c;
    if (!g.g.loaded) return HBM_ESTATE;
    if (hipSetDevice(g.device) != hipSuccess) return HBM_EDEVICE;
    if (hipStreamSynchronize(g.stream) != hipSuccess) return HBM_EDEVICE;
    hbm_server *s = new (std::nothrow) hbm_server;
    if (!s) return HBM_ENOMEM;
    s->root.device = g.device;
    s->root.num_cus = g.num_cus;
    s->root.ic_tier1 = g.ic_tier1;
    s->root.ic_t1_budget = g.ic_t1_budget;
    s->root.block_sets = g.block_sets;
    s->root.lt_lw = g.lt_lw;
    s->root.t2_queue = g.t2_queue;
    s->root.t2_per_cu = g.t2_per_cu;
    if (hipStreamCreateWithFlags(&s->root.stream, hipStreamNonBlocking) != hipSuccess) {
        delete s;
        return HBM_EDEVICE;
    }
    s->rootL.device = g.device;
    s->rootL.num_cus = g.num_cus;
    s->rootL.select_graph = g.select_graph;  // the selector thread drives the greedy launches
    if (hipStreamCreateWithFlags(&s->rootL.stream, hipStreamNonBlocking) != hipSuccess) {
        (void)hipStreamDestroy(s->root.stream);
        delete s;
        return HBM_EDEVICE;
    }
    s->budget = store_budget;
    s->max_active = max_active;
    s->enc = g.s.enc_req;
    s->warmup_frac = g.s.warmup_frac;
    s->hot_frac = g.s.hot_frac;
    s->hot_min_density = g.s.hot_min_density;
    s->implicit_roots = g.s.implicit_roots;
    s->containers = g.s.containers;
    s->graph = g.g;
    s->graph.borrowed = true;
    s->t0 = std::chrono::steady_clock::now();
    try {
        s->worker = std::thread([s] { s->loop(); });
        s->worker_sel = std::thread([s] { s->loop_select(); });
    } catch (...) {
        {
            std::lock_guard<std::mutex> lk(s->mu);
            s->stop = true;
        }
        s->cv.notify_all();
        s->cvL.notify_all();
        if (s->worker.joinable()) s->worker.join();
        (void)hipStreamDestroy(s->root.stream);
        (void)hipStreamDestroy(s->rootL.stream);
        delete s;
        return HBM_ENOMEM;
    }
    *out = s;
    return HBM_OK;
}

void hbm_server_destroy(hbm_server *s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv.notify_all();
    s->cvL.notify_all();
    if (s->worker.joinable()) s->worker.join();
    if (s->worker_sel.joinable()) s->worker_sel.join();
    (void)hipSetDevice(s->root.device);
    (void)hipStreamSynchronize(s->root.stream);
    (void)hipStreamSynchronize(s->rootL.stream);
    for (auto &sp : s->slots) {
        Ctx &c = *sp->c;
        try {
            hbm::select_free(c);
            hbm::store_free(c);
            for (hbm::Buf *b : {&c.scan_tmp, &c.ctrl_arena, &c.tails, &c.bkeys, &c.dctr, &c.xmeta, &c.pfind,
                                &c.spill0, &c.spill, &c.spill2})
                hbm::buf_free(c, *b);
            hbm::stage_free(c);
        } catch (...) {
        }
    }
    try {
        hbm::select_free(s->root);
        hbm::select_free(s->rootL);
        for (hbm::Buf *b : {&s->root.scan_tmp, &s->root.ctrl_arena, &s->root.tails, &s->root.bkeys,
                            &s->root.dctr, &s->root.xmeta, &s->root.pfind, &s->root.spill0, &s->root.spill,
                            &s->root.spill2})
            hbm::buf_free(s->root, *b);
        hbm::stage_free(s->root);
        for (hbm::Buf *b : {&s->rootL.scan_tmp, &s->rootL.ctrl_arena, &s->rootL.tails, &s->rootL.bkeys, &s->rootL.dctr,
                            &s->rootL.xmeta, &s->rootL.pfind, &s->rootL.spill0, &s->rootL.spill,
                            &s->rootL.spill2})
            hbm::buf_free(s->rootL, *b);
        hbm::stage_free(s->rootL);
    } catch (...) {
    }
    (void)hipStreamDestroy(s->root.stream);
    (void)hipStreamDestroy(s->rootL.stream);
    delete s;
}

const char *hbm_server_last_error(const hbm_server *s) { return s ? s->error.c_str() : "null server"; }

hbm_status hbm_server_submit(hbm_server *s, const hbm_query *q, int64_t *ticket) {
    if (!s || !q || !ticket) return HBM_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->broken) return HBM_EDEVICE;
    hbm::Ticket t;
    t.id = s->next_id++;
    t.q = *q;
    t.t_submit = s->now_ms();
    s->queue.push_back(t);
    s->results[t.id] = hbm::Result{};
    s->results[t.id].t_submit = t.t_submit;
    s->stats.submitted++;
    *ticket = t.id;
    s->events++;
    s->cv.notify_all();
    return HBM_OK;
}

hbm_status hbm_server_poll(hbm_server *s, int64_t ticket, int32_t wait, int32_t *seeds, uint64_t *gains,
                           hbm_imm_stats *stats, hbm_serve_info *info) {
    if (!s || !info) return HBM_EINVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->results.find(ticket);
    if (it == s->results.end()) return HBM_EINVAL;
    if (wait) s->cv_done.wait(lk, [&] { return s->results[ticket].done; });
    const hbm::Result &R = it->second;
    std::memset(info, 0, sizeof(*info));
    info->done = R.done ? 1 : 0;
    info->t_submit_ms = R.t_submit;
    info->t_admit_ms = R.t_admit;
    info->t_done_ms = R.t_done;
    info->preemptions = R.preemptions;
    info->status = R.status;
    if (!R.done) return HBM_OK;
    if (R.status == HBM_OK) {
        if (seeds) std::memcpy(seeds, R.seeds.data(), R.seeds.size() * 4);
        if (gains) std::memcpy(gains, R.gains.data(), R.gains.size() * 8);
        if (stats) *stats = R.st;
    } else {
        std::strncpy(info->error, R.error.c_str(), sizeof(info->error) - 1);
    }
    s->results.erase(it);
    return HBM_OK;
}

hbm_status hbm_server_get_stats(hbm_server *s, hbm_server_stats *out) {
    if (!s || !out) return HBM_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    *out = s->stats;
    out->active = s->active;
    out->queued = (int64_t)s->queue.size();
    return s->broken ? HBM_EDEVICE : HBM_OK;
}

}  // extern "C"
