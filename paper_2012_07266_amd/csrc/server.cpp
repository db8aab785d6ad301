// Serving loop: continuous batching of independent simulation requests on
// one GPU (the paper's use case of many fast simulations across cosmologies,
// introduction and Results; each request is a full MADLens forward model).
//
// Two host threads share the request queue:
//  - admission: takes queued requests in arrival order while fewer than
//    max_active run and their HBM footprint fits the budget.  It reuses an
//    idle arena of the same shape (new cosmology uploaded with
//    pm_reconfigure), else frees idle arenas, least recently used first,
//    and creates one on a stream of its own.  It then enqueues the seeded
//    initial conditions and hands the slot to the issue thread.
//  - issue, in one of two forms:
//    streams: keeps up to `depth` chunks of PM steps (pm_run: steps with the
//    projection of their shells) in flight on every running slot,
//    round-robin over slots, so the kernels of different requests overlap
//    on the device (as far as the device's hardware queues let streams run
//    side by side);
//    batched: attaches every running slot to the batch of its shape
//    (pm_batch_*: one launch per pass over the batch's slots, replayed from
//    a HIP graph) and keeps up to `depth` batched steps in flight per batch,
//    so same-shape requests step together in one set of launches whatever
//    the number of hardware queues.
//    When a slot has issued its last step it copies the maps to pinned host
//    memory; when that copy completes it hands the maps to the request and
//    returns the arena to the idle pool.
// The same kernels run as for a lone simulation, and paint and projection
// accumulate in fixed point, so a request's maps are bitwise the same alone
// and in any mix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/madlens.h"

namespace {

using clk = std::chrono::steady_clock;

struct Req {
    int64_t id = 0;
    pm_request r{};
    std::vector<double> z;
    std::vector<double> agrid;
    double t_submit = 0, t_admit = 0, t_done = 0;
    int state = 0;   // 0 queued, 1 running, 2 finished
    int status = 0;  // PM_OK or the error that ended it
    size_t need = 0;
    size_t kbytes = 0;
    std::vector<unsigned char> kappa;
};

struct Key {
    int np, nm, npix, nsrc, dtype;
    bool operator==(const Key& o) const {
        return np == o.np && nm == o.nm && npix == o.npix && nsrc == o.nsrc && dtype == o.dtype;
    }
};

struct Slot {
    pm_sim* sim = nullptr;
    hipStream_t st = nullptr;
    void* kdev = nullptr;
    void* khost = nullptr;
    size_t kbytes = 0;
    size_t bytes = 0;  // HBM held: arena + maps
    Key key{};
    std::shared_ptr<Req> req;
    int next = 0;
    std::deque<hipEvent_t> inflight;
    std::vector<hipEvent_t> spare;
    hipEvent_t done_ev = nullptr;
    bool finishing = false;
    double last_used = 0;

    void destroy() {
        if (sim) pm_destroy(sim);
        for (hipEvent_t e : inflight) (void)hipEventDestroy(e);
        for (hipEvent_t e : spare) (void)hipEventDestroy(e);
        if (done_ev) (void)hipEventDestroy(done_ev);
        if (kdev) (void)hipFree(kdev);
        if (khost) (void)hipHostFree(khost);
        if (st) (void)hipStreamDestroy(st);
        sim = nullptr;
        kdev = khost = nullptr;
        st = nullptr;
        done_ev = nullptr;
        inflight.clear();
        spare.clear();
    }
};

size_t elem_size(int dtype) { return dtype == PM_F64 ? 8 : 4; }

Key key_of(const pm_request& r) {
    return Key{r.p.np, r.p.nm, r.l.npix, r.l.nsrc, r.p.dtype};
}

}  // namespace

struct pm_srv {
    size_t budget = 0;
    int max_active = 1;
    int batch_cap = 0;  // 0: the streams form; else batches of this many slots
    int depth = 2;   // chunks in flight per request
    int chunk = 1;   // steps per chunk (1: finest interleaving)
    clk::time_point t0 = clk::now();

    std::mutex mu;
    std::condition_variable cv;
    std::deque<std::shared_ptr<Req>> queue;
    std::unordered_map<int64_t, std::shared_ptr<Req>> reqs;
    std::vector<std::unique_ptr<Slot>> idle;
    std::deque<std::unique_ptr<Slot>> ready;
    size_t used = 0;
    int running = 0;  // admitted and not finished
    int64_t next_id = 1;
    int64_t submitted = 0, completed = 0, failed = 0;
    int peak_running = 0;
    size_t peak_used = 0;
    bool stop = false;

    std::thread admit_thr, issue_thr;

    double now() const { return std::chrono::duration<double>(clk::now() - t0).count(); }

    void note_peaks() {
        peak_running = std::max(peak_running, running);
        peak_used = std::max(peak_used, used);
    }

    // Called with mu held: the request ends with `status`.
    void finish_locked(const std::shared_ptr<Req>& q, int status) {
        q->status = status;
        q->state = 2;
        q->t_done = now();
        if (status == PM_OK) ++completed;
        else ++failed;
        cv.notify_all();
    }

    void release_locked(std::unique_ptr<Slot> s) {
        s->req.reset();
        s->next = 0;
        s->finishing = false;
        s->last_used = now();
        idle.push_back(std::move(s));
        --running;
        cv.notify_all();
    }

    void admit_loop();
    void issue_loop();
    void issue_loop_batched();

    // Called with mu held: hand the maps over and return the slot.
    void complete_locked(std::unique_ptr<Slot> own, int rc) {
        Req& q = *own->req;
        if (rc == PM_OK)
            q.kappa.assign(reinterpret_cast<unsigned char*>(own->khost),
                           reinterpret_cast<unsigned char*>(own->khost) + own->kbytes);
        finish_locked(own->req, rc);
        release_locked(std::move(own));
    }
};

void pm_srv::admit_loop() {
    for (;;) {
        std::shared_ptr<Req> q;
        std::unique_ptr<Slot> slot;
        std::vector<std::unique_ptr<Slot>> victims;
        {
            std::unique_lock<std::mutex> lk(mu);
            cv.wait(lk, [&] { return stop || (!queue.empty() && running < max_active); });
            if (stop) return;
            q = queue.front();
            Key k = key_of(q->r);
            auto it = std::find_if(idle.begin(), idle.end(),
                                   [&](const std::unique_ptr<Slot>& s) { return s->key == k; });
            if (it != idle.end()) {
                slot = std::move(*it);
                idle.erase(it);
            } else {
                // evict idle arenas, least recently used first, until it fits
                std::sort(idle.begin(), idle.end(), [](const auto& a, const auto& b) {
                    return a->last_used < b->last_used;
                });
                size_t freed = 0, i = 0;
                while (used - freed + q->need > budget && i < idle.size()) freed += idle[i++]->bytes;
                if (used - freed + q->need > budget) {
                    if (running == 0) {  // can never fit
                        queue.pop_front();
                        finish_locked(q, PM_ENOMEM);
                    } else {
                        cv.wait(lk);  // a completion frees memory
                    }
                    continue;
                }
                for (size_t j = 0; j < i; ++j) victims.push_back(std::move(idle[j]));
                idle.erase(idle.begin(), idle.begin() + i);
                used -= freed;
                used += q->need;
            }
            queue.pop_front();
            q->state = 1;
            ++running;
            note_peaks();
        }
        for (auto& v : victims) v->destroy();
        victims.clear();

        int rc = PM_OK;
        if (!slot) {
            slot.reset(new Slot);
            slot->key = key_of(q->r);
            slot->kbytes = q->kbytes;
            slot->bytes = q->need;
            if (hipStreamCreateWithFlags(&slot->st, hipStreamNonBlocking) != hipSuccess ||
                hipMalloc(&slot->kdev, slot->kbytes) != hipSuccess ||
                hipHostMalloc(&slot->khost, slot->kbytes, hipHostMallocDefault) != hipSuccess ||
                hipEventCreateWithFlags(&slot->done_ev, hipEventDisableTiming) != hipSuccess)
                rc = PM_ENOMEM;
            if (rc == PM_OK) rc = pm_create(&q->r.p, &q->r.l, slot->st, &slot->sim);
        } else {
            rc = pm_reconfigure(slot->sim, &q->r.p, &q->r.l);
        }
        if (rc == PM_OK) rc = pm_init_ic_seed(slot->sim, q->r.seed, q->r.a_start);
        if (rc == PM_OK && hipMemsetAsync(slot->kdev, 0, slot->kbytes, slot->st) != hipSuccess)
            rc = PM_EDEVICE;
        std::lock_guard<std::mutex> lk(mu);
        if (rc != PM_OK) {
            finish_locked(q, rc);
            used -= slot->bytes;
            slot->destroy();
            --running;
            cv.notify_all();
            continue;
        }
        q->t_admit = now();
        slot->req = q;
        ready.push_back(std::move(slot));
    }
}

void pm_srv::issue_loop() {
    if (batch_cap > 0) return issue_loop_batched();
    std::vector<std::unique_ptr<Slot>> active;
    for (;;) {
        {
            std::lock_guard<std::mutex> lk(mu);
            while (!ready.empty()) {
                active.push_back(std::move(ready.front()));
                ready.pop_front();
            }
            if (stop && active.empty() && running == 0) return;
        }
        bool progress = false;
        for (size_t i = 0; i < active.size();) {
            Slot& s = *active[i];
            Req& q = *s.req;
            while (!s.inflight.empty() && hipEventQuery(s.inflight.front()) == hipSuccess) {
                s.spare.push_back(s.inflight.front());
                s.inflight.pop_front();
                progress = true;
            }
            int rc = PM_OK;
            while (rc == PM_OK && !s.finishing && (int)s.inflight.size() < depth &&
                   s.next < q.r.nsteps) {
                // a chunk of steps with their shells (pm_run: each readout also
                // starts the next step of the chunk)
                const int m = std::min(chunk, q.r.nsteps - s.next);
                rc = pm_run(s.sim, &q.agrid[s.next], m, s.kdev);
                hipEvent_t e = nullptr;
                if (!s.spare.empty()) {
                    e = s.spare.back();
                    s.spare.pop_back();
                } else if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
                    rc = PM_EDEVICE;
                }
                if (rc == PM_OK && hipEventRecord(e, s.st) != hipSuccess) rc = PM_EDEVICE;
                if (e) s.inflight.push_back(e);
                s.next += m;
                progress = true;
            }
            if (rc == PM_OK && !s.finishing && s.next == q.r.nsteps) {
                if (hipMemcpyAsync(s.khost, s.kdev, s.kbytes, hipMemcpyDeviceToHost, s.st) !=
                        hipSuccess ||
                    hipEventRecord(s.done_ev, s.st) != hipSuccess)
                    rc = PM_EDEVICE;
                s.finishing = true;
            }
            bool done = rc != PM_OK || (s.finishing && hipEventQuery(s.done_ev) == hipSuccess);
            if (!done) {
                ++i;
                continue;
            }
            // the stream is drained: sticky device status, then hand over
            if (hipStreamSynchronize(s.st) != hipSuccess && rc == PM_OK) rc = PM_EDEVICE;
            int dev = pm_sync(s.sim);
            if (rc == PM_OK) rc = dev;
            while (!s.inflight.empty()) {
                s.spare.push_back(s.inflight.front());
                s.inflight.pop_front();
            }
            std::unique_ptr<Slot> own = std::move(active[i]);
            active.erase(active.begin() + i);
            std::lock_guard<std::mutex> lk(mu);
            if (rc == PM_OK) {
                q.kappa.assign(reinterpret_cast<unsigned char*>(own->khost),
                               reinterpret_cast<unsigned char*>(own->khost) + own->kbytes);
            }
            finish_locked(own->req, rc);
            release_locked(std::move(own));
            progress = true;
        }
        if (!progress) std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
}

// The batched form.  One batch per shape (Np, Nm, npix, nsrc, dtype), each
// on a stream of its own; a slot stays attached from admission to its last
// step.  Per batch, up to `depth` steps are in flight; after the step that
// ends a slot's grid, the copy of its maps follows on the batch's stream.
void pm_srv::issue_loop_batched() {
    struct B {
        Key key{};
        pm_batch* b = nullptr;
        hipStream_t st = nullptr;
        std::vector<std::unique_ptr<Slot>> slots;
        std::vector<int> left;  // steps still to issue, per slot
        std::deque<hipEvent_t> inflight;
        std::vector<hipEvent_t> spare;
    };
    std::vector<std::unique_ptr<B>> batches;
    auto batch_for = [&](const Key& k, const pm_request& r) -> B* {
        for (auto& b : batches)
            if (b->key == k) return b.get();
        std::unique_ptr<B> nb(new B);
        nb->key = k;
        if (hipStreamCreateWithFlags(&nb->st, hipStreamNonBlocking) != hipSuccess) return nullptr;
        if (pm_batch_create(&r.p, &r.l, max_active, 1, nb->st, &nb->b) != PM_OK) {
            (void)hipStreamDestroy(nb->st);
            return nullptr;
        }
        batches.push_back(std::move(nb));
        return batches.back().get();
    };
    for (;;) {
        std::vector<std::unique_ptr<Slot>> fresh;
        {
            std::lock_guard<std::mutex> lk(mu);
            while (!ready.empty()) {
                fresh.push_back(std::move(ready.front()));
                ready.pop_front();
            }
            bool any = false;
            for (auto& b : batches) any = any || !b->slots.empty();
            if (stop && fresh.empty() && !any && running == 0) break;
        }
        bool progress = !fresh.empty();
        for (auto& s : fresh) {
            Req& q = *s->req;
            B* b = batch_for(s->key, q.r);
            int rc = b ? pm_batch_attach(b->b, s->sim, q.agrid.data(), q.r.nsteps, nullptr)
                       : PM_EDEVICE;
            if (rc == PM_OK) rc = pm_batch_lens(b->b, s->sim, s->kdev);
            if (rc != PM_OK) {
                std::lock_guard<std::mutex> lk(mu);
                finish_locked(s->req, rc);
                release_locked(std::move(s));
                continue;
            }
            b->slots.push_back(std::move(s));
            b->left.push_back(q.r.nsteps);
        }
        for (auto& bp : batches) {
            B& b = *bp;
            while (!b.inflight.empty() && hipEventQuery(b.inflight.front()) == hipSuccess) {
                b.spare.push_back(b.inflight.front());
                b.inflight.pop_front();
                progress = true;
            }
            bool work = false;
            for (int l : b.left) work = work || l > 0;
            int rc = PM_OK;
            while (rc == PM_OK && work && (int)b.inflight.size() < depth) {
                rc = pm_batch_step(b.b, nullptr);
                work = false;
                for (size_t i = 0; i < b.slots.size() && rc == PM_OK; ++i) {
                    if (b.left[i] <= 0) continue;
                    if (--b.left[i] == 0) {  // its last step: the maps follow
                        Slot& s = *b.slots[i];
                        if (hipMemcpyAsync(s.khost, s.kdev, s.kbytes, hipMemcpyDeviceToHost, b.st) !=
                                hipSuccess ||
                            hipEventRecord(s.done_ev, b.st) != hipSuccess)
                            rc = PM_EDEVICE;
                        s.finishing = true;
                    }
                    work = work || b.left[i] > 0;
                }
                hipEvent_t e = nullptr;
                if (!b.spare.empty()) {
                    e = b.spare.back();
                    b.spare.pop_back();
                } else if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
                    rc = PM_EDEVICE;
                }
                if (e && hipEventRecord(e, b.st) != hipSuccess) rc = PM_EDEVICE;
                if (e) b.inflight.push_back(e);
                progress = true;
            }
            for (size_t i = 0; i < b.slots.size();) {
                Slot& s = *b.slots[i];
                const bool done = rc != PM_OK ||
                                  (s.finishing && hipEventQuery(s.done_ev) == hipSuccess);
                if (!done) {
                    ++i;
                    continue;
                }
                int st = rc;
                if (st == PM_OK) st = pm_sync(s.sim);  // the handle's sticky status
                int rd = pm_batch_detach(b.b, s.sim);
                if (st == PM_OK) st = rd;
                std::unique_ptr<Slot> own = std::move(b.slots[i]);
                b.slots.erase(b.slots.begin() + i);
                b.left.erase(b.left.begin() + i);
                std::lock_guard<std::mutex> lk(mu);
                complete_locked(std::move(own), st);
                progress = true;
            }
        }
        if (!progress) std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
    for (auto& b : batches) {
        (void)hipStreamSynchronize(b->st);
        for (hipEvent_t e : b->inflight) (void)hipEventDestroy(e);
        for (hipEvent_t e : b->spare) (void)hipEventDestroy(e);
        pm_batch_destroy(b->b);
        (void)hipStreamDestroy(b->st);
    }
}

extern "C" {

int pm_srv_create(size_t hbm_budget, int32_t max_active, pm_srv** out) {
    return pm_srv_create_ex(hbm_budget, max_active, 0, out);
}

int pm_srv_create_ex(size_t hbm_budget, int32_t max_active, int32_t batched, pm_srv** out) {
    if (!out || max_active < 1 || hbm_budget == 0 || batched < 0) return PM_EINVAL;
    *out = nullptr;
    pm_srv* s = new (std::nothrow) pm_srv;
    if (!s) return PM_ENOMEM;
    s->budget = hbm_budget;
    s->max_active = max_active;
    s->batch_cap = batched ? max_active : 0;
    try {
        s->admit_thr = std::thread([s] { s->admit_loop(); });
        s->issue_thr = std::thread([s] { s->issue_loop(); });
    } catch (...) {
        {
            std::lock_guard<std::mutex> lk(s->mu);
            s->stop = true;
        }
        s->cv.notify_all();
        if (s->admit_thr.joinable()) s->admit_thr.join();
        if (s->issue_thr.joinable()) s->issue_thr.join();
        delete s;
        return PM_ENOMEM;
    }
    *out = s;
    return PM_OK;
}

int pm_srv_submit(pm_srv* s, const pm_request* r, int64_t* id_out) {
    if (!s || !r || !id_out) return PM_EINVAL;
    if (r->nsteps < 1 || !(r->a_start > 0 && r->a_start < r->a_end && r->a_end <= 1.0))
        return PM_EINVAL;
    size_t fp = pm_footprint(&r->p, &r->l);
    if (fp == 0) return PM_EINVAL;
    auto q = std::make_shared<Req>();
    q->r = *r;
    q->z.assign(r->l.z_src, r->l.z_src + r->l.nsrc);
    q->r.l.z_src = q->z.data();
    // step boundaries a_i = a_start + i (a_end - a_start) / nsteps, last = a_end
    const double step = (r->a_end - r->a_start) / r->nsteps;
    q->agrid.resize(r->nsteps + 1);
    for (int i = 0; i <= r->nsteps; ++i) q->agrid[i] = i * step + r->a_start;
    q->agrid[r->nsteps] = r->a_end;
    q->kbytes = (size_t)r->l.nsrc * r->l.npix * r->l.npix * elem_size(r->p.dtype);
    q->need = fp + ((q->kbytes + 255) & ~size_t(255));
    if (q->need > s->budget) return PM_ENOMEM;
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) return PM_ESTATE;
    q->id = s->next_id++;
    q->t_submit = s->now();
    s->reqs[q->id] = q;
    s->queue.push_back(q);
    ++s->submitted;
    s->cv.notify_all();
    *id_out = q->id;
    return PM_OK;
}

int pm_srv_wait(pm_srv* s, int64_t id, double timeout_s) {
    if (!s) return PM_EINVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(id);
    if (it == s->reqs.end()) return PM_EINVAL;
    std::shared_ptr<Req> q = it->second;
    auto pred = [&] { return q->state == 2; };
    if (timeout_s < 0) s->cv.wait(lk, pred);
    else if (!s->cv.wait_for(lk, std::chrono::duration<double>(timeout_s), pred)) return PM_EAGAIN;
    return PM_OK;
}

int pm_srv_result(pm_srv* s, int64_t id, void* kappa_host, double times[3]) {
    if (!s) return PM_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(id);
    if (it == s->reqs.end()) return PM_EINVAL;
    std::shared_ptr<Req> q = it->second;
    if (q->state != 2) return PM_EAGAIN;
    if (times) {
        times[0] = q->t_submit;
        times[1] = q->t_admit;
        times[2] = q->t_done;
    }
    if (q->status == PM_OK && kappa_host) std::memcpy(kappa_host, q->kappa.data(), q->kappa.size());
    int st = q->status;
    s->reqs.erase(it);
    return st;
}

int pm_srv_stats_get(pm_srv* s, pm_srv_stats* out) {
    if (!s || !out) return PM_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    out->submitted = s->submitted;
    out->completed = s->completed;
    out->failed = s->failed;
    out->running = s->running;
    out->queued = (int32_t)s->queue.size();
    out->peak_running = s->peak_running;
    out->bytes_in_use = s->used;
    out->peak_bytes = s->peak_used;
    out->now = s->now();
    return PM_OK;
}

int pm_srv_destroy(pm_srv* s) {
    if (!s) return PM_EINVAL;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        // queued requests are dropped; running ones finish
        for (auto& q : s->queue) s->finish_locked(q, PM_ESTATE);
        s->queue.clear();
    }
    s->cv.notify_all();
    s->admit_thr.join();
    s->issue_thr.join();
    for (auto& sl : s->ready) sl->destroy();
    for (auto& sl : s->idle) sl->destroy();
    delete s;
    return PM_OK;
}

}  // extern "C"
