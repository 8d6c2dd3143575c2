// serve.hip -- request loop that keeps the graph resident and interleaves walk
// queries with update batches (the paper's ordering rule, Sec. 6 item ii:
// every update submitted before a query is applied before that query runs,
// and none submitted after it).
//
// A scheduler thread admits requests in FIFO order.  Walk queries run on
// max_inflight slots (HIP streams at default priority) and their device buffers
// count against the HBM budget.  When a slot is free, the small walk queries
// waiting at the head of the queue for the same graph version -- up to
// max_batch of them, BATCH_WALKS walks in all, and the budget -- are merged
// into one persistent launch on that slot (continuous batching: one work queue
// over all their walks), so a burst of small queries costs one launch instead
// of one each and a slot per query.  A larger query runs alone, so that no
// small query waits for it.  An update batch waits until every query
// submitted before it has finished, then runs on the update stream; queries
// submitted after it wait for it.  Results do not depend on the mix: a query's
// walks are keyed by (seed, walk id) and the graph it sees is fixed by its
// epoch (the number of update batches submitted before it).
#include "dev.h"
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>
#include <string.h>

namespace {

using Clock = std::chrono::steady_clock;
constexpr uint64_t BATCH_WALKS = 16384;  // walks of the queries merged into one launch

struct Req {
    uint64_t ticket = 0;
    int kind = 0;  // 0 walk query, 1 update batch
    uint64_t epoch = 0;
    // walk query
    std::vector<uint32_t> starts;
    uint32_t length = 0;
    uint64_t seed = 0, base = 0;
    // update batch
    std::vector<uint32_t> isrc, idst, iw, dsrc, ddst;
    // runtime
    int slot = -1;
    uint64_t bytes = 0;
    uint32_t* d_buf = nullptr;      // starts, then paths
    uint32_t* h_paths = nullptr;    // pinned result
    uint64_t* d_steps = nullptr;
    uint64_t* h_steps = nullptr;
    hipEvent_t done_ev = nullptr;
    Clock::time_point t_submit, t_start, t_done;
    int status = 0;
    bool finished = false;
    bingo_update_stats ustats{};
};

}  // namespace

struct bingo_server {
    bingo_graph* g = nullptr;
    uint32_t max_inflight = 8;
    uint32_t max_batch = 1;
    uint64_t budget = 0;
    std::vector<hipStream_t> streams;
    std::vector<bool> busy;
    hipStream_t ustream = nullptr;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Req*> pending;
    std::vector<Req*> inflight;
    std::map<uint64_t, Req*> all;
    uint64_t next_ticket = 1;
    uint64_t submitted_updates = 0;  // epoch of the next request
    uint64_t applied_updates = 0;
    uint64_t used_bytes = 0;
    // pinned host result buffers, reused by power-of-two size class
    std::map<uint64_t, std::vector<void*>> pinned_free;
    bool stop = false;
    std::thread worker;
    int sticky_error = 0;
};

namespace {

uint64_t pin_class(uint64_t bytes) {
    uint64_t c = 4096;
    while (c < bytes) c <<= 1;
    return c;
}
// lock held
void* pin_get(bingo_server* s, uint64_t bytes) {
    const uint64_t c = pin_class(bytes);
    auto& v = s->pinned_free[c];
    if (!v.empty()) { void* p = v.back(); v.pop_back(); return p; }
    void* p = nullptr;
    if (hipHostMalloc(&p, c, 0) != hipSuccess) return nullptr;
    return p;
}
void pin_put(bingo_server* s, void* p, uint64_t bytes) {
    if (p) s->pinned_free[pin_class(bytes)].push_back(p);
}

void finish_req(bingo_server* s, Req* r, int status) {
    r->status = status;
    r->t_done = Clock::now();
    r->finished = true;
}

// Called with the lock held; returns true if it changed state.
bool try_admit(bingo_server* s, std::unique_lock<std::mutex>& lk) {
    if (s->pending.empty()) return false;
    Req* r = s->pending.front();
    if (r->kind == 1) {
        // an update runs once every older query has finished
        if (!s->inflight.empty()) return false;
        s->pending.pop_front();
        r->t_start = Clock::now();
        lk.unlock();
        int rc = BINGO_OK;
        const uint64_t ni = r->isrc.size(), nd = r->dsrc.size();
        uint32_t* d = nullptr;
        const uint64_t words = 3 * ni + 2 * nd;
        if (words) {
            if (hipMallocAsync((void**)&d, words * 4, s->ustream) != hipSuccess) rc = BINGO_E_OOM;
            if (rc == BINGO_OK) {
                uint32_t* p = d;
                auto put = [&](const std::vector<uint32_t>& v) {
                    if (!v.empty()) hipMemcpyAsync(p, v.data(), v.size() * 4, hipMemcpyHostToDevice, s->ustream);
                    p += v.size();
                };
                put(r->isrc); put(r->idst); put(r->iw); put(r->dsrc); put(r->ddst);
            }
        }
        if (rc == BINGO_OK)
            rc = bingo_update_batch(s->g, ni, d, d + ni, d + 2 * ni, nd, d + 3 * ni, d + 3 * ni + nd, s->ustream,
                                    &r->ustats);
        if (d) hipFreeAsync(d, s->ustream);
        hipStreamSynchronize(s->ustream);
        lk.lock();
        s->applied_updates++;
        finish_req(s, r, rc);
        s->cv_done.notify_all();
        return true;
    }
    // walk queries: their epoch's updates must be applied, and a slot and memory must be free
    if (r->epoch != s->applied_updates) return false;
    int slot = -1;
    for (uint32_t i = 0; i < s->max_inflight; ++i)
        if (!s->busy[i]) { slot = (int)i; break; }
    if (slot < 0) return false;
    // the front query and the small walk queries of the same epoch right behind it
    std::vector<Req*> batch;
    uint64_t extra = 0, walks = 0;
    for (Req* q : s->pending) {
        if (batch.size() >= s->max_batch || q->kind != 0 || q->epoch != r->epoch) break;
        const uint64_t nw = q->starts.size();
        if (!batch.empty() && walks + nw > BATCH_WALKS) break;
        walks += nw;
        q->bytes = (nw + nw * ((uint64_t)q->length + 1)) * 4 + 8;
        // over the budget only when nothing else holds memory and the batch is empty
        if (s->budget && s->used_bytes + extra + q->bytes > s->budget && !(s->inflight.empty() && batch.empty()))
            break;
        batch.push_back(q);
        extra += q->bytes;
    }
    if (batch.empty()) return false;
    for (size_t i = 0; i < batch.size(); ++i) s->pending.pop_front();
    s->busy[slot] = true;
    hipStream_t st = s->streams[slot];
    std::vector<bingo_walk_query> qs;
    int rc = BINGO_OK;
    for (Req* q : batch) {
        q->slot = slot;
        s->used_bytes += q->bytes;
        s->inflight.push_back(q);
        q->t_start = Clock::now();
        const uint64_t nw = q->starts.size(), pw = nw * ((uint64_t)q->length + 1);
        if (rc == BINGO_OK &&
            hipMallocAsync((void**)&q->d_buf, std::max<uint64_t>(nw + pw, 1) * 4 + 32, st) != hipSuccess) {
            q->d_buf = nullptr;
            rc = BINGO_E_OOM;
        }
        if (rc == BINGO_OK && !(q->h_paths = (uint32_t*)pin_get(s, std::max<uint64_t>(pw, 1) * 4 + 32)))
            rc = BINGO_E_OOM;
        if (rc != BINGO_OK) continue;
        q->h_steps = (uint64_t*)(q->h_paths + std::max<uint64_t>(pw, 1) + 1);
        q->h_steps = (uint64_t*)(((uintptr_t)q->h_steps + 7) & ~(uintptr_t)7);
        uint32_t* d_starts = q->d_buf;
        uint32_t* d_paths = q->d_buf + nw;
        q->d_steps = (uint64_t*)(((uintptr_t)(d_paths + pw) + 7) & ~(uintptr_t)7);
        if (nw) hipMemcpyAsync(d_starts, q->starts.data(), nw * 4, hipMemcpyHostToDevice, st);
        qs.push_back(bingo_walk_query{nw, d_starts, q->base, q->length, 0u, q->seed, d_paths, q->d_steps});
    }
    if (rc == BINGO_OK) {
        if (qs.size() == 1)
            rc = bingo_walk(s->g, qs[0].n_walks, qs[0].d_starts, qs[0].walk_id_base, qs[0].length, qs[0].seed,
                            qs[0].d_paths, qs[0].d_steps_taken, BINGO_WALK_PERSISTENT, st);
        else
            rc = bingo_walk_batch(s->g, (uint32_t)qs.size(), qs.data(), st);
    }
    for (size_t i = 0; i < batch.size(); ++i) {
        Req* q = batch[i];
        if (rc == BINGO_OK) {
            const uint64_t pw = qs[i].n_walks * ((uint64_t)q->length + 1);
            if (pw) hipMemcpyAsync(q->h_paths, qs[i].d_paths, pw * 4, hipMemcpyDeviceToHost, st);
            hipMemcpyAsync(q->h_steps, q->d_steps, 8, hipMemcpyDeviceToHost, st);
        }
        if (q->d_buf) hipFreeAsync(q->d_buf, st);
        q->d_buf = nullptr;
        hipEventCreateWithFlags(&q->done_ev, hipEventDisableTiming);
        hipEventRecord(q->done_ev, st);
    }
    if (rc != BINGO_OK) {
        // release what was taken and fail the batch's requests
        for (Req* q : batch) {
            hipEventSynchronize(q->done_ev);
            hipEventDestroy(q->done_ev);
            q->done_ev = nullptr;
            s->used_bytes -= q->bytes;
            s->inflight.erase(std::find(s->inflight.begin(), s->inflight.end(), q));
            finish_req(s, q, rc);
        }
        s->busy[slot] = false;
        s->cv_done.notify_all();
    }
    return true;
}

bool reap(bingo_server* s) {
    bool any = false;
    for (size_t i = 0; i < s->inflight.size();) {
        Req* r = s->inflight[i];
        if (hipEventQuery(r->done_ev) == hipSuccess) {
            hipEventDestroy(r->done_ev);
            r->done_ev = nullptr;
            s->busy[r->slot] = false;
            s->used_bytes -= r->bytes;
            s->inflight.erase(s->inflight.begin() + i);
            finish_req(s, r, BINGO_OK);
            any = true;
        } else {
            ++i;
        }
    }
    if (any) s->cv_done.notify_all();
    return any;
}

void worker_main(bingo_server* s) {
    std::unique_lock<std::mutex> lk(s->mu);
    while (true) {
        bool progressed = reap(s);
        while (try_admit(s, lk)) progressed = true;
        if (s->stop && s->pending.empty() && s->inflight.empty()) break;
        if (!progressed) {
            if (s->inflight.empty())
                s->cv_work.wait_for(lk, std::chrono::milliseconds(50));
            else
                s->cv_work.wait_for(lk, std::chrono::microseconds(20));
        }
    }
}

}  // namespace

extern "C" {

int bingo_server_create(bingo_graph* g, const bingo_server_config* cfg, bingo_server** out) {
    if (!g || g->radix_base != 2 || !cfg || !out || cfg->struct_size != sizeof(bingo_server_config))
        return BINGO_E_INVALID;
    if (cfg->max_inflight == 0 || cfg->max_inflight > 64) return BINGO_E_INVALID;
    if (cfg->max_batch > BINGO_WALK_BATCH_MAX || cfg->reserved) return BINGO_E_INVALID;
    if (int rc = ppr_drain(g)) return rc;
    *out = nullptr;
    bingo_server* s = new bingo_server();
    s->g = g;
    s->max_inflight = cfg->max_inflight;
    s->max_batch = std::max<uint32_t>(1, cfg->max_batch);
    s->budget = cfg->hbm_budget_bytes;
    s->streams.resize(s->max_inflight);
    s->busy.assign(s->max_inflight, false);
    for (auto& st : s->streams)
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) { delete s; return BINGO_E_HIP; }
    if (hipStreamCreateWithFlags(&s->ustream, hipStreamNonBlocking) != hipSuccess) { delete s; return BINGO_E_HIP; }
    s->worker = std::thread(worker_main, s);
    *out = s;
    return BINGO_OK;
}

int bingo_server_submit_walk(bingo_server* s, uint64_t n_walks, const uint32_t* h_starts, uint32_t length,
                             uint64_t seed, uint64_t walk_id_base, uint64_t* ticket) {
    if (!s || !ticket || (n_walks && !h_starts) || length == 0xFFFFFFFFu) return BINGO_E_INVALID;
    Req* r = new Req();
    r->kind = 0;
    r->starts.assign(h_starts, h_starts + n_walks);
    r->length = length;
    r->seed = seed;
    r->base = walk_id_base;
    r->t_submit = Clock::now();
    std::lock_guard<std::mutex> lk(s->mu);
    r->ticket = s->next_ticket++;
    r->epoch = s->submitted_updates;
    s->all[r->ticket] = r;
    s->pending.push_back(r);
    *ticket = r->ticket;
    s->cv_work.notify_one();
    return BINGO_OK;
}

int bingo_server_submit_update(bingo_server* s, uint64_t n_ins, const uint32_t* h_ins_src, const uint32_t* h_ins_dst,
                               const uint32_t* h_ins_w, uint64_t n_del, const uint32_t* h_del_src,
                               const uint32_t* h_del_dst, uint64_t* ticket) {
    if (!s || !ticket) return BINGO_E_INVALID;
    if (n_ins && (!h_ins_src || !h_ins_dst || !h_ins_w)) return BINGO_E_INVALID;
    if (n_del && (!h_del_src || !h_del_dst)) return BINGO_E_INVALID;
    Req* r = new Req();
    r->kind = 1;
    r->isrc.assign(h_ins_src, h_ins_src + n_ins);
    r->idst.assign(h_ins_dst, h_ins_dst + n_ins);
    r->iw.assign(h_ins_w, h_ins_w + n_ins);
    r->dsrc.assign(h_del_src, h_del_src + n_del);
    r->ddst.assign(h_del_dst, h_del_dst + n_del);
    r->t_submit = Clock::now();
    std::lock_guard<std::mutex> lk(s->mu);
    r->ticket = s->next_ticket++;
    r->epoch = s->submitted_updates++;
    s->all[r->ticket] = r;
    s->pending.push_back(r);
    *ticket = r->ticket;
    s->cv_work.notify_one();
    return BINGO_OK;
}

int bingo_server_wait(bingo_server* s, uint64_t ticket, uint32_t* h_paths, uint64_t cap_words,
                      bingo_request_info* info) {
    if (!s) return BINGO_E_INVALID;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->all.find(ticket);
    if (it == s->all.end()) return BINGO_E_INVALID;
    Req* r = it->second;
    s->cv_done.wait(lk, [&] { return r->finished; });
    const uint64_t pw = r->kind == 0 ? r->starts.size() * ((uint64_t)r->length + 1) : 0;
    int rc = r->status;
    if (rc == BINGO_OK && r->kind == 0 && h_paths) {
        if (cap_words < pw) return BINGO_E_CAPACITY;  // the request stays available
        memcpy(h_paths, r->h_paths, pw * 4);
    }
    if (info) {
        memset(info, 0, sizeof(*info));
        info->kind = (uint32_t)r->kind;
        info->status = rc;
        info->epoch = r->epoch;
        info->queue_us = std::chrono::duration<double, std::micro>(r->t_start - r->t_submit).count();
        info->latency_us = std::chrono::duration<double, std::micro>(r->t_done - r->t_submit).count();
        info->steps = (r->kind == 0 && rc == BINGO_OK && r->h_steps) ? *r->h_steps : 0;
        info->path_words = pw;
        if (r->kind == 1) {
            info->updates_applied = r->ustats.inserted + r->ustats.deleted;
            info->updates_not_found = r->ustats.not_found;
        }
    }
    if (r->h_paths) pin_put(s, r->h_paths, std::max<uint64_t>(pw, 1) * 4 + 32);
    s->all.erase(it);
    delete r;
    return rc;
}

int bingo_server_destroy(bingo_server* s) {
    if (!s) return BINGO_E_INVALID;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        s->cv_work.notify_one();
    }
    if (s->worker.joinable()) s->worker.join();
    for (auto& kv : s->all) {
        if (kv.second->h_paths) hipHostFree(kv.second->h_paths);
        delete kv.second;
    }
    for (auto& kv : s->pinned_free)
        for (void* p : kv.second) hipHostFree(p);
    for (auto st : s->streams) hipStreamDestroy(st);
    if (s->ustream) hipStreamDestroy(s->ustream);
    delete s;
    return BINGO_OK;
}

}  // extern "C"
