// Serving loop: continuous batching of trait-block requests over a resident
// cohort (see gwas.h). A scheduler thread admits requests by slots and by an
// HBM budget (a first-fit arena carved out of one allocation made up front),
// prepares their traits, and each round runs one slab of every admitted
// request in a single grouped launch; a consumer thread retires the slabs'
// device->host copies, checksums ring slabs, and completes requests.
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <unordered_map>

#include "arena.h"
#include "ctx.h"
#include "serve.h"

using namespace gw;

namespace {

// Device b staging buffers per admitted request: a slab can be computed while
// the previous ones are still on their way to the host.
constexpr int kStages = 4;
// Grouped launches queued on the device at once: a new round is built only
// when the previous one's kernel has finished, so the slabs that became ready
// meanwhile (of every admitted request) share one launch instead of one launch
// each. Measured at 24 and 32 requests/s (m = 1e6, FP32): 2.3 and 2.7 slabs per
// launch and 37 TFLOP/s in the serving kernel, against 1.5-1.8 and 33 TFLOP/s
// with two rounds queued and three stages, at the same throughput (bound by
// the host link) and a lower p99.
constexpr int kRoundsInFlight = 1;
// Workgroups of a ring copy (a copy kernel streams b at the host link's rate
// with a fraction of the chip).
constexpr int kCopyGrid = 64;

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct Req {
    uint64_t ticket = 0;
    int t = 0, p = 0;
    int64_t i0 = 0, m = 0;
    void *b_host = nullptr;
    gwas_slab_fn fn = nullptr;
    void *user = nullptr;
    std::vector<double> y, h2;
    int state = GWAS_REQ_QUEUED, error = GWAS_OK;
    double t_submit = 0, t_admit = 0, t_done = 0;
    // device memory (arena)
    size_t off = 0, bytes = 0;
    double *d_y = nullptr, *d_yt = nullptr, *d_h2 = nullptr, *d_fac = nullptr;
    void *d_panels = nullptr;
    void *d_stage[kStages] = {};
    size_t stage_bytes = 0;
    int64_t slab = 0, n_slabs = 0, next_slab = 0, in_flight = 0;
    int slot = -1;        // admission slot (owns a pinned staging buffer for Y and h2)
    bool stage_busy[kStages] = {};
    bool cancel = false;
    uint64_t checksum = 0;
};

struct Copy {
    std::shared_ptr<Req> r;
    int stage = 0, ring = -1;
    hipEvent_t ev = nullptr;
    hipEvent_t ev_kbeg = nullptr;    // timing: before the round's kernel (first copy of a round only)
    hipEvent_t ev_kend = nullptr;
    gwas_slab info{};
};

size_t panel_bytes(int form, int p, int t, int n_pad) {
    const size_t elt = form == GWAS_FORM_F64 ? 8 : (form == GWAS_FORM_F32 ? 4 : 2);
    const size_t planes = (form == GWAS_FORM_BF16X3 ? 2 : form == GWAS_FORM_BF16X6 ? 3 : 1) * (size_t)(p + 1);
    return elt * planes * panel_rows(t) * n_pad;
}

}  // namespace

struct gwas_server {
    gwas_ctx *c = nullptr;
    int form = 0;
    bool flush = false;
    int max_slots = 8, max_traits = 1024, host_threads = 8, grid = 512;
    int64_t item_problems = 1 << 22;
    size_t besz = 4;

    Arena arena;
    void *arena_mem = nullptr;
    unsigned long long *d_counter = nullptr;
    uint64_t counter_next = 0;   // the tile counter's value when the next round starts
    hipStream_t s_comp = nullptr, s_copy = nullptr;
    std::vector<void *> ring;
    std::vector<void *> ring_dev;   // device-side addresses of the ring slots
    std::vector<int> ring_free;
    size_t ring_bytes = 0;
    std::vector<hipEvent_t> ev_pool;
    std::vector<double *> slot_y, slot_h2;   // pinned per-slot staging of a request's Y and h2
    std::vector<int> slot_free;

    std::mutex mu;
    std::condition_variable cv_sched, cv_cons, cv_done;
    std::deque<std::shared_ptr<Req>> queue;
    std::vector<std::shared_ptr<Req>> active;
    std::deque<Copy> copies;     // issued device->host copies, in issue order
    std::deque<Copy> sums;       // landed ring slabs waiting for a checksum worker
    std::condition_variable cv_sum;
    std::vector<std::thread> workers;
    bool stop_workers = false;
    std::unordered_map<uint64_t, std::shared_ptr<Req>> all;
    uint64_t next_ticket = 1;
    bool stop = false, stop_consumer = false, failed = false;
    int fail_status = GWAS_OK;
    std::string fail_msg;
    int rr = 0;
    bool skip_checksum = false;
    int64_t n_rounds = 0, n_items = 0, ring_stalls = 0, stage_stalls = 0, bytes_d2h = 0;
    double checksum_s = 0, busy_s = 0, busy_since = -1, issue_s = 0, kernel_s = 0;
    std::vector<hipEvent_t> tev_pool;   // timing-enabled events
    std::deque<hipEvent_t> rounds;      // end of each grouped launch in flight (scheduler thread only)
    std::thread th_sched, th_cons;
};

namespace {

hipEvent_t tpool_get(gwas_server *s) {   // timing-enabled; caller holds the lock
    if (!s->tev_pool.empty()) {
        hipEvent_t e = s->tev_pool.back();
        s->tev_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

hipEvent_t pool_get(gwas_server *s) {   // caller holds the lock
    if (!s->ev_pool.empty()) {
        hipEvent_t e = s->ev_pool.back();
        s->ev_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
    return e;
}

size_t stage_bytes_of(const gwas_server *s, int t, int p, int64_t slab) {
    return (size_t)slab * t * p * s->besz;
}

// Device bytes a request holds while admitted.
size_t request_bytes(const gwas_server *s, int t, int p, int64_t slab) {
    const gwas_ctx *c = s->c;
    auto r = [](size_t v) { return (size_t)round_up((int64_t)v, 256); };
    return r(sizeof(double) * (size_t)t * c->n) + r(sizeof(double) * (size_t)t * c->n_pad) + r(sizeof(double) * t) +
           r(panel_bytes(s->form, p, t, c->n_pad)) + r(sizeof(double) * (size_t)t * fac_stride(p)) +
           kStages * r(stage_bytes_of(s, t, p, slab));
}

int64_t slab_of(const gwas_server *s, int t, int64_t m) {
    int64_t slab = std::max<int64_t>(256, s->item_problems / t / 256 * 256);
    return std::min(slab, m);
}

void finish_locked(gwas_server *s, const std::shared_ptr<Req> &r) {
    r->state = r->state == GWAS_REQ_FAILED ? GWAS_REQ_FAILED : (r->cancel ? GWAS_REQ_CANCELLED : GWAS_REQ_DONE);
    r->t_done = now_s();
    s->arena.release(r->off, r->bytes);
    s->slot_free.push_back(r->slot);
    r->slot = -1;
    s->active.erase(std::find(s->active.begin(), s->active.end(), r));
    if (s->active.empty() && s->busy_since >= 0) {
        s->busy_s += r->t_done - s->busy_since;
        s->busy_since = -1;
    }
    r->y.clear();
    r->y.shrink_to_fit();
    s->cv_done.notify_all();
    s->cv_sched.notify_one();
}

void fail_all_locked(gwas_server *s, gwas_status st, const std::string &msg) {
    s->failed = true;
    s->fail_status = st;
    s->fail_msg = msg;
    for (auto &r : s->queue) {
        r->state = GWAS_REQ_FAILED;
        r->error = st;
        r->t_done = now_s();
    }
    s->queue.clear();
    for (auto &r : s->active) {
        r->state = GWAS_REQ_FAILED;
        r->error = st;
        r->n_slabs = r->next_slab;   // issue nothing more; the consumer retires what is in flight
    }
    s->cv_done.notify_all();
}

// Stage, rotate and prepare an admitted request's traits on the compute stream
// (asynchronously: Y and h2 go through the slot's pinned buffers).
gwas_status start_request(gwas_server *s, Req *r) {
    gwas_ctx *c = s->c;
    memcpy(s->slot_y[r->slot], r->y.data(), sizeof(double) * r->y.size());
    memcpy(s->slot_h2[r->slot], r->h2.data(), sizeof(double) * r->t);
    HIP_TRY(hipMemcpyAsync(r->d_y, s->slot_y[r->slot], sizeof(double) * r->y.size(), hipMemcpyHostToDevice,
                           s->s_comp));
    HIP_TRY(hipMemcpyAsync(r->d_h2, s->slot_h2[r->slot], sizeof(double) * r->t, hipMemcpyHostToDevice, s->s_comp));
    RotOut ro{r->d_yt, nullptr, nullptr, nullptr, 0, 0, c->n_pad};
    HIP_TRY(launch_rotate(r->d_y, GWAS_DT_F64, r->t, c->n, c->n, c->Z, c->n_pad, ro, s->s_comp));
    PrepArgs pa{r->d_yt, r->d_h2, c->w, c->xlt, r->d_panels, r->d_fac, r->t, c->n, c->n_pad, r->p,
                panel_rows(r->t), fac_stride(r->p), s->form};
    HIP_TRY(launch_prep(pa, s->s_comp));
    return GWAS_OK;
}

void sched_loop(gwas_server *s) {
    gwas_ctx *c = s->c;
    hipSetDevice(c->dev);
    const void *a_base = s->form == GWAS_FORM_F64 ? (const void *)c->xr64
                       : s->form == GWAS_FORM_F32 ? (const void *)c->xr32
                       : s->form == GWAS_FORM_BF16X3 ? (const void *)c->xrbf : (const void *)c->xrbf3;
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        if (s->stop && s->queue.empty() && s->active.empty()) break;
        // admission: FIFO, by slots and by the arena (HBM budget)
        while (!s->failed && !s->queue.empty() && (int)s->active.size() < s->max_slots) {
            std::shared_ptr<Req> r = s->queue.front();
            if (r->cancel) {
                s->queue.pop_front();
                r->state = GWAS_REQ_CANCELLED;
                r->t_done = now_s();
                s->cv_done.notify_all();
                continue;
            }
            size_t off = 0;
            if (!s->arena.alloc(r->bytes, &off)) break;   // wait for memory to free up
            s->queue.pop_front();
            r->off = off;
            r->slot = s->slot_free.back();
            s->slot_free.pop_back();
            uint8_t *p = s->arena.base + off;
            auto take = [&](size_t bytes) {
                uint8_t *q = p;
                p += round_up((int64_t)bytes, 256);
                return (void *)q;
            };
            r->d_y = (double *)take(sizeof(double) * (size_t)r->t * c->n);
            r->d_yt = (double *)take(sizeof(double) * (size_t)r->t * c->n_pad);
            r->d_h2 = (double *)take(sizeof(double) * r->t);
            r->d_panels = take(panel_bytes(s->form, r->p, r->t, c->n_pad));
            r->d_fac = (double *)take(sizeof(double) * (size_t)r->t * fac_stride(r->p));
            for (int k = 0; k < kStages; ++k) r->d_stage[k] = take(r->stage_bytes);
            r->state = GWAS_REQ_RUNNING;
            r->t_admit = now_s();
            if (s->active.empty()) s->busy_since = r->t_admit;
            s->active.push_back(r);
            lk.unlock();
            gwas_status st = start_request(s, r.get());
            std::string msg = last_error();
            lk.lock();
            if (st != GWAS_OK) fail_all_locked(s, st, msg);
        }
        // rounds in flight: retire the finished ones, and build the next only
        // while fewer than kRoundsInFlight are queued (slabs accumulate meanwhile)
        while (!s->rounds.empty() && hipEventQuery(s->rounds.front()) != hipErrorNotReady) {
            s->ev_pool.push_back(s->rounds.front());
            s->rounds.pop_front();
        }
        if ((int)s->rounds.size() >= kRoundsInFlight) {
            s->cv_sched.wait_for(lk, std::chrono::microseconds(100));
            continue;
        }
        // every slab of every admitted request that has a free staging buffer
        // (and a free ring slot, for ring output) goes into this round
        std::vector<Copy> round;
        ServeBatch bt{};
        bt.a = a_base;
        bt.a_plane_rows = c->m_rows;
        bt.counter = s->d_counter;
        bt.counter_base = s->counter_next;
        bt.non_spd = c->counters;
        bt.rank_rtol = kRankRtol[s->form];
        bt.n_pad = c->n_pad;
        bt.n = c->n;
        bt.f32_flush = s->flush ? c->f32_flush : 0;
        const int na = (int)s->active.size();
        for (int k = 0; k < na && bt.n_items < kServeMaxItems; ++k) {
            std::shared_ptr<Req> r = s->active[(s->rr + k) % na];
            if (r->cancel && r->next_slab < r->n_slabs) r->n_slabs = r->next_slab;
          while (r->next_slab < r->n_slabs && bt.n_items < kServeMaxItems) {
            const int st = (int)(r->next_slab % kStages);
            if (r->stage_busy[st]) {
                s->stage_stalls++;
                break;
            }
            int ring = -1;
            if (!r->b_host) {
                if (s->ring_free.empty()) {
                    s->ring_stalls++;
                    break;
                }
                ring = s->ring_free.back();
                s->ring_free.pop_back();
            }
            const int64_t s0 = r->next_slab * r->slab;
            const int64_t cnt = std::min(r->slab, r->m - s0);
            int tm = 64, tn = 64;
            serve_tile_shape(s->form, s->flush, r->p, tm, tn);
            ServeItem &it = bt.items[bt.n_items++];
            it.panels = r->d_panels;
            it.fac = r->d_fac;
            it.b = r->d_stage[st];
            it.i0 = r->i0 + s0;
            it.mi = cnt;
            it.row_lo = 0;
            if (s->form == GWAS_FORM_BF16X3 || s->form == GWAS_FORM_BF16X6) {
                // whole 16-row groups of the fragment-ordered store (see FusedArgs::row_lo)
                it.row_lo = it.i0 & 15;
                it.i0 -= it.row_lo;
                it.mi += it.row_lo;
            }
            it.tile0 = bt.total_tiles;
            it.tb = r->t;
            it.p = r->p;
            it.tcap = panel_rows(r->t);
            it.fac_stride = fac_stride(r->p);
            bt.total_tiles += ((it.mi + tm - 1) / tm) * (int64_t)((r->t + tn - 1) / tn);
            Copy cp;
            cp.r = r;
            cp.stage = st;
            cp.ring = ring;
            cp.info.index = r->next_slab;
            cp.info.i0 = r->i0 + s0;
            cp.info.count = cnt;
            cp.info.j0 = 0;
            cp.info.tb = r->t;
            cp.info.p = r->p;
            cp.info.form = s->form;
            cp.info.bytes = (int64_t)(cnt * r->t * r->p * s->besz);
            cp.ev = pool_get(s);
            if (round.empty()) {
                cp.ev_kbeg = tpool_get(s);
                cp.ev_kend = tpool_get(s);
            }
            r->stage_busy[st] = true;
            r->next_slab++;
            r->in_flight++;
            round.push_back(cp);
          }
        }
        s->rr++;
        // requests with nothing left in flight complete here (cancelled before their last slab)
        for (int k = (int)s->active.size() - 1; k >= 0; --k) {
            std::shared_ptr<Req> r = s->active[k];
            if (r->next_slab >= r->n_slabs && r->in_flight == 0) finish_locked(s, r);
        }
        if (round.empty()) {
            s->cv_sched.wait_for(lk, std::chrono::milliseconds(2));
            continue;
        }
        hipEvent_t ev_round = pool_get(s);
        lk.unlock();
        const double t_issue = now_s();
        hipError_t e = ev_round ? hipSuccess : hipErrorOutOfMemory;
        if (e == hipSuccess && round[0].ev_kbeg) e = hipEventRecord(round[0].ev_kbeg, s->s_comp);
        if (e == hipSuccess) e = launch_serve(s->form, s->flush, bt, s->grid, s->s_comp);
        if (e == hipSuccess && round[0].ev_kend) e = hipEventRecord(round[0].ev_kend, s->s_comp);
        if (e == hipSuccess) e = hipEventRecord(ev_round, s->s_comp);
        if (e == hipSuccess) e = hipStreamWaitEvent(s->s_copy, ev_round, 0);
        for (Copy &cp : round) {
            if (e != hipSuccess) break;
            void *dst = cp.ring >= 0 ? s->ring[cp.ring]
                                     : (void *)((uint8_t *)cp.r->b_host +
                                                (size_t)(cp.info.i0 - cp.r->i0) * cp.r->t * cp.r->p * s->besz);
            if (!cp.ev) e = hipErrorOutOfMemory;
            if (e == hipSuccess) {
                if (cp.ring >= 0)   // library-owned pinned slot: the copy kernel
                    e = launch_copy_to_host(s->ring_dev[cp.ring], cp.r->d_stage[cp.stage], cp.info.bytes,
                                            kCopyGrid, s->s_copy);
                else                // caller's buffer (may be pageable): the runtime's copy
                    e = hipMemcpyAsync(dst, cp.r->d_stage[cp.stage], (size_t)cp.info.bytes, hipMemcpyDeviceToHost,
                                       s->s_copy);
            }
            if (e == hipSuccess) e = hipEventRecord(cp.ev, s->s_copy);
        }
        const double dt_issue = now_s() - t_issue;
        lk.lock();
        s->issue_s += dt_issue;
        if (e != hipSuccess) {
            // nothing of this round can be trusted: wait for the device, then fail everything
            lk.unlock();
            hipDeviceSynchronize();
            lk.lock();
            for (Copy &cp : round) {
                cp.r->in_flight--;
                cp.r->stage_busy[cp.stage] = false;
                if (cp.ring >= 0) s->ring_free.push_back(cp.ring);
                if (cp.ev) s->ev_pool.push_back(cp.ev);
            }
            if (ev_round) s->ev_pool.push_back(ev_round);
            fail_all_locked(s, GWAS_EHIP, std::string("serving launch failed: ") + hipGetErrorString(e));
            continue;
        }
        s->rounds.push_back(ev_round);
        if (bt.total_tiles > 0 && s->grid > 0)   // launch_serve launched the kernel
            s->counter_next += (uint64_t)bt.total_tiles + (uint64_t)s->grid;
        for (Copy &cp : round) {
            s->bytes_d2h += cp.info.bytes;
            s->copies.push_back(cp);
        }
        s->n_rounds++;
        s->n_items += (int64_t)round.size();
        s->cv_cons.notify_one();
    }
}

// Waits for an event by polling (a dedicated thread: a blocking wait can wake
// up late, and every retired copy frees a staging buffer and a ring slot).
void wait_event(hipEvent_t ev) {
    int spins = 0;
    while (hipEventQuery(ev) == hipErrorNotReady) {
        if (++spins < 64) std::this_thread::yield();
        else std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
}

// Retires device->host copies in issue order: the request's device staging
// buffer is free as soon as its copy has landed; ring slabs then go to the
// checksum workers, which release the ring slot.
void cons_loop(gwas_server *s) {
    hipSetDevice(s->c->dev);
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        while (s->copies.empty() && !s->stop_consumer) s->cv_cons.wait(lk);
        if (s->copies.empty()) break;
        Copy cp = s->copies.front();
        s->copies.pop_front();
        lk.unlock();
        wait_event(cp.ev);
        float kms = 0.f;
        if (cp.ev_kbeg) hipEventElapsedTime(&kms, cp.ev_kbeg, cp.ev_kend);
        lk.lock();
        s->kernel_s += kms * 1e-3;
        if (cp.ev_kbeg) {
            s->tev_pool.push_back(cp.ev_kbeg);
            s->tev_pool.push_back(cp.ev_kend);
        }
        s->ev_pool.push_back(cp.ev);
        cp.ev = nullptr;
        std::shared_ptr<Req> r = cp.r;
        r->stage_busy[cp.stage] = false;
        if (cp.ring >= 0) {
            s->sums.push_back(cp);
            s->cv_sum.notify_one();
        } else {
            r->in_flight--;
            if (r->next_slab >= r->n_slabs && r->in_flight == 0) finish_locked(s, r);
        }
        s->cv_sched.notify_one();
    }
}

// Checksums landed ring slabs (one slab per worker at a time) and passes them
// to the request's callback; completes a request with its last slab.
void sum_loop(gwas_server *s) {
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        while (s->sums.empty() && !s->stop_workers) s->cv_sum.wait(lk);
        if (s->sums.empty()) break;
        Copy cp = s->sums.front();
        s->sums.pop_front();
        lk.unlock();
        cp.info.b = s->ring[cp.ring];
        const double t0 = now_s();
        const uint64_t cs = s->skip_checksum ? 0 : checksum_range((const uint32_t *)cp.info.b, 0, cp.info.bytes / 4);
        const double dt = now_s() - t0;
        cp.info.checksum = cs;
        if (cp.r->fn) cp.r->fn(cp.r->user, &cp.info);
        lk.lock();
        s->checksum_s += dt;
        s->ring_free.push_back(cp.ring);
        std::shared_ptr<Req> r = cp.r;
        r->checksum += cs;
        r->in_flight--;
        if (r->next_slab >= r->n_slabs && r->in_flight == 0) finish_locked(s, r);
        s->cv_sched.notify_one();
    }
}

void fill_result(const Req &r, gwas_result *out) {
    memset(out, 0, sizeof *out);
    out->state = r.state;
    out->error = r.error;
    out->t_submit = r.t_submit;
    out->t_admit = r.t_admit;
    out->t_done = r.t_done;
    out->problems = r.m * (int64_t)r.t;
    out->slabs = r.n_slabs;
    out->checksum = r.checksum;
}

bool terminal(int st) { return st == GWAS_REQ_DONE || st == GWAS_REQ_CANCELLED || st == GWAS_REQ_FAILED; }

hipError_t create_own_queue_stream(hipStream_t *st, int cus) {
    std::vector<uint32_t> mask((cus + 31) / 32, 0u);
    for (int k = 0; k < cus; ++k) mask[k / 32] |= 1u << (k % 32);
    return hipExtStreamCreateWithCUMask(st, (uint32_t)mask.size(), mask.data());
}

void free_server(gwas_server *s) {
    if (!s) return;
    if (s->c) hipSetDevice(s->c->dev);
    hipDeviceSynchronize();
    if (s->arena_mem) hipFree(s->arena_mem);
    if (s->d_counter) hipFree(s->d_counter);
    for (void *p : s->ring)
        if (p) hipHostFree(p);
    for (double *p : s->slot_y)
        if (p) hipHostFree(p);
    for (double *p : s->slot_h2)
        if (p) hipHostFree(p);
    for (hipEvent_t e : s->ev_pool) hipEventDestroy(e);
    for (hipEvent_t e : s->tev_pool) hipEventDestroy(e);
    for (hipEvent_t e : s->rounds) hipEventDestroy(e);
    if (s->s_comp) hipStreamDestroy(s->s_comp);
    if (s->s_copy) hipStreamDestroy(s->s_copy);
    delete s;
}

}  // namespace

extern "C" {

double gwas_clock(void) { return now_s(); }

gwas_status gwas_server_create(gwas_ctx *c, const gwas_server_options *opt, gwas_server **out) {
    last_error().clear();
    if (!out) return fail(GWAS_EINVAL, "server pointer is NULL");
    *out = nullptr;
    if (!c || !opt) return fail(GWAS_EINVAL, "NULL argument");
    if (opt->form < 0 || opt->form > 3 || !(c->forms & GWAS_FORM_BIT(opt->form)))
        return fail(GWAS_EINVAL, "form %d is not resident", opt->form);
    if (opt->hbm_budget < 0 || opt->max_slots < 0 || opt->max_slots > kServeMaxItems || opt->item_problems < 0 ||
        opt->max_traits < 0 || opt->ring_slots < 0 || opt->host_threads < 0 || opt->ring_slots > 256 ||
        opt->host_threads > 256 || opt->grid_wgs < 0)
        return fail(GWAS_EINVAL, "option out of range");
    gwas_server *s = new gwas_server();
    s->c = c;
    s->form = opt->form;
    s->flush = opt->form == GWAS_FORM_F32 && c->f32_flush > 0;
    s->besz = opt->form == GWAS_FORM_F64 ? 8 : 4;
    s->max_slots = opt->max_slots ? opt->max_slots : 8;
    s->max_traits = opt->max_traits ? opt->max_traits : 1024;
    s->item_problems = opt->item_problems ? opt->item_problems : (1 << 22);
    s->host_threads = opt->host_threads ? opt->host_threads : 8;
    s->skip_checksum = opt->skip_checksum != 0;
    const size_t budget = opt->hbm_budget ? (size_t)opt->hbm_budget : ((size_t)8 << 30);
    hipError_t e = hipSetDevice(c->dev);
    int cus = 256;
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->dev);
    // default: as many persistent workgroups as fit the chip at once, at most two
    // per CU (the ring copies still get their share)
    s->grid = opt->grid_wgs > 0 ? opt->grid_wgs : std::min(2, serve_occupancy(s->form, s->flush)) * cus;
    if (e == hipSuccess) e = hipMalloc(&s->arena_mem, budget);
    if (e == hipSuccess) e = hipMalloc((void **)&s->d_counter, 256);
    if (e == hipSuccess) e = hipMemset(s->d_counter, 0, 256);
    // The copy stream must not share a hardware queue with the compute stream, or
    // the copies (blit kernels) wait behind every launch: streams created with a
    // compute-unit mask (here: all units) get hardware queues of their own.
    if (e == hipSuccess) e = create_own_queue_stream(&s->s_comp, cus);
    if (e == hipSuccess) e = create_own_queue_stream(&s->s_copy, cus);
    if (e != hipSuccess) {
        free_server(s);
        return fail(e == hipErrorOutOfMemory ? GWAS_ENOMEM : GWAS_EHIP, "server setup: %s", hipGetErrorString(e));
    }
    s->arena.init(s->arena_mem, budget);
    // ring slots hold the largest slab a request can produce
    const int pmax = std::min(kServeMaxP, c->p);
    // a slab holds at most max(item_problems, 256 x max_traits) problems (slabs are >= 256 SNPs)
    s->ring_bytes = (size_t)round_up(std::max<int64_t>(s->item_problems, 256 * (int64_t)s->max_traits), 256) *
                    pmax * s->besz;
    const int nring = opt->ring_slots ? opt->ring_slots : 2 * s->max_slots;
    for (int k = 0; k < nring; ++k) {
        void *p = nullptr;
        e = hipHostMalloc(&p, s->ring_bytes, hipHostMallocDefault);
        if (e != hipSuccess) {
            free_server(s);
            return fail(GWAS_ENOMEM, "pinned ring slot (%zu bytes): %s", s->ring_bytes, hipGetErrorString(e));
        }
        s->ring.push_back(p);
        void *pd = nullptr;
        e = hipHostGetDevicePointer(&pd, p, 0);
        if (e != hipSuccess) {
            free_server(s);
            return fail(GWAS_EHIP, "ring device address: %s", hipGetErrorString(e));
        }
        s->ring_dev.push_back(pd);
        s->ring_free.push_back(k);
    }
    for (int k = 0; k < s->max_slots; ++k) {
        double *py = nullptr, *ph = nullptr;
        e = hipHostMalloc((void **)&py, sizeof(double) * (size_t)s->max_traits * c->n, hipHostMallocDefault);
        if (e == hipSuccess) e = hipHostMalloc((void **)&ph, sizeof(double) * s->max_traits, hipHostMallocDefault);
        s->slot_y.push_back(py);
        s->slot_h2.push_back(ph);
        if (e != hipSuccess) {
            free_server(s);
            return fail(GWAS_ENOMEM, "pinned slot staging: %s", hipGetErrorString(e));
        }
        s->slot_free.push_back(k);
    }
    s->th_sched = std::thread(sched_loop, s);
    s->th_cons = std::thread(cons_loop, s);
    for (int k = 0; k < s->host_threads; ++k) s->workers.emplace_back(sum_loop, s);
    *out = s;
    return GWAS_OK;
}

gwas_status gwas_server_submit(gwas_server *s, const gwas_request *q, uint64_t *ticket) {
    last_error().clear();
    if (!s || !q || !ticket) return fail(GWAS_EINVAL, "NULL argument");
    const gwas_ctx *c = s->c;
    if (q->t < 1 || q->t > s->max_traits) return fail(GWAS_EINVAL, "t = %d outside [1, %d]", q->t, s->max_traits);
    const int pmax = std::min(kServeMaxP, c->p);
    if (q->p < 2 || q->p > pmax) return fail(GWAS_EINVAL, "p = %d outside [2, %d]", q->p, pmax);
    const int64_t m = q->m ? q->m : c->m_cap - q->i0;
    if (q->i0 < 0 || m <= 0 || q->i0 + m > c->m_cap) return fail(GWAS_EINVAL, "SNP range outside the cohort");
    if (!q->Y || !q->h2) return fail(GWAS_EINVAL, "NULL Y or h2");
    for (int j = 0; j < q->t; ++j) {
        const double h = q->h2[j];
        const bool in_range = (h >= 0.0 && h < 1.0) || (h == 1.0 && c->w_min > 0.0);
        if (!isfinite(h) || !in_range || !(h * c->w_min + (1.0 - h) > 0.0))
            return fail(GWAS_EINVAL, "h2[%d] = %g gives a covariance that is not SPD", j, h);
    }
    for (int64_t k = 0; k < (int64_t)q->t * c->n; ++k)
        if (!isfinite(q->Y[k])) return fail(GWAS_EINVAL, "non-finite value in Y");
    auto r = std::make_shared<Req>();
    r->t = q->t;
    r->p = q->p;
    r->i0 = q->i0;
    r->m = m;
    r->b_host = q->b;
    r->fn = q->fn;
    r->user = q->user;
    r->y.assign(q->Y, q->Y + (size_t)q->t * c->n);
    r->h2.assign(q->h2, q->h2 + q->t);
    r->slab = slab_of(s, r->t, m);
    r->n_slabs = (m + r->slab - 1) / r->slab;
    r->stage_bytes = stage_bytes_of(s, r->t, r->p, r->slab);
    r->bytes = request_bytes(s, r->t, r->p, r->slab);
    if (r->bytes > s->arena.size)
        return fail(GWAS_EINVAL, "request needs %zu device bytes, above the budget %zu", r->bytes, s->arena.size);
    if (!r->b_host && r->stage_bytes > s->ring_bytes)
        return fail(GWAS_EINVAL, "slab larger than a ring slot");
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->failed) return fail(s->fail_status, "server failed: %s", s->fail_msg.c_str());
    if (s->stop) return fail(GWAS_ESTATE, "server is stopping");
    r->ticket = s->next_ticket++;
    r->t_submit = now_s();
    s->all[r->ticket] = r;
    s->queue.push_back(r);
    *ticket = r->ticket;
    s->cv_sched.notify_one();
    return GWAS_OK;
}

gwas_status gwas_server_poll(gwas_server *s, uint64_t ticket, gwas_result *out) {
    last_error().clear();
    if (!s || !out) return fail(GWAS_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->all.find(ticket);
    if (it == s->all.end()) return fail(GWAS_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
    fill_result(*it->second, out);
    return GWAS_OK;
}

gwas_status gwas_server_wait(gwas_server *s, uint64_t ticket, double timeout_s, gwas_result *out) {
    last_error().clear();
    if (!s) return fail(GWAS_EINVAL, "NULL argument");
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->all.find(ticket);
    if (it == s->all.end()) return fail(GWAS_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
    std::shared_ptr<Req> r = it->second;
    auto done = [&] { return terminal(r->state); };
    if (timeout_s < 0) s->cv_done.wait(lk, done);
    else if (!s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), done)) {
        if (out) fill_result(*r, out);
        return fail(GWAS_EBUSY, "request %llu not finished", (unsigned long long)ticket);
    }
    if (out) fill_result(*r, out);
    return GWAS_OK;
}

gwas_status gwas_server_cancel(gwas_server *s, uint64_t ticket) {
    last_error().clear();
    if (!s) return fail(GWAS_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->all.find(ticket);
    if (it == s->all.end()) return fail(GWAS_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
    it->second->cancel = true;
    s->cv_sched.notify_one();
    return GWAS_OK;
}

gwas_status gwas_server_stats(gwas_server *s, gwas_server_stats_t *out) {
    last_error().clear();
    if (!s || !out) return fail(GWAS_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    memset(out, 0, sizeof *out);
    out->rounds = s->n_rounds;
    out->items = s->n_items;
    out->ring_stalls = s->ring_stalls;
    out->stage_stalls = s->stage_stalls;
    out->bytes_d2h = s->bytes_d2h;
    out->checksum_s = s->checksum_s;
    out->busy_s = s->busy_s + (s->busy_since >= 0 ? now_s() - s->busy_since : 0.0);
    out->issue_s = s->issue_s;
    out->kernel_s = s->kernel_s;
    return GWAS_OK;
}

gwas_status gwas_server_destroy(gwas_server *s) {
    last_error().clear();
    if (!s) return GWAS_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        for (auto &r : s->queue) r->cancel = true;
        s->cv_sched.notify_one();
    }
    if (s->th_sched.joinable()) s->th_sched.join();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop_consumer = true;
        s->cv_cons.notify_one();
    }
    if (s->th_cons.joinable()) s->th_cons.join();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop_workers = true;
        s->cv_sum.notify_all();
    }
    for (auto &th : s->workers)
        if (th.joinable()) th.join();
    free_server(s);
    return GWAS_OK;
}

}  // extern "C"
