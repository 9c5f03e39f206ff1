// Serving loop: continuous batching of single bootstrap requests.
//
// Requests of any table (any t, t', r) are admitted into device-resident
// slots as memory allows.  Every launch ("tick") advances each resident
// ciphertext by `chunk` CMux steps, its accumulator staying in device memory
// between ticks, so a request that arrives while others are on the GPU joins
// them at the next tick instead of waiting for a whole batch to drain.  The
// slots are split into two partitions with a stream each; while one
// partition's tick runs, the host harvests and relaunches the other, so the
// two overlap on the device.  Ciphertexts that reach step n are key-switched in
// the same tick and their results copied back.
//
// Contexts whose bootstraps run the global-accumulator path (the wide ring
// modulus, rings of degree 16384) are served the same way with that path's
// kernels: a tick is `chunk` CMux launches over every resident component, each
// ciphertext at its own step (a ciphertext that reaches step n inside the tick
// carries its accumulator over), the accumulators in two device arenas.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <set>
#include <thread>
#include <unordered_map>
#include <unordered_set>

#include "device_internal.hpp"

namespace mm {

using clk = std::chrono::steady_clock;

namespace {

// Buddy allocator over accumulator units (one unit = the (a, b) pair of one
// ring component); a ciphertext with vector length r takes a block of
// 2^ceil(log2 r) units, r <= 2^top.
struct Buddy {
    std::vector<std::set<uint32_t>> free_;
    uint32_t top = 3;
    // aligned blocks of at most 2^top units, largest first, cover [0, units)
    void init(uint32_t units, uint32_t top_order)
    {
        top = top_order;
        free_.assign(top + 1, {});
        uint32_t u = 0;
        for (int o = (int)top; o >= 0; o--)
            while (u + (1u << o) <= units) {
                free_[o].insert(u);
                u += 1u << o;
            }
    }
    // the largest order that init left a block of
    uint32_t largest() const
    {
        for (int o = (int)top; o >= 0; o--)
            if (!free_[o].empty()) return (uint32_t)o;
        return 0;
    }
    int64_t alloc(uint32_t order)
    {
        uint32_t o = order;
        while (o <= top && free_[o].empty()) o++;
        if (o > top) return -1;
        uint32_t start = *free_[o].begin();
        free_[o].erase(free_[o].begin());
        while (o > order) {  // split, keep the lower half
            o--;
            free_[o].insert(start + (1u << o));
        }
        return start;
    }
    void release(uint32_t start, uint32_t order)
    {
        while (order < top) {
            const uint32_t buddy = start ^ (1u << order);
            auto it = free_[order].find(buddy);
            if (it == free_[order].end()) break;
            free_[order].erase(it);
            start = std::min(start, buddy);
            order++;
        }
        free_[order].insert(start);
    }
};

uint32_t order_of(uint32_t r)
{
    uint32_t o = 0;
    while ((1u << o) < r) o++;
    return o;
}

struct Req {
    uint64_t ticket;
    int table;
    std::vector<uint32_t> ct;
    clk::time_point t0;
    int cls;  // 0: at most 4 components, 1: wider
};

struct Active {
    uint64_t ticket;
    int table;
    uint32_t slot, unit, order, step;
    clk::time_point t0;
    int cls;
};

struct Result {
    std::vector<uint32_t> ct;
    double ms;
};

template <class T>
struct DevHost {
    T *d = nullptr;
    T *h = nullptr;
    size_t cap = 0;
    void reserve(size_t n)
    {
        if (n <= cap) return;
        release();
        const size_t want = std::max<size_t>(n * 2, 256);
        if (hipMalloc((void **)&d, want * sizeof(T)) != hipSuccess ||
            hipHostMalloc((void **)&h, want * sizeof(T), hipHostMallocDefault) != hipSuccess)
            throw Error(MM_ENOMEM, "server staging allocation failed");
        cap = want;
    }
    void release()
    {
        if (d) hipFree(d);
        if (h) hipHostFree(h);
        d = nullptr;
        h = nullptr;
        cap = 0;
    }
};

struct Part {
    hipStream_t st = nullptr;
    hipEvent_t ev = nullptr;
    bool busy = false;
    std::vector<Active> active, finishing;
    DevHost<dev::WaveTask> tasks;
    DevHost<int32_t> rows, stage_rows;
    DevHost<uint32_t> out, stage, qout;
    uint64_t *part = nullptr;
    size_t part_cap = 0;
    // global-accumulator path: task list (fresh components' initialisations, then
    // every resident component's steps), component-0 offsets of the finishing
    // ciphertexts, their extracted samples, and the arena holding this partition's
    // current accumulators
    DevHost<dev::WideTask> wtasks;
    DevHost<uint64_t> woff;
    uint32_t *ext = nullptr;
    size_t ext_cap = 0;
    int cur = 0;
};

}  // namespace

struct Server {
    mm_ctx *c = nullptr;
    uint32_t chunk = 64, max_cts = 0, units = 0;
    bool global = false;     // the global-accumulator path (one launch per CMux step)
    bool switchable = false; // fused-kernel context whose light ticks take the global path
    size_t unit_words = 0;   // words of one unit in one arena
    uint32_t top_block = 3;  // order of the largest block the arena holds
    uint32_t *d_acc = nullptr, *d_ct = nullptr, *d_ext = nullptr;
    Buddy buddy;
    std::vector<uint32_t> free_slots;
    Part part[2];
    std::mutex mu;
    std::condition_variable cv;
    std::deque<Req> pending[2];  // by class: at most 4 components, and wider
    size_t pending_cap = 1u << 20;
    std::unordered_map<uint64_t, Result> done;
    std::unordered_set<uint64_t> live;  // issued tickets whose result is not ready yet
    std::vector<double> lat;            // latencies of the last LAT_CAP completed requests (a ring)
    size_t lat_next = 0;
    static constexpr size_t LAT_CAP = size_t(1) << 20;
    uint64_t next_ticket = 1, completed = 0, refused = 0;
    // admission by expected latency (0: off): a request is refused when the
    // requests of its class (at most 4 components, or wider: each class has a partition
    // and a rate of its own) queued and in flight, over that class's recent completion
    // rate (its last RECENT completions up to now), exceed max_latency_ms (Little's law:
    // that quotient is the time a request admitted now can expect to wait for its
    // result); until a class has 64 completions, all requests and all completions count
    double max_latency_ms = 0.0;
    uint64_t in_flight = 0;             // admitted to device slots, result not harvested
    uint64_t in_flight_cls[2] = {0, 0};  // the same by class
    std::deque<clk::time_point> recent, recent_cls[2];
    static constexpr size_t RECENT = 4096;
    bool have_first = false;
    clk::time_point t_first, t_last;
    std::atomic<bool> stop{false};
    std::thread th;
    int next_admit = 0;

    void loop();
    bool harvest(Part &p);
    void launch(Part &p);
    void launch_global(Part &p, const std::vector<Active> &fresh);
    uint64_t submit(int table, const uint32_t *ct, clk::time_point t0, int *rc);
    ~Server();
};

Server::~Server()
{
    hipSetDevice(c->dev->id);
    for (auto &p : part) {
        if (p.st) hipStreamSynchronize(p.st);
        p.tasks.release();
        p.rows.release();
        p.stage_rows.release();
        p.out.release();
        p.stage.release();
        p.qout.release();
        p.wtasks.release();
        p.woff.release();
        if (p.part) hipFree(p.part);
        if (p.ext) hipFree(p.ext);
        if (p.ev) hipEventDestroy(p.ev);
        if (p.st) hipStreamDestroy(p.st);
    }
    if (d_acc) hipFree(d_acc);
    if (d_ct) hipFree(d_ct);
    if (d_ext) hipFree(d_ext);
}

#define SRV_HIP(expr)                                                                               \
    do {                                                                                            \
        hipError_t e_ = (expr);                                                                     \
        if (e_ != hipSuccess)                                                                       \
            throw ::mm::Error(MM_EDEVICE, std::string(#expr) + " failed: " + hipGetErrorString(e_)); \
    } while (0)

Server *server_start(mm_ctx &c, size_t budget, uint32_t chunk)
{
    MM_REQUIRE(chunk >= 1 && chunk <= c.p.n, "chunk_steps must be in [1, n]");
    MM_REQUIRE(c.p.N <= 16384, "the server takes rings of up to 16384 coefficients");
    Device &d = ensure_device(c);
    const size_t N = c.p.N, W = c.p.n + 1;
    const bool global = c.wide || !dev::device_supports_n(c.p.N);
    // at N = 1024 a tick that leaves compute units idle runs the global-accumulator
    // kernels (each component on its own compute unit), a heavier one the fused kernel
    const bool switchable = !global && N == 1024 && dev::wide_supports_wpp((uint32_t)N, 1, 4);
    // per ciphertext slot: input, extracted sample, key-switch partial row; per unit:
    // one (a, b) pair (with every residue; in each of two arenas when ticks may take the
    // global path)
    const size_t per_ct = (W + N + 1) * 4 + W * 8;
    const size_t unit_words = 2 * (size_t)primes_of(c) * N;
    const size_t per_unit = (global || switchable ? 2 : 1) * unit_words * 4;
    const size_t fit = budget / (per_ct + per_unit);
    const size_t units = global ? std::min<size_t>(fit, size_t(1) << 24) : fit / 8 * 8;
    MM_REQUIRE(units >= (global ? 1 : 8), "HBM budget too small for one slot group");
    auto *s = new Server();
    s->c = &c;
    s->chunk = chunk;
    s->global = global;
    s->switchable = switchable;
    s->unit_words = unit_words;
    s->units = (uint32_t)units;
    s->max_cts = (uint32_t)units;
    try {
        if (hipMalloc((void **)&s->d_acc, units * per_unit) != hipSuccess ||
            hipMalloc((void **)&s->d_ct, (size_t)s->max_cts * W * 4) != hipSuccess ||
            (!global && hipMalloc((void **)&s->d_ext, (size_t)s->max_cts * (N + 1) * 4) != hipSuccess))
            throw Error(MM_ENOMEM, "server arena allocation failed");
        s->buddy.init(s->units, global ? 10 : 3);
        s->top_block = s->buddy.largest();
        s->free_slots.resize(s->max_cts);
        for (uint32_t i = 0; i < s->max_cts; i++) s->free_slots[i] = s->max_cts - 1 - i;
        for (auto &p : s->part) {
            SRV_HIP(hipStreamCreateWithFlags(&p.st, hipStreamNonBlocking));
            SRV_HIP(hipEventCreateWithFlags(&p.ev, hipEventDisableTiming));
        }
    } catch (...) {
        delete s;
        throw;
    }
    s->th = std::thread([s] { s->loop(); });
    return s;
}

void server_stop(Server *s)
{
    if (!s) return;
    s->stop = true;
    s->cv.notify_all();
    if (s->th.joinable()) s->th.join();
    delete s;
}

uint64_t Server::submit(int table, const uint32_t *ct, clk::time_point t0, int *rc)
{
    const size_t W = c->p.n + 1;
    bool ok;
    int cls = 0;
    {
        std::lock_guard<std::mutex> gc(c->lock);  // the table list may grow under this lock
        ok = table >= 0 && (size_t)table < c->tables.size() && c->tables[table].g_id < 0;
        if (ok) {
            const uint32_t r = c->tables[table].r;
            ok = global ? order_of(r) <= top_block : r * (uint32_t)dev::waves_per_poly(c->p.N) <= 8;
            cls = r > 4 ? 1 : 0;
        }
    }
    std::lock_guard<std::mutex> g(mu);
    if (!ok) {
        // unknown table, a general table (two bootstraps; not served), too wide a
        // group, or (global path) more components than the arena holds
        *rc = MM_EINVAL;
        return 0;
    }
    if (stop) {
        *rc = MM_ESTATE;  // the serving loop has stopped (a device error ends it; see mm_last_error)
        return 0;
    }
    if (pending[0].size() + pending[1].size() >= pending_cap) {
        *rc = MM_EBUSY;
        return 0;
    }
    if (max_latency_ms > 0) {
        // completions arrive in bursts (a tick at a time): the rate is taken up to now,
        // not up to the last burst, over a window of several ticks
        const auto now = clk::now();
        auto expected_ms = [&](const std::deque<clk::time_point> &rec, double backlog) {
            const double span = std::chrono::duration<double, std::milli>(now - rec.front()).count();
            return span > 0 ? backlog * span / (double)rec.size() : 0.0;
        };
        double e = 0.0;
        if (recent_cls[cls].size() >= 64)
            e = expected_ms(recent_cls[cls], (double)(pending[cls].size() + in_flight_cls[cls]));
        else if (recent.size() >= 64)
            e = expected_ms(recent, (double)(pending[0].size() + pending[1].size() + in_flight));
        if (e > max_latency_ms) {
            refused++;
            *rc = MM_EBUSY;
            return 0;
        }
    }
    Req r{next_ticket++, table, std::vector<uint32_t>(ct, ct + W), t0, cls};
    live.insert(r.ticket);
    if (!have_first) {
        have_first = true;
        t_first = t0;
    }
    const uint64_t ticket = r.ticket;
    pending[cls].push_back(std::move(r));
    cv.notify_all();
    *rc = MM_OK;
    return ticket;
}

// Collect the results of a finished tick.  Returns true if it harvested.
bool Server::harvest(Part &p)
{
    if (!p.busy) return false;
    if (hipEventQuery(p.ev) != hipSuccess) return false;
    const size_t W = c->p.n + 1;
    const auto now = clk::now();
    std::lock_guard<std::mutex> g(mu);
    for (size_t k = 0; k < p.finishing.size(); k++) {
        const Active &a = p.finishing[k];
        Result res{std::vector<uint32_t>(p.out.h + k * W, p.out.h + (k + 1) * W),
                   std::chrono::duration<double, std::milli>(now - a.t0).count()};
        if (lat.size() < LAT_CAP) lat.push_back(res.ms);
        else lat[lat_next] = res.ms;
        lat_next = (lat_next + 1) % LAT_CAP;
        live.erase(a.ticket);
        done.emplace(a.ticket, std::move(res));
        free_slots.push_back(a.slot);
        buddy.release(a.unit, a.order);
        completed++;
        in_flight--;
        const int cls = a.cls;
        in_flight_cls[cls]--;
        recent.push_back(now);
        if (recent.size() > RECENT) recent.pop_front();
        recent_cls[cls].push_back(now);
        if (recent_cls[cls].size() > RECENT) recent_cls[cls].pop_front();
    }
    if (!p.finishing.empty()) t_last = now;
    p.finishing.clear();
    p.busy = false;
    return true;
}

// Admit what fits, then enqueue one tick of this partition.
void Server::launch(Part &p)
{
    const uint32_t N = c->p.N, W = c->p.n + 1, n = c->p.n;
    std::vector<Active> fresh;
    std::vector<Req> fresh_req;
    std::lock_guard<std::mutex> dev_lock(c->lock);  // tables and device state; taken before mu
    {
        std::lock_guard<std::mutex> g(mu);
        // each partition admits one class (at most 4 components, or wider), so that
        // the groups of a tick are alike and every ciphertext advances the full chunk;
        // a partition with nothing in flight and an empty queue of its own takes the other class
        const int own = (int)(&p - part);
        for (int k : {own, own ^ 1}) {
            if (k != own && !(p.active.empty() && fresh.empty())) break;
            std::deque<Req> &queue = pending[k];
            while (!queue.empty() && !free_slots.empty()) {
                const Req &q = queue.front();
                const uint32_t order = order_of(c->tables[q.table].r);
                const int64_t unit = buddy.alloc(order);
                if (unit < 0) break;  // no accumulator memory: wait for completions
                Active a{q.ticket, q.table, free_slots.back(), (uint32_t)unit, order, 0, q.t0, q.cls};
                free_slots.pop_back();
                in_flight++;
                in_flight_cls[q.cls]++;
                fresh.push_back(a);
                fresh_req.push_back(std::move(queue.front()));
                queue.pop_front();
            }
        }
    }
    if (fresh.empty() && p.active.empty()) return;
    Device &d = ensure_device(*c);
    if (!fresh.empty()) {
        p.stage.reserve(fresh.size() * W);
        p.stage_rows.reserve(fresh.size());
        for (size_t k = 0; k < fresh.size(); k++) {
            std::memcpy(p.stage.h + k * W, fresh_req[k].ct.data(), W * 4);
            p.stage_rows.h[k] = (int32_t)fresh[k].slot;
        }
        SRV_HIP(hipMemcpyAsync(p.stage.d, p.stage.h, fresh.size() * W * 4, hipMemcpyHostToDevice, p.st));
        SRV_HIP(hipMemcpyAsync(p.stage_rows.d, p.stage_rows.h, fresh.size() * 4, hipMemcpyHostToDevice, p.st));
        dev::launch_scatter_rows(p.stage.d, d_ct, p.stage_rows.d, fresh.size(), W, p.st);
        p.active.insert(p.active.end(), fresh.begin(), fresh.end());
    }
    bool glob = global;
    if (switchable) {
        // the rule of the batched path's default schedule: at most two components per
        // compute unit, or four where the components cannot take two-wave slots
        uint64_t comps = 0;
        bool wide8 = false;
        for (auto &a : p.active) {
            comps += c->tables[a.table].r;
            wide8 |= c->tables[a.table].r > 4;
        }
        glob = comps <= 2ull * (uint64_t)d.num_cu || (wide8 && comps <= 4ull * (uint64_t)d.num_cu);
    }
    if (glob) {
        launch_global(p, fresh);
        return;
    }
    // one task per resident ciphertext, packed into 8-wave groups; under light
    // load the groups hold at most 4 components (one wave per SIMD), and a
    // ciphertext that still needs all 8 slots (two waves per SIMD, about 1.5x
    // slower per step) advances 2/3 of the steps when the tick also holds narrower
    // ones, so its group does not set the length of the tick for the others
    const uint32_t wpp = (uint32_t)dev::waves_per_poly(c->p.N);
    uint64_t comps = 0;
    for (auto &a : p.active) comps += c->tables[a.table].r;
    const uint32_t cap = spread_cap(d, comps, 8, wpp);
    bool narrow = false, wide = false;
    for (auto &a : p.active) (c->tables[a.table].r > cap ? wide : narrow) = true;
    const uint32_t wide_chunk = narrow && wide ? std::max<uint32_t>(1, chunk * 2 / 3) : chunk;
    auto steps_of = [&](const Active &a) { return c->tables[a.table].r > cap ? wide_chunk : chunk; };
    std::vector<dev::WaveTask> cts(p.active.size());
    for (size_t k = 0; k < p.active.size(); k++) {
        const Active &a = p.active[k];
        const Table &t = c->tables[a.table];
        dev::WaveTask &w = cts[k];
        w.ct = (int32_t)a.slot;
        w.r = t.r;
        w.tv_off = (uint32_t)t.dev_offset;
        w.q_in = t.q_in;
        w.i0 = a.step;
        w.steps = steps_of(a);
        w.flags = (a.step == 0 ? dev::TASK_INIT : 0u) | dev::TASK_STORE | dev::TASK_EXTRACT;
        w.acc_off = (uint64_t)a.unit * 2 * N;
    }
    // a light tick of ciphertexts of at most 4 components (the partition of that
    // class) runs two waves per component, 4 components per group, where the ring
    // has that kernel: each step about 13 % shorter than with one wave per component
    const bool slots2 = wpp == 1 && cap < 8 && !wide && dev::br_supports_wpp(N, 2);
    auto tasks = slots2 ? pack_tasks(cts, 8, 2, 0) : pack_tasks(cts, 8, wpp, cap);
    p.tasks.reserve(tasks.size());
    std::memcpy(p.tasks.h, tasks.data(), tasks.size() * sizeof(dev::WaveTask));
    SRV_HIP(hipMemcpyAsync(p.tasks.d, p.tasks.h, tasks.size() * sizeof(dev::WaveTask), hipMemcpyHostToDevice, p.st));
    dev::BrArgs A = br_args(*c, d);
    A.tasks = p.tasks.d;
    A.num_groups = (int)(tasks.size() / 8);  // 8-wave groups (any r <= 8)
    A.steps = (int)chunk;
    A.ct_in = d_ct;
    // the partition's current arena, read and written in place
    A.acc_state = switchable ? d_acc + (size_t)p.cur * units * unit_words : d_acc;
    A.ext_out = d_ext;
    dev::launch_blind_rotate(N, A, 8, std::min(A.num_groups, d.num_cu), p.st, slots2 ? 2 : 0);

    // ciphertexts that reach step n in this tick: key switch and copy back
    std::vector<Active> keep;
    p.finishing.clear();
    for (auto &a : p.active) {
        const uint32_t st = steps_of(a);
        if (a.step + st >= n) p.finishing.push_back(a);
        else {
            a.step += st;
            keep.push_back(a);
        }
    }
    p.active.swap(keep);
    const size_t F = p.finishing.size();
    if (F) {
        p.rows.reserve(F);
        p.qout.reserve(F);
        p.out.reserve(F * W);
        for (size_t k = 0; k < F; k++) {
            p.rows.h[k] = (int32_t)p.finishing[k].slot;
            p.qout.h[k] = c->tables[p.finishing[k].table].q_in;
        }
        SRV_HIP(hipMemcpyAsync(p.rows.d, p.rows.h, F * 4, hipMemcpyHostToDevice, p.st));
        SRV_HIP(hipMemcpyAsync(p.qout.d, p.qout.h, F * 4, hipMemcpyHostToDevice, p.st));
        const KsSched ks = ks_default(*c, d, F);
        const size_t need = ks_part_words(*c, ks, F);
        if (p.part_cap < need) {
            SRV_HIP(hipStreamSynchronize(p.st));
            if (p.part) SRV_HIP(hipFree(p.part));
            p.part = nullptr;
            p.part_cap = 0;
            if (hipMalloc((void **)&p.part, need * 2 * 8) != hipSuccess) throw Error(MM_ENOMEM, "server key-switch buffer");
            p.part_cap = need * 2;
        }
        enqueue_keyswitch(*c, d, d_ext, p.rows.d, F, p.out.d, p.qout.d, 0, ks, p.part, p.st);
        SRV_HIP(hipMemcpyAsync(p.out.h, p.out.d, F * W * 4, hipMemcpyDeviceToHost, p.st));
    }
    SRV_HIP(hipGetLastError());
    SRV_HIP(hipEventRecord(p.ev, p.st));
    p.busy = true;
}

// One tick on the global-accumulator path: initialise the fresh ciphertexts'
// accumulators in the partition's current arena, `chunk` CMux launches over every
// resident component (each from its own ciphertext's step), then extraction, key
// switch and copy-back of the ciphertexts that reached step n.
void Server::launch_global(Part &p, const std::vector<Active> &fresh)
{
    const uint32_t N = c->p.N, W = c->p.n + 1, n = c->p.n;
    Device &d = *c->dev;
    const int npr = primes_of(*c);
    uint32_t *arena[2] = {d_acc, d_acc + (size_t)units * unit_words};
    auto task = [&](const Active &a, uint32_t j, uint32_t i0) {
        const Table &t = c->tables[a.table];
        return dev::WideTask{(int32_t)a.slot, j, t.r, t.q_in, (uint32_t)t.dev_offset, i0, (uint64_t)a.unit * unit_words};
    };
    std::vector<dev::WideTask> list;
    for (auto &a : fresh)
        for (uint32_t j = 0; j < c->tables[a.table].r; j++) list.push_back(task(a, j, 0));
    const size_t n_init = list.size();
    for (auto &a : p.active)
        for (uint32_t j = 0; j < c->tables[a.table].r; j++) list.push_back(task(a, j, a.step));
    const size_t n_step = list.size() - n_init;
    p.wtasks.reserve(list.size());
    std::memcpy(p.wtasks.h, list.data(), list.size() * sizeof(dev::WideTask));
    SRV_HIP(hipMemcpyAsync(p.wtasks.d, p.wtasks.h, list.size() * sizeof(dev::WideTask), hipMemcpyHostToDevice, p.st));
    dev::WideArgs A = wide_args(*c, d);
    A.ct_in = d_ct;
    if (n_init) {
        A.tasks = p.wtasks.d;
        A.acc_wr = arena[p.cur];
        dev::launch_wide_init(N, npr, A, (uint32_t)n_init, p.st);
    }
    A.tasks = p.wtasks.d + n_init;
    const int wpp = switchable ? light_global_wpp(*c) : 0;
    const bool ps = prime_split(*c, d, n_step);
    const int dg = switchable ? light_global_dg(*c, d, n_step) : ps ? prime_split_dg(*c, d, n_step) : 1;
    for (uint32_t s = 0; s < chunk; s++) {
        A.step = s;
        A.acc_rd = arena[p.cur];
        A.acc_wr = arena[p.cur ^ 1];
        dev::launch_wide_step(N, npr, c->keys, A, (uint32_t)n_step, p.st, wpp, dg, ps);
        p.cur ^= 1;
    }
    std::vector<Active> keep;
    p.finishing.clear();
    for (auto &a : p.active) {
        if (a.step + chunk >= n) p.finishing.push_back(a);
        else {
            a.step += chunk;
            keep.push_back(a);
        }
    }
    p.active.swap(keep);
    const size_t F = p.finishing.size();
    if (F) {
        p.woff.reserve(F);
        p.qout.reserve(F);
        p.out.reserve(F * W);
        for (size_t k = 0; k < F; k++) {
            p.woff.h[k] = (uint64_t)p.finishing[k].unit * unit_words;
            p.qout.h[k] = c->tables[p.finishing[k].table].q_in;
        }
        SRV_HIP(hipMemcpyAsync(p.woff.d, p.woff.h, F * 8, hipMemcpyHostToDevice, p.st));
        SRV_HIP(hipMemcpyAsync(p.qout.d, p.qout.h, F * 4, hipMemcpyHostToDevice, p.st));
        const KsSched ks = ks_default(*c, d, F);
        const size_t need = ks_part_words(*c, ks, F);
        if (p.part_cap < need || p.ext_cap < F) {
            SRV_HIP(hipStreamSynchronize(p.st));
            if (p.part_cap < need) {
                if (p.part) SRV_HIP(hipFree(p.part));
                p.part = nullptr;
                p.part_cap = 0;
                if (hipMalloc((void **)&p.part, need * 2 * 8) != hipSuccess)
                    throw Error(MM_ENOMEM, "server key-switch buffer");
                p.part_cap = need * 2;
            }
            if (p.ext_cap < F) {
                if (p.ext) SRV_HIP(hipFree(p.ext));
                p.ext = nullptr;
                p.ext_cap = 0;
                if (hipMalloc((void **)&p.ext, F * 2 * (N + 1) * 4) != hipSuccess)
                    throw Error(MM_ENOMEM, "server extraction buffer");
                p.ext_cap = F * 2;
            }
        }
        A.acc_rd = arena[p.cur];
        dev::launch_wide_extract(N, npr, A, p.woff.d, F, p.ext, p.st);
        enqueue_keyswitch(*c, d, p.ext, nullptr, F, p.out.d, p.qout.d, 0, ks, p.part, p.st);
        SRV_HIP(hipMemcpyAsync(p.out.h, p.out.d, F * W * 4, hipMemcpyDeviceToHost, p.st));
    }
    SRV_HIP(hipGetLastError());
    SRV_HIP(hipEventRecord(p.ev, p.st));
    p.busy = true;
}

void Server::loop()
{
    try {
        hipSetDevice(c->dev->id);
        for (;;) {
            bool progress = false;
            for (int k = 0; k < 2; k++) {
                Part &p = part[(next_admit + k) & 1];
                progress |= harvest(p);
                if (!p.busy) {
                    launch(p);
                    progress |= p.busy;
                }
            }
            next_admit ^= 1;
            const bool idle = !part[0].busy && !part[1].busy;
            std::unique_lock<std::mutex> g(mu);
            if (idle && pending[0].empty() && pending[1].empty()) {
                if (stop) break;
                cv.wait_for(g, std::chrono::milliseconds(5));
            } else if (!progress) {
                g.unlock();
                std::this_thread::sleep_for(std::chrono::microseconds(50));
            }
        }
    } catch (const std::exception &e) {
        std::lock_guard<std::mutex> g(c->lock);
        c->err = std::string("server: ") + e.what();
        stop = true;
    }
}

}  // namespace mm

struct mm_server {
    mm::Server *s;
};

namespace {

template <class F>
int srv_guard(mm_ctx *c, F &&f)
{
    try {
        f();
        return MM_OK;
    } catch (const mm::Error &e) {
        if (c) c->err = e.what();
        return e.code;
    } catch (const std::bad_alloc &) {
        return MM_ENOMEM;
    } catch (const std::exception &e) {
        if (c) c->err = e.what();
        return MM_EDEVICE;
    }
}

}  // namespace

extern "C" {

int mm_server_start(mm_ctx *ctx, size_t hbm_budget_bytes, uint32_t chunk_steps, mm_server **out)
{
    if (!ctx || !out) return MM_EINVAL;
    if (ctx->server) return MM_ESTATE;
    return srv_guard(ctx, [&] {
        mm::Server *s;
        {
            std::lock_guard<std::mutex> g(ctx->lock);
            s = mm::server_start(*ctx, hbm_budget_bytes, chunk_steps);
        }
        ctx->server = s;
        *out = new mm_server{s};
    });
}

int mm_submit(mm_server *h, int table_id, const uint32_t *ct, uint64_t *ticket)
{
    if (!h || !h->s || !ct || !ticket) return MM_EINVAL;
    int rc = MM_OK;
    *ticket = h->s->submit(table_id, ct, mm::clk::now(), &rc);
    return rc;
}

int mm_poll(mm_server *h, uint64_t ticket, uint32_t *ct_out)
{
    if (!h || !h->s || !ct_out) return MM_EINVAL;
    mm::Server &s = *h->s;
    std::lock_guard<std::mutex> g(s.mu);
    auto it = s.done.find(ticket);
    if (it == s.done.end()) {
        if (!s.live.count(ticket)) return MM_EINVAL;  // never issued, or already collected
        return s.stop ? MM_ESTATE : MM_EAGAIN;        // a stopped loop will not finish it
    }
    std::memcpy(ct_out, it->second.ct.data(), it->second.ct.size() * 4);
    s.done.erase(it);
    return MM_OK;
}

int mm_server_set_admission(mm_server *h, double max_latency_ms)
{
    if (!h || !h->s || !(max_latency_ms >= 0)) return MM_EINVAL;
    std::lock_guard<std::mutex> g(h->s->mu);
    h->s->max_latency_ms = max_latency_ms;
    return MM_OK;
}

int mm_server_refused(mm_server *h, uint64_t *refused)
{
    if (!h || !h->s || !refused) return MM_EINVAL;
    std::lock_guard<std::mutex> g(h->s->mu);
    *refused = h->s->refused;
    return MM_OK;
}

int mm_server_stats(mm_server *h, double *p50_ms, double *p99_ms, double *boots_per_s, uint64_t *completed)
{
    if (!h || !h->s) return MM_EINVAL;
    mm::Server &s = *h->s;
    std::lock_guard<std::mutex> g(s.mu);
    std::vector<double> v(s.lat);
    auto pct = [&](double q) {
        if (v.empty()) return 0.0;
        size_t k = (size_t)(q * (v.size() - 1) + 0.5);
        std::nth_element(v.begin(), v.begin() + k, v.end());
        return v[k];
    };
    if (p50_ms) *p50_ms = pct(0.50);
    if (p99_ms) *p99_ms = pct(0.99);
    if (boots_per_s) {
        const double secs = s.completed ? std::chrono::duration<double>(s.t_last - s.t_first).count() : 0.0;
        *boots_per_s = secs > 0 ? (double)s.completed / secs : 0.0;
    }
    if (completed) *completed = s.completed;
    return MM_OK;
}

int mm_server_stop(mm_server *h)
{
    if (!h || !h->s) return MM_EINVAL;
    mm_ctx *c = h->s->c;
    mm::server_stop(h->s);
    if (c) c->server = nullptr;
    delete h;
    return MM_OK;
}

int mm_server_replay(mm_server *h, const int *table_ids, const uint32_t *ct_in, const int64_t *arrival_ns,
                     size_t count, uint32_t *ct_out, double *latency_ms)
{
    if (!h || !h->s || (count && (!table_ids || !ct_in || !arrival_ns || !ct_out || !latency_ms))) return MM_EINVAL;
    mm::Server &s = *h->s;
    const size_t W = s.c->p.n + 1;
    const auto start = mm::clk::now();
    std::vector<uint64_t> tickets(count, 0);
    std::vector<char> refused(count, 0);
    std::vector<mm::clk::time_point> t0(count);
    size_t next_poll = 0;
    auto poll_some = [&](bool all) {
        std::lock_guard<std::mutex> g(s.mu);
        while (next_poll < count && (tickets[next_poll] || refused[next_poll])) {
            if (refused[next_poll]) {  // refused by admission: no result, latency -1
                std::memset(ct_out + next_poll * W, 0, W * 4);
                latency_ms[next_poll] = -1.0;
                next_poll++;
                continue;
            }
            auto it = s.done.find(tickets[next_poll]);
            if (it == s.done.end()) {
                if (!all) break;
                return false;
            }
            std::memcpy(ct_out + next_poll * W, it->second.ct.data(), W * 4);
            latency_ms[next_poll] = it->second.ms;
            s.done.erase(it);
            next_poll++;
        }
        return next_poll == count;
    };
    for (size_t k = 0; k < count; k++) {
        t0[k] = start + std::chrono::nanoseconds(arrival_ns[k]);
        for (;;) {  // wait for the scheduled arrival
            const auto now = mm::clk::now();
            if (now >= t0[k]) break;
            const auto gap = t0[k] - now;
            if (gap > std::chrono::microseconds(200)) std::this_thread::sleep_for(gap - std::chrono::microseconds(100));
        }
        for (;;) {
            int rc = MM_OK;
            tickets[k] = s.submit(table_ids[k], ct_in + k * W, t0[k], &rc);
            if (rc == MM_OK) break;
            if (rc != MM_EBUSY) return rc;
            bool shedding;
            {
                std::lock_guard<std::mutex> g(s.mu);
                shedding = s.max_latency_ms > 0;
            }
            if (shedding) {  // refused by admission: recorded, not retried
                refused[k] = 1;
                break;
            }
            std::this_thread::sleep_for(std::chrono::microseconds(100));  // the queue is full: wait
        }
        if ((k & 63) == 63) poll_some(false);
    }
    for (;;) {
        if (poll_some(false) && next_poll == count) break;
        if (s.stop) return MM_EDEVICE;
        std::this_thread::sleep_for(std::chrono::microseconds(200));
    }
    return MM_OK;
}

}  // extern "C"
