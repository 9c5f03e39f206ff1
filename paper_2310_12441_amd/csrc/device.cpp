// Device runtime of the library: key upload, workspace, batching (packing
// ciphertext components into 8-wave groups), HIP-graph capture of the batched
// launch sequence, and the per-row entry points.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <functional>
#include <numeric>
#include <string>

#include "device_internal.hpp"

namespace mm {

void DeviceDeleter::operator()(Device *d) const { delete d; }

void device_release(mm_ctx &c) { c.dev.reset(); }

void *ws(Device &d, int slot, size_t bytes)
{
    DevBuf &b = d.ws[slot];
    if (b.bytes < bytes) {
        HIPC(hipDeviceSynchronize());
        if (b.p) HIPC(hipFree(b.p));
        b.p = nullptr;
        b.bytes = 0;
        const size_t want = std::max<size_t>(bytes + bytes / 4, 4096);
        if (hipMalloc(&b.p, want) != hipSuccess) {
            b.p = nullptr;
            throw Error(MM_ENOMEM, "device workspace allocation failed");
        }
        b.bytes = want;
        d.ws_generation++;
        for (auto &g : d.graphs)
            if (g.exec) hipGraphExecDestroy(g.exec);
        d.graphs.clear();
    }
    return b.p;
}

// Pinned host staging buffer `slot`; waits until its previous use has executed.
void *pinned(Device &d, int slot, size_t bytes)
{
    PinBuf &b = d.pin[slot];
    if (!b.ev) HIPC(hipEventCreateWithFlags(&b.ev, hipEventDisableTiming));
    HIPC(hipEventSynchronize(b.ev));
    if (b.bytes < bytes) {
        if (b.p) HIPC(hipHostFree(b.p));
        b.p = nullptr;
        const size_t want = std::max<size_t>(bytes * 2, 4096);
        if (hipHostMalloc(&b.p, want, hipHostMallocDefault) != hipSuccess) {
            b.p = nullptr;
            b.bytes = 0;
            throw Error(MM_ENOMEM, "pinned staging allocation failed");
        }
        b.bytes = want;
    }
    return b.p;
}

static uint32_t neg_inv_2_32(uint32_t Q)
{
    uint32_t inv = Q;  // Newton: inv = Q^-1 mod 2^32 (Q odd)
    for (int i = 0; i < 5; i++) inv *= 2u - Q * inv;
    return 0u - inv;
}

static uint32_t to_mont(uint32_t x, uint32_t Q) { return (uint32_t)(((uint64_t)x << 32) % Q); }

// BSK in the NTT domain for one prime, times 2^32 / N (Montgomery form with the
// inverse NTT's 1/N folded in), and its digit-offset correction: the blind
// rotation feeds the gadget digits shifted by +B/2 (non-negative, one bit-field
// extract each), i.e. each digit polynomial gains (B/2)(1 + x + ... + x^(N-1));
// in the NTT domain that adds (B/2) NTT(1 + ... + x^(N-1)) sum_{key,row} K/N to
// each output part, and the accumulator starts from minus that sum.
// coeff is [n][K][2l][2][N]; kb has the same layout, corr is [n][2][N].
static void ntt_domain_keys(const mm_ctx &c, const NttTables &T, const uint32_t *coeff, std::vector<uint32_t> &kb,
                            std::vector<uint32_t> &corr)
{
    const mm_params &p = c.p;
    const uint32_t N = p.N, Q = T.Q;
    const size_t polys = (size_t)p.n * c.keys * 2 * p.l * 2;
    kb.assign(polys * N, 0);
    const uint32_t scale = to_mont(T.n_inv, Q);
    parallel_for((int64_t)polys, [&](int64_t t) {
        uint32_t *dst = &kb[(size_t)t * N];
        std::memcpy(dst, coeff + (size_t)t * N, sizeof(uint32_t) * N);
        T.forward(dst);
        for (uint32_t k = 0; k < N; k++) dst[k] = mulmod(dst[k], scale, Q);
    });
    const uint32_t K = c.keys, rows = 2 * p.l;
    corr.assign((size_t)p.n * 2 * N, 0);
    const uint32_t inv_r = [&] {  // 2^-32 mod Q
        uint64_t x = to_mont(1, Q), e = Q - 2, r = 1;
        while (e) {
            if (e & 1) r = mulmod((uint32_t)r, (uint32_t)x, Q);
            x = mulmod((uint32_t)x, (uint32_t)x, Q);
            e >>= 1;
        }
        return (uint32_t)r;
    }();
    const uint32_t half_b = mulmod(1u << (p.log2_B - 1), inv_r, Q);
    std::vector<uint32_t> ones(N, 1u);
    T.forward(ones.data());
    parallel_for((int64_t)p.n * 2, [&](int64_t ip) {
        const size_t i = (size_t)ip / 2, part = (size_t)ip % 2;
        uint32_t *dst = &corr[(i * 2 + part) * N];
        for (uint32_t k = 0; k < N; k++) {
            uint64_t sum = 0;
            for (uint32_t key = 0; key < K; key++)
                for (uint32_t row = 0; row < rows; row++)
                    sum += kb[((((size_t)i * K + key) * rows + row) * 2 + part) * N + k];
            const uint32_t cval = mulmod(mulmod((uint32_t)(sum % Q), half_b, Q), ones[k], Q);
            dst[k] = cval ? Q - cval : 0;
        }
    });
}

void device_init(mm_ctx &c, int id)
{
    if (c.dev && c.dev->id == id) return;
    c.dev.reset();
    std::unique_ptr<Device, DeviceDeleter> d(new Device());
    HIPC(hipSetDevice(id));
    d->id = id;
    hipDeviceProp_t prop;
    HIPC(hipGetDeviceProperties(&prop, id));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        throw Error(MM_EDEVICE, std::string("device is ") + prop.gcnArchName + ", the kernels are built for gfx950");
    d->num_cu = prop.multiProcessorCount;
    const mm_params &p = c.p;
    const uint32_t N = p.N, Q = p.Q;
    MM_REQUIRE(dev::device_supports_n(N) || dev::wide_supports_n(N, 1),
               "device path supports N in {256, 512, ..., 65536}");
    MM_REQUIRE(!c.wide || dev::wide_supports_n(N, 2), "the wide-modulus path supports N in {256, ..., 4096}");
    d->qn = neg_inv_2_32(Q);
    // 2^64 / N mod Q, for the pointwise product of two forward NTTs
    d->c_fix = mulmod(to_mont(to_mont(1, Q), Q), c.ntt.n_inv, Q);

    auto twiddles = [&](const NttTables &T, std::vector<uint32_t> &twf, std::vector<uint32_t> &twi) {
        twf.resize(N);
        twi.resize(N);
        for (uint32_t k = 0; k < N; k++) {
            twf[k] = to_mont(T.fwd[k], T.Q);
            twi[k] = to_mont(T.inv[k], T.Q);
        }
    };
    auto upload = [&](uint32_t **dst, const uint32_t *src, size_t words) {
        if (hipMalloc((void **)dst, words * 4) != hipSuccess) {
            *dst = nullptr;
            throw Error(MM_ENOMEM, "device key allocation failed");
        }
        HIPC(hipMemcpy(*dst, src, words * 4, hipMemcpyHostToDevice));
    };
    std::vector<uint32_t> twf, twi;
    twiddles(c.ntt, twf, twi);
    upload(&d->twf, twf.data(), N);
    upload(&d->twi, twi.data(), N);
    if (!c.wide && dev::split_supports_n(N)) {
        // sub-ring h's stage with m' groups uses the full table's entry M m' + h m' + i'
        const uint32_t NS = dev::SPLIT_NS, M = N / NS;
        std::vector<uint32_t> sf((size_t)M * NS, 0), si((size_t)M * NS, 0);
        for (uint32_t h = 0; h < M; h++)
            for (uint32_t mm = 1; mm < NS; mm <<= 1)
                for (uint32_t g = 0; g < mm; g++) {
                    sf[(size_t)h * NS + mm + g] = twf[M * mm + h * mm + g];
                    si[(size_t)h * NS + mm + g] = twi[M * mm + h * mm + g];
                }
        upload(&d->twf_sub, sf.data(), sf.size());
        upload(&d->twi_sub, si.data(), si.size());
    }
    std::vector<uint32_t> kb, corr;
    if (!c.wide) {
        ntt_domain_keys(c, c.ntt, c.bsk.data(), kb, corr);
    } else {
        // two primes: [n][K][prime][2l][2][N] keys, [n][prime][2][N] corrections
        const size_t per = (size_t)2 * p.l * 2 * N, nk = (size_t)p.n * c.keys;
        std::vector<uint32_t> one(nk * per), kbp, corrp;
        kb.assign(nk * 2 * per, 0);
        corr.assign((size_t)p.n * 2 * 2 * N, 0);
        const NttTables *T[2] = {&c.ntt, &c.ntt2};
        for (size_t pr = 0; pr < 2; pr++) {
            for (size_t ik = 0; ik < nk; ik++)
                std::memcpy(&one[ik * per], &c.bsk[(ik * 2 + pr) * per], per * 4);
            ntt_domain_keys(c, *T[pr], one.data(), kbp, corrp);
            for (size_t ik = 0; ik < nk; ik++) std::memcpy(&kb[(ik * 2 + pr) * per], &kbp[ik * per], per * 4);
            for (size_t i = 0; i < p.n; i++)
                std::memcpy(&corr[(i * 2 + pr) * 2 * N], &corrp[i * 2 * N], 2 * N * 4);
        }
        twiddles(c.ntt2, twf, twi);
        upload(&d->twf2, twf.data(), N);
        upload(&d->twi2, twi.data(), N);
        d->qn2 = neg_inv_2_32(p.Q2);
    }
    upload(&d->bsk, kb.data(), kb.size());
    upload(&d->bsk_corr, corr.data(), corr.size());
    {
        // the key-switching key in column tiles, [i][tile][l_ks B_ks][64], a few
        // coordinates at a time through a host buffer
        const size_t W = p.n + 1, rows = (size_t)p.l_ks << p.log2_Bks, T = (W + 63) / 64;
        const size_t per_i = T * rows * 64;
        if (hipMalloc((void **)&d->ksk, (size_t)N * per_i * 4) != hipSuccess) {
            d->ksk = nullptr;
            throw Error(MM_ENOMEM, "device key allocation failed");
        }
        const size_t chunk = std::max<size_t>(1, ((size_t)64 << 20) / (per_i * 4));
        std::vector<uint32_t> buf(std::min<size_t>(chunk, N) * per_i);
        for (size_t i0 = 0; i0 < N; i0 += chunk) {
            const size_t ni = std::min<size_t>(chunk, N - i0);
            parallel_for((int64_t)(ni * T), [&](int64_t it) {
                const size_t i = i0 + (size_t)it / T, x = (size_t)it % T;
                uint32_t *dst = &buf[(size_t)it * rows * 64];
                for (size_t row = 0; row < rows; row++) {
                    const uint32_t *srow = &c.ksk[(i * rows + row) * W];
                    for (size_t cc = 0; cc < 64; cc++) {
                        const size_t col = x * 64 + cc;
                        dst[row * 64 + cc] = col < W ? srow[col] : 0u;
                    }
                }
            });
            HIPC(hipMemcpy(d->ksk + i0 * per_i, buf.data(), ni * per_i * 4, hipMemcpyHostToDevice));
        }
    }
    HIPC(dev::init_kernel_attributes());
    HIPC(dev::noalloc_scratch_init(id, &d->scratch));
    HIPC(hipStreamCreateWithFlags(&d->own, hipStreamNonBlocking));
    c.dev = std::move(d);
}

Device &ensure_device(mm_ctx &c)
{
    if (!c.dev) {
        int cur = 0;
        HIPC(hipGetDevice(&cur));
        device_init(c, cur);
    }
    HIPC(hipSetDevice(c.dev->id));
    Device &d = *c.dev;
    // (re)upload the test-vector arena when tables were added
    if (d.tables_uploaded != c.tables.size()) {
        size_t words = 0;
        for (auto &t : c.tables) {
            t.dev_offset = words;
            words += t.V.size();
        }
        std::vector<uint32_t> arena(std::max<size_t>(words, 1));
        for (auto &t : c.tables) std::memcpy(&arena[t.dev_offset], t.V.data(), t.V.size() * 4);
        HIPC(hipDeviceSynchronize());
        if (d.tv) HIPC(hipFree(d.tv));
        d.tv = nullptr;
        if (hipMalloc((void **)&d.tv, arena.size() * 4) != hipSuccess) throw Error(MM_ENOMEM, "test vector upload");
        HIPC(hipMemcpy(d.tv, arena.data(), arena.size() * 4, hipMemcpyHostToDevice));
        d.tables_uploaded = c.tables.size();
        for (auto &g : d.graphs)
            if (g.exec) hipGraphExecDestroy(g.exec);
        d.graphs.clear();
    }
    return d;
}

// ------------------------------------------------------------------ staging

static const uint32_t *stage_in(Device &d, int slot, const uint32_t *p, size_t words, bool dptr, hipStream_t st)
{
    if (dptr || words == 0) return p;
    uint32_t *b = (uint32_t *)ws(d, slot, words * 4);
    HIPC(hipMemcpyAsync(b, p, words * 4, hipMemcpyHostToDevice, st));
    return b;
}

static uint32_t *stage_out(Device &d, int slot, uint32_t *p, size_t words, bool dptr)
{
    if (dptr || words == 0) return p;
    return (uint32_t *)ws(d, slot, words * 4);
}

static void finish_out(uint32_t *host, const uint32_t *dev, size_t words, bool dptr, hipStream_t st)
{
    if (!dptr && words) HIPC(hipMemcpyAsync(host, dev, words * 4, hipMemcpyDeviceToHost, st));
    if (!dptr) HIPC(hipStreamSynchronize(st));
}

// ------------------------------------------------------------------ batching

// Pack ciphertexts into groups of gw waves = gw / wpp component slots (wpp
// waves per polynomial), first-fit over r descending, each ciphertext's
// components on consecutive slots of one group.  cts[k] is the task of
// ciphertext k with comp = 0; the result holds gw tasks per group, the wpp
// waves of a slot carrying the same task.  With cap < slots a group takes at
// most cap components (a wider ciphertext still gets a group of its own), so
// that a small batch spreads over more compute units, one wave per SIMD.
std::vector<dev::WaveTask> pack_tasks(const std::vector<dev::WaveTask> &cts, uint32_t gw, uint32_t wpp, uint32_t cap)
{
    const uint32_t slots = gw / wpp;
    cap = std::max<uint32_t>(1, std::min(cap ? cap : slots, slots));
    for (auto &t : cts)
        MM_REQUIRE(t.r >= 1 && t.r <= slots,
                   "a ciphertext's r components times their waves per component must fit one workgroup");
    std::vector<size_t> order(cts.size());
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) { return cts[a].r > cts[b].r; });
    std::vector<dev::WaveTask> tasks;
    std::vector<uint32_t> used;  // slots used per group
    size_t first_open = 0;
    for (size_t o : order) {
        const uint32_t r = cts[o].r, limit = std::max(cap, r);
        size_t g = first_open;
        while (g < used.size() && used[g] + r > limit) g++;
        if (g == used.size()) {
            used.push_back(0);
            dev::WaveTask idle{};
            idle.ct = -1;
            tasks.insert(tasks.end(), gw, idle);
        }
        for (uint32_t j = 0; j < r; j++) {
            dev::WaveTask w = cts[o];
            w.comp = j;
            for (uint32_t v = 0; v < wpp; v++) tasks[g * gw + (used[g] + j) * wpp + v] = w;
        }
        used[g] += r;
        while (first_open < used.size() && used[first_open] >= cap) first_open++;
    }
    return tasks;
}

// Components per group for a batch of `comps` components: the full width,
// or half of it when that still fits every group on its own compute unit.
uint32_t spread_cap(const Device &d, uint64_t comps, uint32_t gw, uint32_t wpp)
{
    const uint32_t slots = gw / wpp;
    if (slots >= 8 && comps <= (uint64_t)(slots / 2) * (uint64_t)d.num_cu) return slots / 2;
    return slots;
}

static std::vector<dev::WaveTask> pack_groups(const mm_ctx &c, const Device &d, const int *ids, size_t count,
                                              uint32_t flags, uint32_t i0, const std::vector<uint64_t> &acc_off,
                                              uint32_t gw = 8, uint32_t wpp = 0)
{
    std::vector<dev::WaveTask> cts(count);
    for (size_t k = 0; k < count; k++) {
        const Table &t = c.tables[ids[k]];
        dev::WaveTask &w = cts[k];
        w.ct = (int32_t)k;
        w.comp = 0;
        w.r = t.r;
        w.tv_off = (uint32_t)t.dev_offset;
        w.q_in = t.q_in;
        w.i0 = i0;
        w.flags = flags;
        w.acc_off = acc_off.empty() ? 0 : acc_off[k];
    }
    uint64_t comps = 0;
    for (auto &t : cts) comps += t.r;
    if (!wpp) wpp = (uint32_t)dev::waves_per_poly(c.p.N);
    return pack_tasks(cts, gw, wpp, spread_cap(d, comps, gw, wpp));
}

// Valid ids; returns how many name general (two-bootstrap) tables.
static size_t check_ids(const mm_ctx &c, const int *ids, size_t count)
{
    MM_REQUIRE(ids || count == 0, "null table ids");
    size_t general = 0;
    for (size_t i = 0; i < count; i++) {
        MM_REQUIRE(ids[i] >= 0 && (size_t)ids[i] < c.tables.size(), "table id out of range");
        general += c.tables[ids[i]].g_id >= 0;
    }
    return general;
}

static dev::WaveTask *upload_tasks(Device &d, const std::vector<dev::WaveTask> &tasks, hipStream_t st)
{
    const size_t bytes = tasks.size() * sizeof(dev::WaveTask);
    void *h = pinned(d, 0, bytes);
    std::memcpy(h, tasks.data(), bytes);
    auto *dt = (dev::WaveTask *)ws(d, WS_TASKS, bytes);
    HIPC(hipMemcpyAsync(dt, h, bytes, hipMemcpyHostToDevice, st));
    HIPC(hipEventRecord(d.pin[0].ev, st));
    return dt;
}

dev::BrArgs br_args(const mm_ctx &c, const Device &d)
{
    dev::BrArgs A{};
    A.ct_stride = c.p.n + 1;
    A.n = c.p.n;
    A.Q = c.p.Q;
    A.qn = d.qn;
    A.log2B = c.p.log2_B;
    A.l = c.p.l;
    A.sg = c.sg;
    A.keys = c.keys;
    A.goff = 0;  // (B/2)(1 + B + ... + B^(l-1)): every digit becomes a non-negative bit field
    for (uint32_t u = 0; u < c.p.l; u++) A.goff += (1u << (c.p.log2_B - 1)) << (u * c.p.log2_B);
    A.bsk = d.bsk;
    A.bsk_corr = d.bsk_corr;
    A.twf = d.twf;
    A.twi = d.twi;
    A.tv = d.tv;
    return A;
}

uint32_t ks_splits(const mm_ctx &c, const Device &d, size_t count)
{
    const size_t col_tiles = (c.p.n + 1 + 63) / 64;
    const size_t ct_tiles = (count + 4 * dev::KS_CTS_PER_WAVE - 1) / (4 * dev::KS_CTS_PER_WAVE);
    const size_t target = 2 * (size_t)d.num_cu;
    size_t P = (target + col_tiles * ct_tiles - 1) / (col_tiles * ct_tiles);
    P = std::max<size_t>(1, std::min<size_t>(P, c.p.N / 8));
    return (uint32_t)P;
}

// Splits of the i range for the one-ciphertext-per-lane key switch: as many as
// keep the launch within one round of two workgroups per compute unit.
static uint32_t ks_lanes_splits(const mm_ctx &c, const Device &d, size_t count)
{
    const size_t blocks = ((c.p.n + 1 + 63) / 64) * ((count + 255) / 256);
    return (uint32_t)std::max<size_t>(1, std::min<size_t>(8, 2 * (size_t)d.num_cu / blocks));
}

// Key-switch schedule for `count` samples: one ciphertext per lane for large
// batches, the LDS-tiled kernel with columns in lanes (cpw > 0) for medium
// ones, the i-split kernel for small ones.
KsSched ks_default(const mm_ctx &c, const Device &d, size_t count)
{
    KsSched k;
    const uint32_t rows = c.p.l_ks << c.p.log2_Bks;
    if (count >= 512 && rows <= (uint32_t)dev::KS_TILED_MAX_ROWS) {
        k.cpw = KS_LANES;
        k.P = ks_lanes_splits(c, d, count);
    } else if (count >= 256 && rows <= (uint32_t)dev::KS_TILED_MAX_ROWS) {
        k.cpw = 32;
        const size_t blocks = ((c.p.n + 1 + 63) / 64) * ((count + 4 * k.cpw - 1) / (4 * k.cpw));
        k.P = (uint32_t)std::max<size_t>(1, std::min<size_t>(4, (2 * (size_t)d.num_cu + blocks - 1) / blocks));
    } else {
        k.cpw = 0;
        k.P = ks_splits(c, d, count);
    }
    return k;
}

size_t ks_part_words(const mm_ctx &c, const KsSched &k, size_t count) { return (size_t)k.P * count * (c.p.n + 1); }

// Enqueue key switch + final modulus switch of `count` extracted samples
// (row k of the output is sample rows[k] of ext, or sample k when rows is null).
void enqueue_keyswitch(const mm_ctx &c, Device &d, const uint32_t *ext, const int32_t *rows, size_t count,
                       uint32_t *out, const uint32_t *q_out_per_ct, uint32_t q_out, const KsSched &ks, uint64_t *part,
                       hipStream_t st)
{
    dev::KsArgs K{};
    K.lwe_N = ext;
    K.rows = rows;
    K.ksk = d.ksk;
    K.col_tiles = (c.p.n + 1 + 63) / 64;
    K.part = part;
    K.count = count;
    K.n = c.p.n;
    K.N = c.p.N;
    K.Q = c.p.Q;
    K.log2Bks = c.p.log2_Bks;
    K.l_ks = c.p.l_ks;
    if (ks.cpw == KS_LANES) dev::launch_keyswitch_lanes(K, ks.P, st);
    else if (ks.cpw > 0) dev::launch_keyswitch_tiled(K, ks.cpw, ks.P, st);
    else dev::launch_keyswitch(K, ks.P, st);
    dev::launch_ks_finalize(part, ext, rows, out, count, c.p.n, c.p.N, ks.P, c.p.Q, q_out_per_ct, q_out, st);
}

static uint32_t max_r(const mm_ctx &c, const int *ids, size_t count)
{
    uint32_t m = 1;
    for (size_t i = 0; i < count; i++) m = std::max(m, c.tables[ids[i]].r);
    return m;
}

static std::string shape_key(const mm_ctx &c, const int *ids, size_t count)
{
    uint64_t sum_r = 0;
    for (size_t i = 0; i < count; i++) sum_r += c.tables[ids[i]].r;
    return std::to_string(c.p.N) + "/" + std::to_string(count) + "/" + std::to_string(sum_r) + "/" +
           std::to_string(max_r(c, ids, count));
}

// The global-accumulator path (accumulators in device memory, one launch per
// CMux step): the wide modulus, rings above 8192, and tables whose components
// do not fit one workgroup (r N / 1024 > 8).
static bool use_global(const mm_ctx &c, const int *ids, size_t count)
{
    return c.wide || !dev::device_supports_n(c.p.N) || max_r(c, ids, count) * (uint32_t)dev::waves_per_poly(c.p.N) > 8;
}

int primes_of(const mm_ctx &c) { return c.wide ? 2 : 1; }

// Blind-rotation shapes of the global path: one workgroup per component and
// CMux step (NTT schedule 0; rings up to 16384), or the ring split into
// sub-rings of 8192 (schedule 3; one prime, rings of 16384 and more); with two
// primes also one workgroup per component and prime (5), of two digit groups
// (6, N = 1024 and 2048).
static std::vector<int> global_shapes(const mm_ctx &c)
{
    if (c.wide) {
        std::vector<int> v{0};
        if (dev::wide_supports_ps(c.p.N, 2)) v.push_back(5);
        if (dev::wide_supports_ps(c.p.N, 2, 2)) v.push_back(6);
        return v;
    }
    if (!dev::split_supports_n(c.p.N)) return {0};
    if (c.p.N > 16384) return {3};
    return {0, 3};
}

// The global-accumulator shape as a schedule of batches the fused kernel holds
// (one prime, rings up to 8192).
static bool global_ok(const mm_ctx &c) { return !c.wide && dev::device_supports_n(c.p.N); }

// Waves per component of that shape for batches that leave the device mostly idle:
// twice the usual where the kernel exists (N = 512, 1024), else the usual.
int light_global_wpp(const mm_ctx &c)
{
    const int w2 = 2 * dev::wide_waves_per_poly(c.p.N);
    return dev::wide_supports_wpp(c.p.N, 1, w2) ? w2 : 0;
}

// One workgroup per component and prime (two primes) for batches of up to 16
// components per compute unit.  Measured at the paper-margin parameters (N = 2048,
// ternary, ms per bootstrap call, both shapes): one ciphertext 19.2 against 38.6,
// 256 components 30.2 against 41.5, 1024 87.7 against 94.8, 4096 332.1 against
// 335.3; 8192 669.2 against 663.2 (the shared digit fields computed twice).
bool prime_split(const mm_ctx &c, const Device &d, uint64_t comps)
{
    return c.wide && dev::wide_supports_ps(c.p.N, 2) && comps <= 16ull * (uint64_t)d.num_cu;
}

// Digit groups of those workgroups: two (N = 1024, 2048) while both primes' workgroups
// of every component fit one per compute unit (one ciphertext at N = 2048, t = 2^12:
// 18.7 against 19.9 ms; 256 components 34.6 against 29.0 ms), else one.
int prime_split_dg(const mm_ctx &c, const Device &d, uint64_t comps)
{
    return prime_split(c, d, comps) && dev::wide_supports_ps(c.p.N, 2, 2) && 2 * comps <= (uint64_t)d.num_cu ? 2
                                                                                                            : 1;
}

// Digit groups per component of light global-path work: two (each group of
// light_global_wpp waves taking every other digit) for batches of at most two
// components per compute unit where that kernel exists, else one.
int light_global_dg(const mm_ctx &c, const Device &d, uint64_t comps)
{
    const int w2 = light_global_wpp(c);
    return w2 && dev::wide_supports_dg(c.p.N, primes_of(c), w2) && comps <= 2ull * (uint64_t)d.num_cu ? 2 : 1;
}

// Two waves per component (N = 512, 1024, r <= 4): for batches that do not
// fill every compute unit, both waves of a slot share one component's work.
static bool wide_slots_ok(const mm_ctx &c, const int *ids, size_t count)
{
    return dev::br_supports_wpp(c.p.N, 2) && dev::waves_per_poly(c.p.N) == 1 && max_r(c, ids, count) <= 4;
}

static uint64_t sum_r(const mm_ctx &c, const int *ids, size_t count)
{
    uint64_t s = 0;
    for (size_t i = 0; i < count; i++) s += c.tables[ids[i]].r;
    return s;
}

// Candidate schedules for a batch: blind-rotation shape (8-wave groups, 4-wave
// groups, 8-wave groups of 2-wave slots) x key-switch tiling.
static std::vector<Sched> candidates(const mm_ctx &c, const Device &d, const int *ids, size_t count)
{
    std::vector<Sched> out;
    const bool narrow_ok = max_r(c, ids, count) * (uint32_t)dev::waves_per_poly(c.p.N) <= 4;
    std::vector<KsSched> ks{ks_default(c, d, count)};
    const uint32_t rows = c.p.l_ks << c.p.log2_Bks;
    auto add = [&](KsSched k) {
        for (auto &o : ks)
            if (o.cpw == k.cpw && o.P == k.P) return;
        ks.push_back(k);
    };
    if (rows <= (uint32_t)dev::KS_TILED_MAX_ROWS && count >= 64)
        for (int cpw : {16, 32, 64})
            for (uint32_t P : {1u, 2u, 4u}) add(KsSched{cpw, P});
    if (rows <= (uint32_t)dev::KS_TILED_MAX_ROWS && count >= 256)
        for (uint32_t P : {2u, 3u, 4u, 6u}) add(KsSched{KS_LANES, P});
    if (count < 256) ks.push_back(KsSched{0, ks_splits(c, d, count)});
    if (use_global(c, ids, count)) {
        for (int shape : global_shapes(c))
            for (auto &k : ks) out.push_back(Sched{0, k, shape == 3 ? dev::SPLIT_WAVES : 0, shape});
        return out;
    }
    for (int gw : {8, 4}) {
        if (gw == 4 && !narrow_ok) continue;
        for (auto &k : ks) out.push_back(Sched{gw, k});
    }
    if (wide_slots_ok(c, ids, count))
        for (auto &k : ks) out.push_back(Sched{8, k, 2});
    if (dev::br_supports_lane_swap(c.p.N))
        for (int gw : {8, 4}) {
            if (gw == 4 && !narrow_ok) continue;
            for (auto &k : ks) out.push_back(Sched{gw, k, 0, 1});
        }
    if (dev::waves_per_poly(c.p.N) == 1)
        for (int gw : {8, 4}) {
            if (gw == 4 && !narrow_ok) continue;
            for (auto &k : ks) out.push_back(Sched{gw, k, 0, 2});
        }
    // the global-accumulator shape (one workgroup per component and CMux step, each
    // on its own compute unit): for small batches the components of one ciphertext
    // then run side by side instead of sharing one compute unit
    if (global_ok(c)) {
        for (auto &k : ks) out.push_back(Sched{0, k});
        if (const int w2 = light_global_wpp(c)) {
            for (auto &k : ks) out.push_back(Sched{0, k, w2});
            // two digit groups per component (schedule 4): half a step's dependent
            // chain per compute unit, for batches with compute units to spare
            if (dev::wide_supports_dg(c.p.N, 1, w2))
                for (auto &k : ks) out.push_back(Sched{0, k, w2, 4});
        }
    }
    return out;
}

static Sched schedule_for(const mm_ctx &c, const Device &d, const int *ids, size_t count)
{
    auto it = d.tuned.find(shape_key(c, ids, count));
    if (it != d.tuned.end()) {
        auto cand = candidates(c, d, ids, count);
        if (it->second >= 0 && (size_t)it->second < cand.size()) return cand[it->second];
    }
    if (use_global(c, ids, count)) {
        const uint64_t comps = sum_r(c, ids, count);
        if (prime_split(c, d, comps))
            return Sched{0, ks_default(c, d, count), 0, prime_split_dg(c, d, comps) == 2 ? 6 : 5};
        const int shape = global_shapes(c).front();
        return Sched{0, ks_default(c, d, count), shape == 3 ? dev::SPLIT_WAVES : 0, shape};
    }
    // untuned, at N = 1024 (the ring of the paper-shaped parameters, measured for
    // r = 4 and 8 at 1024 to 16384 components; at N = 512 the fused kernel measured
    // faster up to 8192 components): the global-accumulator shape with four
    // waves per component (one component per workgroup: small workgroups, up to eight
    // waves per SIMD) where it measured fastest -- batches that leave the device mostly
    // idle (at most two components per compute unit, or four where the components
    // cannot take two-wave slots: one ciphertext 7.4 ms instead of 14.2 ms, or 25.9 ms
    // at r = 8) and batches of more than 16 components per compute unit (188.8 against
    // 203.8 ms for 16,384); in between the fused kernel (two-wave slots up to four
    // components per compute unit, 14.6 against 16.5 ms at 1024; one wave per component
    // up to 16 per compute unit, 25.6 against 27.4 ms at 2048).  Up to two components
    // per compute unit, two digit groups per component (6.5 against 7.4 ms for one
    // ciphertext, 12.2 against 12.7 ms for 512 components; 20.3 against 18.2 ms at 1024)
    const uint64_t comps = sum_r(c, ids, count), cu = (uint64_t)d.num_cu;
    const bool two_wave = wide_slots_ok(c, ids, count);
    if (global_ok(c) && c.p.N == 1024 && light_global_wpp(c) &&
        (comps <= 2 * cu || (!two_wave && comps <= 4 * cu) || comps > 16 * cu))
        return Sched{0, ks_default(c, d, count), light_global_wpp(c), light_global_dg(c, d, comps) == 2 ? 4 : 0};
    return Sched{8, ks_default(c, d, count), comps <= 4 * cu && two_wave ? 2 : 0};
}

static int br_grid(const Device &d, int groups, int gw) { return std::min(groups, d.num_cu * (gw == 4 ? 2 : 1)); }

// Output modulus per ciphertext: q_out, or each table's q_in when q_out = 0
// (a scalar when they agree, else a device vector written on st).
static const uint32_t *resolve_q_out(const mm_ctx &c, Device &d, const int *ids, size_t count, uint32_t &q_out,
                                     hipStream_t st)
{
    if (q_out != 0) return nullptr;
    bool same = true;
    for (size_t i = 1; i < count; i++) same &= c.tables[ids[i]].q_in == c.tables[ids[0]].q_in;
    if (same) {
        q_out = c.tables[ids[0]].q_in;
        return nullptr;
    }
    uint32_t *h = (uint32_t *)pinned(d, 1, count * 4);
    for (size_t i = 0; i < count; i++) h[i] = c.tables[ids[i]].q_in;
    uint32_t *dq = (uint32_t *)ws(d, WS_QOUT, count * 4);
    HIPC(hipMemcpyAsync(dq, h, count * 4, hipMemcpyHostToDevice, st));
    HIPC(hipEventRecord(d.pin[1].ev, st));
    return dq;
}

// The instantiated graph of a launch sequence, captured on first use of its key.
static hipGraphExec_t graph_for(Device &d, const std::string &k, const std::function<void(hipStream_t)> &body)
{
    for (auto &g : d.graphs)
        if (g.key == k) return g.exec;
    hipGraph_t graph;
    hipGraphExec_t exec = nullptr;
    HIPC(hipStreamBeginCapture(d.own, hipStreamCaptureModeThreadLocal));
    body(d.own);
    HIPC(hipStreamEndCapture(d.own, &graph));
    HIPC(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
    HIPC(hipGraphDestroy(graph));
    if (d.graphs.size() >= 12) {
        hipGraphExecDestroy(d.graphs.front().exec);
        d.graphs.erase(d.graphs.begin());
    }
    d.graphs.push_back({k, exec});
    return exec;
}

// Run a blind-rotation part and a key-switch part on st: eager, one graph, or
// (with timing on) two graphs with HIP events around each.
static void run_sequence(Device &d, const std::string &key, bool use_graph, hipStream_t st,
                         const std::function<void(hipStream_t)> &br, const std::function<void(hipStream_t)> &ks)
{
    const bool timed = d.timing;
    if (!use_graph) {
        if (timed) HIPC(hipEventRecord(d.tev[0], st));
        br(st);
        if (timed) HIPC(hipEventRecord(d.tev[1], st));
        ks(st);
        if (timed) HIPC(hipEventRecord(d.tev[2], st));
        HIPC(hipGetLastError());
        return;
    }
    if (!timed) {
        hipGraphExec_t g = graph_for(d, key + "/all", [&](hipStream_t s) {
            br(s);
            ks(s);
        });
        HIPC(hipGraphLaunch(g, st));
    } else {
        hipGraphExec_t g1 = graph_for(d, key + "/br", br);
        hipGraphExec_t g2 = graph_for(d, key + "/ks", ks);
        HIPC(hipEventRecord(d.tev[0], st));
        HIPC(hipGraphLaunch(g1, st));
        HIPC(hipEventRecord(d.tev[1], st));
        HIPC(hipGraphLaunch(g2, st));
        HIPC(hipEventRecord(d.tev[2], st));
    }
}

static void bootstrap_wide(mm_ctx &c, Device &d, const int *ids, const uint32_t *d_in, size_t count,
                           uint32_t *d_out, uint32_t q_out, bool use_graph, hipStream_t st, const Sched &S);

// The batched path for ciphertexts already on the device.
static void bootstrap_batch(mm_ctx &c, Device &d, const int *ids, const uint32_t *d_in, size_t count, uint32_t *d_out,
                            uint32_t q_out, bool use_graph, hipStream_t st, const Sched *force = nullptr)
{
    const Sched S = force ? *force : schedule_for(c, d, ids, count);
    if (use_global(c, ids, count) || S.gw == 0) {
        bootstrap_wide(c, d, ids, d_in, count, d_out, q_out, use_graph, st, S);
        return;
    }
    const uint32_t N = c.p.N;
    auto tasks = pack_groups(c, d, ids, count, dev::TASK_INIT | dev::TASK_EXTRACT, 0, {}, (uint32_t)S.gw,
                             (uint32_t)S.wpp);
    const int groups = (int)(tasks.size() / S.gw);
    uint32_t q_scalar = q_out;
    const uint32_t *qv = resolve_q_out(c, d, ids, count, q_scalar, st);
    // allocate every buffer before a capture
    uint32_t *ext = (uint32_t *)ws(d, WS_EXT, count * (N + 1) * 4);
    uint64_t *part = (uint64_t *)ws(d, WS_PART, ks_part_words(c, S.ks, count) * 8);
    dev::WaveTask *dt = upload_tasks(d, tasks, st);

    dev::BrArgs A = br_args(c, d);
    A.tasks = dt;
    A.num_groups = groups;
    A.steps = (int)c.p.n;
    A.ct_in = d_in;
    A.ext_out = ext;
    A.acc_state = nullptr;
    const int grid = br_grid(d, groups, S.gw);

    const std::string key = std::to_string(count) + "/" + std::to_string(groups) + "/" + std::to_string(S.gw) + "/" +
                            std::to_string(S.wpp) + "/" + std::to_string(S.ntt) + "/" + std::to_string(S.ks.cpw) +
                            "/" + std::to_string(S.ks.P) +
                            "/" + std::to_string(q_scalar) +
                            "/" + std::to_string((uintptr_t)qv) + "/" + std::to_string((uintptr_t)d_in) + "/" +
                            std::to_string((uintptr_t)d_out) + "/" + std::to_string(d.ws_generation);
    run_sequence(
        d, key, use_graph, st, [&](hipStream_t s) { dev::launch_blind_rotate(N, A, S.gw, grid, s, S.wpp, S.ntt); },
        [&](hipStream_t s) { enqueue_keyswitch(c, d, ext, nullptr, count, d_out, qv, q_scalar, S.ks, part, s); });
}

// ------------------------------------------------------------------ wide ring modulus

dev::WideArgs wide_args(const mm_ctx &c, const Device &d)
{
    const mm_params &p = c.p;
    dev::WideArgs A{};
    A.ct_stride = p.n + 1;
    A.n = p.n;
    A.Q[0] = p.Q;
    A.qn[0] = d.qn;
    A.log2B = p.log2_B;
    A.l = p.l;
    A.sg = c.sg;
    if (c.wide) {
        A.Q[1] = p.Q2;
        A.qn[1] = d.qn2;
        A.crt_cq = (p.Q + p.Q2 - 1) / p.Q2 * p.Q2;
        A.crt_inv = to_mont(powmod(p.Q % p.Q2, p.Q2 - 2, p.Q2), p.Q2);
        A.Qw = c.Qw;
    } else {
        A.Qw = p.Q;  // one prime: the 31-bit ring modulus itself
    }
    A.goff = 0;
    for (uint32_t u = 0; u < p.l; u++) A.goff += (uint64_t)(1u << (p.log2_B - 1)) << (u * p.log2_B);
    A.bsk = d.bsk;
    A.bsk_corr = d.bsk_corr;
    A.twf0 = d.twf;
    A.twi0 = d.twi;
    A.twf1 = d.twf2;
    A.twi1 = d.twi2;
    A.tv = d.tv;
    return A;
}

// One task per (ciphertext, component); accumulators of 2N words per component
// and prime laid out ciphertext after ciphertext.  Returns the total words.
static uint64_t wide_tasks(const mm_ctx &c, const int *ids, size_t count, std::vector<dev::WideTask> &tasks,
                           std::vector<uint64_t> &offs)
{
    const uint64_t N = c.p.N;
    uint64_t words = 0;
    tasks.clear();
    offs.resize(count);
    for (size_t i = 0; i < count; i++) {
        const Table &tb = c.tables[ids[i]];
        offs[i] = words;
        for (uint32_t j = 0; j < tb.r; j++)
            tasks.push_back({(int32_t)i, j, tb.r, tb.q_in, (uint32_t)tb.dev_offset, 0, words});
        words += (uint64_t)tb.r * 2 * primes_of(c) * N;
    }
    return words;
}

// Upload the task list and the per-ciphertext offsets through pinned staging.
static void upload_wide(Device &d, const std::vector<dev::WideTask> &tasks, const std::vector<uint64_t> &offs,
                        dev::WideTask **dt, uint64_t **doff, hipStream_t st)
{
    const size_t tb = tasks.size() * sizeof(dev::WideTask), ob = offs.size() * 8;
    char *h = (char *)pinned(d, 0, tb + ob);
    std::memcpy(h, tasks.data(), tb);
    std::memcpy(h + tb, offs.data(), ob);
    *dt = (dev::WideTask *)ws(d, WS_TASKS, tb);
    *doff = (uint64_t *)ws(d, WS_WOFF, std::max<size_t>(ob, 8));
    HIPC(hipMemcpyAsync(*dt, h, tb, hipMemcpyHostToDevice, st));
    if (ob) HIPC(hipMemcpyAsync(*doff, h + tb, ob, hipMemcpyHostToDevice, st));
    HIPC(hipEventRecord(d.pin[0].ev, st));
}

// The split-ring buffers (digit polynomials, sub-ring products) of num_tasks
// components, from the workspace, into A; before any capture.
static void split_buffers(const mm_ctx &c, Device &d, dev::WideArgs &A, size_t num_tasks)
{
    const size_t N = c.p.N;
    A.M = (uint32_t)(N / dev::SPLIT_NS);
    A.dig = (uint32_t *)ws(d, WS_DIG, num_tasks * c.keys * c.p.l * 2 * N * 4);
    A.outb = (uint32_t *)ws(d, WS_OUTB, num_tasks * 2 * N * 4);
    A.twf_sub = d.twf_sub;
    A.twi_sub = d.twi_sub;
}

// ACC init and `steps` CMux launches (three per step for a split ring, A.M > 0);
// returns the buffer holding the result.
static uint32_t *enqueue_wide_rotation(const mm_ctx &c, dev::WideArgs A, uint32_t *buf0, uint32_t *buf1,
                                       uint32_t num_tasks, uint32_t steps, hipStream_t s, int wpp = 0, int dg = 1,
                                       bool ps = false)
{
    const uint32_t N = c.p.N;
    uint32_t *buf[2] = {buf0, buf1};
    A.acc_wr = buf[0];
    dev::launch_wide_init(N, primes_of(c), A, num_tasks, s);
    for (uint32_t i = 0; i < steps; i++) {
        A.step = i;
        A.acc_rd = buf[i & 1];
        A.acc_wr = buf[(i + 1) & 1];
        if (A.M) dev::launch_split_step(N, c.keys, A, num_tasks, s);
        else dev::launch_wide_step(N, primes_of(c), c.keys, A, num_tasks, s, wpp, dg, ps);
    }
    return buf[steps & 1];
}

static void bootstrap_wide(mm_ctx &c, Device &d, const int *ids, const uint32_t *d_in, size_t count,
                           uint32_t *d_out, uint32_t q_out, bool use_graph, hipStream_t st, const Sched &S)
{
    const uint32_t N = c.p.N;
    const KsSched &ks = S.ks;
    std::vector<dev::WideTask> tasks;
    std::vector<uint64_t> offs;
    const uint64_t words = wide_tasks(c, ids, count, tasks, offs);
    uint32_t q_scalar = q_out;
    const uint32_t *qv = resolve_q_out(c, d, ids, count, q_scalar, st);
    uint32_t *ext = (uint32_t *)ws(d, WS_EXT, count * (N + 1) * 4);
    uint64_t *part = (uint64_t *)ws(d, WS_PART, ks_part_words(c, ks, count) * 8);
    uint32_t *acc0 = (uint32_t *)ws(d, WS_ACC, words * 4);
    uint32_t *acc1 = (uint32_t *)ws(d, WS_ACC2, words * 4);
    dev::WideArgs A = wide_args(c, d);
    if (S.ntt == 3) split_buffers(c, d, A, tasks.size());
    dev::WideTask *dt;
    uint64_t *doff;
    upload_wide(d, tasks, offs, &dt, &doff, st);
    A.tasks = dt;
    A.ct_in = d_in;
    const uint32_t nt = (uint32_t)tasks.size();
    const std::string key = "wide/" + std::to_string(S.ntt) + "/" + std::to_string(S.wpp) + "/" + std::to_string(count) + "/" + std::to_string(nt) + "/" +
                            std::to_string(ks.cpw) + "/" + std::to_string(ks.P) + "/" + std::to_string(q_scalar) +
                            "/" + std::to_string((uintptr_t)qv) + "/" + std::to_string((uintptr_t)d_in) + "/" +
                            std::to_string((uintptr_t)d_out) + "/" + std::to_string(d.ws_generation);
    run_sequence(
        d, key, use_graph, st,
        [&](hipStream_t s) {
            dev::WideArgs B = A;
            B.acc_rd = enqueue_wide_rotation(c, A, acc0, acc1, nt, c.p.n, s, S.ntt == 3 ? 0 : S.wpp,
                                             S.ntt == 4 || S.ntt == 6 ? 2 : 1, S.ntt == 5 || S.ntt == 6);
            dev::launch_wide_extract(N, primes_of(c), B, doff, count, ext, s);
        },
        [&](hipStream_t s) { enqueue_keyswitch(c, d, ext, nullptr, count, d_out, qv, q_scalar, ks, part, s); });
}

static void blind_rotate_wide(mm_ctx &c, Device &d, const int *ids, const uint32_t *d_in, size_t count,
                              uint32_t steps, uint32_t *d_acc, hipStream_t st)
{
    std::vector<dev::WideTask> tasks;
    std::vector<uint64_t> offs;
    const uint64_t words = wide_tasks(c, ids, count, tasks, offs);
    uint32_t *acc0 = (uint32_t *)ws(d, WS_ACC, words * 4);
    uint32_t *acc1 = (uint32_t *)ws(d, WS_ACC2, words * 4);
    dev::WideArgs A = wide_args(c, d);
    if (schedule_for(c, d, ids, count).ntt == 3) split_buffers(c, d, A, tasks.size());
    dev::WideTask *dt;
    uint64_t *doff;
    upload_wide(d, tasks, offs, &dt, &doff, st);
    A.tasks = dt;
    A.ct_in = d_in;
    const uint32_t nt = (uint32_t)tasks.size();
    A.acc_rd = enqueue_wide_rotation(c, A, acc0, acc1, nt, steps, st);
    if (c.wide) dev::launch_wide_export(c.p.N, A, nt, d_acc, st);
    else HIPC(hipMemcpyAsync(d_acc, A.acc_rd, words * 4, hipMemcpyDeviceToDevice, st));  // already [comp][part][N]
    HIPC(hipGetLastError());
}

void run_bootstrap(mm_ctx &c, const int *ids, const uint32_t *ct_in, size_t count, uint32_t *ct_out, uint32_t q_out,
                   uint32_t flags, void *stream)
{
    const size_t general = check_ids(c, ids, count);
    MM_REQUIRE(general == 0 || general == count, "a call takes only general tables or none of them");
    MM_REQUIRE(q_out == 0 || q_out == c.p.Q || (q_out >= 2 && q_out < c.p.Q), "q_out must be 0, Q or in [2, Q)");
    if (count == 0) return;
    Device &d = ensure_device(c);
    hipStream_t st = (hipStream_t)stream;
    const bool dptr = flags & MM_DEVICE_PTRS;
    const size_t W = c.p.n + 1;
    const uint32_t *d_in = stage_in(d, WS_IN, ct_in, count * W, dptr, st);
    uint32_t *d_out = stage_out(d, WS_OUT, ct_out, count * W, dptr);
    auto pass = [&](const int *pid, const uint32_t *in, uint32_t *out, uint32_t qo) {
        if (flags & MM_PLAIN) {
            for (size_t i = 0; i < count; i++) bootstrap_batch(c, d, pid + i, in + i * W, 1, out + i * W, qo, false, st);
        } else {
            bootstrap_batch(c, d, pid, in, count, out, qo, true, st);
        }
    };
    if (general == 0) {
        pass(ids, d_in, d_out, q_out);
    } else {
        // general f: sign bootstrap, top-bit removal, then the extended f
        std::vector<int> g_ids(count), f_ids(count);
        uint32_t *hq = (uint32_t *)pinned(d, 1, count * 8);
        for (size_t i = 0; i < count; i++) {
            const Table &tb = c.tables[ids[i]];
            g_ids[i] = tb.g_id;
            f_ids[i] = tb.F_id;
            hq[2 * i] = tb.q_in;
            hq[2 * i + 1] = (uint32_t)((uint64_t)(tb.t / 2) * (tb.q_in / (2 * tb.t)) % tb.q_in);
        }
        uint32_t *dq = (uint32_t *)ws(d, WS_GENQ, count * 8);
        uint32_t *tmp = (uint32_t *)ws(d, WS_GEN1, count * W * 4);
        uint32_t *comb = (uint32_t *)ws(d, WS_GEN2, count * W * 4);
        HIPC(hipMemcpyAsync(dq, hq, count * 8, hipMemcpyHostToDevice, st));
        HIPC(hipEventRecord(d.pin[1].ev, st));
        pass(g_ids.data(), d_in, tmp, 0);
        dev::launch_lwe_combine(d_in, tmp, comb, count, (uint32_t)W, dq, st);
        pass(f_ids.data(), comb, d_out, q_out);
    }
    HIPC(hipGetLastError());
    finish_out(ct_out, d_out, count * W, dptr, st);
}

void run_blind_rotate(mm_ctx &c, const int *ids, const uint32_t *ct_in, size_t count, uint32_t steps,
                      uint32_t *acc_out, uint32_t flags, void *stream)
{
    MM_REQUIRE(check_ids(c, ids, count) == 0, "blind rotation takes nega-cyclic tables");
    MM_REQUIRE(steps <= c.p.n, "steps must be <= n");
    if (count == 0) return;
    Device &d = ensure_device(c);
    hipStream_t st = (hipStream_t)stream;
    const bool dptr = flags & MM_DEVICE_PTRS;
    const uint32_t N = c.p.N;
    std::vector<uint64_t> off(count);
    uint64_t words = 0;
    for (size_t i = 0; i < count; i++) {
        off[i] = words;
        words += (uint64_t)c.tables[ids[i]].r * 2 * N;
    }
    const uint32_t *d_in = stage_in(d, WS_IN, ct_in, count * (c.p.n + 1), dptr, st);
    if (use_global(c, ids, count)) {  // with the wide modulus uint64 entries: two words each
        const uint64_t out_words = c.wide ? 2 * words : words;
        uint32_t *d_out = stage_out(d, WS_OUT, acc_out, out_words, dptr);
        blind_rotate_wide(c, d, ids, d_in, count, steps, d_out, st);
        finish_out(acc_out, d_out, out_words, dptr, st);
        return;
    }
    uint32_t *d_acc = stage_out(d, WS_ACC, acc_out, words, dptr);
    auto tasks = pack_groups(c, d, ids, count, dev::TASK_INIT | dev::TASK_STORE, 0, off);
    dev::WaveTask *dt = upload_tasks(d, tasks, st);
    dev::BrArgs A = br_args(c, d);
    A.tasks = dt;
    A.num_groups = (int)(tasks.size() / 8);
    A.steps = (int)steps;
    A.ct_in = d_in;
    A.acc_state = d_acc;
    dev::launch_blind_rotate(N, A, 8, std::min(A.num_groups, d.num_cu), st);
    HIPC(hipGetLastError());
    finish_out(acc_out, d_acc, words, dptr, st);
}

void run_external_product(mm_ctx &c, uint32_t i, const uint32_t *in, size_t count, uint32_t *out, uint32_t flags,
                          void *stream)
{
    MM_REQUIRE(!c.wide, "mm_external_product is not available with a wide ring modulus");
    MM_REQUIRE(dev::device_supports_n(c.p.N), "mm_external_product supports N up to 8192");
    MM_REQUIRE(i < c.p.n * c.keys, "key index must be < K n");
    if (count == 0) return;
    Device &d = ensure_device(c);
    hipStream_t st = (hipStream_t)stream;
    const bool dptr = flags & MM_DEVICE_PTRS;
    const size_t words = count * 2 * c.p.N;
    const uint32_t *din = stage_in(d, WS_IN, in, words, dptr, st);
    uint32_t *dout = stage_out(d, WS_OUT, out, words, dptr);
    dev::launch_external_product(c.p.N, din, dout, count, d.bsk + (size_t)i * 4 * c.p.l * c.p.N, d.twf, d.twi, c.p.Q,
                                 d.qn, c.p.log2_B, c.p.l, c.sg, st);
    HIPC(hipGetLastError());
    finish_out(out, dout, words, dptr, st);
}

void run_negacyclic_mul(mm_ctx &c, const uint32_t *a, const uint32_t *b, size_t count, uint32_t *out, uint32_t flags,
                        void *stream)
{
    MM_REQUIRE(dev::device_supports_n(c.p.N), "mm_negacyclic_mul supports N up to 8192");
    if (count == 0) return;
    Device &d = ensure_device(c);
    hipStream_t st = (hipStream_t)stream;
    const bool dptr = flags & MM_DEVICE_PTRS;
    const size_t words = count * c.p.N;
    const uint32_t *da = stage_in(d, WS_IN, a, words, dptr, st);
    const uint32_t *db = stage_in(d, WS_IN2, b, words, dptr, st);
    uint32_t *dout = stage_out(d, WS_OUT, out, words, dptr);
    dev::launch_negacyclic_mul(c.p.N, da, db, dout, count, d.twf, d.twi, c.p.Q, d.qn, d.c_fix, st);
    HIPC(hipGetLastError());
    finish_out(out, dout, words, dptr, st);
}

void run_modswitch(mm_ctx &c, const uint32_t *in, size_t count, uint32_t q_from, uint32_t q_to, uint32_t *out,
                   uint32_t flags, void *stream)
{
    MM_REQUIRE(q_from >= 2 && q_to >= 2 && q_from <= (1u << 31) && q_to <= (1u << 31), "moduli out of range");
    if (count == 0) return;
    Device &d = ensure_device(c);
    hipStream_t st = (hipStream_t)stream;
    const bool dptr = flags & MM_DEVICE_PTRS;
    const uint32_t *din = stage_in(d, WS_IN, in, count, dptr, st);
    uint32_t *dout = stage_out(d, WS_OUT, out, count, dptr);
    dev::launch_modswitch(din, dout, count, q_from, q_to, st);
    HIPC(hipGetLastError());
    finish_out(out, dout, count, dptr, st);
}

void run_sample_extract(mm_ctx &c, const uint32_t *rlwe, size_t count, uint32_t *lwe, uint32_t flags, void *stream)
{
    if (count == 0) return;
    Device &d = ensure_device(c);
    hipStream_t st = (hipStream_t)stream;
    const bool dptr = flags & MM_DEVICE_PTRS;
    const uint32_t N = c.p.N;
    const uint32_t *din = stage_in(d, WS_IN, rlwe, count * 2 * N, dptr, st);
    uint32_t *dout = stage_out(d, WS_OUT, lwe, count * (N + 1), dptr);
    dev::launch_sample_extract(din, dout, count, N, c.p.Q, st);
    HIPC(hipGetLastError());
    finish_out(lwe, dout, count * (N + 1), dptr, st);
}

void run_keyswitch(mm_ctx &c, const uint32_t *lwe_N, size_t count, uint32_t *lwe_n, uint32_t flags, void *stream)
{
    if (count == 0) return;
    Device &d = ensure_device(c);
    hipStream_t st = (hipStream_t)stream;
    const bool dptr = flags & MM_DEVICE_PTRS;
    const uint32_t N = c.p.N, W = c.p.n + 1;
    const uint32_t *din = stage_in(d, WS_IN, lwe_N, count * (N + 1), dptr, st);
    uint32_t *dout = stage_out(d, WS_OUT, lwe_n, count * W, dptr);
    const KsSched ks = ks_default(c, d, count);
    uint64_t *part = (uint64_t *)ws(d, WS_PART, ks_part_words(c, ks, count) * 8);
    enqueue_keyswitch(c, d, din, nullptr, count, dout, nullptr, c.p.Q, ks, part, st);
    HIPC(hipGetLastError());
    finish_out(lwe_n, dout, count * W, dptr, st);
}

// The key switch with its partial sums in the device's fixed scratch array: no
// allocation, no staging, no schedule lookup that could upload anything.
void run_keyswitch_noalloc(mm_ctx &c, const uint32_t *lwe_N, size_t count, uint32_t *lwe_n, void *stream)
{
    if (!c.dev) throw Error(MM_ESTATE, "mm_keyswitch_noalloc needs mm_device_init first (it allocates nothing)");
    const size_t W = c.p.n + 1, per_split = count * W * sizeof(uint64_t);
    MM_REQUIRE(per_split <= dev::NOALLOC_SCRATCH_BYTES,
               "mm_keyswitch_noalloc: count * (n + 1) * 8 bytes exceeds its 64 MiB scratch");
    if (count == 0) return;
    Device &d = *c.dev;
    HIPC(hipSetDevice(d.id));
    MM_REQUIRE(d.scratch != nullptr, "no device scratch");
    KsSched ks = ks_default(c, d, count);
    ks.P = (uint32_t)std::max<size_t>(1, std::min<size_t>(ks.P, dev::NOALLOC_SCRATCH_BYTES / per_split));
    enqueue_keyswitch(c, d, lwe_N, nullptr, count, lwe_n, nullptr, c.p.Q, ks, (uint64_t *)d.scratch,
                      (hipStream_t)stream);
    HIPC(hipGetLastError());
}

void set_timing(mm_ctx &c, bool on)
{
    Device &d = ensure_device(c);
    if (on && !d.tev[0])
        for (auto &e : d.tev) HIPC(hipEventCreate(&e));
    d.timing = on;
}

void last_timing(mm_ctx &c, float *br_ms, float *ks_ms)
{
    Device &d = ensure_device(c);
    if (!d.timing || !d.tev[0]) throw Error(MM_ESTATE, "timing is not enabled");
    HIPC(hipEventSynchronize(d.tev[2]));
    float a = 0, b = 0;
    HIPC(hipEventElapsedTime(&a, d.tev[0], d.tev[1]));
    HIPC(hipEventElapsedTime(&b, d.tev[1], d.tev[2]));
    if (br_ms) *br_ms = a;
    if (ks_ms) *ks_ms = b;
}

int schedule_count(mm_ctx &c, const int *ids, size_t count)
{
    MM_REQUIRE(check_ids(c, ids, count) == 0, "schedules are per nega-cyclic table batch");
    MM_REQUIRE(count > 0, "empty batch");
    Device &d = ensure_device(c);
    return (int)candidates(c, d, ids, count).size();
}

void set_schedule(mm_ctx &c, const int *ids, size_t count, int choice)
{
    const int n = schedule_count(c, ids, count);
    MM_REQUIRE(choice >= 0 && choice < n, "schedule index out of range");
    c.dev->tuned[shape_key(c, ids, count)] = choice;
}

void describe_schedule(mm_ctx &c, const int *ids, size_t count, int choice, int *gw, int *cpw, int *P, int *wpp,
                       int *ks_kernel, int *ntt)
{
    const int n = schedule_count(c, ids, count);
    MM_REQUIRE(choice < n, "schedule index out of range");
    Device &d = *c.dev;
    const Sched S = choice >= 0 ? candidates(c, d, ids, count)[choice] : schedule_for(c, d, ids, count);
    if (gw) *gw = S.gw;
    if (cpw) *cpw = S.ks.cpw == KS_LANES ? 64 : S.ks.cpw;
    if (ks_kernel) *ks_kernel = S.ks.cpw == KS_LANES ? 2 : (S.ks.cpw > 0 ? 1 : 0);
    if (ntt) *ntt = S.ntt;
    if (P) *P = (int)S.ks.P;
    if (wpp) *wpp = S.wpp ? S.wpp : (S.gw == 0 ? dev::wide_waves_per_poly(c.p.N) : dev::waves_per_poly(c.p.N));
}

// The global-accumulator path: time each blind-rotation shape (at N = 16384 one
// workgroup per component, or the ring split into sub-rings) with the default key
// switch, one untimed run first; then each key-switch candidate on the samples the
// last run extracted.
static int autotune_global(mm_ctx &c, Device &d, const int *ids, const uint32_t *d_in, uint32_t *d_out,
                           size_t count)
{
    hipStream_t st = d.own;
    auto cand = candidates(c, d, ids, count);
    hipEvent_t ev[2];
    HIPC(hipEventCreate(&ev[0]));
    HIPC(hipEventCreate(&ev[1]));
    int best_shape = cand[0].ntt;
    size_t best_k = 0;
    try {
        const std::vector<int> shapes = global_shapes(c);
        float best = 1e30f;
        for (int shape : shapes) {
            size_t k0 = 0;
            while (cand[k0].ntt != shape) k0++;  // the shape's first candidate: the default key switch
            bootstrap_batch(c, d, ids, d_in, count, d_out, 0, false, st, &cand[k0]);
            if (shapes.size() == 1) break;
            HIPC(hipEventRecord(ev[0], st));
            bootstrap_batch(c, d, ids, d_in, count, d_out, 0, false, st, &cand[k0]);
            HIPC(hipEventRecord(ev[1], st));
            HIPC(hipEventSynchronize(ev[1]));
            float ms = 0;
            HIPC(hipEventElapsedTime(&ms, ev[0], ev[1]));
            if (ms < best) {
                best = ms;
                best_shape = shape;
            }
        }
        // the extracted samples of the last run stay in the workspace (a later
        // request for the same slot and size returns the same buffer)
        const uint32_t *ext = (const uint32_t *)ws(d, WS_EXT, count * (c.p.N + 1) * 4);
        size_t part_words = 0;
        for (auto &S : cand) part_words = std::max(part_words, ks_part_words(c, S.ks, count));
        uint64_t *part = (uint64_t *)ws(d, WS_PART, part_words * 8);
        HIPC(hipStreamSynchronize(st));
        float best_ks = 1e30f;
        for (size_t k = 0; k < cand.size(); k++) {
            if (cand[k].ntt != best_shape) continue;
            enqueue_keyswitch(c, d, ext, nullptr, count, d_out, nullptr, c.p.Q, cand[k].ks, part, st);
            HIPC(hipEventRecord(ev[0], st));
            enqueue_keyswitch(c, d, ext, nullptr, count, d_out, nullptr, c.p.Q, cand[k].ks, part, st);
            HIPC(hipEventRecord(ev[1], st));
            HIPC(hipEventSynchronize(ev[1]));
            float ms = 0;
            HIPC(hipEventElapsedTime(&ms, ev[0], ev[1]));
            if (ms < best_ks) {
                best_ks = ms;
                best_k = k;
            }
        }
    } catch (...) {
        hipEventDestroy(ev[0]);
        hipEventDestroy(ev[1]);
        throw;
    }
    HIPC(hipEventDestroy(ev[0]));
    HIPC(hipEventDestroy(ev[1]));
    d.tuned[shape_key(c, ids, count)] = (int)best_k;
    return (int)best_k;
}

// Time each blind-rotation shape (group width, waves per component; with the
// default key switch) and each key-switch tiling (with the first shape) on this
// batch, one untimed run each first, and remember the fastest combination for
// the batch shape.
int run_autotune(mm_ctx &c, const int *ids, const uint32_t *ct_in, size_t count)
{
    MM_REQUIRE(check_ids(c, ids, count) == 0, "autotuning takes nega-cyclic tables");
    MM_REQUIRE(count > 0, "empty batch");
    Device &d = ensure_device(c);
    const size_t W = c.p.n + 1;
    hipStream_t st = d.own;
    const uint32_t *d_in = stage_in(d, WS_IN, ct_in, count * W, false, st);
    uint32_t *d_out = stage_out(d, WS_OUT, nullptr, count * W, false);
    HIPC(hipStreamSynchronize(st));
    if (use_global(c, ids, count)) return autotune_global(c, d, ids, d_in, d_out, count);
    auto cand = candidates(c, d, ids, count);
    const bool was_timed = d.timing;
    if (!d.tev[0])
        for (auto &e : d.tev) HIPC(hipEventCreate(&e));
    d.timing = true;
    const KsSched ks0 = cand[0].ks;
    const Sched first = cand[0];
    float best_br = 1e30f, best_ks = 1e30f;
    Sched br_best = first;
    KsSched ks_best = ks0;
    for (size_t k = 0; k < cand.size(); k++) {
        const Sched &S = cand[k];
        const bool default_ks = S.ks.cpw == ks0.cpw && S.ks.P == ks0.P;
        const bool first_shape = S.gw == first.gw && S.wpp == first.wpp && S.ntt == first.ntt;
        if (!default_ks && !first_shape) continue;  // each key-switch tiling is timed once
        bootstrap_batch(c, d, ids, d_in, count, d_out, 0, false, st, &S);
        HIPC(hipStreamSynchronize(st));
        bootstrap_batch(c, d, ids, d_in, count, d_out, 0, false, st, &S);
        HIPC(hipEventSynchronize(d.tev[2]));
        float br = 0, ks = 0;
        HIPC(hipEventElapsedTime(&br, d.tev[0], d.tev[1]));
        HIPC(hipEventElapsedTime(&ks, d.tev[1], d.tev[2]));
        if (default_ks && br < best_br) {
            best_br = br;
            br_best = S;
        }
        if (first_shape && ks < best_ks) {
            best_ks = ks;
            ks_best = S.ks;
        }
    }
    d.timing = was_timed;
    int choice = 0;
    for (size_t k = 0; k < cand.size(); k++)
        if (cand[k].gw == br_best.gw && cand[k].wpp == br_best.wpp && cand[k].ntt == br_best.ntt &&
            cand[k].ks.cpw == ks_best.cpw && cand[k].ks.P == ks_best.P)
            choice = (int)k;
    d.tuned[shape_key(c, ids, count)] = choice;
    return choice;
}

}  // namespace mm

mm_ctx::~mm_ctx()
{
    if (server) mm::server_stop(server);
    server = nullptr;
    dev.reset();
}
