/* Drives every entry point of the C ABI (include/mmpm.h) twice over, for the
 * host AddressSanitizer build (`python -m paper_2310_12441_amd.build --asan`):
 * the library's host runtime and this program are instrumented, the GPU code is
 * the product's.  Keys come from a counter-based generator of this file
 * (splitmix64) with zero errors, so every output must decrypt to f(m) exactly at
 * the ring modulus; the paths are checked against each other: plain = batched
 * = device pointers = served, every schedule gives the same bits, the steps one
 * by one compose to the bootstrap.  Exit status 0 when every check holds. */
#include <hip/hip_runtime_api.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

#include "mmpm.h"

static const uint32_t Q = 2147352577u, Q2 = 8380417u;
static uint64_t g_state;
static int g_fails;

/* splitmix64 (Steele, Lea and Flood, 2014): one 64-bit output per counter step */
static uint64_t next64(void)
{
    uint64_t z = (g_state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
static uint32_t below(uint32_t b) { return (uint32_t)(next64() % b); }

#define CHECK(ctx, call)                                                                                     \
    do {                                                                                                     \
        int rc_ = (call);                                                                                    \
        if (rc_ != MM_OK) {                                                                                  \
            fprintf(stderr, "%s:%d: %s returned %d: %s\n", __FILE__, __LINE__, #call, rc_, mm_last_error(ctx)); \
            exit(1);                                                                                         \
        }                                                                                                    \
    } while (0)
#define EXPECT(cond, what)                                                              \
    do {                                                                                \
        if (!(cond)) {                                                                  \
            fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, what); \
            g_fails++;                                                                  \
        }                                                                               \
    } while (0)
#define EXPECT_RC(call, code)                                                                                  \
    do {                                                                                                       \
        int rc_ = (call);                                                                                      \
        if (rc_ != (code)) {                                                                                   \
            fprintf(stderr, "%s:%d: %s returned %d, expected %d\n", __FILE__, __LINE__, #call, rc_, (code)); \
            g_fails++;                                                                                         \
        }                                                                                                      \
    } while (0)

static void *xmalloc(size_t bytes)
{
    void *p = calloc(bytes ? bytes : 1, 1);
    if (!p) {
        fprintf(stderr, "out of host memory\n");
        exit(1);
    }
    return p;
}

static mm_params params(uint32_t n, uint32_t N, uint32_t log2_B, uint32_t l, uint32_t ternary, uint32_t q2)
{
    mm_params p = {n, N, Q, log2_B, l, 4, 8, ternary, q2};
    return p;
}

/* A key set from the generator, every error zero. */
static mm_ctx *keys(const mm_params *p)
{
    const size_t K = 1 + p->ternary, rows = (size_t)p->n * K * 2 * p->l * p->N;
    const size_t ks = (size_t)p->N * p->l_ks * (1u << p->log2_Bks);
    int32_t *s = xmalloc(p->n * 4), *bsk_e = xmalloc(rows * 4), *ksk_e = xmalloc(ks * 4);
    uint32_t *z = xmalloc(p->N * 4), *bsk_a = xmalloc(rows * 4), *ksk_a = xmalloc(ks * p->n * 4);
    uint64_t *wide = p->Q2 ? xmalloc(rows * 8) : NULL;
    for (uint32_t i = 0; i < p->n; i++) s[i] = p->ternary ? (int32_t)below(3) - 1 : (int32_t)below(2);
    for (uint32_t i = 0; i < p->N; i++) z[i] = below(2);
    for (size_t i = 0; i < rows; i++) {
        bsk_a[i] = below(Q);
        if (wide) wide[i] = next64() % ((uint64_t)Q * p->Q2);
    }
    for (size_t i = 0; i < ks * p->n; i++) ksk_a[i] = below(Q);
    mm_key_draws d = {s, z, bsk_a, bsk_e, ksk_a, ksk_e, wide};
    mm_ctx *ctx = NULL;
    CHECK((mm_ctx *)NULL, mm_keygen(p, &d, &ctx));
    free(s);
    free(bsk_e);
    free(ksk_e);
    free(z);
    free(bsk_a);
    free(ksk_a);
    free(wide);
    return ctx;
}

/* f: Z_t -> Z_t' with f(m + t/2) = -f(m) mod t' */
static uint32_t *negacyclic(uint32_t t, uint32_t t_out)
{
    uint32_t *f = xmalloc(t * 4);
    for (uint32_t m = 0; m < t / 2; m++) {
        f[m] = below(t_out);
        f[m + t / 2] = (t_out - f[m]) % t_out;
    }
    return f;
}

/* count noise-free encryptions of m at (q, t) */
static uint32_t *encrypt(mm_ctx *ctx, uint32_t n, uint32_t q, uint32_t t, const uint32_t *m, size_t count)
{
    uint32_t *mask = xmalloc(count * n * 4), *ct = xmalloc(count * (n + 1) * 4);
    int32_t *err = xmalloc(count * 4);
    for (size_t i = 0; i < count * n; i++) mask[i] = below(q);
    CHECK(ctx, mm_encrypt(ctx, q, t, m, count, mask, err, ct));
    free(mask);
    free(err);
    return ct;
}

static int same(const void *a, const void *b, size_t words) { return memcmp(a, b, words * 4) == 0; }

/* The output decrypts to f(m) at the ring modulus (q_out = Q). */
static void expect_decrypts(mm_ctx *ctx, const uint32_t *out, size_t count, const int *ids, const uint32_t *const *fs,
                            const int *fidx, const uint32_t *m, const uint32_t *t_out)
{
    uint32_t *got = xmalloc(4);
    mm_params p;
    CHECK(ctx, mm_get_params(ctx, &p));
    for (size_t c = 0; c < count; c++) {
        CHECK(ctx, mm_decrypt(ctx, Q, t_out[c], out + c * (p.n + 1), 1, got));
        EXPECT(got[0] == fs[fidx[c]][m[c]], "bootstrap decrypts to f(m)");
        (void)ids;
    }
    free(got);
}

/* ---------------------------------------------------------------- the 31-bit ring, N = 1024 */
static void case_paper_ring(void)
{
    mm_params p = params(32, 1024, 7, 4, 0, 0);
    mm_ctx *ctx = keys(&p);
    const uint32_t n = p.n, N = p.N, W = n + 1;
    CHECK(ctx, mm_device_init(ctx, 0));
    /* tables: (t, r) = (4096, 4), (16384, 8), (256, 1); a general table (64, 2) */
    const uint32_t tt[3] = {4096, 16384, 256}, rr[3] = {4, 8, 1};
    uint32_t *f[3];
    int tid[3];
    for (int k = 0; k < 3; k++) {
        f[k] = negacyclic(tt[k], tt[k]);
        CHECK(ctx, mm_table_create(ctx, tt[k], tt[k], rr[k], 0, f[k], &tid[k]));
        uint32_t t, to, r, q;
        CHECK(ctx, mm_table_info(ctx, tid[k], &t, &to, &r, &q));
        EXPECT(t == tt[k] && r == rr[k] && q == 2 * N * rr[k], "table_info");
        uint32_t *V = xmalloc((size_t)r * N * 4);
        CHECK(ctx, mm_table_export(ctx, tid[k], V, (size_t)r * N));
        free(V);
    }
    /* a mixed batch */
    const size_t B = 48;
    int ids[48], cls[48];
    uint32_t m[48], tout[48];
    uint32_t *ct = xmalloc(B * W * 4);
    for (size_t c = 0; c < B; c++) {
        cls[c] = (int)(c % 3);
        ids[c] = tid[cls[c]];
        m[c] = below(tt[cls[c]]);
        tout[c] = tt[cls[c]];
        uint32_t *one = encrypt(ctx, n, 2 * N * rr[cls[c]], tt[cls[c]], &m[c], 1);
        memcpy(ct + c * W, one, W * 4);
        free(one);
    }
    uint32_t *out = xmalloc(B * W * 4), *out2 = xmalloc(B * W * 4);
    CHECK(ctx, mm_bootstrap(ctx, ids, ct, B, out, Q, 0, NULL));
    expect_decrypts(ctx, out, B, ids, (const uint32_t *const *)f, cls, m, tout);
    CHECK(ctx, mm_bootstrap(ctx, ids, ct, B, out2, Q, MM_PLAIN, NULL));
    EXPECT(same(out, out2, B * W), "plain = batched");
    /* device pointers on the null stream */
    uint32_t *d_in = NULL, *d_out = NULL;
    if (hipMalloc((void **)&d_in, B * W * 4) != hipSuccess || hipMalloc((void **)&d_out, B * W * 4) != hipSuccess) {
        fprintf(stderr, "hipMalloc failed\n");
        exit(1);
    }
    if (hipMemcpy(d_in, ct, B * W * 4, hipMemcpyHostToDevice) != hipSuccess) exit(1);
    CHECK(ctx, mm_bootstrap(ctx, ids, d_in, B, d_out, Q, MM_DEVICE_PTRS, NULL));
    memset(out2, 0, B * W * 4);
    if (hipMemcpy(out2, d_out, B * W * 4, hipMemcpyDeviceToHost) != hipSuccess) exit(1);
    EXPECT(same(out, out2, B * W), "device pointers = host pointers");
    /* every schedule, then autotuning, then timing */
    int ns = 0, choice = -1;
    CHECK(ctx, mm_schedule_count(ctx, ids, B, &ns));
    EXPECT(ns > 4, "schedule candidates");
    for (int k = 0; k < ns; k++) {
        int v[6];
        CHECK(ctx, mm_schedule_describe(ctx, ids, B, k, &v[0], &v[1], &v[2], &v[3], &v[4], &v[5]));
        CHECK(ctx, mm_set_schedule(ctx, ids, B, k));
        CHECK(ctx, mm_bootstrap(ctx, ids, ct, B, out2, Q, 0, NULL));
        EXPECT(same(out, out2, B * W), "every schedule gives the same bits");
    }
    CHECK(ctx, mm_autotune(ctx, ids, ct, B, &choice));
    EXPECT(choice >= 0 && choice < ns, "autotune choice");
    CHECK(ctx, mm_set_timing(ctx, 1));
    CHECK(ctx, mm_bootstrap(ctx, ids, ct, B, out2, Q, 0, NULL));
    float br = 0, ksm = 0;
    CHECK(ctx, mm_last_timing(ctx, &br, &ksm));
    EXPECT(br > 0 && ksm > 0, "kernel timing");
    CHECK(ctx, mm_set_timing(ctx, 0));
    EXPECT(same(out, out2, B * W), "timed = untimed");
    /* the steps one by one for the first ciphertext (r = 4, q_in = 2Nr) */
    {
        uint32_t ms[8], ms2[8];
        for (int k = 0; k < 8; k++) ms[k] = below(1u << 20);
        CHECK(ctx, mm_modswitch(ctx, ms, 8, 1u << 20, 4096, ms2, 0, NULL));
        for (int k = 0; k < 8; k++)
            EXPECT(ms2[k] == (uint32_t)(((2ull * ms[k] * 4096 + (1u << 20)) / (2ull << 20)) % 4096), "modswitch");
        uint32_t *acc = xmalloc((size_t)4 * 2 * N * 4), *lweN = xmalloc((N + 1) * 4), *lwen = xmalloc(W * 4);
        CHECK(ctx, mm_blind_rotate(ctx, ids, ct, 1, n, acc, 0, NULL));
        CHECK(ctx, mm_sample_extract(ctx, acc, 1, lweN, 0, NULL));
        CHECK(ctx, mm_keyswitch(ctx, lweN, 1, lwen, 0, NULL));
        EXPECT(same(lwen, out, W), "steps compose to the bootstrap");
        /* the allocation-free key switch on device pointers */
        uint32_t *dN = NULL, *dn = NULL;
        if (hipMalloc((void **)&dN, (N + 1) * 4) != hipSuccess || hipMalloc((void **)&dn, W * 4) != hipSuccess) exit(1);
        if (hipMemcpy(dN, lweN, (N + 1) * 4, hipMemcpyHostToDevice) != hipSuccess) exit(1);
        CHECK(ctx, mm_keyswitch_noalloc(ctx, dN, 1, dn, NULL));
        memset(lwen, 0, W * 4);
        if (hipMemcpy(lwen, dn, W * 4, hipMemcpyDeviceToHost) != hipSuccess) exit(1);
        EXPECT(same(lwen, out, W), "allocation-free key switch");
        hipFree(dN);
        hipFree(dn);
        /* external product and negacyclic product run; a x 1 = a */
        uint32_t *rl = xmalloc((size_t)2 * N * 4), *rl2 = xmalloc((size_t)2 * N * 4), *rl3 = xmalloc((size_t)2 * N * 4);
        for (uint32_t k = 0; k < 2 * N; k++) rl[k] = below(Q);
        CHECK(ctx, mm_external_product(ctx, 3, rl, 1, rl2, 0, NULL));
        CHECK(ctx, mm_external_product(ctx, 3, rl, 1, rl3, 0, NULL));
        EXPECT(same(rl2, rl3, 2 * N), "external product is deterministic");
        uint32_t *one = xmalloc(N * 4);
        one[0] = 1;
        CHECK(ctx, mm_negacyclic_mul(ctx, rl, one, 1, rl2, 0, NULL));
        EXPECT(same(rl, rl2, N), "a x 1 = a");
        free(one);
        free(rl);
        free(rl2);
        free(rl3);
        free(acc);
        free(lweN);
        free(lwen);
    }
    /* a general f: plaintext modulus 2t, m in [0, t) */
    {
        const uint32_t t = 64, r = 2, q = 2 * N * r;
        uint32_t *fg = xmalloc(t * 4), mg[16], outg[16];
        for (uint32_t k = 0; k < t; k++) fg[k] = below(t);
        int gid;
        CHECK(ctx, mm_table_create_general(ctx, t, t, r, 0, fg, &gid));
        int gids[16];
        for (int k = 0; k < 16; k++) {
            gids[k] = gid;
            mg[k] = below(t);
        }
        uint32_t *cg = encrypt(ctx, n, q, 2 * t, mg, 16);
        uint32_t *og = xmalloc(16 * W * 4);
        CHECK(ctx, mm_bootstrap(ctx, gids, cg, 16, og, Q, 0, NULL));
        CHECK(ctx, mm_decrypt(ctx, Q, t, og, 16, outg));
        for (int k = 0; k < 16; k++) EXPECT(outg[k] == fg[mg[k]], "general f decrypts to f(m)");
        int mix[2] = {gid, tid[0]};
        EXPECT_RC(mm_bootstrap(ctx, mix, ct, 2, og, Q, 0, NULL), MM_EINVAL);
        free(fg);
        free(cg);
        free(og);
    }
    /* serving: submit/poll, then a replayed burst with admission */
    {
        uint32_t *alone = xmalloc(B * W * 4);
        CHECK(ctx, mm_bootstrap(ctx, ids, ct, B, alone, 0, 0, NULL));
        mm_server *srv = NULL;
        EXPECT_RC(mm_server_start(ctx, 1024, 7, &srv), MM_EINVAL);
        CHECK(ctx, mm_server_start(ctx, 256u << 20, 7, &srv));
        EXPECT_RC(mm_server_start(ctx, 256u << 20, 7, &srv), MM_ESTATE);
        uint64_t tickets[48];
        for (size_t c = 0; c < B; c++) CHECK(ctx, mm_submit(srv, ids[c], ct + c * W, &tickets[c]));
        uint64_t bogus;
        EXPECT_RC(mm_submit(srv, 99, ct, &bogus), MM_EINVAL);
        EXPECT_RC(mm_poll(srv, 123456789, out2), MM_EINVAL);
        size_t left = B;
        char *got = xmalloc(B);
        const time_t t0 = time(NULL);
        while (left && time(NULL) - t0 < 60) {
            for (size_t c = 0; c < B; c++) {
                if (got[c]) continue;
                int rc = mm_poll(srv, tickets[c], out2 + c * W);
                if (rc == MM_OK) {
                    got[c] = 1;
                    left--;
                } else if (rc != MM_EAGAIN) {
                    fprintf(stderr, "poll returned %d\n", rc);
                    exit(1);
                }
            }
        }
        EXPECT(left == 0, "every served request completes");
        EXPECT(same(out2, alone, B * W), "served = alone");
        EXPECT_RC(mm_poll(srv, tickets[0], out2), MM_EINVAL);
        int64_t arr[48];
        for (size_t c = 0; c < B; c++) arr[c] = 0;
        double lat[48];
        CHECK(ctx, mm_server_set_admission(srv, 0.001));
        EXPECT_RC(mm_server_set_admission(srv, -1.0), MM_EINVAL);
        CHECK(ctx, mm_server_replay(srv, ids, ct, arr, B, out2, lat));
        for (size_t c = 0; c < B; c++)
            if (lat[c] >= 0) EXPECT(same(out2 + c * W, alone + c * W, W), "replayed = alone");
        uint64_t refused = 0, done = 0;
        double p50, p99, bps;
        CHECK(ctx, mm_server_refused(srv, &refused));
        CHECK(ctx, mm_server_stats(srv, &p50, &p99, &bps, &done));
        EXPECT(done + refused == 2 * B, "completed + refused = submitted");
        CHECK(ctx, mm_server_stop(srv));
        free(got);
        free(alone);
    }
    /* error paths */
    {
        int bad = 77;
        EXPECT_RC(mm_bootstrap(ctx, &bad, ct, 1, out2, Q, 0, NULL), MM_EINVAL);
        uint32_t g2[4] = {1, 2, 3, 4};
        int dummy;
        EXPECT_RC(mm_table_create(ctx, 4, 4, 1, 0, g2, &dummy), MM_EINVAL); /* not nega-cyclic */
        EXPECT_RC(mm_table_create(ctx, 16, 16, 2000, 0, g2, &dummy), MM_EINVAL);
        mm_params bp = params(4, 100, 7, 4, 0, 0);
        mm_ctx *none = NULL;
        uint32_t zero[1] = {0};
        int32_t izero[1] = {0};
        mm_key_draws d = {izero, zero, zero, izero, zero, izero, NULL};
        EXPECT_RC(mm_keygen(&bp, &d, &none), MM_EINVAL);
        EXPECT(mm_last_error(NULL) != NULL, "keygen error message");
    }
    hipFree(d_in);
    hipFree(d_out);
    for (int k = 0; k < 3; k++) free(f[k]);
    free(ct);
    free(out);
    free(out2);
    mm_free(ctx);
}

/* ---------------------------------------------------------------- 54-bit ring modulus, ternary */
static void case_wide(void)
{
    mm_params p = params(8, 256, 15, 4, 1, Q2);
    mm_ctx *ctx = keys(&p);
    const uint32_t n = p.n, N = p.N, W = n + 1, t = 16, r = 4, q = 2 * N * r;
    uint32_t *f = negacyclic(t, t);
    int tid;
    CHECK(ctx, mm_table_create(ctx, t, t, r, 0, f, &tid));
    const size_t B = 16;
    int ids[16], fi[16];
    uint32_t m[16], tout[16];
    for (size_t c = 0; c < B; c++) {
        ids[c] = tid;
        fi[c] = 0;
        m[c] = below(t);
        tout[c] = t;
    }
    uint32_t *ct = encrypt(ctx, n, q, t, m, B);
    uint32_t *out = xmalloc(B * W * 4), *out2 = xmalloc(B * W * 4);
    CHECK(ctx, mm_bootstrap(ctx, ids, ct, B, out, Q, 0, NULL));
    const uint32_t *fs[1] = {f};
    expect_decrypts(ctx, out, B, ids, fs, fi, m, tout);
    CHECK(ctx, mm_bootstrap(ctx, ids, ct, B, out2, Q, MM_PLAIN, NULL));
    EXPECT(same(out, out2, B * W), "wide: plain = batched");
    int ns = 0, choice = -1;
    CHECK(ctx, mm_schedule_count(ctx, ids, B, &ns));
    for (int k = 0; k < ns; k++) {
        CHECK(ctx, mm_set_schedule(ctx, ids, B, k));
        CHECK(ctx, mm_bootstrap(ctx, ids, ct, B, out2, Q, 0, NULL));
        EXPECT(same(out, out2, B * W), "wide: every schedule gives the same bits");
    }
    CHECK(ctx, mm_autotune(ctx, ids, ct, B, &choice));
    uint32_t *acc = xmalloc((size_t)B * r * 2 * N * 8);
    CHECK(ctx, mm_blind_rotate(ctx, ids, ct, B, 2, acc, 0, NULL));
    EXPECT_RC(mm_external_product(ctx, 0, acc, 1, acc, 0, NULL), MM_EINVAL);
    uint32_t *alone = xmalloc(B * W * 4);
    CHECK(ctx, mm_bootstrap(ctx, ids, ct, B, alone, 0, 0, NULL));
    mm_server *srv = NULL;
    CHECK(ctx, mm_server_start(ctx, 16u << 20, 3, &srv));
    int64_t arr[16];
    double lat[16];
    for (size_t c = 0; c < B; c++) arr[c] = (int64_t)c * 1000000;
    CHECK(ctx, mm_server_replay(srv, ids, ct, arr, B, out2, lat));
    EXPECT(same(out2, alone, B * W), "wide: served = alone");
    CHECK(ctx, mm_server_stop(srv));
    free(alone);
    free(acc);
    free(f);
    free(ct);
    free(out);
    free(out2);
    mm_free(ctx);
}

/* ---------------------------------------------------------------- a ring split into sub-rings */
static void case_split(void)
{
    mm_params p = params(2, 32768, 7, 4, 0, 0);
    mm_ctx *ctx = keys(&p);
    const uint32_t n = p.n, N = p.N, W = n + 1, t = 16384, q = 2 * N;
    uint32_t *f = negacyclic(t, t);
    int tid;
    CHECK(ctx, mm_table_create(ctx, t, t, 1, 0, f, &tid));
    int ids[2] = {tid, tid}, fi[2] = {0, 0};
    uint32_t m[2] = {below(t), below(t)}, tout[2] = {t, t};
    uint32_t *ct = encrypt(ctx, n, q, t, m, 2);
    uint32_t *out = xmalloc(2 * W * 4), *out2 = xmalloc(2 * W * 4);
    CHECK(ctx, mm_bootstrap(ctx, ids, ct, 2, out, Q, 0, NULL));
    const uint32_t *fs[1] = {f};
    expect_decrypts(ctx, out, 2, ids, fs, fi, m, tout);
    CHECK(ctx, mm_bootstrap(ctx, ids, ct, 2, out2, Q, MM_PLAIN, NULL));
    EXPECT(same(out, out2, 2 * W), "split ring: plain = batched");
    int ns = 0;
    CHECK(ctx, mm_schedule_count(ctx, ids, 2, &ns));
    EXPECT(ns >= 1, "split ring schedules");
    mm_server *srv = NULL;
    EXPECT_RC(mm_server_start(ctx, 256u << 20, 1, &srv), MM_EINVAL);
    free(f);
    free(ct);
    free(out);
    free(out2);
    mm_free(ctx);
}

int main(void)
{
    for (int round = 0; round < 2; round++) {
        g_state = 0x5EED0000u + (uint64_t)round;
        case_paper_ring();
        printf("round %d: N = 1024 done\n", round);
        fflush(stdout);
        case_wide();
        printf("round %d: 54-bit ring done\n", round);
        fflush(stdout);
        case_split();
        printf("round %d: split ring done\n", round);
        fflush(stdout);
    }
    if (g_fails) {
        fprintf(stderr, "%d checks failed\n", g_fails);
        return 1;
    }
    printf("abi driver: every check passed\n");
    return 0;
}
