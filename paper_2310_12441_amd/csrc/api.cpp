// extern "C" boundary: argument checks and exception-to-status translation.
#include <cstring>
#include <new>

#include "mmpm_internal.hpp"

namespace {

thread_local std::string g_keygen_err;

template <class F>
int guard(mm_ctx *c, F &&f)
{
    try {
        f();
        return MM_OK;
    } catch (const mm::Error &e) {
        if (c) c->err = e.what();
        else g_keygen_err = e.what();
        return e.code;
    } catch (const std::bad_alloc &) {
        if (c) c->err = "host allocation failed";
        else g_keygen_err = "host allocation failed";
        return MM_ENOMEM;
    } catch (const std::exception &e) {
        if (c) c->err = e.what();
        else g_keygen_err = e.what();
        return MM_EDEVICE;
    }
}

}  // namespace

extern "C" {

int mm_keygen(const mm_params *p, const mm_key_draws *draws, mm_ctx **out)
{
    if (!out) return MM_EINVAL;
    *out = nullptr;
    mm_ctx *c = nullptr;
    int rc = guard(nullptr, [&] {
        MM_REQUIRE(p && draws, "null argument");
        mm::validate_params(*p);
        c = new mm_ctx();
        c->p = *p;
        try {
            mm::keygen(*c, *draws);
        } catch (...) {
            delete c;
            c = nullptr;
            throw;
        }
    });
    if (rc == MM_OK) *out = c;
    return rc;
}

void mm_free(mm_ctx *ctx) { delete ctx; }

const char *mm_last_error(const mm_ctx *ctx) { return ctx ? ctx->err.c_str() : g_keygen_err.c_str(); }

int mm_get_params(const mm_ctx *ctx, mm_params *out)
{
    if (!ctx || !out) return MM_EINVAL;
    *out = ctx->p;
    return MM_OK;
}

int mm_export_bsk(const mm_ctx *ctx, uint32_t *out, size_t words)
{
    if (!ctx || !out) return MM_EINVAL;
    if (words < ctx->bsk.size()) return MM_EINVAL;
    if (!ctx->wide) {
        std::memcpy(out, ctx->bsk.data(), ctx->bsk.size() * 4);
        return MM_OK;
    }
    // [ik][limb][row][part][N] residues -> [ik][row][part][N] uint64 at Q Q2
    const size_t N = ctx->p.N, per = (size_t)2 * ctx->p.l * 2 * N;  // words of one limb of one key
    const size_t keys = ctx->bsk.size() / (2 * per);
    for (size_t ik = 0; ik < keys; ik++)
        for (size_t w = 0; w < per; w++) {
            const uint64_t v = mm::crt2(ctx->bsk[(ik * 2 + 0) * per + w], ctx->bsk[(ik * 2 + 1) * per + w],
                                        ctx->p.Q, ctx->p.Q2);
            std::memcpy(out + 2 * (ik * per + w), &v, 8);
        }
    return MM_OK;
}

int mm_export_ksk(const mm_ctx *ctx, uint32_t *out, size_t words)
{
    if (!ctx || !out) return MM_EINVAL;
    if (words < ctx->ksk.size()) return MM_EINVAL;
    std::memcpy(out, ctx->ksk.data(), ctx->ksk.size() * 4);
    return MM_OK;
}

int mm_device_init(mm_ctx *ctx, int device)
{
    if (!ctx) return MM_EINVAL;
    std::lock_guard<std::mutex> g(ctx->lock);
    return guard(ctx, [&] { mm::device_init(*ctx, device); });
}

int mm_table_create(mm_ctx *ctx, uint32_t t, uint32_t t_out, uint32_t r, uint32_t q_in, const uint32_t *f, int *id)
{
    if (!ctx || !f || !id) return MM_EINVAL;
    std::lock_guard<std::mutex> g(ctx->lock);
    return guard(ctx, [&] { *id = mm::table_create(*ctx, t, t_out, r, q_in, f); });
}

int mm_table_create_general(mm_ctx *ctx, uint32_t t, uint32_t t_out, uint32_t r, uint32_t q_in, const uint32_t *f,
                            int *id)
{
    if (!ctx || !f || !id) return MM_EINVAL;
    std::lock_guard<std::mutex> g(ctx->lock);
    return guard(ctx, [&] { *id = mm::table_create_general(*ctx, t, t_out, r, q_in, f); });
}

int mm_table_info(const mm_ctx *ctx, int id, uint32_t *t, uint32_t *t_out, uint32_t *r, uint32_t *q_in)
{
    if (!ctx || id < 0 || (size_t)id >= ctx->tables.size()) return MM_EINVAL;
    const mm::Table &tb = ctx->tables[id];
    if (t) *t = tb.t;
    if (t_out) *t_out = tb.t_out;
    if (r) *r = tb.r;
    if (q_in) *q_in = tb.q_in;
    return MM_OK;
}

int mm_table_export(const mm_ctx *ctx, int id, uint32_t *V, size_t words)
{
    if (!ctx || !V || id < 0 || (size_t)id >= ctx->tables.size()) return MM_EINVAL;
    const mm::Table &tb = ctx->tables[id];
    if (tb.V.empty() || words < tb.V.size()) return MM_EINVAL;
    if (!ctx->wide) {
        std::memcpy(V, tb.V.data(), tb.V.size() * 4);
        return MM_OK;
    }
    const size_t N = ctx->p.N;  // [r][limb][N] -> [r][N] uint64
    for (size_t b = 0; b < tb.r; b++)
        for (size_t a = 0; a < N; a++) {
            const uint64_t v = mm::crt2(tb.V[(b * 2 + 0) * N + a], tb.V[(b * 2 + 1) * N + a], ctx->p.Q, ctx->p.Q2);
            std::memcpy(V + 2 * (b * N + a), &v, 8);
        }
    return MM_OK;
}

int mm_encrypt(const mm_ctx *ctx, uint32_t q, uint32_t t, const uint32_t *m, size_t count, const uint32_t *mask,
               const int32_t *err, uint32_t *ct)
{
    if (!ctx || (count && (!m || !mask || !err || !ct))) return MM_EINVAL;
    return guard(const_cast<mm_ctx *>(ctx), [&] { mm::encrypt(*ctx, q, t, m, count, mask, err, ct); });
}

int mm_decrypt(const mm_ctx *ctx, uint32_t q, uint32_t t, const uint32_t *ct, size_t count, uint32_t *m)
{
    if (!ctx || (count && (!ct || !m))) return MM_EINVAL;
    return guard(const_cast<mm_ctx *>(ctx), [&] { mm::decrypt(*ctx, q, t, ct, count, m); });
}

int mm_bootstrap(mm_ctx *ctx, const int *table_ids, const uint32_t *ct_in, size_t count, uint32_t *ct_out,
                 uint32_t q_out, uint32_t flags, void *stream)
{
    if (!ctx || (count && (!ct_in || !ct_out))) return MM_EINVAL;
    std::lock_guard<std::mutex> g(ctx->lock);
    return guard(ctx, [&] { mm::run_bootstrap(*ctx, table_ids, ct_in, count, ct_out, q_out, flags, stream); });
}

int mm_modswitch(mm_ctx *ctx, const uint32_t *in, size_t count, uint32_t q_from, uint32_t q_to, uint32_t *out,
                 uint32_t flags, void *stream)
{
    if (!ctx || (count && (!in || !out))) return MM_EINVAL;
    std::lock_guard<std::mutex> g(ctx->lock);
    return guard(ctx, [&] { mm::run_modswitch(*ctx, in, count, q_from, q_to, out, flags, stream); });
}

int mm_blind_rotate(mm_ctx *ctx, const int *table_ids, const uint32_t *ct_in, size_t count, uint32_t steps,
                    uint32_t *acc_out, uint32_t flags, void *stream)
{
    if (!ctx || (count && (!ct_in || !acc_out))) return MM_EINVAL;
    std::lock_guard<std::mutex> g(ctx->lock);
    return guard(ctx, [&] { mm::run_blind_rotate(*ctx, table_ids, ct_in, count, steps, acc_out, flags, stream); });
}

int mm_external_product(mm_ctx *ctx, uint32_t i, const uint32_t *in, size_t count, uint32_t *out, uint32_t flags,
                        void *stream)
{
    if (!ctx || (count && (!in || !out))) return MM_EINVAL;
    std::lock_guard<std::mutex> g(ctx->lock);
    return guard(ctx, [&] { mm::run_external_product(*ctx, i, in, count, out, flags, stream); });
}

int mm_sample_extract(mm_ctx *ctx, const uint32_t *rlwe, size_t count, uint32_t *lwe, uint32_t flags, void *stream)
{
    if (!ctx || (count && (!rlwe || !lwe))) return MM_EINVAL;
    std::lock_guard<std::mutex> g(ctx->lock);
    return guard(ctx, [&] { mm::run_sample_extract(*ctx, rlwe, count, lwe, flags, stream); });
}

int mm_keyswitch(mm_ctx *ctx, const uint32_t *lwe_N, size_t count, uint32_t *lwe_n, uint32_t flags, void *stream)
{
    if (!ctx || (count && (!lwe_N || !lwe_n))) return MM_EINVAL;
    std::lock_guard<std::mutex> g(ctx->lock);
    return guard(ctx, [&] { mm::run_keyswitch(*ctx, lwe_N, count, lwe_n, flags, stream); });
}

int mm_keyswitch_noalloc(mm_ctx *ctx, const uint32_t *lwe_N, size_t count, uint32_t *lwe_n, void *stream)
{
    if (!ctx || (count && (!lwe_N || !lwe_n))) return MM_EINVAL;
    std::lock_guard<std::mutex> g(ctx->lock);
    return guard(ctx, [&] { mm::run_keyswitch_noalloc(*ctx, lwe_N, count, lwe_n, stream); });
}

int mm_negacyclic_mul(mm_ctx *ctx, const uint32_t *a, const uint32_t *b, size_t count, uint32_t *out, uint32_t flags,
                      void *stream)
{
    if (!ctx || (count && (!a || !b || !out))) return MM_EINVAL;
    std::lock_guard<std::mutex> g(ctx->lock);
    return guard(ctx, [&] { mm::run_negacyclic_mul(*ctx, a, b, count, out, flags, stream); });
}

int mm_set_timing(mm_ctx *ctx, int enable)
{
    if (!ctx) return MM_EINVAL;
    std::lock_guard<std::mutex> g(ctx->lock);
    return guard(ctx, [&] { mm::set_timing(*ctx, enable != 0); });
}

int mm_last_timing(mm_ctx *ctx, float *blind_rotate_ms, float *keyswitch_ms)
{
    if (!ctx) return MM_EINVAL;
    std::lock_guard<std::mutex> g(ctx->lock);
    return guard(ctx, [&] { mm::last_timing(*ctx, blind_rotate_ms, keyswitch_ms); });
}

int mm_autotune(mm_ctx *ctx, const int *table_ids, const uint32_t *ct_in, size_t count, int *choice)
{
    if (!ctx || !choice || (count && (!ct_in || !table_ids))) return MM_EINVAL;
    std::lock_guard<std::mutex> g(ctx->lock);
    return guard(ctx, [&] { *choice = mm::run_autotune(*ctx, table_ids, ct_in, count); });
}

int mm_schedule_count(mm_ctx *ctx, const int *table_ids, size_t count, int *n)
{
    if (!ctx || !n || !table_ids) return MM_EINVAL;
    std::lock_guard<std::mutex> g(ctx->lock);
    return guard(ctx, [&] { *n = mm::schedule_count(*ctx, table_ids, count); });
}

int mm_set_schedule(mm_ctx *ctx, const int *table_ids, size_t count, int choice)
{
    if (!ctx || !table_ids) return MM_EINVAL;
    std::lock_guard<std::mutex> g(ctx->lock);
    return guard(ctx, [&] { mm::set_schedule(*ctx, table_ids, count, choice); });
}

int mm_schedule_describe(mm_ctx *ctx, const int *table_ids, size_t count, int choice, int *group_waves,
                         int *ks_cts_per_wave, int *ks_splits, int *waves_per_component, int *ks_kernel,
                         int *ntt_schedule)
{
    if (!ctx || !table_ids) return MM_EINVAL;
    std::lock_guard<std::mutex> g(ctx->lock);
    return guard(ctx, [&] {
        mm::describe_schedule(*ctx, table_ids, count, choice, group_waves, ks_cts_per_wave, ks_splits,
                              waves_per_component, ks_kernel, ntt_schedule);
    });
}

}  // extern "C"
