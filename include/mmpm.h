/*
 * mmpm.h -- C ABI of the BootMMPM functional bootstrap on AMD Instinct
 * MI355X (gfx950).
 *
 * The library bootstraps LWE ciphertexts whose plaintexts are large (t up to
 * 2^14 and beyond) through a look-up table spread over a vector of r
 * negacyclic polynomials, following Algorithm 1 (BootMMPM) of "Large-Plaintext
 * Functional Bootstrapping in FHE with Small Bootstrapping Keys"
 * (arXiv 2310.12441), with a binary LWE secret s and a binary ring secret z.
 *
 * Conventions shared by every call
 *   * Q is an odd prime with Q = 1 mod 2N and Q < 2^31; every residue is a
 *     uint32 in [0, Q) (or [0, q) for LWE ciphertexts at modulus q).
 *   * An LWE ciphertext of dimension d is d+1 consecutive uint32: a_0..a_{d-1}, b,
 *     with phase b - <a, s> (Sec. 2 item (8)).
 *   * An RLWE pair is (a, b), N words each, phase b - a z (Sec. 2 item (12)).
 *   * Ownership: the caller owns every buffer it passes; the library copies
 *     what it keeps.  A context owns its keys, tables and device memory.
 *   * Errors: every int-returning call returns MM_OK (0) or a negative MM_E*
 *     code, never throws, and keeps a message readable with mm_last_error().
 *   * Threads: calls on distinct contexts are independent.  Calls on one
 *     context must not overlap, except mm_submit / mm_poll / mm_server_stats,
 *     which are safe from any thread while a server runs.
 *   * Device pointers: with MM_DEVICE_PTRS every ciphertext buffer is device
 *     memory on the context's device and the call is asynchronous on `stream`
 *     (a hipStream_t, or NULL for the null stream); without it buffers are host
 *     memory and the call returns when results are in them.
 */
#ifndef MMPM_H
#define MMPM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MM_OK 0
#define MM_EINVAL (-1)   /* bad parameter, size or id */
#define MM_ENOMEM (-2)   /* host or device allocation failed */
#define MM_EDEVICE (-3)  /* a HIP call failed; see mm_last_error */
#define MM_EBUSY (-4)    /* serving: request refused by admission */
#define MM_EAGAIN (-5)   /* serving: result not ready yet */
#define MM_ESTATE (-6)   /* call not valid in the current state */

/* flags */
#define MM_DEVICE_PTRS 1u /* ciphertext buffers are device pointers */
#define MM_PLAIN 2u       /* bootstrap one ciphertext at a time (per-ciphertext launches) */

typedef struct mm_ctx mm_ctx;
typedef struct mm_server mm_server;

/* Ring and gadget parameters of one key set (Alg. 1 inputs).
 * n: LWE dimension; N: ring degree, a power of two in [64, 65536] (the device
 * path takes 256 ... 65536; above 1024 one polynomial spans N / 1024 waves; a
 * batch whose tables all have r * N / 1024 <= 8 runs the fused persistent
 * kernel, any other batch, and every batch at N >= 16384, the global-
 * accumulator path: accumulators in device memory, one launch per CMux step
 * (three for a ring split into sub-rings of 8192 coefficients: the NTT stages
 * that mix sub-rings run through device memory; always above 16384, a
 * schedule choice at 16384), r up to 1024 -- so the TFHE-shaped rings of the
 * comparison in Sec. 5 reach N = 65536 and MMPM tables r = 16 and beyond);
 * Q: ring modulus (odd prime, Q = 1 mod 2N, Q < 2^31); log2_B, l:
 * the blind-rotation gadget base 2^log2_B and length, l * log2_B <= 32 and
 * log2_B <= 15; log2_Bks, l_ks: the key-switch base and length,
 * l_ks * log2_Bks >= bits(Q) so the key-switch digits are exact; ternary: 0 for
 * a binary LWE secret (one RGSW key and one external product per step), 1 for a
 * ternary one (keys for s+ and s-, two external products per step, Alg. 1 as
 * printed).  K = 1 + ternary keys per coordinate.
 *
 * Q2 = 0 is the default.  Q2 != 0 selects a wide ring modulus Q_w = Q Q2 for
 * the blind rotation (the parameter regime of the experiments in Sec. 5, where
 * log Q = 54 and the gadget base is 2^15): Q2 is a second odd prime, Q2 != Q,
 * Q2 = 1 mod 2N, Q2 < 2^31; the accumulator and the bootstrapping key hold two
 * residues per coefficient (mod Q and mod Q2); the gadget needs log2_B <= 16,
 * l <= 8, l * log2_B <= 62 and sg = max(0, bits(Q_w) - l log2_B).  Everything
 * on the LWE side stays at Q: after sample extraction every coefficient is
 * switched Q_w -> Q by rounding (round(x / Q2), Sec. 2 item (9)), then the key
 * switch and the final switch run at Q as in the default mode.  Tables may then
 * have r up to 1024, because the accumulator of a ciphertext lives in device
 * memory, one (ciphertext, component) pair per workgroup and one launch per
 * CMux step.  In this mode mm_external_product, the schedule calls
 * (mm_autotune, mm_schedule_*) and the server return MM_EINVAL; mm_export_bsk,
 * mm_table_export and mm_blind_rotate give uint64 values in [0, Q_w) (two
 * words each, the low word first). */
typedef struct {
    uint32_t n, N, Q, log2_B, l, log2_Bks, l_ks, ternary;
    uint32_t Q2;
} mm_params;

/* The random material of a key set, drawn by the caller (host memory, read
 * only during mm_keygen).  The library takes draws instead of a seed so that it
 * holds no random generator of its own: a checker builds the same keys from the
 * same arrays, and the caller picks the generator and its seed.
 *   s      n values in {0,1} (binary) or {-1,0,1} (ternary)   LWE secret
 *   z      N values in {0,1}           RLWE secret
 *   bsk_a  n * K * 2l * N in [0, Q)    RGSW masks, [i][key][row][coeff]
 *   bsk_e  n * K * 2l * N small ints   RGSW errors, same layout
 *   ksk_a  N * l_ks * B_ks * n in [0,Q) key-switch masks, [i][j][v][k]
 *   ksk_e  N * l_ks * B_ks small ints  key-switch errors, [i][j][v]
 *   bsk_a_wide  with Q2 != 0 only: n * K * 2l * N uint64 in [0, Q Q2), the
 *          RGSW masks at the wide modulus (bsk_a is then not read)  */
typedef struct {
    const int32_t *s;
    const uint32_t *z, *bsk_a;
    const int32_t *bsk_e;
    const uint32_t *ksk_a;
    const int32_t *ksk_e;
    const uint64_t *bsk_a_wide;
} mm_key_draws;

/* Build a key set (host only; no GPU needed).
 * BSK_{i,k} = RGSW_z(m) with m = s_i (binary), or m = max(s_i, 0) for k = 0 and
 * max(-s_i, 0) for k = 1 (ternary): rows u < l are (a_u, a_u z + e_u + m g_u),
 * rows l+u are (a_{l+u} + m g_u, a_{l+u} z + e_{l+u}), g_u = 2^(sg + u log2_B)
 * mod Q with sg = max(0, bits(Q) - l log2_B) (Alg. 1 inputs; Sec. 2 item (14)).
 * KSK[i][j][v] = LWE_s(v z_i B_ks^j), v in [0, B_ks) including 0 (Sec. 2 item
 * (11)).  On success *out owns a new context.  MM_EINVAL for bad parameters. */
int mm_keygen(const mm_params *p, const mm_key_draws *draws, mm_ctx **out);

/* Release a context, its device memory and any server it runs.  NULL is a no-op. */
void mm_free(mm_ctx *ctx);

/* Message of the last failed call on ctx (or of the last failed mm_keygen when
 * ctx is NULL).  The string stays valid until the next call on ctx. */
const char *mm_last_error(const mm_ctx *ctx);

int mm_get_params(const mm_ctx *ctx, mm_params *out);

/* Coefficient-form keys, for checking: bsk as [n][K][2l][2][N] (part 0 = a),
 * ksk as [N][l_ks][B_ks][n+1].  `words` is the capacity of out (with Q2 != 0
 * the bsk entries are uint64 at Q Q2, two words each). */
int mm_export_bsk(const mm_ctx *ctx, uint32_t *out, size_t words);
int mm_export_ksk(const mm_ctx *ctx, uint32_t *out, size_t words);

/* Select device `device`, convert the bootstrapping key to the NTT domain and
 * upload both keys.  Called implicitly by the first device call. */
int mm_device_init(mm_ctx *ctx, int device);

/* Register a look-up table f: Z_t -> Z_t' held in r polynomials (Sec. 3,
 * Example 2; Alg. 1 input v_test), 1 <= r <= 1024.  Requires t, t' even, t | 2Nr, f nega-cyclic
 * (f[m + t/2] = -f[m] mod t', Definition 1) with entries in [0, t').  q_in is
 * the modulus of the ciphertexts bootstrapped with this table (0 selects 2Nr, so
 * the first modulus switch is the identity); 2 <= q_in <= 2^31.  The test vector
 * holds, at entry b and coefficient a, floor(Q/t') times the canonical residue of
 * f'(-(a r + b)), where f' extends f to Z_2Nr by rounding to the nearest multiple
 * of 2Nr/t (ties upward).  *id receives the table id. */
int mm_table_create(mm_ctx *ctx, uint32_t t, uint32_t t_out, uint32_t r, uint32_t q_in,
                    const uint32_t *f, int *id);
int mm_table_info(const mm_ctx *ctx, int id, uint32_t *t, uint32_t *t_out, uint32_t *r,
                  uint32_t *q_in);

/* Register an arbitrary (not nega-cyclic) f: Z_t -> Z_t', t entries in [0, t'),
 * evaluated by two bootstraps (Sec. 4, functional bootstrapping of a general
 * f): ciphertexts for this table encrypt x = m + b t in Z_2t (plaintext modulus
 * 2t, m in [0, t), b an unknown top bit) at modulus q_in (0 selects 2Nr);
 * requires t even, 2t | 2Nr.  The first bootstrap evaluates the nega-cyclic
 * g(x) = t/2 for x in [0, t), -t/2 for x in [t, 2t); ct + ct_g - (0, (t/2)
 * floor(q_in / 2t)) then encrypts m; the second evaluates the nega-cyclic
 * extension F(y) = f(y), F(y + t) = -f(y).  The output encrypts f(m) with
 * plaintext modulus t'.  A single mm_bootstrap call takes either only such
 * tables or none of them (MM_EINVAL otherwise); mm_table_info reports t and the
 * vector length r. */
int mm_table_create_general(mm_ctx *ctx, uint32_t t, uint32_t t_out, uint32_t r, uint32_t q_in,
                            const uint32_t *f, int *id);
/* The scaled test vector of table id as [r][N] (uint64 at Q Q2, two words
 * per entry, when Q2 != 0). */
int mm_table_export(const mm_ctx *ctx, int id, uint32_t *V, size_t words);

/* LWE encryption under s (Sec. 2 item (8)): ct_c = (a_c, <a_c, s> + m_c floor(q/t)
 * + e_c mod q) with caller-drawn masks a (count x n, in [0, q)) and errors e.
 * Host buffers; ct is count x (n+1). */
int mm_encrypt(const mm_ctx *ctx, uint32_t q, uint32_t t, const uint32_t *m, size_t count,
               const uint32_t *mask, const int32_t *err, uint32_t *ct);

/* LWE decryption under s (Sec. 2 item (8), the phase of eq. def:phase):
 * m_c = round((b - <a, s> mod q) / floor(q/t)) mod t (ties upward). Host buffers. */
int mm_decrypt(const mm_ctx *ctx, uint32_t q, uint32_t t, const uint32_t *ct, size_t count,
               uint32_t *m);

/* BootMMPM(ct, f) (Alg. 1) for `count` ciphertexts, ciphertext c bootstrapped
 * with table table_ids[c] (tables may differ in t, t', r and q_in):
 * modulus switch q_in -> 2Nr, ACC = Phi(b')(0, V), n CMux steps
 * ACC += (Phi(-a'_i) ACC - ACC) x BSK_{i,0} [+ (Phi(a'_i) ACC - ACC) x BSK_{i,1}
 * for a ternary secret] (eq. cmux:BP), sample extraction of entry 0, key switch
 * z -> s, modulus switch Q -> q_out.  ct_in holds count x (n+1) words at each
 * table's q_in; ct_out receives count x (n+1) words at q_out, where q_out = 0
 * keeps each table's q_in and q_out = Q skips the final switch.  By default the
 * whole batch runs as one persistent fused launch sequence (captured in a HIP
 * graph); MM_PLAIN runs one ciphertext at a time.  Both give identical bits. */
int mm_bootstrap(mm_ctx *ctx, const int *table_ids, const uint32_t *ct_in, size_t count,
                 uint32_t *ct_out, uint32_t q_out, uint32_t flags, void *stream);

/* ---- the same path one step at a time (each a row of the hot path) ---- */

/* Modulus switch round(x q_to / q_from) (ties upward) of `count` residues (Sec. 2 item (9)). */
int mm_modswitch(mm_ctx *ctx, const uint32_t *in, size_t count, uint32_t q_from, uint32_t q_to,
                 uint32_t *out, uint32_t flags, void *stream);

/* Blind rotation only: for ciphertext c (at its table's q_in), the accumulator
 * after the modulus switch, the initialisation and the first `steps` CMux steps
 * (steps <= n).  acc_out receives, for each c in order, r_c x 2 x N words
 * ([component][part][coeff], part 0 = a); with Q2 != 0 each entry is a uint64
 * at Q Q2 (two words, so 2 r_c x 2 x N words per ciphertext). */
int mm_blind_rotate(mm_ctx *ctx, const int *table_ids, const uint32_t *ct_in, size_t count,
                    uint32_t steps, uint32_t *acc_out, uint32_t flags, void *stream);

/* One external product g^{-1}(in) x BSK (eq. def:gsw) for `count` RLWE pairs
 * in = [count][2][N] -> out, same layout, with RGSW key i < K n (key k of
 * coordinate j is i = j K + k). */
int mm_external_product(mm_ctx *ctx, uint32_t i, const uint32_t *in, size_t count, uint32_t *out,
                        uint32_t flags, void *stream);

/* Constant-term extraction (eq. equ-sam-extr) of `count` RLWE pairs
 * [count][2][N] -> [count][N+1]. */
int mm_sample_extract(mm_ctx *ctx, const uint32_t *rlwe, size_t count, uint32_t *lwe,
                      uint32_t flags, void *stream);

/* Key switch z -> s (eq. equ-key-swi) of `count` LWE_N ciphertexts at Q
 * [count][N+1] -> [count][n+1] at Q. */
int mm_keyswitch(mm_ctx *ctx, const uint32_t *lwe_N, size_t count, uint32_t *lwe_n,
                 uint32_t flags, void *stream);

/* The key switch of mm_keyswitch (with the final residues at Q) for callers
 * that cannot allocate device memory: code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc.  lwe_N and lwe_n are device
 * pointers ([count][N+1] and [count][n+1], the caller's), the call is
 * asynchronous on `stream` and calls no hipMalloc/hipFree nor any allocating
 * routine: the partial sums live in a fixed 64 MiB device array per GPU (held
 * until the process ends), so count * (n + 1) * 8 must not exceed 64 MiB
 * (MM_EINVAL otherwise; 13,290 samples at n = 630).  mm_device_init must have
 * run on the context (MM_ESTATE otherwise).  Every call on one GPU shares that
 * array: calls that overlap on one GPU (other streams, other contexts or
 * threads) race and must be serialised by the caller.  Same bits as
 * mm_keyswitch. */
int mm_keyswitch_noalloc(mm_ctx *ctx, const uint32_t *lwe_N, size_t count, uint32_t *lwe_n,
                         void *stream);

/* Negacyclic products a_c * b_c in Z_Q[x]/(x^N+1) through the device NTT:
 * a, b, out are [count][N]. */
int mm_negacyclic_mul(mm_ctx *ctx, const uint32_t *a, const uint32_t *b, size_t count,
                      uint32_t *out, uint32_t flags, void *stream);

/* ---- kernel timing ---- */

/* With enable != 0, every batched mm_bootstrap on ctx records HIP events on
 * its stream around the blind-rotation kernel and around the key-switch
 * kernels (inside the captured graph).  mm_last_timing waits for the events
 * of the last such call and returns both durations in milliseconds. */
int mm_set_timing(mm_ctx *ctx, int enable);
int mm_last_timing(mm_ctx *ctx, float *blind_rotate_ms, float *keyswitch_ms);

/* ---- autotuning ---- */

/* Time the kernel schedules that fit this batch shape (ciphertexts per
 * workgroup slot packing, waves per component, NTT stage schedule, key-switch
 * kernel and tiling) on the device and remember the fastest for the shape (N,
 * sum of r, count).  mm_bootstrap uses the remembered schedule.  *choice
 * receives the chosen schedule index.  Untuned batches at N = 1024 that leave
 * the device mostly idle (at most two components per compute unit, or four when
 * no two-wave slots fit), or that hold more than 16 components per compute unit,
 * take the global-accumulator shape with four waves per component (each
 * component a small workgroup of its own; up to two components per compute
 * unit, with two digit groups of four waves: NTT schedule 4 below); that
 * shape, with its usual and with
 * twice the waves (N = 512, 1024), is a candidate for every batch the fused
 * kernel holds.  A batch on the global-accumulator path
 * (see mm_params; the wide modulus among others) has one or two blind-rotation
 * shapes (two primes: one workgroup per component, or per component and
 * prime; N = 16384: one workgroup per component, or the split ring): this call
 * times each shape once, then each key switch on the extracted samples. */
int mm_autotune(mm_ctx *ctx, const int *table_ids, const uint32_t *ct_in, size_t count,
                int *choice);

/* Number of candidate schedules for this batch shape, and pinning one of
 * them (0 <= choice < *n) for the shape without timing; every schedule gives
 * identical results. */
int mm_schedule_count(mm_ctx *ctx, const int *table_ids, size_t count, int *n);
int mm_set_schedule(mm_ctx *ctx, const int *table_ids, size_t count, int choice);

/* What schedule `choice` of this batch shape is (choice < 0: the one in use):
 * waves per blind-rotation workgroup (8 or 4; 0 on the global-accumulator
 * path, one workgroup per component and CMux step), ciphertexts per wave of the
 * key switch (0 = the i-split key switch), the number of i splits, waves per
 * ring component (1 up to N = 1024 and N / 1024 above by default; 2 at N = 512
 * and 1024 for batches that do not fill the device, r <= 4; on the global path
 * the waves of its workgroup, N / 512 up to 4096 and N / 1024 above), the key-switch
 * kernel (0: i split over workgroups, per-thread sums; 1: KSK rows staged in
 * LDS, one output column per lane; 2: KSK rows staged in LDS, one ciphertext
 * per lane) and the NTT stage schedule of the blind rotation (0: every
 * cross-lane exchange through LDS, the two polynomials of an NTT in lockstep;
 * 1: the last exchange between NTT phases by wavefront lane swaps
 * (v_permlane16/32_swap), the others through LDS; 2: LDS exchanges with the two
 * polynomials staggered, one's relayout in flight while the other's
 * butterflies run; 3, global path only: the ring split into sub-rings of 8192,
 * the stages that mix them in separate launches; 4, the global-accumulator shape
 * at N = 1024 with one prime: two groups of four waves per component, each
 * taking every other gadget digit and one part's inverse NTT, for batches
 * that leave compute units idle; 5, the global-accumulator path with two primes:
 * one workgroup per component and prime, the default up to 16 components per
 * compute unit; 6, those workgroups with two digit groups, N = 1024 and 2048,
 * the default while all of them fit one per compute unit).  Any output pointer may be NULL. */
int mm_schedule_describe(mm_ctx *ctx, const int *table_ids, size_t count, int choice, int *group_waves,
                         int *ks_cts_per_wave, int *ks_splits, int *waves_per_component, int *ks_kernel,
                         int *ntt_schedule);

/* ---- serving: continuous batching ---- */

/* Start a server on ctx (one per context; MM_ESTATE if one runs).  It keeps as
 * many in-flight ciphertexts as their device state (accumulators, inputs,
 * outputs) fits in hbm_budget_bytes (MM_EINVAL below one 8-component group);
 * chunk_steps in [1, n].  Two partitions, one for requests of at most 4
 * components and one for wider ones, alternate launches; each launch advances
 * every resident ciphertext of its partition by chunk_steps CMux steps (2/3 of
 * that for the wider ones when a partition holds both kinds), so a request
 * admitted while others run joins them at the next launch.  At N = 1024 a tick
 * whose partition holds at most two components per compute unit (four when it
 * holds r = 8 ciphertexts) runs the global-accumulator kernels instead, with the
 * four waves per component of the batched path's default, two digit groups of them
 * up to two components per compute unit (the accumulators then
 * live in two arenas, so the budget counts 2 x 2 x N words per component at
 * N = 1024, 2 x N elsewhere).  Tables of general
 * f are not served, nor, at the default modulus and N <= 8192, tables with
 * r N/1024 > 8.  A context on the global-accumulator path (Q2 != 0, or
 * N = 16384) is served with that path's kernels: each launch ("tick") is
 * chunk_steps CMux launches over every resident component, each ciphertext at
 * its own step, with accumulators in two device arenas (rings up to 16384;
 * MM_EINVAL above; the budget then counts
 * 2 x 2 x N words per component and residue); any r up to 1024 whose block of
 * 2^ceil(log2 r) components fits the budget is served (MM_EINVAL at submission
 * otherwise).
 * The handle stays valid until mm_server_stop; mm_free of the context stops a
 * running server too, after which the handle must not be used. */
int mm_server_start(mm_ctx *ctx, size_t hbm_budget_bytes, uint32_t chunk_steps, mm_server **out);

/* Queue one ciphertext (n+1 words at its table's q_in, host memory).  The
 * result is at the table's q_in.  MM_EBUSY when the queue is full, MM_EINVAL
 * for a table the server does not take, MM_ESTATE once the serving loop has
 * stopped after a device error (mm_last_error of the context says which).
 * *ticket identifies the request for mm_poll. */
int mm_submit(mm_server *s, int table_id, const uint32_t *ct, uint64_t *ticket);

/* Copy the result of `ticket` into ct_out (n+1 words) once ready; MM_EAGAIN
 * before that, MM_ESTATE if the serving loop stopped before finishing it,
 * MM_EINVAL for a ticket never issued or already collected (a ticket can be
 * collected once). */
int mm_poll(mm_server *s, uint64_t ticket, uint32_t *ct_out);

/* Latency percentiles (submit to result ready, ms) over the last 2^20 completed
 * requests, and completed bootstraps per second since start. */
int mm_server_stats(mm_server *s, double *p50_ms, double *p99_ms, double *boots_per_s,
                    uint64_t *completed);

/* Admission by expected latency (load shedding): with max_latency_ms > 0,
 * mm_submit refuses a request with MM_EBUSY when the requests of its class (at
 * most 4 components, or wider) queued and in flight, divided by that class's
 * recent completion rate (its last 4096 completions, counted up to the time of
 * the call), exceed max_latency_ms: by Little's law the time a request admitted
 * now can expect to wait for its result.  The check starts after 64 completions
 * (all classes' requests and completions count until the request's class has
 * 64); 0 (the default) admits every request while the queue has room.
 * mm_server_refused reports how many requests admission has refused since the
 * server started. */
int mm_server_set_admission(mm_server *s, double max_latency_ms);
int mm_server_refused(mm_server *s, uint64_t *refused);

/* Stop the server after its in-flight work completes. */
int mm_server_stop(mm_server *s);

/* Replay a request trace: request k (table table_ids[k], ciphertext
 * ct_in + k(n+1)) arrives arrival_ns[k] ns after the call starts; the call
 * submits each at its time, collects every result into ct_out + k(n+1) and
 * latency_ms[k], and returns when all are done.  A request the queue cannot
 * take is submitted again until it can; with admission on
 * (mm_server_set_admission) a refused request is not retried: its latency is
 * -1 and its output words are zero. */
int mm_server_replay(mm_server *s, const int *table_ids, const uint32_t *ct_in,
                     const int64_t *arrival_ns, size_t count, uint32_t *ct_out,
                     double *latency_ms);

#ifdef __cplusplus
}
#endif

#endif /* MMPM_H */
