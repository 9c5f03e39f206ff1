/*
 * mmpm_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow CPU statement of the BootMMPM functional bootstrap
 * (Algorithm 1 of "Large-Plaintext Functional Bootstrapping in FHE with Small
 * Bootstrapping Keys", arXiv 2310.12441) for a binary or ternary LWE secret s
 * and a binary ring secret z.  It exists so that tests, the smoke check and the
 * benchmark's CPU baseline can check the HIP library against something that a
 * reader can compare with the paper line by line.  No product code may call
 * it, and it shares no code, header or table with the HIP library.
 *
 * Conventions (the readings of the paper that fix the output bit pattern):
 *   * Polynomials live in Z_Q[x]/(x^N+1) as N coefficients in [0, Q).
 *   * An RLWE pair is stored (a, b) with phase b - a*z (Sec. 2 item (12)).
 *   * An RLWE vector of dimension r is r such pairs: acc[j][part][N], part 0 = a,
 *     part 1 = b (Sec. 4, "r-dimensional RLWE vector").
 *   * An RGSW key is 2l rows, each an RLWE pair (a, b).  Rows u < l carry the
 *     message on b, rows l+u carry it on a: the phase of (def:phase3) with the
 *     matrix columns read as (b, a).  Digits of b multiply rows u < l and
 *     digits of a multiply rows l+u (eq. def:gsw).
 *   * The gadget is signed and possibly truncated: the centred residue is
 *     rounded to a multiple of 2^sg, sg = max(0, bits(Q) - l*log2 B), then split
 *     into l balanced base-B digits whose top digit absorbs the final carry
 *     (Sec. 2 item (10) uses unsigned exact digits; see the decomposition note).
 *   * Rounding x*q'/q is round-half-up: floor((2 x q' + q) / (2 q)) (item (9)).
 *
 * Every loop here is the literal definition: schoolbook negacyclic products
 * with int64 accumulation, explicit monomial matrices for the rotation, and
 * an explicit sum for the key switch.  There is no NTT in this file.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ----------------------------------------------------------------------- */
/* Integers mod Q                                                          */
/* ----------------------------------------------------------------------- */

static uint32_t mod_i64(int64_t x, uint32_t Q)
{
    int64_t r = x % (int64_t)Q;
    return (uint32_t)(r < 0 ? r + (int64_t)Q : r);
}

static uint32_t neg_mod(uint32_t x, uint32_t Q) { return x ? Q - x : 0; }

static uint32_t bits_of(uint32_t Q)
{
    uint32_t b = 0;
    while (b < 32 && (Q >> b)) b++;
    return b;
}

/* floor(a / b) for b > 0 and any sign of a */
static int64_t floor_div(int64_t a, int64_t b)
{
    int64_t q = a / b;
    if ((a % b != 0) && (a < 0)) q -= 1;
    return q;
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Modulus switch q_from -> q_to of one residue: round(x q_to / q_from), half up
 * (Sec. 2 item (9)). */
uint32_t orc_modswitch(uint32_t x, uint32_t q_from, uint32_t q_to)
{
    uint64_t num = 2ull * (uint64_t)x * (uint64_t)q_to + (uint64_t)q_from;
    return (uint32_t)((num / (2ull * (uint64_t)q_from)) % (uint64_t)q_to);
}

void orc_modswitch_vec(const uint32_t *in, uint64_t count, uint32_t q_from, uint32_t q_to,
                       uint32_t *out)
{
    for (uint64_t i = 0; i < count; i++) out[i] = orc_modswitch(in[i], q_from, q_to);
}

/* ----------------------------------------------------------------------- */
/* Negacyclic polynomials (Sec. 2 item (6): R_{N,Q} = Z_Q[x]/(x^N+1))      */
/* ----------------------------------------------------------------------- */

/* acc += small * big in Z[x]/(x^N+1), with |small| tiny so that int64 holds
 * the sum: x^j * x^m = x^(j+m) if j+m < N, else -x^(j+m-N). */
static void nega_mac_small(int64_t *acc, const int32_t *small, const uint32_t *big, uint32_t N)
{
    /* big < Q < 2^31, so it is also a non-negative int32 and each term is a
     * 32 x 32 -> 64-bit signed product */
    const int32_t *bigs = (const int32_t *)big;
    const int64_t n = (int64_t)N;
    for (int64_t j = 0; j < n; j++) {
        const int64_t d = small[j];
        if (d == 0) continue;
        const int32_t *lo = bigs - j;     /* lo[k] = big[k - j],     k >= j */
        const int32_t *hi = bigs + n - j; /* hi[k] = big[N + k - j], k <  j */
        for (int64_t k = j; k < n; k++) acc[k] += d * (int64_t)lo[k];
        for (int64_t k = 0; k < j; k++) acc[k] -= d * (int64_t)hi[k];
    }
}

/* out = a * b in Z_Q[x]/(x^N+1), both operands arbitrary residues. */
void orc_poly_mul(uint32_t N, uint32_t Q, const uint32_t *a, const uint32_t *b, uint32_t *out)
{
    for (uint32_t k = 0; k < N; k++) {
        uint64_t pos = 0, neg = 0;
        for (uint32_t j = 0; j <= k; j++) pos = (pos + (uint64_t)a[j] * b[k - j]) % Q;
        for (uint32_t j = k + 1; j < N; j++) neg = (neg + (uint64_t)a[j] * b[N + k - j]) % Q;
        out[k] = (uint32_t)((pos + Q - neg) % Q);
    }
}

/* out = x^e * p in Z_Q[x]/(x^N+1), any e >= 0 (x^(2N) = 1, x^N = -1). */
static void monomial_mul(uint64_t e, const uint32_t *p, uint32_t *out, uint32_t N, uint32_t Q)
{
    const uint64_t twoN = 2ull * N;
    for (uint32_t i = 0; i < N; i++) {
        uint64_t m = ((uint64_t)i + e) % twoN;
        if (m < N) out[m] = p[i];
        else out[m - N] = neg_mod(p[i], Q);
    }
}

void orc_monomial_mul(uint32_t N, uint32_t Q, uint64_t e, const uint32_t *p, uint32_t *out)
{
    monomial_mul(e, p, out, N, Q);
}

/* ----------------------------------------------------------------------- */
/* The MMPM representation Phi of Z_{2Nr} (Sec. 3, Example 1)             */
/* ----------------------------------------------------------------------- */

/* Entry (row j) of Phi(c) for c = a r + b, a in [2N], b in [r], by (ex1:BPc):
 * the top-right block x^(a+1) I_b puts, in row j < b, x^(a+1) at column
 * r - b + j; the bottom-left block x^a I_(r-b) puts, in row j >= b, x^a at
 * column j - b.  Returns the column and writes the exponent. */
static uint32_t phi_row(uint32_t r, uint64_t c, uint32_t N, uint32_t j, uint64_t *expo)
{
    const uint64_t M = 2ull * N * r;
    c %= M;
    const uint64_t a = c / r;
    const uint32_t b = (uint32_t)(c % r);
    if (j < b) {
        *expo = a + 1;
        return r - b + j;
    }
    *expo = a;
    return j - b;
}

/* Column index and exponent of row j of Phi(c), exported for the pins. */
uint32_t orc_phi_entry(uint32_t N, uint32_t r, uint64_t c, uint32_t j, uint64_t *expo)
{
    return phi_row(r, c, N, j, expo);
}

/* out = Phi(c) v for v in (Z_Q[x]/(x^N+1))^r stored as r polys of N:
 * out_j = x^(e_j) v_(col_j), the matrix-vector product with one monomial per row. */
void orc_rotate(uint32_t N, uint32_t r, uint32_t Q, uint64_t c, const uint32_t *v, uint32_t *out)
{
    for (uint32_t j = 0; j < r; j++) {
        uint64_t e;
        uint32_t col = phi_row(r, c, N, j, &e);
        monomial_mul(e, v + (size_t)col * N, out + (size_t)j * N, N, Q);
    }
}

/* ----------------------------------------------------------------------- */
/* Nega-cyclic extension and the test polynomial vector                    */
/* ----------------------------------------------------------------------- */

/* f'(x) on Z_M, M = 2Nr, Delta = M / t: x = m Delta + e with -Delta/2 <= e <
 * Delta/2 maps to f(m mod t) (Sec. 2 item (7); the boundary e = -Delta/2 that
 * the strict inequality leaves open is assigned by rounding half up). */
static uint32_t f_ext(uint64_t x, const uint32_t *f, uint32_t t, uint64_t M)
{
    const uint64_t D = M / t;
    const uint64_t m = ((x % M) + D / 2) / D;
    return f[m % t];
}

/* V = v_test * floor(Q / t'): entry b, coefficient a holds f'(-(a r + b)) as
 * its canonical residue in [0, t'), scaled by floor(Q/t') (eq. equ:test-use;
 * Alg. 1, phase accumulation initialisation). */
void orc_test_vector(uint32_t N, uint32_t r, uint32_t Q, uint32_t t, uint32_t t_out,
                     const uint32_t *f, uint32_t *V)
{
    const uint64_t M = 2ull * N * r;
    const uint64_t dq = Q / t_out;
    for (uint32_t b = 0; b < r; b++)
        for (uint32_t a = 0; a < N; a++) {
            const uint64_t p = (uint64_t)a * r + b;
            const uint32_t val = f_ext((M - p) % M, f, t, M) % t_out;
            V[(size_t)b * N + a] = (uint32_t)((dq * val) % Q);
        }
}

/* ----------------------------------------------------------------------- */
/* Gadget decomposition                                                    */
/* ----------------------------------------------------------------------- */

uint32_t orc_gadget_shift(uint32_t Q, uint32_t log2B, uint32_t l)
{
    const uint32_t used = l * log2B, bq = bits_of(Q);
    return bq > used ? bq - used : 0;
}

/* g_u = 2^(sg + u log2B) mod Q */
uint32_t orc_gadget(uint32_t Q, uint32_t log2B, uint32_t l, uint32_t u)
{
    const uint32_t e = orc_gadget_shift(Q, log2B, l) + u * log2B;
    uint64_t g = 1;
    for (uint32_t i = 0; i < e; i++) g = (g * 2) % Q;
    return (uint32_t)g;
}

/* Signed digits of x in [0, Q): sum_u d_u g_u = x - err (mod Q), |err| <= 2^(sg-1). */
void orc_decompose(uint32_t Q, uint32_t log2B, uint32_t l, uint32_t x, int32_t *d)
{
    const uint32_t sg = orc_gadget_shift(Q, log2B, l);
    const int64_t B = (int64_t)1 << log2B;
    const int64_t xc = (x > (Q - 1) / 2) ? (int64_t)x - (int64_t)Q : (int64_t)x;
    int64_t y = sg ? floor_div(xc + ((int64_t)1 << (sg - 1)), (int64_t)1 << sg) : xc;
    for (uint32_t u = 0; u + 1 < l; u++) {
        int64_t dig = ((y % B) + B) % B;
        y = (y - dig) / B;
        if (dig >= B / 2) {
            dig -= B;
            y += 1;
        }
        d[u] = (int32_t)dig;
    }
    d[l - 1] = (int32_t)y;
}

/* ----------------------------------------------------------------------- */
/* Keys (Alg. 1 inputs; Sec. 2 items (11), (14))                           */
/* ----------------------------------------------------------------------- */

/* RGSW_z(m) with m in {0,1} from masks a[2l][N] and errors e[2l][N]:
 * row u < l  : (a_u,               a_u z + e_u + m g_u)
 * row l + u  : (a_{l+u} + m g_u,   a_{l+u} z + e_{l+u})
 * out[row][part][N]. */
static void rgsw_encrypt(uint32_t N, uint32_t Q, uint32_t log2B, uint32_t l, uint32_t m,
                         const int32_t *z, const uint32_t *a, const int32_t *e, uint32_t *out)
{
    int64_t *acc = (int64_t *)malloc(sizeof(int64_t) * N);
    for (uint32_t row = 0; row < 2 * l; row++) {
        const uint32_t *ar = a + (size_t)row * N;
        const int32_t *er = e + (size_t)row * N;
        uint32_t *oa = out + ((size_t)row * 2 + 0) * N;
        uint32_t *ob = out + ((size_t)row * 2 + 1) * N;
        const uint32_t g = orc_gadget(Q, log2B, l, row % l);
        for (uint32_t k = 0; k < N; k++) acc[k] = er[k];
        nega_mac_small(acc, z, ar, N);
        for (uint32_t k = 0; k < N; k++) {
            oa[k] = ar[k];
            ob[k] = mod_i64(acc[k], Q);
        }
        if (m) {
            if (row < l) ob[0] = (uint32_t)(((uint64_t)ob[0] + g) % Q);
            else oa[0] = (uint32_t)(((uint64_t)oa[0] + g) % Q);
        }
    }
    free(acc);
}

/* Bootstrapping keys (Alg. 1 inputs).  keys = 1 (binary s): BSK_i = RGSW_z(s_i).
 * keys = 2 (ternary s): BSK_{i,0} = RGSW_z(s_i+), BSK_{i,1} = RGSW_z(s_i-),
 * s+ = max(s, 0), s- = max(-s, 0) (eq. d:pm).  bsk[i][key][row][part][N];
 * masks and errors bsk_a/bsk_e are [i][key][row][N]. */
void orc_keygen_bsk(uint32_t n, uint32_t N, uint32_t Q, uint32_t log2B, uint32_t l, uint32_t keys,
                    const int32_t *s, const uint32_t *z, const uint32_t *bsk_a, const int32_t *bsk_e,
                    uint32_t *bsk)
{
    int32_t *zi = (int32_t *)malloc(sizeof(int32_t) * N);
    for (uint32_t k = 0; k < N; k++) zi[k] = (int32_t)z[k];
    const size_t per = (size_t)2 * l * N;
#pragma omp parallel for schedule(dynamic)
    for (int64_t ik = 0; ik < (int64_t)n * keys; ik++) {
        const int64_t i = ik / keys, key = ik % keys;
        const uint32_t m = key == 0 ? (s[i] > 0 ? (uint32_t)s[i] : 0u) : (s[i] < 0 ? (uint32_t)(-s[i]) : 0u);
        rgsw_encrypt(N, Q, log2B, l, m, zi, bsk_a + (size_t)ik * per, bsk_e + (size_t)ik * per,
                     bsk + (size_t)ik * per * 2);
    }
    free(zi);
}

/* Key-switching keys KSK[i][j][v] = LWE_s(v z_i B_ks^j) in Z_Q^(n+1)
 * (Sec. 2 item (11), Alg. 1 inputs), digit value v = 0 included. */
void orc_keygen_ksk(uint32_t n, uint32_t N, uint32_t Q, uint32_t log2Bks, uint32_t lks,
                    const int32_t *s, const uint32_t *z, const uint32_t *ksk_a,
                    const int32_t *ksk_e, uint32_t *ksk)
{
    const uint32_t Bks = 1u << log2Bks;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < (int64_t)N; i++) {
        uint64_t pw = 1; /* B_ks^j mod Q */
        for (uint32_t j = 0; j < lks; j++) {
            for (uint32_t v = 0; v < Bks; v++) {
                const size_t row = ((size_t)i * lks + j) * Bks + v;
                const uint32_t *al = ksk_a + row * n;
                uint32_t *o = ksk + row * (n + 1);
                int64_t dot = 0;
                for (uint32_t k = 0; k < n; k++) {
                    o[k] = al[k];
                    dot = (dot + (int64_t)al[k] * s[k]) % (int64_t)Q;
                }
                const uint64_t msg = ((uint64_t)v * z[i] % Q) * pw % Q;
                o[n] = mod_i64(dot + ksk_e[row] + (int64_t)msg, Q);
            }
            pw = pw * Bks % Q;
        }
    }
}

/* ----------------------------------------------------------------------- */
/* LWE encryption / decryption (Sec. 2 item (8))                           */
/* ----------------------------------------------------------------------- */

/* b = <a, s> + m floor(q/t) + e mod q; ct[i] = (a_0..a_{n-1}, b). */
/* <a, s> mod q for an integer secret */
static int64_t dot_mod(const uint32_t *a, const int32_t *s, uint32_t n, uint32_t q)
{
    int64_t dot = 0;
    for (uint32_t k = 0; k < n; k++) dot = (dot + (int64_t)a[k] * s[k]) % (int64_t)q;
    return dot < 0 ? dot + q : dot;
}

void orc_encrypt(uint32_t n, uint32_t q, uint32_t t, const int32_t *s, const uint32_t *m,
                 const uint32_t *a, const int32_t *e, uint64_t count, uint32_t *ct)
{
    const uint64_t delta = q / t;
    for (uint64_t c = 0; c < count; c++) {
        const uint32_t *ac = a + c * n;
        uint32_t *o = ct + c * (n + 1);
        for (uint32_t k = 0; k < n; k++) o[k] = ac[k];
        const int64_t dot = dot_mod(ac, s, n, q);
        const int64_t b = dot + (int64_t)((m[c] % t) * delta % q) + e[c];
        o[n] = mod_i64(b, q);
    }
}

/* phase = b - <a, s> mod q = m floor(q/t) + e; m = round(phase / floor(q/t)) mod t. */
void orc_decrypt(uint32_t n, uint32_t q, uint32_t t, const int32_t *s, const uint32_t *ct,
                 uint64_t count, uint32_t *m)
{
    const uint64_t delta = q / t;
    for (uint64_t c = 0; c < count; c++) {
        const uint32_t *o = ct + c * (n + 1);
        const uint64_t dot = (uint64_t)dot_mod(o, s, n, q);
        const uint64_t ph = ((uint64_t)o[n] + q - dot) % q;
        m[c] = (uint32_t)(((ph + delta / 2) / delta) % t);
    }
}

/* phase of an LWE ciphertext, for noise measurements */
void orc_lwe_phase(uint32_t n, uint32_t q, const int32_t *s, const uint32_t *ct, uint64_t count,
                   uint32_t *phase)
{
    for (uint64_t c = 0; c < count; c++) {
        const uint32_t *o = ct + c * (n + 1);
        const uint64_t dot = (uint64_t)dot_mod(o, s, n, q);
        phase[c] = (uint32_t)(((uint64_t)o[n] + q - dot) % q);
    }
}

/* ----------------------------------------------------------------------- */
/* External product and the blind rotation (Sec. 4, Alg. 1)                */
/* ----------------------------------------------------------------------- */

/* out = g^{-1}(in) * C for one RLWE pair in = (a, b) and RGSW C[2l][2][N]
 * (eq. def:gsw): sum_u dec(b)_u C[u] + sum_u dec(a)_u C[l+u]. */
void orc_external_product(uint32_t N, uint32_t Q, uint32_t log2B, uint32_t l,
                          const uint32_t *rgsw, const uint32_t *in, uint32_t *out)
{
    int32_t *dig = (int32_t *)malloc(sizeof(int32_t) * (size_t)2 * l * N);
    int64_t *acc = (int64_t *)calloc((size_t)2 * N, sizeof(int64_t));
    int32_t tmp[64];
    /* dig[u] = digit u of b, dig[l+u] = digit u of a */
    for (uint32_t k = 0; k < N; k++) {
        orc_decompose(Q, log2B, l, in[N + k], tmp);
        for (uint32_t u = 0; u < l; u++) dig[(size_t)u * N + k] = tmp[u];
        orc_decompose(Q, log2B, l, in[k], tmp);
        for (uint32_t u = 0; u < l; u++) dig[(size_t)(l + u) * N + k] = tmp[u];
    }
    for (uint32_t row = 0; row < 2 * l; row++)
        for (uint32_t part = 0; part < 2; part++)
            nega_mac_small(acc + (size_t)part * N, dig + (size_t)row * N,
                           rgsw + ((size_t)row * 2 + part) * N, N);
    for (uint32_t k = 0; k < 2 * N; k++) out[k] = mod_i64(acc[k], Q);
    free(dig);
    free(acc);
}

/* ACC <- Phi(b')(0, V); then for i < steps the CMux of eq. (cmux:BP):
 * ACC <- ACC + (Phi(-a'_i) ACC - ACC) x BSK_{i,0} [+ (Phi(a'_i) ACC - ACC) x BSK_{i,1}],
 * the second term only for a ternary secret (keys = 2), both computed from the
 * same ACC.  ct_ms holds (a'_0..a'_{n-1}, b') in Z_{2Nr}.  acc[j][part][N]. */
static void blind_rotate(uint32_t n, uint32_t N, uint32_t Q, uint32_t log2B, uint32_t l,
                         uint32_t r, uint32_t keys, const uint32_t *bsk, const uint32_t *V,
                         const uint32_t *ct_ms, uint32_t steps, uint32_t *acc, int parallel)
{
    const uint64_t M = 2ull * N * r;
    const size_t comp = (size_t)2 * N;
    uint32_t *rv = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)r * N);
    uint32_t *ra = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)r * N);
    uint32_t *rb = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)r * N);
    uint32_t *D = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)keys * r * comp);

    /* ACC <- Phi(b') (0, V) */
    orc_rotate(N, r, Q, ct_ms[n] % M, V, rv);
    for (uint32_t j = 0; j < r; j++) {
        memset(acc + j * comp, 0, sizeof(uint32_t) * N);
        memcpy(acc + j * comp + N, rv + (size_t)j * N, sizeof(uint32_t) * N);
    }

    for (uint32_t i = 0; i < steps && i < n; i++) {
        for (uint32_t key = 0; key < keys; key++) {
            /* key 0: c = -a'_i (the s+ term); key 1: c = +a'_i (the s- term) */
            const uint64_t a = ct_ms[i] % M;
            const uint64_t c = key == 0 ? (M - a) % M : a;
            for (uint32_t j = 0; j < r; j++) memcpy(rv + (size_t)j * N, acc + j * comp, sizeof(uint32_t) * N);
            orc_rotate(N, r, Q, c, rv, ra);
            for (uint32_t j = 0; j < r; j++) memcpy(rv + (size_t)j * N, acc + j * comp + N, sizeof(uint32_t) * N);
            orc_rotate(N, r, Q, c, rv, rb);
            uint32_t *Dk = D + (size_t)key * r * comp;
            for (uint32_t j = 0; j < r; j++)
                for (uint32_t k = 0; k < N; k++) {
                    Dk[j * comp + k] = (ra[(size_t)j * N + k] + Q - acc[j * comp + k]) % Q;
                    Dk[j * comp + N + k] = (rb[(size_t)j * N + k] + Q - acc[j * comp + N + k]) % Q;
                }
        }
#pragma omp parallel for schedule(static) if (parallel)
        for (int64_t j = 0; j < (int64_t)r; j++) {
            uint32_t *prod = (uint32_t *)malloc(sizeof(uint32_t) * comp);
            for (uint32_t key = 0; key < keys; key++) {
                const uint32_t *rgsw = bsk + ((size_t)i * keys + key) * 2 * l * 2 * N;
                orc_external_product(N, Q, log2B, l, rgsw, D + (size_t)key * r * comp + j * comp, prod);
                for (uint32_t k = 0; k < 2 * N; k++)
                    acc[j * comp + k] = (uint32_t)(((uint64_t)acc[j * comp + k] + prod[k]) % Q);
            }
            free(prod);
        }
    }
    free(rv);
    free(ra);
    free(rb);
    free(D);
}

void orc_blind_rotate(uint32_t n, uint32_t N, uint32_t Q, uint32_t log2B, uint32_t l, uint32_t r,
                      uint32_t keys, const uint32_t *bsk, const uint32_t *V, const uint32_t *ct_ms,
                      uint32_t steps, uint32_t *acc)
{
    blind_rotate(n, N, Q, log2B, l, r, keys, bsk, V, ct_ms, steps, acc, 1);
}

/* Constant-term extraction of (A, B) (eq. equ-sam-extr):
 * (A_0, -A_{N-1}, ..., -A_1; B_0). */
void orc_sample_extract(uint32_t N, uint32_t Q, const uint32_t *rlwe, uint32_t *lwe)
{
    lwe[0] = rlwe[0];
    for (uint32_t k = 1; k < N; k++) lwe[k] = neg_mod(rlwe[N - k], Q);
    lwe[N] = rlwe[N];
}

/* Key switch z -> s (eq. equ-key-swi): (0^n, b) - sum_{i<N, j<l_ks} KSK[i][j][d_ij],
 * d_ij = floor(A_i / B_ks^j) mod B_ks. */
void orc_keyswitch(uint32_t n, uint32_t N, uint32_t Q, uint32_t log2Bks, uint32_t lks,
                   const uint32_t *ksk, const uint32_t *lwe_N, uint32_t *lwe_n)
{
    const uint64_t Bks = 1ull << log2Bks;
    uint64_t *acc = (uint64_t *)calloc((size_t)n + 1, sizeof(uint64_t));
    for (uint32_t i = 0; i < N; i++) {
        uint64_t pw = 1;
        for (uint32_t j = 0; j < lks; j++) {
            const uint64_t d = ((uint64_t)lwe_N[i] / pw) % Bks;
            const uint32_t *row = ksk + (((size_t)i * lks + j) * Bks + d) * (n + 1);
            for (uint32_t k = 0; k <= n; k++) acc[k] = (acc[k] + row[k]) % Q;
            pw *= Bks;
        }
    }
    for (uint32_t k = 0; k < n; k++) lwe_n[k] = neg_mod((uint32_t)acc[k], Q);
    lwe_n[n] = (uint32_t)(((uint64_t)lwe_N[N] + Q - acc[n]) % Q);
    free(acc);
}

/* ----------------------------------------------------------------------- */
/* Algorithm 1 end to end                                                  */
/* ----------------------------------------------------------------------- */

/* BootMMPM(ct, f) for one ciphertext at modulus q_in.
 * steps: ModulusSwitch q_in -> 2Nr; ACC init; n CMux steps; SampleExtract of
 * entry 0; KeySwitch; ModulusSwitch Q -> q_out (skipped when q_out == Q).
 * Optional outputs (NULL to skip): acc_out (r*2*N), ext_out (N+1), ks_out (n+1). */
static void bootstrap_one(uint32_t n, uint32_t N, uint32_t Q, uint32_t log2B, uint32_t l,
                          uint32_t log2Bks, uint32_t lks, uint32_t r, uint32_t keys, const uint32_t *bsk,
                          const uint32_t *ksk, const uint32_t *V, uint32_t q_in,
                          uint32_t q_out, const uint32_t *ct, uint32_t *out,
                          uint32_t *acc_out, uint32_t *ext_out, uint32_t *ks_out, int parallel)
{
    const uint32_t M = 2u * N * r;
    uint32_t *ms = (uint32_t *)malloc(sizeof(uint32_t) * (n + 1));
    uint32_t *acc = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)r * 2 * N);
    uint32_t *ext = (uint32_t *)malloc(sizeof(uint32_t) * (N + 1));
    uint32_t *ks = (uint32_t *)malloc(sizeof(uint32_t) * (n + 1));
    orc_modswitch_vec(ct, n + 1, q_in, M, ms);
    blind_rotate(n, N, Q, log2B, l, r, keys, bsk, V, ms, n, acc, parallel);
    orc_sample_extract(N, Q, acc, ext);
    orc_keyswitch(n, N, Q, log2Bks, lks, ksk, ext, ks);
    if (q_out == Q) memcpy(out, ks, sizeof(uint32_t) * (n + 1));
    else orc_modswitch_vec(ks, n + 1, Q, q_out, out);
    if (acc_out) memcpy(acc_out, acc, sizeof(uint32_t) * (size_t)r * 2 * N);
    if (ext_out) memcpy(ext_out, ext, sizeof(uint32_t) * (N + 1));
    if (ks_out) memcpy(ks_out, ks, sizeof(uint32_t) * (n + 1));
    free(ms);
    free(acc);
    free(ext);
    free(ks);
}

void orc_bootstrap(uint32_t n, uint32_t N, uint32_t Q, uint32_t log2B, uint32_t l,
                   uint32_t log2Bks, uint32_t lks, uint32_t r, uint32_t keys, const uint32_t *bsk,
                   const uint32_t *ksk, const uint32_t *V, uint32_t q_in, uint32_t q_out,
                   const uint32_t *ct, uint32_t *out, uint32_t *acc_out, uint32_t *ext_out,
                   uint32_t *ks_out)
{
    bootstrap_one(n, N, Q, log2B, l, log2Bks, lks, r, keys, bsk, ksk, V, q_in, q_out, ct, out,
                  acc_out, ext_out, ks_out, 1);
}

/* Many ciphertexts of one table, one thread per ciphertext. */
void orc_bootstrap_many(uint32_t n, uint32_t N, uint32_t Q, uint32_t log2B, uint32_t l,
                        uint32_t log2Bks, uint32_t lks, uint32_t r, uint32_t keys, const uint32_t *bsk,
                        const uint32_t *ksk, const uint32_t *V, uint32_t q_in, uint32_t q_out,
                        const uint32_t *ct, uint64_t count, uint32_t *out)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t c = 0; c < (int64_t)count; c++)
        bootstrap_one(n, N, Q, log2B, l, log2Bks, lks, r, keys, bsk, ksk, V, q_in, q_out,
                      ct + (size_t)c * (n + 1), out + (size_t)c * (n + 1), NULL, NULL, NULL, 0);
}

/* ----------------------------------------------------------------------- */
/* A function that is not nega-cyclic: two bootstraps (Sec. 4, end)       */
/* ----------------------------------------------------------------------- */

/* For f: Z_t -> Z_t' arbitrary, the ciphertext carries x = m + b t in Z_2t,
 * m in [0, t), b an unknown top bit.  The two nega-cyclic tables on Z_2t:
 *   g(x) = t/2 for x in [0, t), -t/2 for x in [t, 2t)   (the sign of x, times t/2)
 *   F(y) = f(y) for y in [0, t), -f(y - t) for y in [t, 2t)   (mod t').
 * g is not the sign table of eq. (rel:mp) as printed: that table is -t/2 on
 * [-t/2, t/2) and t/2 on the rest of [-t, t), so it plus t/2 (eq. rel:sign) is
 * 0 or t according to |x| < t/2, not to the top bit.  g is that table moved by
 * t/2, g(x) = -mp(x - t/2), which is t/2 exactly when b = 0; then
 * x + g(x) - t/2 = m + b t + (t/2 - b t) - t/2 = m for both values of b.
 * Outputs g[2t] in Z_2t and F[2t] in Z_t'. */
void orc_general_tables(uint32_t t, uint32_t t_out, const uint32_t *f, uint32_t *g, uint32_t *F)
{
    for (uint32_t x = 0; x < 2 * t; x++) {
        g[x] = x < t ? t / 2 : 2 * t - t / 2;
        F[x] = x < t ? f[x] % t_out : (t_out - f[x - t] % t_out) % t_out;
    }
}

/* f(m) from Enc_{2t}(m + b t) at modulus q: bootstrap with g (output at q,
 * plaintext modulus 2t), ct' = ct + ct_g - (0, (t/2) floor(q/2t)) so that
 * ct' encrypts x - b t = m, then bootstrap ct' with F (output at q_out). */
void orc_bootstrap_general(uint32_t n, uint32_t N, uint32_t Q, uint32_t log2B, uint32_t l,
                           uint32_t log2Bks, uint32_t lks, uint32_t r, uint32_t keys, const uint32_t *bsk,
                           const uint32_t *ksk, const uint32_t *Vg, const uint32_t *VF, uint32_t q,
                           uint32_t t, uint32_t q_out, const uint32_t *ct, uint32_t *out)
{
    uint32_t *ctg = (uint32_t *)malloc(sizeof(uint32_t) * (n + 1));
    uint32_t *ct2 = (uint32_t *)malloc(sizeof(uint32_t) * (n + 1));
    bootstrap_one(n, N, Q, log2B, l, log2Bks, lks, r, keys, bsk, ksk, Vg, q, q, ct, ctg, NULL, NULL, NULL, 1);
    const uint64_t shift = (uint64_t)(t / 2) * (q / (2 * t)) % q;
    for (uint32_t k = 0; k <= n; k++) ct2[k] = (uint32_t)(((uint64_t)ct[k] + ctg[k]) % q);
    ct2[n] = (uint32_t)(((uint64_t)ct2[n] + q - shift) % q);
    bootstrap_one(n, N, Q, log2B, l, log2Bks, lks, r, keys, bsk, ksk, VF, q, q_out, ct2, out, NULL, NULL,
                  NULL, 1);
    free(ctg);
    free(ct2);
}

/* ----------------------------------------------------------------------- */
/* A wide ring modulus (Sec. 5 experiments: log Q = 54, B = 2^15)          */
/* ----------------------------------------------------------------------- */

/* The same steps with the ring modulus Q_w up to 2^62 held as one uint64 per
 * coefficient (no residue-number split here: Q_w is a single integer).  The
 * LWE side stays 32-bit: after extraction each coefficient is switched from
 * Q_w to the key-switch modulus Q_ks (< 2^31) by rounding, then the key switch
 * and the final switch are the functions above.  Products are reduced with
 * 128-bit integers. */

typedef unsigned __int128 w_u128;
typedef __int128 w_i128;

static uint64_t w_mod(w_i128 x, uint64_t Q)
{
    w_i128 r = x % (w_i128)Q;
    return (uint64_t)(r < 0 ? r + (w_i128)Q : r);
}

static uint64_t w_neg(uint64_t x, uint64_t Q) { return x ? Q - x : 0; }

static uint32_t w_bits(uint64_t Q)
{
    uint32_t b = 0;
    while (b < 64 && (Q >> b)) b++;
    return b;
}

/* out = a * b in Z_Q[x]/(x^N+1), every product reduced mod Q. */
void orc_w_poly_mul(uint32_t N, uint64_t Q, const uint64_t *a, const uint64_t *b, uint64_t *out)
{
    for (uint32_t k = 0; k < N; k++) {
        w_u128 pos = 0, neg = 0;
        for (uint32_t j = 0; j <= k; j++) pos += (w_u128)a[j] * b[k - j] % Q;
        for (uint32_t j = k + 1; j < N; j++) neg += (w_u128)a[j] * b[N + k - j] % Q;
        out[k] = w_mod((w_i128)(pos % Q) - (w_i128)(neg % Q), Q);
    }
}

/* acc += small * big in Z[x]/(x^N+1) with 128-bit accumulators (|small| < 2^31). */
static void w_nega_mac_small(w_i128 *acc, const int64_t *small, const uint64_t *big, uint32_t N)
{
    for (uint32_t j = 0; j < N; j++) {
        const w_i128 d = small[j];
        if (d == 0) continue;
        for (uint32_t k = j; k < N; k++) acc[k] += d * (w_i128)big[k - j];
        for (uint32_t k = 0; k < j; k++) acc[k] -= d * (w_i128)big[N + k - j];
    }
}

static void w_monomial_mul(uint64_t e, const uint64_t *p, uint64_t *out, uint32_t N, uint64_t Q)
{
    const uint64_t twoN = 2ull * N;
    for (uint32_t i = 0; i < N; i++) {
        uint64_t m = ((uint64_t)i + e) % twoN;
        if (m < N) out[m] = p[i];
        else out[m - N] = w_neg(p[i], Q);
    }
}

/* out = Phi(c) v, the rows of (ex1:BPc) as in orc_rotate. */
void orc_w_rotate(uint32_t N, uint32_t r, uint64_t Q, uint64_t c, const uint64_t *v, uint64_t *out)
{
    for (uint32_t j = 0; j < r; j++) {
        uint64_t e;
        uint32_t col = phi_row(r, c, N, j, &e);
        w_monomial_mul(e, v + (size_t)col * N, out + (size_t)j * N, N, Q);
    }
}

/* V = v_test * floor(Q / t') (eq. equ:test-use) at the wide modulus. */
void orc_w_test_vector(uint32_t N, uint32_t r, uint64_t Q, uint32_t t, uint32_t t_out,
                       const uint32_t *f, uint64_t *V)
{
    const uint64_t M = 2ull * N * r;
    const uint64_t dq = Q / t_out;
    for (uint32_t b = 0; b < r; b++)
        for (uint32_t a = 0; a < N; a++) {
            const uint64_t p = (uint64_t)a * r + b;
            const uint32_t val = f_ext((M - p) % M, f, t, M) % t_out;
            V[(size_t)b * N + a] = (uint64_t)((w_u128)dq * val % Q);
        }
}

uint32_t orc_w_gadget_shift(uint64_t Q, uint32_t log2B, uint32_t l)
{
    const uint32_t used = l * log2B, bq = w_bits(Q);
    return bq > used ? bq - used : 0;
}

/* g_u = 2^(sg + u log2B) mod Q */
uint64_t orc_w_gadget(uint64_t Q, uint32_t log2B, uint32_t l, uint32_t u)
{
    const uint32_t e = orc_w_gadget_shift(Q, log2B, l) + u * log2B;
    uint64_t g = 1 % Q;
    for (uint32_t i = 0; i < e; i++) g = (uint64_t)((w_u128)g * 2 % Q);
    return g;
}

/* Signed digits of x in [0, Q): the centred lift rounded to a multiple of
 * 2^sg, then l balanced base-B digits, the top one keeping the carry. */
void orc_w_decompose(uint64_t Q, uint32_t log2B, uint32_t l, uint64_t x, int64_t *d)
{
    const uint32_t sg = orc_w_gadget_shift(Q, log2B, l);
    const w_i128 B = (w_i128)1 << log2B;
    const w_i128 xc = (x > (Q - 1) / 2) ? (w_i128)x - (w_i128)Q : (w_i128)x;
    w_i128 y = xc;
    if (sg) {
        const w_i128 den = (w_i128)1 << sg, num = xc + ((w_i128)1 << (sg - 1));
        y = num / den;
        if (num % den != 0 && num < 0) y -= 1; /* floor */
    }
    for (uint32_t u = 0; u + 1 < l; u++) {
        w_i128 dig = ((y % B) + B) % B;
        y = (y - dig) / B;
        if (dig >= B / 2) {
            dig -= B;
            y += 1;
        }
        d[u] = (int64_t)dig;
    }
    d[l - 1] = (int64_t)y;
}

/* RGSW_z(m), m in {0,1}, rows as in rgsw_encrypt, at the wide modulus. */
static void w_rgsw_encrypt(uint32_t N, uint64_t Q, uint32_t log2B, uint32_t l, uint32_t m,
                           const int64_t *z, const uint64_t *a, const int32_t *e, uint64_t *out)
{
    w_i128 *acc = (w_i128 *)malloc(sizeof(w_i128) * N);
    for (uint32_t row = 0; row < 2 * l; row++) {
        const uint64_t *ar = a + (size_t)row * N;
        const int32_t *er = e + (size_t)row * N;
        uint64_t *oa = out + ((size_t)row * 2 + 0) * N;
        uint64_t *ob = out + ((size_t)row * 2 + 1) * N;
        const uint64_t g = orc_w_gadget(Q, log2B, l, row % l);
        for (uint32_t k = 0; k < N; k++) acc[k] = er[k];
        w_nega_mac_small(acc, z, ar, N);
        for (uint32_t k = 0; k < N; k++) {
            oa[k] = ar[k];
            ob[k] = w_mod(acc[k], Q);
        }
        if (m) {
            if (row < l) ob[0] = (uint64_t)(((w_u128)ob[0] + g) % Q);
            else oa[0] = (uint64_t)(((w_u128)oa[0] + g) % Q);
        }
    }
    free(acc);
}

/* Bootstrapping keys at the wide modulus, same layout and key rule as
 * orc_keygen_bsk: bsk[i][key][row][part][N], masks bsk_a in [0, Q). */
void orc_w_keygen_bsk(uint32_t n, uint32_t N, uint64_t Q, uint32_t log2B, uint32_t l, uint32_t keys,
                      const int32_t *s, const uint32_t *z, const uint64_t *bsk_a, const int32_t *bsk_e,
                      uint64_t *bsk)
{
    int64_t *zi = (int64_t *)malloc(sizeof(int64_t) * N);
    for (uint32_t k = 0; k < N; k++) zi[k] = (int64_t)z[k];
    const size_t per = (size_t)2 * l * N;
#pragma omp parallel for schedule(dynamic)
    for (int64_t ik = 0; ik < (int64_t)n * keys; ik++) {
        const int64_t i = ik / keys, key = ik % keys;
        const uint32_t m = key == 0 ? (s[i] > 0 ? (uint32_t)s[i] : 0u) : (s[i] < 0 ? (uint32_t)(-s[i]) : 0u);
        w_rgsw_encrypt(N, Q, log2B, l, m, zi, bsk_a + (size_t)ik * per, bsk_e + (size_t)ik * per,
                       bsk + (size_t)ik * per * 2);
    }
    free(zi);
}

/* out = g^{-1}(in) * C (eq. def:gsw) at the wide modulus. */
void orc_w_external_product(uint32_t N, uint64_t Q, uint32_t log2B, uint32_t l,
                            const uint64_t *rgsw, const uint64_t *in, uint64_t *out)
{
    int64_t *dig = (int64_t *)malloc(sizeof(int64_t) * (size_t)2 * l * N);
    w_i128 *acc = (w_i128 *)calloc((size_t)2 * N, sizeof(w_i128));
    int64_t tmp[64];
    for (uint32_t k = 0; k < N; k++) {
        orc_w_decompose(Q, log2B, l, in[N + k], tmp);
        for (uint32_t u = 0; u < l; u++) dig[(size_t)u * N + k] = tmp[u];
        orc_w_decompose(Q, log2B, l, in[k], tmp);
        for (uint32_t u = 0; u < l; u++) dig[(size_t)(l + u) * N + k] = tmp[u];
    }
    for (uint32_t row = 0; row < 2 * l; row++)
        for (uint32_t part = 0; part < 2; part++)
            w_nega_mac_small(acc + (size_t)part * N, dig + (size_t)row * N,
                             rgsw + ((size_t)row * 2 + part) * N, N);
    for (uint32_t k = 0; k < 2 * N; k++) out[k] = w_mod(acc[k], Q);
    free(dig);
    free(acc);
}

/* The blind rotation of Alg. 1 at the wide modulus (as blind_rotate above). */
static void w_blind_rotate(uint32_t n, uint32_t N, uint64_t Q, uint32_t log2B, uint32_t l,
                           uint32_t r, uint32_t keys, const uint64_t *bsk, const uint64_t *V,
                           const uint32_t *ct_ms, uint32_t steps, uint64_t *acc, int parallel)
{
    const uint64_t M = 2ull * N * r;
    const size_t comp = (size_t)2 * N;
    uint64_t *rv = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)r * N);
    uint64_t *ra = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)r * N);
    uint64_t *rb = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)r * N);
    uint64_t *D = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)keys * r * comp);

    orc_w_rotate(N, r, Q, ct_ms[n] % M, V, rv);
    for (uint32_t j = 0; j < r; j++) {
        memset(acc + j * comp, 0, sizeof(uint64_t) * N);
        memcpy(acc + j * comp + N, rv + (size_t)j * N, sizeof(uint64_t) * N);
    }
    for (uint32_t i = 0; i < steps && i < n; i++) {
        for (uint32_t key = 0; key < keys; key++) {
            const uint64_t a = ct_ms[i] % M;
            const uint64_t c = key == 0 ? (M - a) % M : a;
            for (uint32_t j = 0; j < r; j++) memcpy(rv + (size_t)j * N, acc + j * comp, sizeof(uint64_t) * N);
            orc_w_rotate(N, r, Q, c, rv, ra);
            for (uint32_t j = 0; j < r; j++) memcpy(rv + (size_t)j * N, acc + j * comp + N, sizeof(uint64_t) * N);
            orc_w_rotate(N, r, Q, c, rv, rb);
            uint64_t *Dk = D + (size_t)key * r * comp;
            for (uint32_t j = 0; j < r; j++)
                for (uint32_t k = 0; k < N; k++) {
                    Dk[j * comp + k] = w_mod((w_i128)ra[(size_t)j * N + k] - (w_i128)acc[j * comp + k], Q);
                    Dk[j * comp + N + k] = w_mod((w_i128)rb[(size_t)j * N + k] - (w_i128)acc[j * comp + N + k], Q);
                }
        }
#pragma omp parallel for schedule(static) if (parallel)
        for (int64_t j = 0; j < (int64_t)r; j++) {
            uint64_t *prod = (uint64_t *)malloc(sizeof(uint64_t) * comp);
            for (uint32_t key = 0; key < keys; key++) {
                const uint64_t *rgsw = bsk + ((size_t)i * keys + key) * 2 * l * 2 * N;
                orc_w_external_product(N, Q, log2B, l, rgsw, D + (size_t)key * r * comp + j * comp, prod);
                for (uint32_t k = 0; k < 2 * N; k++)
                    acc[j * comp + k] = (uint64_t)(((w_u128)acc[j * comp + k] + prod[k]) % Q);
            }
            free(prod);
        }
    }
    free(rv);
    free(ra);
    free(rb);
    free(D);
}

void orc_w_blind_rotate(uint32_t n, uint32_t N, uint64_t Q, uint32_t log2B, uint32_t l, uint32_t r,
                        uint32_t keys, const uint64_t *bsk, const uint64_t *V, const uint32_t *ct_ms,
                        uint32_t steps, uint64_t *acc)
{
    w_blind_rotate(n, N, Q, log2B, l, r, keys, bsk, V, ct_ms, steps, acc, 1);
}

/* round(x q_to / Q_from), half up (Sec. 2 item (9)), for Q_from up to 2^62. */
uint64_t orc_w_modswitch(uint64_t x, uint64_t Q_from, uint64_t q_to)
{
    const w_u128 num = (w_u128)2 * x * q_to + Q_from;
    return (uint64_t)((num / ((w_u128)2 * Q_from)) % q_to);
}

/* Constant-term extraction (eq. equ-sam-extr) of a wide RLWE pair. */
void orc_w_sample_extract(uint32_t N, uint64_t Q, const uint64_t *rlwe, uint64_t *lwe)
{
    lwe[0] = rlwe[0];
    for (uint32_t k = 1; k < N; k++) lwe[k] = w_neg(rlwe[N - k], Q);
    lwe[N] = rlwe[N];
}

/* BootMMPM(ct, f) with the wide ring modulus: modulus switch q_in -> 2Nr; ACC
 * init; n CMux steps at Q_w; extraction; each coefficient switched Q_w -> Q_ks;
 * key switch at Q_ks; switch Q_ks -> q_out (skipped when q_out == Q_ks). */
static void w_bootstrap_one(uint32_t n, uint32_t N, uint64_t Qw, uint32_t log2B, uint32_t l, uint32_t Qks,
                            uint32_t log2Bks, uint32_t lks, uint32_t r, uint32_t keys, const uint64_t *bsk,
                            const uint32_t *ksk, const uint64_t *V, uint32_t q_in, uint32_t q_out,
                            const uint32_t *ct, uint32_t *out, uint32_t *ext_out, int parallel)
{
    const uint32_t M = 2u * N * r;
    uint32_t *ms = (uint32_t *)malloc(sizeof(uint32_t) * (n + 1));
    uint64_t *acc = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)r * 2 * N);
    uint64_t *ext = (uint64_t *)malloc(sizeof(uint64_t) * (N + 1));
    uint32_t *ext32 = (uint32_t *)malloc(sizeof(uint32_t) * (N + 1));
    uint32_t *ks = (uint32_t *)malloc(sizeof(uint32_t) * (n + 1));
    orc_modswitch_vec(ct, n + 1, q_in, M, ms);
    w_blind_rotate(n, N, Qw, log2B, l, r, keys, bsk, V, ms, n, acc, parallel);
    orc_w_sample_extract(N, Qw, acc, ext);
    for (uint32_t k = 0; k <= N; k++) ext32[k] = (uint32_t)orc_w_modswitch(ext[k], Qw, Qks);
    orc_keyswitch(n, N, Qks, log2Bks, lks, ksk, ext32, ks);
    if (q_out == Qks) memcpy(out, ks, sizeof(uint32_t) * (n + 1));
    else orc_modswitch_vec(ks, n + 1, Qks, q_out, out);
    if (ext_out) memcpy(ext_out, ext32, sizeof(uint32_t) * (N + 1));
    free(ms);
    free(acc);
    free(ext);
    free(ext32);
    free(ks);
}

void orc_w_bootstrap(uint32_t n, uint32_t N, uint64_t Qw, uint32_t log2B, uint32_t l, uint32_t Qks,
                     uint32_t log2Bks, uint32_t lks, uint32_t r, uint32_t keys, const uint64_t *bsk,
                     const uint32_t *ksk, const uint64_t *V, uint32_t q_in, uint32_t q_out,
                     const uint32_t *ct, uint32_t *out, uint32_t *ext_out)
{
    w_bootstrap_one(n, N, Qw, log2B, l, Qks, log2Bks, lks, r, keys, bsk, ksk, V, q_in, q_out, ct, out,
                    ext_out, 1);
}

void orc_w_bootstrap_many(uint32_t n, uint32_t N, uint64_t Qw, uint32_t log2B, uint32_t l, uint32_t Qks,
                          uint32_t log2Bks, uint32_t lks, uint32_t r, uint32_t keys, const uint64_t *bsk,
                          const uint32_t *ksk, const uint64_t *V, uint32_t q_in, uint32_t q_out,
                          const uint32_t *ct, uint64_t count, uint32_t *out)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t c = 0; c < (int64_t)count; c++)
        w_bootstrap_one(n, N, Qw, log2B, l, Qks, log2Bks, lks, r, keys, bsk, ksk, V, q_in, q_out,
                        ct + (size_t)c * (n + 1), out + (size_t)c * (n + 1), NULL, 0);
}

/* f not nega-cyclic at the wide ring modulus: the two bootstraps of
 * orc_bootstrap_general (sign table g, then the extension F), each through
 * w_bootstrap_one; the LWE arithmetic between them is at q. */
void orc_w_bootstrap_general(uint32_t n, uint32_t N, uint64_t Qw, uint32_t log2B, uint32_t l, uint32_t Qks,
                             uint32_t log2Bks, uint32_t lks, uint32_t r, uint32_t keys, const uint64_t *bsk,
                             const uint32_t *ksk, const uint64_t *Vg, const uint64_t *VF, uint32_t q, uint32_t t,
                             uint32_t q_out, const uint32_t *ct, uint64_t count, uint32_t *out)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t c = 0; c < (int64_t)count; c++) {
        const uint32_t *ci = ct + (size_t)c * (n + 1);
        uint32_t *ctg = (uint32_t *)malloc(sizeof(uint32_t) * (n + 1));
        uint32_t *ct2 = (uint32_t *)malloc(sizeof(uint32_t) * (n + 1));
        w_bootstrap_one(n, N, Qw, log2B, l, Qks, log2Bks, lks, r, keys, bsk, ksk, Vg, q, q, ci, ctg, NULL, 0);
        const uint64_t shift = (uint64_t)(t / 2) * (q / (2 * t)) % q;
        for (uint32_t k = 0; k <= n; k++) ct2[k] = (uint32_t)(((uint64_t)ci[k] + ctg[k]) % q);
        ct2[n] = (uint32_t)(((uint64_t)ct2[n] + q - shift) % q);
        w_bootstrap_one(n, N, Qw, log2B, l, Qks, log2Bks, lks, r, keys, bsk, ksk, VF, q, q_out, ct2,
                        out + (size_t)c * (n + 1), NULL, 0);
        free(ctg);
        free(ct2);
    }
}
