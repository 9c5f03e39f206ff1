// Host side of the library: parameter checks, key generation, LWE
// encryption/decryption and look-up-table registration.  Nothing here is on
// the bootstrap's hot path; keys are built once and uploaded by device_init.
#include <algorithm>
#include <cstring>
#include <functional>
#include <thread>

#include "mmpm_internal.hpp"

namespace mm {

// Run fn(i) for i in [0, n) on the machine's hardware threads.
void parallel_for(int64_t n, const std::function<void(int64_t)> &fn)
{
    const int64_t T = std::max<int64_t>(1, std::min<int64_t>(n, std::thread::hardware_concurrency()));
    std::vector<std::thread> th;
    for (int64_t t = 0; t < T; t++)
        th.emplace_back([&, t] {
            for (int64_t i = t; i < n; i += T) fn(i);
        });
    for (auto &x : th) x.join();
}

uint32_t powmod(uint32_t a, uint64_t e, uint32_t q)
{
    uint64_t r = 1 % q, b = a % q;
    while (e) {
        if (e & 1) r = r * b % q;
        b = b * b % q;
        e >>= 1;
    }
    return (uint32_t)r;
}

bool is_prime(uint32_t q)
{
    if (q < 2) return false;
    for (uint32_t d = 2; (uint64_t)d * d <= q; d++)
        if (q % d == 0) return false;
    return true;
}

uint32_t bit_length(uint32_t x)
{
    uint32_t b = 0;
    while (x) {
        b++;
        x >>= 1;
    }
    return b;
}

uint32_t bitrev(uint32_t x, uint32_t bits)
{
    uint32_t r = 0;
    for (uint32_t i = 0; i < bits; i++) r |= ((x >> i) & 1u) << (bits - 1 - i);
    return r;
}

uint64_t crt2(uint32_t x1, uint32_t x2, uint32_t Q1, uint32_t Q2)
{
    const uint32_t inv = powmod(Q1 % Q2, Q2 - 2, Q2);  // Q1^-1 mod Q2
    const uint32_t d = submod(x2, x1 % Q2, Q2);
    return (uint64_t)x1 + (uint64_t)Q1 * mulmod(d, inv, Q2);
}

void NttTables::build(uint32_t N_, uint32_t Q_)
{
    N = N_;
    Q = Q_;
    // psi = g^((Q-1)/2N) with psi^N = -1: a primitive 2N-th root of unity
    psi = 0;
    for (uint32_t g = 2; g < 1000000 && !psi; g++) {
        uint32_t c = powmod(g, (Q - 1) / (2 * N), Q);
        if (powmod(c, N, Q) == Q - 1) psi = c;
    }
    if (!psi) throw Error(MM_EINVAL, "no primitive 2N-th root of unity mod Q");
    const uint32_t logN = bit_length(N) - 1;
    const uint32_t psi_inv = powmod(psi, 2ull * N - 1, Q);
    fwd.assign(N, 0);
    inv.assign(N, 0);
    for (uint32_t k = 0; k < N; k++) {
        fwd[k] = powmod(psi, bitrev(k, logN), Q);
        inv[k] = powmod(psi_inv, bitrev(k, logN), Q);
    }
    n_inv = powmod(N, Q - 2, Q);
}

void NttTables::forward(uint32_t *a) const
{
    for (uint32_t m = 1, t = N / 2; m < N; m <<= 1, t >>= 1)
        for (uint32_t i = 0; i < m; i++) {
            const uint32_t w = fwd[m + i];
            for (uint32_t j = 2 * i * t; j < 2 * i * t + t; j++) {
                const uint32_t u = a[j], v = mulmod(a[j + t], w, Q);
                a[j] = addmod(u, v, Q);
                a[j + t] = submod(u, v, Q);
            }
        }
}

void NttTables::inverse(uint32_t *a) const
{
    for (uint32_t m = N / 2, t = 1; m >= 1; m >>= 1, t <<= 1)
        for (uint32_t i = 0; i < m; i++) {
            const uint32_t w = inv[m + i];
            for (uint32_t j = 2 * i * t; j < 2 * i * t + t; j++) {
                const uint32_t u = a[j], v = a[j + t];
                a[j] = addmod(u, v, Q);
                a[j + t] = mulmod(submod(u, v, Q), w, Q);
            }
        }
    for (uint32_t k = 0; k < N; k++) a[k] = mulmod(a[k], n_inv, Q);
}

void validate_params(const mm_params &p)
{
    MM_REQUIRE(p.n >= 1 && p.n <= 4096, "n must be in [1, 4096]");
    MM_REQUIRE(p.N >= 64 && p.N <= 65536 && (p.N & (p.N - 1)) == 0, "N must be a power of two in [64, 65536]");
    MM_REQUIRE(p.Q > 2 && p.Q < (1u << 31), "Q must be below 2^31");
    MM_REQUIRE((p.Q - 1) % (2 * p.N) == 0, "Q must be 1 mod 2N");
    MM_REQUIRE(is_prime(p.Q), "Q must be prime");
    if (p.Q2 == 0) {
        MM_REQUIRE(p.log2_B >= 1 && p.log2_B <= 15 && p.l >= 1 && p.l * p.log2_B <= 32 && p.l <= 8,
                   "gadget needs 1 <= log2_B <= 15, 1 <= l <= 8, l*log2_B <= 32");
    } else {
        MM_REQUIRE(p.Q2 > 2 && p.Q2 < (1u << 31) && p.Q2 != p.Q, "Q2 must be below 2^31 and differ from Q");
        MM_REQUIRE((p.Q2 - 1) % (2 * p.N) == 0, "Q2 must be 1 mod 2N");
        MM_REQUIRE(is_prime(p.Q2), "Q2 must be prime");
        MM_REQUIRE(p.log2_B >= 1 && p.log2_B <= 16 && p.l >= 1 && p.l * p.log2_B <= 62 && p.l <= 8,
                   "wide gadget needs 1 <= log2_B <= 16, 1 <= l <= 8, l*log2_B <= 62");
        // the device joins residues through d1 + c Q2 - d0 in 32 bits, and every
        // digit field (at most B + 1) must be a residue of both primes
        MM_REQUIRE((uint64_t)p.Q + 2ull * p.Q2 < (1ull << 32), "wide mode needs Q + 2 Q2 < 2^32");
        MM_REQUIRE((2ull << p.log2_B) < p.Q2, "wide mode needs 2B < Q2");
    }
    MM_REQUIRE(p.log2_Bks >= 1 && p.log2_Bks <= 8, "log2_Bks must be in [1, 8]");
    MM_REQUIRE(p.l_ks * p.log2_Bks >= bit_length(p.Q) && p.l_ks <= 32,
               "l_ks * log2_Bks must cover bits(Q) (exact key-switch digits)");
    MM_REQUIRE(p.ternary <= 1, "ternary must be 0 or 1");
}

// a * z in Z_Q[x]/(x^N+1) for binary z, through the host NTT
static void mul_by_secret(const NttTables &T, const uint32_t *a, const std::vector<uint32_t> &z_ntt,
                          uint32_t *out)
{
    std::vector<uint32_t> tmp(a, a + T.N);
    T.forward(tmp.data());
    for (uint32_t k = 0; k < T.N; k++) tmp[k] = mulmod(tmp[k], z_ntt[k], T.Q);
    T.inverse(tmp.data());
    std::memcpy(out, tmp.data(), sizeof(uint32_t) * T.N);
}

static uint32_t lift_err(int32_t e, uint32_t Q)
{
    int64_t v = (int64_t)e % (int64_t)Q;
    return (uint32_t)(v < 0 ? v + Q : v);
}

static uint32_t bit_length64(uint64_t x)
{
    uint32_t b = 0;
    while (x) {
        b++;
        x >>= 1;
    }
    return b;
}

// BSK_{i,k} = RGSW_z(m_{i,k}) at Q_w = Q Q2, built limb by limb: row masks are
// the caller's uint64 draws reduced mod each prime, a z is taken through that
// prime's NTT, and g_u = 2^(sg + u log2_B) mod Q_w.  [i][k][limb][row][part][N].
static void keygen_bsk_wide(mm_ctx &c, const mm_key_draws &d)
{
    const mm_params &p = c.p;
    const uint32_t N = p.N, l = p.l, n = p.n, K = c.keys;
    MM_REQUIRE(d.bsk_a_wide, "null wide key draw (bsk_a_wide)");
    const size_t bsk_in = (size_t)n * K * 2 * l * N;
    for (size_t k = 0; k < bsk_in; k++) MM_REQUIRE(d.bsk_a_wide[k] < c.Qw, "bsk_a_wide out of range");
    c.ntt2.build(N, p.Q2);
    const NttTables *T[2] = {&c.ntt, &c.ntt2};
    std::vector<uint32_t> z_ntt[2];
    for (int j = 0; j < 2; j++) {
        z_ntt[j] = c.z;
        T[j]->forward(z_ntt[j].data());
    }
    std::vector<uint64_t> g(l);
    for (uint32_t u = 0; u < l; u++) {
        uint64_t v = 1 % c.Qw;
        for (uint32_t e = 0; e < c.sg + u * p.log2_B; e++) v = (uint64_t)((unsigned __int128)v * 2 % c.Qw);
        g[u] = v;
    }
    c.bsk.assign(bsk_in * 2 * 2, 0);
    parallel_for((int64_t)n * K, [&](int64_t ik) {
        const int64_t i = ik / K, key = ik % K;
        const int32_t si = c.s[i];
        const uint32_t m = key == 0 ? (uint32_t)std::max(si, 0) : (uint32_t)std::max(-si, 0);
        std::vector<uint32_t> a(N);
        for (uint32_t j = 0; j < 2; j++) {
            const uint32_t Qj = T[j]->Q;
            for (uint32_t row = 0; row < 2 * l; row++) {
                const size_t in_off = ((size_t)ik * 2 * l + row) * N;
                uint32_t *oa = &c.bsk[((((size_t)ik * 2 + j) * 2 * l + row) * 2 + 0) * N];
                uint32_t *ob = oa + N;
                for (uint32_t k = 0; k < N; k++) oa[k] = (uint32_t)(d.bsk_a_wide[in_off + k] % Qj);
                mul_by_secret(*T[j], oa, z_ntt[j], ob);
                for (uint32_t k = 0; k < N; k++) ob[k] = addmod(ob[k], lift_err(d.bsk_e[in_off + k], Qj), Qj);
                if (m) {
                    const uint32_t gj = (uint32_t)(g[row % l] % Qj);
                    if (row < l) ob[0] = addmod(ob[0], gj, Qj);
                    else oa[0] = addmod(oa[0], gj, Qj);
                }
            }
        }
    });
}

static void keygen_bsk(mm_ctx &c, const mm_key_draws &d, const std::vector<uint32_t> &z_ntt);
static void keygen_ksk(mm_ctx &c, const mm_key_draws &d);

void keygen(mm_ctx &c, const mm_key_draws &d)
{
    const mm_params &p = c.p;
    c.wide = p.Q2 != 0;
    MM_REQUIRE(d.s && d.z && (c.wide || d.bsk_a) && d.bsk_e && d.ksk_a && d.ksk_e, "null key draw");
    const uint32_t N = p.N, Q = p.Q, l = p.l, n = p.n;
    c.Qw = c.wide ? (uint64_t)Q * p.Q2 : Q;
    const uint32_t bq = bit_length64(c.Qw);
    c.sg = bq > l * p.log2_B ? bq - l * p.log2_B : 0;
    c.gadget.resize(l);
    for (uint32_t u = 0; u < l; u++) c.gadget[u] = c.wide ? 0 : powmod(2, c.sg + u * p.log2_B, Q);
    c.keys = 1 + p.ternary;
    c.s.assign(d.s, d.s + n);
    c.z.assign(d.z, d.z + N);
    for (int32_t v : c.s) MM_REQUIRE(p.ternary ? (v >= -1 && v <= 1) : (v == 0 || v == 1), "s out of range");
    for (uint32_t v : c.z) MM_REQUIRE(v <= 1, "z must be binary");
    c.ntt.build(N, Q);

    std::vector<uint32_t> z_ntt(c.z);
    c.ntt.forward(z_ntt.data());

    // BSK_{i,k} = RGSW_z(m_{i,k}); KSK at Q
    if (c.wide) keygen_bsk_wide(c, d);
    else keygen_bsk(c, d, z_ntt);
    keygen_ksk(c, d);
}

static void keygen_bsk(mm_ctx &c, const mm_key_draws &d, const std::vector<uint32_t> &z_ntt)
{
    const mm_params &p = c.p;
    const uint32_t N = p.N, Q = p.Q, l = p.l, n = p.n, K = c.keys;
    const size_t bsk_in = (size_t)n * K * 2 * l * N;
    for (size_t k = 0; k < bsk_in; k++) MM_REQUIRE(d.bsk_a[k] < Q, "bsk_a out of range");
    c.bsk.assign(bsk_in * 2, 0);
    parallel_for((int64_t)n * K, [&](int64_t ik) {
        const int64_t i = ik / K, key = ik % K;
        const int32_t si = c.s[i];
        const uint32_t m = key == 0 ? (uint32_t)std::max(si, 0) : (uint32_t)std::max(-si, 0);
        for (uint32_t row = 0; row < 2 * l; row++) {
            const size_t in_off = ((size_t)ik * 2 * l + row) * N;
            uint32_t *a = &c.bsk[(((size_t)ik * 2 * l + row) * 2 + 0) * N];
            uint32_t *b = a + N;
            std::memcpy(a, d.bsk_a + in_off, sizeof(uint32_t) * N);
            mul_by_secret(c.ntt, a, z_ntt, b);
            for (uint32_t k = 0; k < N; k++) b[k] = addmod(b[k], lift_err(d.bsk_e[in_off + k], Q), Q);
            if (m) {
                const uint32_t g = c.gadget[row % l];
                if (row < l) b[0] = addmod(b[0], g, Q);
                else a[0] = addmod(a[0], g, Q);
            }
        }
    });
}

// KSK[i][j][v] = (alpha, <alpha, s> + e + v z_i B_ks^j), [i][j][v][n+1], at Q
static void keygen_ksk(mm_ctx &c, const mm_key_draws &d)
{
    const mm_params &p = c.p;
    const uint32_t N = p.N, Q = p.Q, n = p.n, Bks = 1u << p.log2_Bks;
    const size_t ksk_rows = (size_t)N * p.l_ks * Bks;
    for (size_t k = 0; k < ksk_rows * n; k++) MM_REQUIRE(d.ksk_a[k] < Q, "ksk_a out of range");
    c.ksk.assign(ksk_rows * (n + 1), 0);
    parallel_for(N, [&](int64_t i) {
        uint32_t pw = 1;
        for (uint32_t j = 0; j < p.l_ks; j++) {
            for (uint32_t v = 0; v < Bks; v++) {
                const size_t row = ((size_t)i * p.l_ks + j) * Bks + v;
                const uint32_t *al = d.ksk_a + row * n;
                uint32_t *o = &c.ksk[row * (n + 1)];
                uint64_t pos = 0, neg = 0;
                for (uint32_t k = 0; k < n; k++) {
                    o[k] = al[k];
                    if (c.s[k] > 0) pos += al[k];
                    else if (c.s[k] < 0) neg += al[k];
                }
                uint32_t bval = submod((uint32_t)(pos % Q), (uint32_t)(neg % Q), Q);
                bval = addmod(bval, lift_err(d.ksk_e[row], Q), Q);
                bval = addmod(bval, mulmod(mulmod(v, c.z[i], Q), pw, Q), Q);
                o[n] = bval;
            }
            pw = mulmod(pw, Bks, Q);
        }
    });
}

void encrypt(const mm_ctx &c, uint32_t q, uint32_t t, const uint32_t *m, size_t count,
             const uint32_t *mask, const int32_t *err, uint32_t *ct)
{
    const uint32_t n = c.p.n;
    MM_REQUIRE(q >= 2 && t >= 2 && t <= q, "need 2 <= t <= q");
    const uint64_t delta = q / t;
    for (size_t i = 0; i < count; i++) {
        const uint32_t *a = mask + i * n;
        uint32_t *o = ct + i * (n + 1);
        uint64_t pos = 0, neg = 0;
        for (uint32_t k = 0; k < n; k++) {
            MM_REQUIRE(a[k] < q, "mask out of range");
            o[k] = a[k];
            if (c.s[k] > 0) pos += a[k];
            else if (c.s[k] < 0) neg += a[k];
        }
        int64_t b = (int64_t)(pos % q) - (int64_t)(neg % q) + (int64_t)((uint64_t)(m[i] % t) * delta % q) + err[i];
        b %= (int64_t)q;
        if (b < 0) b += q;
        o[n] = (uint32_t)b;
    }
}

void decrypt(const mm_ctx &c, uint32_t q, uint32_t t, const uint32_t *ct, size_t count, uint32_t *m)
{
    const uint32_t n = c.p.n;
    MM_REQUIRE(q >= 2 && t >= 2 && t <= q, "need 2 <= t <= q");
    const uint64_t delta = q / t;
    for (size_t i = 0; i < count; i++) {
        const uint32_t *o = ct + i * (n + 1);
        uint64_t pos = 0, neg = 0;
        for (uint32_t k = 0; k < n; k++) {
            if (c.s[k] > 0) pos += o[k];
            else if (c.s[k] < 0) neg += o[k];
        }
        const uint64_t ph = ((uint64_t)o[n] % q + 2 * (uint64_t)q - pos % q + neg % q) % q;
        m[i] = (uint32_t)(((ph + delta / 2) / delta) % t);
    }
}

int table_create(mm_ctx &c, uint32_t t, uint32_t t_out, uint32_t r, uint32_t q_in, const uint32_t *f)
{
    const uint32_t N = c.p.N;
    MM_REQUIRE(r >= 1 && r <= 1024u, "r must be in [1, 1024]");
    const uint64_t M = 2ull * N * r;
    MM_REQUIRE(M <= (1ull << 31), "2Nr must be <= 2^31");
    MM_REQUIRE(t >= 2 && t % 2 == 0 && M % t == 0, "t must be even and divide 2Nr");
    MM_REQUIRE(t_out >= 2 && t_out % 2 == 0 && t_out <= c.p.Q / 2, "t' must be even and below Q/2");
    if (q_in == 0) q_in = (uint32_t)M;
    MM_REQUIRE(q_in >= 2 && q_in <= (1u << 31), "q_in must be in [2, 2^31]");
    for (uint32_t m = 0; m < t; m++) MM_REQUIRE(f[m] < t_out, "table entry out of range");
    for (uint32_t m = 0; m < t / 2; m++)
        MM_REQUIRE((f[m] + f[m + t / 2]) % t_out == 0, "table is not nega-cyclic");
    Table tb{t, t_out, r, q_in, {}, 0};
    const uint32_t limbs = c.wide ? 2 : 1;
    tb.V.resize((size_t)r * limbs * N);
    const uint64_t delta = M / t, dq = c.Qw / t_out;
    for (uint32_t b = 0; b < r; b++)
        for (uint32_t a = 0; a < N; a++) {
            const uint64_t x = (M - ((uint64_t)a * r + b) % M) % M;  // -(a r + b) mod 2Nr
            const uint64_t m = ((x + delta / 2) / delta) % t;       // nearest multiple of 2Nr/t
            const uint64_t v = (uint64_t)((unsigned __int128)dq * f[m] % c.Qw);
            if (!c.wide) {
                tb.V[(size_t)b * N + a] = (uint32_t)v;
            } else {
                tb.V[((size_t)b * 2 + 0) * N + a] = (uint32_t)(v % c.p.Q);
                tb.V[((size_t)b * 2 + 1) * N + a] = (uint32_t)(v % c.p.Q2);
            }
        }
    c.tables.push_back(std::move(tb));
    return (int)c.tables.size() - 1;
}

// Two nega-cyclic tables on Z_2t carry an arbitrary f: the sign table g and
// the nega-cyclic extension F of f (Sec. 4, general f).
int table_create_general(mm_ctx &c, uint32_t t, uint32_t t_out, uint32_t r, uint32_t q_in, const uint32_t *f)
{
    MM_REQUIRE(t >= 2 && t % 2 == 0, "t must be even");
    MM_REQUIRE(t_out >= 2 && t_out % 2 == 0, "t' must be even");
    for (uint32_t m = 0; m < t; m++) MM_REQUIRE(f[m] < t_out, "table entry out of range");
    std::vector<uint32_t> g(2 * t), F(2 * t);
    for (uint32_t x = 0; x < 2 * t; x++) {
        g[x] = x < t ? t / 2 : 2 * t - t / 2;
        F[x] = x < t ? f[x] : (t_out - f[x - t]) % t_out;
    }
    const int gid = table_create(c, 2 * t, 2 * t, r, q_in, g.data());
    const int fid = table_create(c, 2 * t, t_out, r, q_in, F.data());
    Table tb{t, t_out, r, c.tables[gid].q_in, {}, 0, gid, fid};
    c.tables.push_back(std::move(tb));
    return (int)c.tables.size() - 1;
}

}  // namespace mm
