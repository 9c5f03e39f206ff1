// HIP kernels of the BootMMPM bootstrap for gfx950.
//
// k_blind_rotate: the fused, persistent blind rotation (Alg. 1, first modulus
//   switch, accumulator initialisation and the n CMux steps, then the sample
//   extraction of entry 0).  One workgroup of GW waves owns a "group" of
//   component slots: a slot is W waves (by default one up to N = 1024 and
//   N / 1024 above; two at N = 512 and 1024 for batches that do not fill the
//   device) and holds one component j of one ciphertext, whose RLWE pair (a, b)
//   stays in LDS for all n steps.  Each step the slots read the pair that
//   Phi(-a'_i) brings to them (an index-and-sign remap, eq. ex1:BPc), form
//   D = Phi(-a'_i) ACC - ACC, and add D x BSK_i (the binary CMux of
//   eq. cmux:BP) with a register-resident NTT external product.
// k_keyswitch / k_ks_finalize: the key switch z -> s (eq. equ-key-swi) and the
//   final modulus switch Q -> q_out, batched over ciphertexts.
#include <hip/hip_runtime.h>

#include "device_common.hpp"
#include "kernels.hpp"

namespace mm {
namespace dev {

__host__ __device__ constexpr uint32_t gadget_offset(uint32_t log2B, uint32_t l)
{
    uint32_t off = 0;
    for (uint32_t u = 0; u + 1 < l; u++) off += (1u << (log2B - 1)) << (u * log2B);
    return off;
}

__device__ __forceinline__ uint32_t modswitch_dev(uint32_t x, uint32_t q_from, uint32_t q_to)
{
    if (q_from == q_to) return x;
    const uint64_t num = 2ull * (uint64_t)x * q_to + q_from;
    return (uint32_t)((num / (2ull * q_from)) % q_to);
}

__global__ void k_modswitch(const uint32_t *__restrict__ in, uint32_t *__restrict__ out, size_t count,
                            uint32_t q_from, uint32_t q_to)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x)
        out[i] = modswitch_dev(in[i], q_from, q_to);
}

// Row j of Phi(c), c = a r + b: source component (j - b) mod r and monomial
// exponent a + [j < b] (eq. ex1:BPc).
__device__ __forceinline__ void phi_row(uint32_t c, uint32_t r, uint32_t j, uint32_t &src, uint32_t &e)
{
    const uint32_t a = c / r, b = c - a * r;
    src = (j + r - b) % r;
    e = a + (j < b ? 1u : 0u);
}

// A wave's task, every field moved to scalar registers (the same for all lanes),
// so that the step index, key and ciphertext addresses derived from it stay
// scalar and the per-lane part of each address is one 32-bit offset.
__device__ __forceinline__ WaveTask uniform_task(const WaveTask &t)
{
    WaveTask u;
    u.ct = __builtin_amdgcn_readfirstlane(t.ct);
    u.comp = __builtin_amdgcn_readfirstlane(t.comp);
    u.r = __builtin_amdgcn_readfirstlane(t.r);
    u.tv_off = __builtin_amdgcn_readfirstlane(t.tv_off);
    u.q_in = __builtin_amdgcn_readfirstlane(t.q_in);
    u.i0 = __builtin_amdgcn_readfirstlane(t.i0);
    u.flags = __builtin_amdgcn_readfirstlane(t.flags);
    u.steps = __builtin_amdgcn_readfirstlane(t.steps);
    u.acc_off = ((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(t.acc_off >> 32)) << 32) |
                __builtin_amdgcn_readfirstlane((uint32_t)t.acc_off);
    return u;
}

// LDS per component slot: two accumulator buffers, each a swizzled pair (a, b).
// During a step one holds the current ACC (read by the rotations of every slot
// of the ciphertext) and the other serves the slot's NTT relayouts, then
// receives the updated ACC; the roles swap every step.
template <int N>
struct BrLds {
    static constexpr int BUF_WORDS = 2 * Geo<N>::POLYW;
    static constexpr int COMP_WORDS = 2 * BUF_WORDS;
    static_assert(BUF_WORDS == Geo<N>::SLOTW, "an accumulator buffer doubles as the exchange slot");
};

template <int N, int GW, int KEYS, int W = default_wpp(N), bool PL = false, bool ST = false>
__global__ void __launch_bounds__(64 * GW, 8 / GW) k_blind_rotate(BrArgs A)
{
    using G = Geo<N, W>;
    using LD = BrLds<N>;
    constexpr int E = G::E, P = G::POLYW, WPP = G::WPP, LN = G::LANES;
    static_assert(GW % WPP == 0, "a group holds whole component slots");
    extern __shared__ uint32_t lds[];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform: scalar from here on
    const int cs = wave / WPP;                             // component slot
    const int L = (wave % WPP) * 64 + (threadIdx.x & 63);  // virtual lane of the slot
    uint32_t *const base = lds + cs * LD::COMP_WORDS;
    // two waves per polynomial at N <= 1024: a second exchange slot per component
    // after the accumulator buffers, so that consecutive relayouts alternate between
    // the two and each needs one workgroup barrier instead of two
    constexpr bool DS = WPP == 2 && N <= 1024;
    uint32_t *const slot2 = lds + (GW / WPP) * LD::COMP_WORDS + cs * G::SLOTW;
    const ModQ m{A.Q, A.qn};
    const GadgetC g{A.log2B, A.l, A.sg, A.goff};

    for (int grp = blockIdx.x; grp < A.num_groups; grp += gridDim.x) {
        const WaveTask T = uniform_task(A.tasks[grp * GW + wave]);
        const bool has = T.ct >= 0;
        const uint32_t r = has ? T.r : 1u, M = 2u * N * r;
        const uint32_t *ct = A.ct_in + (size_t)(has ? T.ct : 0) * A.ct_stride;
        __syncthreads();  // the previous group's last rotated reads are done
        int cur = 0;      // buffer holding the current accumulator

        // ---- accumulator: Phi(b') (0, V) or the stored state, into buffer 0
        if (has && (T.flags & TASK_INIT)) {
            const uint32_t bq = __builtin_amdgcn_readfirstlane(modswitch_dev(ct[A.n], T.q_in, M));
            uint32_t src, e;
            phi_row(bq, r, T.comp, src, e);
            const uint32_t *V = A.tv + T.tv_off + (size_t)src * N;
#pragma unroll
            for (int k = 0; k < E; k++) {
                const uint32_t idx = LN * k + L;
                const uint32_t i2 = (idx + 2 * N - (e % (2 * N))) % (2 * N);
                const uint32_t v = V[i2 & (N - 1)];
                base[swz(idx)] = 0;
                base[P + swz(idx)] = (i2 >= N) ? (v ? A.Q - v : 0) : v;
            }
        } else if (has) {
            const uint32_t *S = A.acc_state + T.acc_off + (size_t)T.comp * 2 * N;
#pragma unroll
            for (int k = 0; k < E; k++) {
                base[swz(LN * k + L)] = S[LN * k + L];
                base[P + swz(LN * k + L)] = S[N + LN * k + L];
            }
        }

        // D = Phi(c) ACC - ACC for this slot's component: coefficient idx of x^e v is
        // v[(idx - e) mod 2N], negated when that index is >= N; a negated source enters
        // D as Q - v (Q is read as 0 by the decomposition)
        auto rotated_diff = [&](uint32_t c, const uint32_t *accl, uint32_t(&D)[2][E]) {
            uint32_t src, e;
            phi_row(c, r, T.comp, src, e);
            const uint32_t *sp = accl + ((int)src - (int)T.comp) * LD::COMP_WORDS;
            const uint32_t rb = (uint32_t)(L + 2 * N - (e % (2 * N)));
#pragma unroll
            for (int k = 0; k < E; k++) {
                const uint32_t i2 = (rb + LN * k) & (2 * N - 1);
                const int a = swz(i2 & (N - 1));
                uint32_t va = sp[a], vb = sp[P + a];
                if (i2 & N) {
                    va = A.Q - va;
                    vb = A.Q - vb;
                }
                const int o = swz(LN * k + L);
                D[0][k] = sub_q(va, accl[o], A.Q);
                D[1][k] = sub_q(vb, accl[P + o], A.Q);
            }
        };

        // ---- the CMux steps (eq. cmux:BP): the s+ term with Phi(-a'_i), and for a
        // ternary secret the s- term with Phi(a'_i), both read from the current buffer,
        // which no slot writes during the step, so one barrier per step suffices.
        // When a polynomial spans several waves its NTTs synchronise the whole
        // workgroup, so every wave runs them (idle slots on zeros, results dropped).
        const uint32_t lim = T.steps ? min(T.steps, (uint32_t)A.steps) : (uint32_t)A.steps;
        for (int s = 0; s < A.steps; s++) {
            const uint32_t i = T.i0 + (uint32_t)s;
            const bool active = has && i < A.n && (uint32_t)s < lim;
            const bool run = active || WPP > 1;
            uint32_t *const accl = base + cur * LD::BUF_WORDS;        // current ACC
            uint32_t *const nxt = base + (cur ^ 1) * LD::BUF_WORDS;   // exchange slot, then next ACC
            __syncthreads();  // every current accumulator is written
            uint32_t D[2][E];
            uint32_t ai = 0;
            if (active) {
                ai = __builtin_amdgcn_readfirstlane(modswitch_dev(ct[i], T.q_in, M));
                rotated_diff((M - ai) % M, accl, D);  // -a'_i mod 2Nr
            } else if (WPP > 1) {
#pragma unroll
                for (int k = 0; k < E; k++) D[0][k] = D[1][k] = 0;
            }
            uint32_t o[2][E];
            const uint32_t ik = active ? i : 0u;
            const uint32_t *K = A.bsk + (size_t)ik * KEYS * (4u * A.l * N);
            int par = 0;  // relayouts since the step's barrier (which slot the next one uses)
            if (run) {
                // start from the digit-offset correction of coordinate i, in the
                // layout of the forward NTT's output
                const uint32_t *C0 = A.bsk_corr + (size_t)ik * 2 * N + phase_lane<N, W, PL>(G::NPH - 1, L) * E;
#pragma unroll
                for (int k = 0; k < E; k++) {
                    const int v = phase_reg<N, W, PL>(G::NPH - 1, k);
                    o[0][k] = C0[v];
                    o[1][k] = C0[N + v];
                }
                ext_mac<N, true, W, (W == 1), DS, PL, ST>(D[0], D[1], K, nxt, A.twf, L, m, g, o, slot2, &par);
            }
            if (KEYS == 2) {
                if (active) rotated_diff(ai, accl, D);  // +a'_i from the same accumulator
                if (run)
                    ext_mac<N, true, W, (W == 1), DS, PL, ST>(D[0], D[1], K + 4u * A.l * N, nxt, A.twf, L, m, g, o,
                                                              slot2, &par);
            }
            if (run) {
                __asm__ volatile("" ::: "memory");
                ntt_inv<N, 2, W, (W == 1), DS, PL, ST>(o, nxt, A.twi, L, m, slot2, &par);
            }
            if (WPP > 1) __syncthreads();  // every lane of the slot has left the exchange slot
            if (active) {
#pragma unroll
                for (int k = 0; k < E; k++) {
                    const int a = swz(LN * k + L);
                    nxt[a] = add_q(accl[a], o[0][k], A.Q);
                    nxt[P + a] = add_q(accl[P + a], o[1][k], A.Q);
                }
            } else if (has) {
#pragma unroll
                for (int k = 0; k < E; k++) {  // past step n: carry the accumulator over
                    const int a = swz(LN * k + L);
                    nxt[a] = accl[a];
                    nxt[P + a] = accl[P + a];
                }
            }
            cur ^= 1;
        }

        // ---- results (each slot reads back only its own lanes of its accumulator)
        if (!has) continue;
        const uint32_t *accl = base + cur * LD::BUF_WORDS;
        if (T.flags & TASK_STORE) {
            uint32_t *S = A.acc_state + T.acc_off + (size_t)T.comp * 2 * N;
#pragma unroll
            for (int k = 0; k < E; k++) {
                S[LN * k + L] = accl[swz(LN * k + L)];
                S[N + LN * k + L] = accl[P + swz(LN * k + L)];
            }
        }
        if ((T.flags & TASK_EXTRACT) && T.comp == 0 && T.i0 + lim >= A.n) {
            // (A_0, -A_{N-1}, ..., -A_1; B_0) (eq. equ-sam-extr)
            uint32_t *o = A.ext_out + (size_t)T.ct * (N + 1);
#pragma unroll
            for (int k = 0; k < E; k++) {
                const uint32_t idx = LN * k + L;
                const uint32_t v = accl[swz(idx)];
                o[(N - idx) & (N - 1)] = idx ? (v ? A.Q - v : 0) : v;
            }
            if (L == 0) o[N] = accl[P + swz(0)];
        }
    }
}

// One external product per polynomial slot (WPP waves): in/out [count][2][N].
// A slot past the end computes on item 0 and stores nothing, so that every
// wave reaches the workgroup barriers of a multi-wave NTT.
template <int N>
__global__ void __launch_bounds__(512) k_external_product(const uint32_t *__restrict__ in, uint32_t *__restrict__ out,
                                                          size_t count, const uint32_t *__restrict__ K,
                                                          const uint32_t *twf, const uint32_t *twi, uint32_t Q,
                                                          uint32_t qn, uint32_t log2B, uint32_t l, uint32_t sg)
{
    using G = Geo<N>;
    constexpr int E = G::E, LN = G::LANES;
    extern __shared__ uint32_t lds[];
    const int wave = threadIdx.x >> 6, item = wave / G::WPP;
    const int L = (wave % G::WPP) * 64 + (threadIdx.x & 63);
    const size_t c0 = (size_t)blockIdx.x * (blockDim.x / LN) + item;
    if (G::WPP == 1 && c0 >= count) return;
    const bool ok = c0 < count;
    const size_t c = ok ? c0 : 0;
    uint32_t *slot = lds + item * G::SLOTW;
    const ModQ m{Q, qn};
    const GadgetC g{log2B, l, sg, gadget_offset(log2B, l)};
    uint32_t D[2][E], o[2][E];
#pragma unroll
    for (int k = 0; k < E; k++) {
        D[0][k] = in[c * 2 * N + LN * k + L];
        D[1][k] = in[c * 2 * N + N + LN * k + L];
    }
    external_product<N>(D[0], D[1], K, slot, twf, twi, L, m, g, o);
    if (!ok) return;
#pragma unroll
    for (int k = 0; k < E; k++) {
        out[c * 2 * N + LN * k + L] = o[0][k];
        out[c * 2 * N + N + LN * k + L] = o[1][k];
    }
}

// a * b through the NTT, one product per polynomial slot: [count][N] each.
// c_fix = 2^64 / N mod Q undoes two Montgomery factors and the missing 1/N.
template <int N>
__global__ void __launch_bounds__(512) k_negacyclic_mul(const uint32_t *__restrict__ a, const uint32_t *__restrict__ b,
                                                        uint32_t *__restrict__ out, size_t count, const uint32_t *twf,
                                                        const uint32_t *twi, uint32_t Q, uint32_t qn, uint32_t c_fix)
{
    using G = Geo<N>;
    constexpr int E = G::E, LN = G::LANES;
    extern __shared__ uint32_t lds[];
    const int wave = threadIdx.x >> 6, item = wave / G::WPP;
    const int L = (wave % G::WPP) * 64 + (threadIdx.x & 63);
    const size_t c0 = (size_t)blockIdx.x * (blockDim.x / LN) + item;
    if (G::WPP == 1 && c0 >= count) return;
    const bool ok = c0 < count;
    const size_t c = ok ? c0 : 0;
    uint32_t *slot = lds + item * G::SLOTW;
    const ModQ m{Q, qn};
    uint32_t x[2][E];
#pragma unroll
    for (int k = 0; k < E; k++) {
        x[0][k] = a[c * N + LN * k + L];
        x[1][k] = b[c * N + LN * k + L];
    }
    ntt_fwd<N, 2>(x, slot, twf, L, m);
    uint32_t y[1][E];
#pragma unroll
    for (int k = 0; k < E; k++) y[0][k] = mont_mul(mont_mul(x[0][k], x[1][k], m), c_fix, m);
    ntt_inv<N, 1>(y, slot, twi, L, m);
    if (!ok) return;
#pragma unroll
    for (int k = 0; k < E; k++) out[c * N + LN * k + L] = y[0][k];
}

// Sample extraction of [count][2][N] pairs.
__global__ void k_sample_extract(const uint32_t *__restrict__ rlwe, uint32_t *__restrict__ lwe, size_t count,
                                 uint32_t N, uint32_t Q)
{
    const size_t total = count * (N + 1);
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (size_t)gridDim.x * blockDim.x) {
        const size_t c = t / (N + 1);
        const uint32_t k = (uint32_t)(t - c * (N + 1));
        const uint32_t *A = rlwe + c * 2 * N;
        uint32_t v;
        if (k == N) v = A[N];
        else if (k == 0) v = A[0];
        else v = A[N - k] ? Q - A[N - k] : 0;
        lwe[t] = v;
    }
}

// Key switch, partial sums: thread (col, ct) adds KSK[i][j][d_ij(ct)][col] over
// the (i, j) pairs of split z (i in [i_begin, i_end)).  part[(z count + ct)(n+1) + col].
__global__ void __launch_bounds__(256) k_keyswitch(KsArgs A)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint32_t col = blockIdx.x * 64 + lane;
    const uint32_t W = A.n + 1;
    const uint32_t iper = (A.N + gridDim.z - 1) / gridDim.z;
    const uint32_t i_begin = blockIdx.z * iper, i_end = min(A.N, i_begin + iper);
    const uint32_t Bm = (1u << A.log2Bks) - 1;
    constexpr int CPW = KS_CTS_PER_WAVE;
    uint64_t acc[CPW];
    const uint32_t *src[CPW];
    bool ok[CPW];
#pragma unroll
    for (int q = 0; q < CPW; q++) {
        const size_t ct = ((size_t)blockIdx.y * 4 + wave) * CPW + q;
        ok[q] = ct < A.count;
        const size_t srow = ok[q] ? (A.rows ? (size_t)A.rows[ct] : ct) : 0;
        src[q] = A.lwe_N + srow * (A.N + 1);
        acc[q] = 0;
    }
    if (col < W) {
        for (uint32_t i = i_begin; i < i_end; i++) {
            const uint32_t *rowbase = A.ksk + ((size_t)i * A.col_tiles + blockIdx.x) * A.l_ks * (Bm + 1) * 64 + lane;
#pragma unroll
            for (int q = 0; q < CPW; q++) {
                const uint32_t a = __builtin_amdgcn_readfirstlane(src[q][i]);
                for (uint32_t j = 0; j < A.l_ks; j++) {
                    const uint32_t sh = j * A.log2Bks;
                    const uint32_t d = sh < 32 ? (a >> sh) & Bm : 0u;
                    acc[q] += rowbase[(j * (Bm + 1) + d) * 64];
                }
            }
        }
#pragma unroll
        for (int q = 0; q < CPW; q++) {
            const size_t ct = ((size_t)blockIdx.y * 4 + wave) * CPW + q;
            if (ok[q]) A.part[((size_t)blockIdx.z * A.count + ct) * W + col] = acc[q] % A.Q;
        }
    }
}

// Key switch for large batches.  A workgroup (4 waves) owns 64 columns of the
// output and 4 CPW ciphertexts; for each input coordinate i it stages the
// l_ks x B_ks candidate rows KSK[i][*][*][cols] in LDS (double-buffered through
// registers) and every wave adds, for each of its CPW ciphertexts, the l_ks rows
// its digits select.  KSK traffic: one read of the column slice per ciphertext
// tile.  Partial sums over the i-split blockIdx.z go to part (reduced mod Q).
template <int CPW, bool L8>
__global__ void __launch_bounds__(256) k_keyswitch_tiled(KsArgs A)
{
    constexpr int ROWS = KS_TILED_MAX_ROWS;  // l_ks * B_ks <= 128
    __shared__ uint32_t tile[2][ROWS * 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint32_t W = A.n + 1, Bks = 1u << A.log2Bks, rows = A.l_ks * Bks;
    const uint32_t col0 = blockIdx.x * 64, col = col0 + lane;
    const uint32_t iper = (A.N + gridDim.z - 1) / gridDim.z;
    const uint32_t i_begin = blockIdx.z * iper, i_end = min(A.N, i_begin + iper);
    const size_t ct_base = ((size_t)blockIdx.y * 4 + wave) * CPW;
    // lane q of the wave reads coordinate i of ciphertext ct_base + q (q < CPW)
    const size_t my_ct = ct_base + (lane < CPW ? lane : 0);
    const bool my_ok = lane < CPW && my_ct < A.count;
    const uint32_t *my_src = A.lwe_N + (my_ok ? (A.rows ? (size_t)A.rows[my_ct] : my_ct) : 0) * (A.N + 1);
    uint32_t acc[CPW];
#pragma unroll
    for (int q = 0; q < CPW; q++) acc[q] = 0;

    // each thread moves ceil(rows*64/256) words of a tile (rows need not be a
    // multiple of 4: l_ks * B_ks = 62 with B_ks = 2 and l_ks = 31)
    const uint32_t tile_words = rows * 64;
    const int per_thread = (int)((tile_words + 255) / 256);
    uint32_t stage[ROWS / 4];
    auto fetch = [&](uint32_t i) {
        const uint32_t *base = A.ksk + ((size_t)i * A.col_tiles + blockIdx.x) * tile_words;
#pragma unroll
        for (int k = 0; k < ROWS / 4; k++) {
            const uint32_t e = threadIdx.x + 256u * k;
            if (k < per_thread) stage[k] = e < tile_words ? base[e] : 0u;
        }
    };
    auto put = [&](int b) {
#pragma unroll
        for (int k = 0; k < ROWS / 4; k++) {
            const uint32_t e = threadIdx.x + 256u * k;
            if (k < per_thread && e < tile_words) tile[b][e] = stage[k];
        }
    };
    if (i_begin < i_end) {
        fetch(i_begin);
        put(0);
    }
    __syncthreads();
    int b = 0;
    for (uint32_t i = i_begin; i < i_end; i++) {
        if (i + 1 < i_end) fetch(i + 1);
        const uint32_t mine = my_ok ? my_src[i] : 0u;
        if constexpr (L8) {
            // eight digits of log2Bks bits: unrolled, one scalar extract per row
            const uint32_t *tl = &tile[b][lane];
#pragma unroll
            for (int q = 0; q < CPW; q++) {
                uint32_t a = __builtin_amdgcn_readlane(mine, q);
                __asm__ volatile("" : "+s"(a) :: "memory");  // one ciphertext at a time
                uint32_t s0 = 0, s1 = 0;
#pragma unroll
                for (int j = 0; j < 8; j += 2) {
                    const uint32_t d0 = (a >> (j * A.log2Bks)) & (Bks - 1);
                    const uint32_t d1 = (a >> ((j + 1) * A.log2Bks)) & (Bks - 1);
                    s0 = add_q(s0, tl[((uint32_t)j * Bks + d0) * 64], A.Q);
                    s1 = add_q(s1, tl[((uint32_t)(j + 1) * Bks + d1) * 64], A.Q);
                }
                acc[q] = add_q(acc[q], add_q(s0, s1, A.Q), A.Q);
            }
        } else {
#pragma unroll
            for (int q = 0; q < CPW; q++) {
                const uint32_t a = __builtin_amdgcn_readlane(mine, q);
                uint32_t s = 0;
                for (uint32_t j = 0; j < A.l_ks; j++) {
                    const uint32_t sh = j * A.log2Bks;
                    const uint32_t d = sh < 32 ? (a >> sh) & (Bks - 1) : 0u;
                    s = add_q(s, tile[b][(j * Bks + d) * 64 + lane], A.Q);
                }
                acc[q] = add_q(acc[q], s, A.Q);
            }
        }
        __syncthreads();
        if (i + 1 < i_end) put(b ^ 1);
        __syncthreads();
        b ^= 1;
    }
    if (col < W) {
#pragma unroll
        for (int q = 0; q < CPW; q++) {
            const size_t ct = ct_base + q;
            if (ct < A.count) A.part[((size_t)blockIdx.z * A.count + ct) * W + col] = acc[q];
        }
    }
}

// Key switch for large batches with one ciphertext per lane.  A workgroup
// (4 waves) owns 256 ciphertexts and 64 output columns; for each input
// coordinate i it stages the l_ks x B_ks candidate rows KSK[i][*][*][cols] in
// LDS (double-buffered through registers, rows padded to 66 words), and every
// lane forms the LDS addresses of the l_ks rows its own digits select once per
// i, then adds the 64 columns of those rows to 64-bit sums in registers, two
// rows at a time summed in 32 bits first (both below Q < 2^31).  The digit
// work is thus spread over the lanes and amortised over 64 columns; lanes
// whose digits agree read the same LDS words (broadcasts), and the 66-word row
// pitch puts the B_ks candidates of one digit on distinct banks.  KSK traffic:
// one read of the column slice per 256 ciphertexts.  Partial sums over the
// i-split blockIdx.z go to part (not reduced; every sum < 2^31 l_ks N).
constexpr int KSL_COLS = KS_TILE_COLS, KSL_PITCH = 66, KSL_CTS = 256, KSL_CHUNK = 32;

template <bool FULL>
__global__ void __launch_bounds__(256, 2) k_keyswitch_lanes(KsArgs A)
{
    constexpr int ROWS = KS_TILED_MAX_ROWS, V4 = ROWS * KSL_COLS / 4 / 256;
    __shared__ __align__(16) uint32_t tile[2][ROWS * KSL_PITCH];
    const uint32_t W = A.n + 1, Bks = 1u << A.log2Bks, rows = FULL ? (uint32_t)ROWS : A.l_ks * Bks;
    const uint32_t col0 = blockIdx.x * KSL_COLS;
    const uint32_t iper = (A.N + gridDim.z - 1) / gridDim.z;
    const uint32_t i_begin = blockIdx.z * iper, i_end = min(A.N, i_begin + iper);
    const size_t ct = (size_t)blockIdx.y * KSL_CTS + threadIdx.x;
    const bool ok = ct < A.count;
    const uint32_t *src = A.lwe_N + (ok ? (A.rows ? (size_t)A.rows[ct] : ct) : 0) * (A.N + 1);
    uint64_t acc[KSL_COLS];
#pragma unroll
    for (int c = 0; c < KSL_COLS; c++) acc[c] = 0;

    // staging: the tile of coordinate i is rows x 64 contiguous words; thread t
    // moves the 4-word pieces t + 256 k (row (t + 256 k) >> 4, column 4 (t & 15))
    const uint32_t tile4 = rows * KSL_COLS / 4;
    uint4 stage[V4];
    auto fetch = [&](uint32_t i) {
        const uint4 *base = reinterpret_cast<const uint4 *>(A.ksk + ((size_t)i * A.col_tiles + blockIdx.x) * rows * KSL_COLS);
#pragma unroll
        for (int k = 0; k < V4; k++) {
            const uint32_t e4 = threadIdx.x + 256u * k;
            if (FULL || e4 < tile4) stage[k] = base[e4];
        }
    };
    auto put = [&](int b) {
#pragma unroll
        for (int k = 0; k < V4; k++) {
            const uint32_t e4 = threadIdx.x + 256u * k;
            if (FULL || e4 < tile4) {
                uint32_t *d = &tile[b][(e4 >> 4) * KSL_PITCH + 4 * (e4 & 15)];
                *reinterpret_cast<uint2 *>(d) = make_uint2(stage[k].x, stage[k].y);
                *reinterpret_cast<uint2 *>(d + 2) = make_uint2(stage[k].z, stage[k].w);
            }
        }
    };
    // acc += row0 + row1 (64 columns each), or row0 alone, 16 columns at a time
    // (the compiler is kept from hoisting every LDS read of the rows: registers)
    auto add2 = [&](const uint32_t *r0, const uint32_t *r1) {
#pragma unroll
        for (int c0 = 0; c0 < KSL_COLS; c0 += KSL_CHUNK) {
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int c = c0; c < c0 + KSL_CHUNK; c += 2) {
                const uint2 x = *reinterpret_cast<const uint2 *>(r0 + c);
                const uint2 y = *reinterpret_cast<const uint2 *>(r1 + c);
                acc[c] += (uint64_t)(x.x + y.x);
                acc[c + 1] += (uint64_t)(x.y + y.y);
            }
        }
    };
    auto add1 = [&](const uint32_t *r0) {
#pragma unroll
        for (int c0 = 0; c0 < KSL_COLS; c0 += KSL_CHUNK) {
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int c = c0; c < c0 + KSL_CHUNK; c += 2) {
                const uint2 x = *reinterpret_cast<const uint2 *>(r0 + c);
                acc[c] += (uint64_t)x.x;
                acc[c + 1] += (uint64_t)x.y;
            }
        }
    };
    if (i_begin < i_end) {
        fetch(i_begin);
        put(0);
    }
    __syncthreads();
    int b = 0;
    for (uint32_t i = i_begin; i < i_end; i++) {
        if (i + 1 < i_end) fetch(i + 1);
        const uint32_t a = src[i];
        const uint32_t *tb = tile[b];
        // the row of each digit, two rows at a time (the digit loop stays rolled:
        // unrolled, the compiler keeps too many row reads in flight)
        auto digit = [&](uint32_t j) {
            const uint32_t sh = j * A.log2Bks;
            return sh < 32 ? (a >> sh) & (Bks - 1) : 0u;
        };
        uint32_t j = 0;
        for (; j + 1 < A.l_ks; j += 2)
            add2(tb + (j * Bks + digit(j)) * KSL_PITCH, tb + ((j + 1) * Bks + digit(j + 1)) * KSL_PITCH);
        if (j < A.l_ks) add1(tb + (j * Bks + digit(j)) * KSL_PITCH);
        __syncthreads();
        if (i + 1 < i_end) put(b ^ 1);
        __syncthreads();
        b ^= 1;
    }
    if (ok) {
        uint64_t *o = A.part + ((size_t)blockIdx.z * A.count + ct) * W + col0;
#pragma unroll
        for (int c = 0; c < KSL_COLS; c++)
            if (col0 + c < W) o[c] = acc[c];
    }
}

// (0^n, b) - sum of the partials, then the modulus switch Q -> q_out
// (q_out = Q keeps the residues).  out[ct][n+1].
__global__ void k_ks_finalize(const uint64_t *__restrict__ part, const uint32_t *__restrict__ lwe_N,
                              const int32_t *__restrict__ rows, uint32_t *__restrict__ out, size_t count, uint32_t n, uint32_t N, uint32_t splits,
                              uint32_t Q, const uint32_t *__restrict__ q_out_per_ct, uint32_t q_out)
{
    const uint32_t W = n + 1;
    const size_t total = count * W;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (size_t)gridDim.x * blockDim.x) {
        const size_t ct = t / W;
        const uint32_t col = (uint32_t)(t - ct * W);
        uint64_t s = 0;
        for (uint32_t z = 0; z < splits; z++) s += part[((size_t)z * count + ct) * W + col];
        const uint32_t v = (uint32_t)(s % Q);
        uint32_t x;
        if (col < n) x = v ? Q - v : 0;
        else {
            const size_t srow = rows ? (size_t)rows[ct] : ct;
            const uint32_t b = lwe_N[srow * (N + 1) + N];
            x = b >= v ? b - v : b + Q - v;
        }
        const uint32_t qo = q_out_per_ct ? q_out_per_ct[ct] : q_out;
        out[t] = (qo == Q) ? x : modswitch_dev(x, Q, qo);
    }
}

// dst[rows[k]] = src[k] for rows of W words (staged ciphertexts into their slots).
__global__ void k_scatter_rows(const uint32_t *__restrict__ src, uint32_t *__restrict__ dst,
                               const int32_t *__restrict__ rows, size_t count, uint32_t W)
{
    const size_t total = count * W;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (size_t)gridDim.x * blockDim.x) {
        const size_t k = t / W;
        dst[(size_t)rows[k] * W + (t - k * W)] = src[t];
    }
}

void launch_scatter_rows(const uint32_t *src, uint32_t *dst, const int32_t *rows, size_t count, uint32_t W,
                         hipStream_t st)
{
    const size_t total = count * W;
    const int grid = (int)std::min<size_t>((total + 255) / 256, 4096);
    hipLaunchKernelGGL(k_scatter_rows, dim3(std::max(grid, 1)), dim3(256), 0, st, src, dst, rows, count, W);
}

// out = ct + tmp - (0, shift) mod q, per ciphertext (q, shift) = qs[2c], qs[2c+1]:
// removes the top bit found by the sign bootstrap of a general f.
__global__ void k_lwe_combine(const uint32_t *__restrict__ ct, const uint32_t *__restrict__ tmp,
                              uint32_t *__restrict__ out, size_t count, uint32_t W, const uint32_t *__restrict__ qs)
{
    const size_t total = count * W;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (size_t)gridDim.x * blockDim.x) {
        const size_t c = t / W;
        const uint32_t k = (uint32_t)(t - c * W);
        const uint64_t q = qs[2 * c];
        uint64_t v = ((uint64_t)ct[t] + tmp[t]) % q;
        if (k == W - 1) v = (v + q - qs[2 * c + 1] % q) % q;
        out[t] = (uint32_t)v;
    }
}

void launch_lwe_combine(const uint32_t *ct, const uint32_t *tmp, uint32_t *out, size_t count, uint32_t W,
                        const uint32_t *qs, hipStream_t st)
{
    const size_t total = count * W;
    const int grid = (int)std::min<size_t>((total + 255) / 256, 4096);
    hipLaunchKernelGGL(k_lwe_combine, dim3(std::max(grid, 1)), dim3(256), 0, st, ct, tmp, out, count, W, qs);
}

// ------------------------------------------------------------------ launchers

// Two waves per polynomial at N = 512 and 1024 (half the registers' work per
// wave: lower latency for batches too small to fill the chip).
constexpr bool br_wide_slots(int N) { return N == 512 || N == 1024; }

template <int N, int GW, int KEYS, int W = default_wpp(N), bool PL = false, bool ST = false>
static hipError_t br_attr_n()
{
    return hipFuncSetAttribute((const void *)k_blind_rotate<N, GW, KEYS, W, PL, ST>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)br_lds_bytes(N, GW, W));
}

// NTT schedule 1 (the lane-swap exchange) exists where one wave holds a
// polynomial and the next-to-last phase has R = 2: N = 256 and 1024.
template <int N>
constexpr bool br_lane_swap()
{
    if constexpr (default_wpp(N) == 1) return pl_ok<N, 1>();
    else return false;
}

template <int N>
static hipError_t br_attr_all()
{
    hipError_t e = br_attr_n<N, 8, 1>();
    if (e == hipSuccess) e = br_attr_n<N, 8, 2>();
    if constexpr (Geo<N>::WPP <= 4) {
        if (e == hipSuccess) e = br_attr_n<N, 4, 1>();
        if (e == hipSuccess) e = br_attr_n<N, 4, 2>();
    }
    if constexpr (br_wide_slots(N)) {
        if (e == hipSuccess) e = br_attr_n<N, 8, 1, 2>();
        if (e == hipSuccess) e = br_attr_n<N, 8, 2, 2>();
    }
    if constexpr (br_lane_swap<N>()) {
        if (e == hipSuccess) e = br_attr_n<N, 8, 1, 1, true>();
        if (e == hipSuccess) e = br_attr_n<N, 8, 2, 1, true>();
        if (e == hipSuccess) e = br_attr_n<N, 4, 1, 1, true>();
        if (e == hipSuccess) e = br_attr_n<N, 4, 2, 1, true>();
    }
    if constexpr (Geo<N>::WPP == 1) {
        if (e == hipSuccess) e = br_attr_n<N, 8, 1, 1, false, true>();
        if (e == hipSuccess) e = br_attr_n<N, 8, 2, 1, false, true>();
        if (e == hipSuccess) e = br_attr_n<N, 4, 1, 1, false, true>();
        if (e == hipSuccess) e = br_attr_n<N, 4, 2, 1, false, true>();
    }
    return e;
}

template <int N>
static hipError_t slot_attr_n()
{
    const int lds = (int)((512 / Geo<N>::LANES) * Geo<N>::SLOTW * sizeof(uint32_t));
    hipError_t e = hipFuncSetAttribute((const void *)k_external_product<N>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (e == hipSuccess)
        e = hipFuncSetAttribute((const void *)k_negacyclic_mul<N>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    return e;
}

template <int N>
static hipError_t attr_n()
{
    hipError_t e = br_attr_all<N>();
    if (e == hipSuccess) e = slot_attr_n<N>();
    return e;
}

hipError_t init_kernel_attributes()
{
    hipError_t e = attr_n<256>();
    if (e == hipSuccess) e = attr_n<512>();
    if (e == hipSuccess) e = attr_n<1024>();
    if (e == hipSuccess) e = attr_n<2048>();
    if (e == hipSuccess) e = attr_n<4096>();
    if (e == hipSuccess) e = attr_n<8192>();
    return e;
}

bool device_supports_n(uint32_t N)
{
    return N == 256 || N == 512 || N == 1024 || N == 2048 || N == 4096 || N == 8192;
}

int waves_per_poly(uint32_t N) { return N > 1024 ? (int)(N / 1024) : 1; }

template <int N, int KEYS>
static void launch_br_nk(const BrArgs &A, int gw, int grid, hipStream_t st, int wpp, int ntt)
{
    if constexpr (Geo<N>::WPP == 1) {
        if (ntt == 2 && (wpp == 0 || wpp == 1)) {
            if (gw == 4)
                hipLaunchKernelGGL((k_blind_rotate<N, 4, KEYS, 1, false, true>), dim3(grid), dim3(256),
                                   br_lds_bytes(N, 4), st, A);
            else
                hipLaunchKernelGGL((k_blind_rotate<N, 8, KEYS, 1, false, true>), dim3(grid), dim3(512),
                                   br_lds_bytes(N, 8), st, A);
            return;
        }
    }
    if constexpr (br_lane_swap<N>()) {
        if (ntt == 1 && (wpp == 0 || wpp == 1)) {
            if (gw == 4)
                hipLaunchKernelGGL((k_blind_rotate<N, 4, KEYS, 1, true>), dim3(grid), dim3(256), br_lds_bytes(N, 4),
                                   st, A);
            else
                hipLaunchKernelGGL((k_blind_rotate<N, 8, KEYS, 1, true>), dim3(grid), dim3(512), br_lds_bytes(N, 8),
                                   st, A);
            return;
        }
    }
    if constexpr (br_wide_slots(N)) {
        if (wpp == 2) {
            hipLaunchKernelGGL((k_blind_rotate<N, 8, KEYS, 2>), dim3(grid), dim3(512), br_lds_bytes(N, 8, 2), st, A);
            return;
        }
    }
    if constexpr (Geo<N>::WPP <= 4) {
        if (gw == 4) {
            hipLaunchKernelGGL((k_blind_rotate<N, 4, KEYS>), dim3(grid), dim3(256), br_lds_bytes(N, 4), st, A);
            return;
        }
    }
    hipLaunchKernelGGL((k_blind_rotate<N, 8, KEYS>), dim3(grid), dim3(512), br_lds_bytes(N, 8), st, A);
}

template <int N>
static void launch_br_n(const BrArgs &A, int gw, int grid, hipStream_t st, int wpp, int ntt)
{
    if (A.keys == 2) launch_br_nk<N, 2>(A, gw, grid, st, wpp, ntt);
    else launch_br_nk<N, 1>(A, gw, grid, st, wpp, ntt);
}

void launch_blind_rotate(uint32_t N, const BrArgs &A, int gw, int grid, hipStream_t st, int wpp, int ntt)
{
    switch (N) {
    case 256: launch_br_n<256>(A, gw, grid, st, wpp, ntt); break;
    case 512: launch_br_n<512>(A, gw, grid, st, wpp, ntt); break;
    case 1024: launch_br_n<1024>(A, gw, grid, st, wpp, ntt); break;
    case 2048: launch_br_n<2048>(A, gw, grid, st, wpp, ntt); break;
    case 4096: launch_br_n<4096>(A, gw, grid, st, wpp, ntt); break;
    case 8192: launch_br_n<8192>(A, gw, grid, st, wpp, ntt); break;
    default: break;
    }
}

bool br_supports_wpp(uint32_t N, int wpp) { return wpp == waves_per_poly(N) || (wpp == 2 && br_wide_slots((int)N)); }

bool br_supports_lane_swap(uint32_t N)
{
    return (N == 256 && br_lane_swap<256>()) || (N == 512 && br_lane_swap<512>()) ||
           (N == 1024 && br_lane_swap<1024>());
}

template <int N>
static size_t br_lds_n(int gw, int wpp)
{
    const int w = wpp ? wpp : Geo<N>::WPP;
    const size_t extra = (w == 2 && N <= 1024) ? (size_t)Geo<N>::SLOTW : 0;  // the second exchange slot
    return (size_t)(gw / w) * (BrLds<N>::COMP_WORDS + extra) * sizeof(uint32_t);
}

size_t br_lds_bytes(uint32_t N, int gw, int wpp)
{
    switch (N) {
    case 256: return br_lds_n<256>(gw, wpp);
    case 512: return br_lds_n<512>(gw, wpp);
    case 1024: return br_lds_n<1024>(gw, wpp);
    case 2048: return br_lds_n<2048>(gw, wpp);
    case 4096: return br_lds_n<4096>(gw, wpp);
    default: return br_lds_n<8192>(gw, wpp);
    }
}

// Blocks of 4 waves (8 when one polynomial spans 8 waves); one item per slot.
template <int N>
static void slot_launch_shape(size_t count, dim3 &grid, dim3 &block, size_t &lds)
{
    const int threads = std::max(256, Geo<N>::LANES);
    const int items = threads / Geo<N>::LANES;
    grid = dim3((unsigned)((count + items - 1) / items));
    block = dim3(threads);
    lds = (size_t)items * Geo<N>::SLOTW * sizeof(uint32_t);
}

template <int N>
static void launch_ep_n(const uint32_t *in, uint32_t *out, size_t count, const uint32_t *K, const uint32_t *twf,
                        const uint32_t *twi, uint32_t Q, uint32_t qn, uint32_t log2B, uint32_t l, uint32_t sg,
                        hipStream_t st)
{
    dim3 grid, block;
    size_t lds;
    slot_launch_shape<N>(count, grid, block, lds);
    hipLaunchKernelGGL(k_external_product<N>, grid, block, lds, st, in, out, count, K, twf, twi, Q, qn, log2B, l, sg);
}

void launch_external_product(uint32_t N, const uint32_t *in, uint32_t *out, size_t count, const uint32_t *K,
                             const uint32_t *twf, const uint32_t *twi, uint32_t Q, uint32_t qn, uint32_t log2B,
                             uint32_t l, uint32_t sg, hipStream_t st)
{
    switch (N) {
    case 256: launch_ep_n<256>(in, out, count, K, twf, twi, Q, qn, log2B, l, sg, st); break;
    case 512: launch_ep_n<512>(in, out, count, K, twf, twi, Q, qn, log2B, l, sg, st); break;
    case 1024: launch_ep_n<1024>(in, out, count, K, twf, twi, Q, qn, log2B, l, sg, st); break;
    case 2048: launch_ep_n<2048>(in, out, count, K, twf, twi, Q, qn, log2B, l, sg, st); break;
    case 4096: launch_ep_n<4096>(in, out, count, K, twf, twi, Q, qn, log2B, l, sg, st); break;
    case 8192: launch_ep_n<8192>(in, out, count, K, twf, twi, Q, qn, log2B, l, sg, st); break;
    default: break;
    }
}

template <int N>
static void launch_pm_n(const uint32_t *a, const uint32_t *b, uint32_t *out, size_t count, const uint32_t *twf,
                        const uint32_t *twi, uint32_t Q, uint32_t qn, uint32_t c_fix, hipStream_t st)
{
    dim3 grid, block;
    size_t lds;
    slot_launch_shape<N>(count, grid, block, lds);
    hipLaunchKernelGGL(k_negacyclic_mul<N>, grid, block, lds, st, a, b, out, count, twf, twi, Q, qn, c_fix);
}

void launch_negacyclic_mul(uint32_t N, const uint32_t *a, const uint32_t *b, uint32_t *out, size_t count,
                           const uint32_t *twf, const uint32_t *twi, uint32_t Q, uint32_t qn, uint32_t c_fix,
                           hipStream_t st)
{
    switch (N) {
    case 256: launch_pm_n<256>(a, b, out, count, twf, twi, Q, qn, c_fix, st); break;
    case 512: launch_pm_n<512>(a, b, out, count, twf, twi, Q, qn, c_fix, st); break;
    case 1024: launch_pm_n<1024>(a, b, out, count, twf, twi, Q, qn, c_fix, st); break;
    case 2048: launch_pm_n<2048>(a, b, out, count, twf, twi, Q, qn, c_fix, st); break;
    case 4096: launch_pm_n<4096>(a, b, out, count, twf, twi, Q, qn, c_fix, st); break;
    case 8192: launch_pm_n<8192>(a, b, out, count, twf, twi, Q, qn, c_fix, st); break;
    default: break;
    }
}

void launch_modswitch(const uint32_t *in, uint32_t *out, size_t count, uint32_t q_from, uint32_t q_to, hipStream_t st)
{
    const int grid = (int)std::min<size_t>((count + 255) / 256, 4096);
    hipLaunchKernelGGL(k_modswitch, dim3(std::max(grid, 1)), dim3(256), 0, st, in, out, count, q_from, q_to);
}

void launch_sample_extract(const uint32_t *rlwe, uint32_t *lwe, size_t count, uint32_t N, uint32_t Q, hipStream_t st)
{
    const size_t total = count * (N + 1);
    const int grid = (int)std::min<size_t>((total + 255) / 256, 4096);
    hipLaunchKernelGGL(k_sample_extract, dim3(std::max(grid, 1)), dim3(256), 0, st, rlwe, lwe, count, N, Q);
}

void launch_keyswitch_tiled(const KsArgs &A, int cpw, uint32_t splits, hipStream_t st)
{
    const uint32_t W = A.n + 1;
    const uint32_t cts_per_block = 4u * cpw;
    dim3 grid((W + 63) / 64, (uint32_t)((A.count + cts_per_block - 1) / cts_per_block), splits);
    const bool l8 = A.l_ks == 8 && 8 * A.log2Bks <= 32;  // eight digits, all inside the word
    switch (cpw) {
    case 16:
        if (l8) hipLaunchKernelGGL((k_keyswitch_tiled<16, true>), grid, dim3(256), 0, st, A);
        else hipLaunchKernelGGL((k_keyswitch_tiled<16, false>), grid, dim3(256), 0, st, A);
        break;
    case 32:
        if (l8) hipLaunchKernelGGL((k_keyswitch_tiled<32, true>), grid, dim3(256), 0, st, A);
        else hipLaunchKernelGGL((k_keyswitch_tiled<32, false>), grid, dim3(256), 0, st, A);
        break;
    default:
        if (l8) hipLaunchKernelGGL((k_keyswitch_tiled<64, true>), grid, dim3(256), 0, st, A);
        else hipLaunchKernelGGL((k_keyswitch_tiled<64, false>), grid, dim3(256), 0, st, A);
        break;
    }
}

void launch_keyswitch_lanes(const KsArgs &A, uint32_t splits, hipStream_t st)
{
    dim3 grid(A.col_tiles, (uint32_t)((A.count + KSL_CTS - 1) / KSL_CTS), splits);
    const bool full = (A.l_ks << A.log2Bks) == (uint32_t)KS_TILED_MAX_ROWS;
    if (full) hipLaunchKernelGGL(k_keyswitch_lanes<true>, grid, dim3(256), 0, st, A);
    else hipLaunchKernelGGL(k_keyswitch_lanes<false>, grid, dim3(256), 0, st, A);
}

void launch_keyswitch(const KsArgs &A, uint32_t splits, hipStream_t st)
{
    const uint32_t W = A.n + 1;
    const uint32_t cts_per_block = 4 * KS_CTS_PER_WAVE;
    dim3 grid((W + 63) / 64, (uint32_t)((A.count + cts_per_block - 1) / cts_per_block), splits);
    hipLaunchKernelGGL(k_keyswitch, grid, dim3(256), 0, st, A);
}

void launch_ks_finalize(const uint64_t *part, const uint32_t *lwe_N, const int32_t *rows, uint32_t *out, size_t count,
                        uint32_t n, uint32_t N, uint32_t splits, uint32_t Q, const uint32_t *q_out_per_ct,
                        uint32_t q_out, hipStream_t st)
{
    const size_t total = count * (n + 1);
    const int grid = (int)std::min<size_t>((total + 255) / 256, 8192);
    hipLaunchKernelGGL(k_ks_finalize, dim3(std::max(grid, 1)), dim3(256), 0, st, part, lwe_N, rows, out, count, n, N,
                       splits, Q, q_out_per_ct, q_out);
}

}  // namespace dev
}  // namespace mm
