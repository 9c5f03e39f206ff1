// HIP kernels of the blind rotation at a wide ring modulus Q_w = Q0 Q1 (two
// primes below 2^31, e.g. a 54-bit Q_w as in the experiments of Sec. 5).
//
// The accumulator of a ciphertext can be far larger than a workgroup (r up to
// 1024 components), so it lives in device memory as [component][part][prime][N]
// residues, double-buffered, and every CMux step is one launch over all
// (ciphertext, component) pairs: the launch boundary is the barrier between
// steps.  Workgroup k_wide_step (N / 512 waves by default) owns one pair for one step:
//   1. reads its own component and the one that Phi(-a'_i) brings to it (index
//      and sign remap of the source, eq. ex1:BPc), both primes, and forms
//      D = Phi(-a'_i) ACC_j - ACC_j;
//   2. joins the two residues of each coefficient into one integer in [0, Q_w)
//      (Chinese remainders), centres it and cuts it into l digit fields of the
//      signed gadget (offset by B/2, Sec. 2 item (10));
//   3. for each prime: forward NTT of every digit polynomial, product with
//      BSK_i in the NTT domain (eq. def:gsw), inverse NTT;
//   4. writes ACC_j + D x BSK_i into the other buffer.
// A ternary secret adds the second term of Alg. 1 (Phi(+a'_i), BSK_i^-) from
// the same ACC before step 3's inverse NTT.
//
// The same kernels, instantiated for one prime (NPR = 1), are the global-
// accumulator path of the default 31-bit ring modulus: for tables whose r
// components do not fit one workgroup's LDS (r N / 1024 > 8, e.g. r = 16 at
// N = 1024), for rings of 16384 and more (one polynomial over 16 waves, or the
// split ring below), which the fused persistent kernel cannot hold, and, with
// four waves per component at N = 1024, the faster shape for the largest and the
// lightest batches the fused kernel could hold.  Layouts are the wide ones with the
// prime index dropped: a component is [part][N], key blocks [n][keys][2l][2][N].
// Variants: two digit groups per workgroup (DG), one workgroup per prime (PS), and
// an XCD-aware order of work items (xcd_item).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "device_common.hpp"
#include "kernels.hpp"

namespace mm {
namespace dev {

// a' = round(x M / q) (Sec. 2 item (9)), ties upward.
__device__ __forceinline__ uint32_t wide_modswitch(uint32_t x, uint32_t q, uint32_t M)
{
    return (uint32_t)(((2ull * x * M + q) / (2ull * q)) % M);
}

// Row j of Phi(c) for c = a r + b (eq. ex1:BPc): source component (j - b) mod r
// and monomial x^(a + [j < b]), returned as a shift e in [0, N) and a sign.
struct WideRow {
    uint32_t src, e;
    bool neg;
};

__device__ __forceinline__ WideRow wide_row(uint32_t c, uint32_t r, uint32_t j, uint32_t N)
{
    const uint32_t a = c / r, b = c - a * r;
    WideRow w;
    w.src = j >= b ? j - b : j + r - b;
    uint32_t e = (a + (j < b ? 1u : 0u)) % (2 * N);
    w.neg = e >= N;
    w.e = w.neg ? e - N : e;
    return w;
}

// Coefficient idx of x^e p (negacyclic, e < N): p[idx - e], negated when the
// index wraps; `neg` folds in a further x^N = -1.
__device__ __forceinline__ uint32_t wide_rot_load(const uint32_t *p, uint32_t idx, const WideRow &w, uint32_t N,
                                                  uint32_t Q)
{
    const uint32_t v = p[(idx - w.e) & (N - 1)];
    const bool flip = (idx < w.e) != w.neg;
    return (flip && v) ? Q - v : v;
}

template <int N, int NPR>
__global__ __launch_bounds__(256) void k_wide_init(WideArgs A)
{
    const WideTask T = A.tasks[blockIdx.x];
    const uint32_t M = 2u * N * T.r;
    const uint32_t *ct = A.ct_in + (size_t)T.ct * A.ct_stride;
    const uint32_t b = wide_modswitch(ct[A.ct_stride - 1], T.q_in, M);
    const WideRow w = wide_row(b, T.r, T.comp, N);
    uint32_t *acc = A.acc_wr + T.acc_off + (size_t)T.comp * 2 * NPR * N;
    for (uint32_t idx = threadIdx.x; idx < (uint32_t)N; idx += blockDim.x) {
#pragma unroll
        for (int pr = 0; pr < NPR; pr++) {
            const uint32_t *v = A.tv + T.tv_off + ((size_t)w.src * NPR + pr) * N;
            acc[pr * N + idx] = 0;                                              // part a
            acc[NPR * N + pr * N + idx] = wide_rot_load(v, idx, w, N, A.Q[pr]);  // part b
        }
    }
}

// W waves per polynomial: N / 512 (8 coefficients per lane) and at least three
// waves per SIMD hide the accumulator loads and the workgroup barriers of the
// relayouts.  Measured at N = 2048, binary secret, 16384 components, per 512
// steps: 982 ms with 16 coefficients per lane and 2 waves per SIMD, 904 ms with
// 8 and 2, 794 ms with 8 and 3 (735 ms once relayouts addressed LDS from one base
// per side), 810 ms with 8 and 4 (spills).
// At N >= 8192 (one prime only) 16 coefficients per lane: N / 1024 waves, 16
// at N = 16384, the most one workgroup holds.
constexpr int wide_wpp(int N) { return N > 4096 ? N / 1024 : (N > 512 ? N / 512 : 1); }

// Work item of workgroup b of a grid of g: the hardware deals workgroups to the eight
// XCDs in turn (b mod 8), each with its own L2; this mapping gives each XCD a contiguous
// eighth of the items (the rest, g mod 8, in order), so the components of one
// ciphertext -- which read each other's accumulators through the rotation -- share an L2.
__device__ __forceinline__ uint32_t xcd_item(uint32_t b, uint32_t g)
{
    const uint32_t full = g / 8 * 8;
    return b < full ? (b % 8) * (full / 8) + b / 8 : b;
}

// Waves per EU the compiler is asked to leave room for: three (measured best at
// N = 2048), or what a workgroup of 16 waves leaves anyway.
constexpr int wide_min_waves(int W) { return W >= 16 ? 4 : 3; }

// DG = 2: two groups of W waves per workgroup share one component's step: group g
// takes the digits u = g, g + 2, ... of the forward NTTs and products, the two
// groups' products meet in LDS, and group g runs the inverse NTT of part g --
// half the dependent chain of a step for a component on one compute unit, the
// shape for batches that leave compute units idle.
//
// PS (two primes): two workgroups per component, one per prime (work item = 2 task +
// prime): both form the digit fields from both residues, each runs the NTTs, key
// products and inverse NTT of its own prime and writes that prime's residues --
// for batches with compute units to spare, half the dependent chain of a step.
// With DG = 2 as well, each such workgroup splits its prime's digits over two groups.
template <int N, int KEYS, int NPR, int W = wide_wpp(N), int DG = 1, bool PS = false>
__global__ __launch_bounds__(64 * W * DG) __attribute__((amdgpu_waves_per_eu(wide_min_waves(W)))) void k_wide_step(WideArgs A)
{
    using G = Geo<N, W>;
    constexpr int E = G::E;
    static_assert(DG == 1 || (DG == 2 && (NPR == 1 || PS) && W < 16),
                  "two digit groups: one prime per workgroup, up to 8 waves each");
    static_assert(!PS || NPR == 2, "one workgroup per prime: two primes");
    // digit fields: l log2 B bits fit 32 with one prime (31-bit Q), up to 62 with two
    using Y = typename std::conditional<NPR == 1, uint32_t, uint64_t>::type;
    // a ternary secret keeps the first key's digit fields in LDS (each lane reads
    // back only its own), so each key's fields are formed once per step
    // (one array for both, so no alignment gap: three workgroups per CU at N = 2048)
    constexpr bool Y_LDS = KEYS == 2 && (G::SLOTW * 4 + 2 * N * 8) <= 65536;
    static_assert(G::SLOTW % 2 == 0, "the slot ends on an 8-byte boundary");
    // issue priority around the relayouts (see relayout): on where they are wave-private,
    // and with a ternary secret, which measured 5 % faster at N = 2048 (binary: 1 % slower)
    constexpr bool PRIO = W == 1 || KEYS == 2;
    // a binary secret leaves LDS to spare: a second exchange slot, so that
    // consecutive relayouts alternate and each needs one workgroup barrier, not two
    // (a third of the LDS a ternary workgroup needs, so occupancy is unchanged);
    // not at N = 16384, where one slot takes 136 KB
    constexpr bool DS = KEYS == 1 && W > 1 && 2 * G::SLOTW * 4 <= 160 * 1024;
    // 16 waves (N = 16384): the forward NTTs take one digit polynomial at a time
    constexpr bool ONE_AT_A_TIME = W >= 16;
    constexpr int GS64 = G::SLOTW / 2 + (Y_LDS ? 2 * N : 0) + (DS ? G::SLOTW / 2 : 0);  // per group
    __shared__ uint64_t lds64[GS64 * DG];
    const int grp = DG > 1 ? (int)(threadIdx.x / (64 * W)) : 0;  // wave-uniform
    uint32_t *const slot = reinterpret_cast<uint32_t *>(lds64 + grp * GS64);
    uint64_t *const ylds = lds64 + grp * GS64 + G::SLOTW / 2;
    uint32_t *const slot2 = slot + G::SLOTW;  // DS only (ylds is ternary only)
    int par = 0;                              // relayouts so far: which slot the next one uses
    const uint32_t item = xcd_item(blockIdx.x, gridDim.x);
    const WideTask T = A.tasks[PS ? item / 2 : item];
    const int L = DG > 1 ? (int)(threadIdx.x % (64 * W)) : (int)threadIdx.x;
    constexpr size_t CW = (size_t)2 * NPR * N, PW = (size_t)NPR * N;  // words per component, per part
    const uint32_t *own = A.acc_rd + T.acc_off + (size_t)T.comp * CW;
    uint32_t *wr = A.acc_wr + T.acc_off + (size_t)T.comp * CW;
    // the primes this workgroup computes: both, or its own with PS
    const int pr_lo = PS ? (int)(item % 2) : 0, pr_hi = PS ? pr_lo + 1 : NPR;
    const uint32_t i = T.i0 + A.step;  // this task's CMux step
    if (i >= A.n) {
        // past step n - 1 (a ciphertext that finishes inside a sequence of launches):
        // carry the component over to the buffer the next launch reads
        if constexpr (PS) {
            for (uint32_t w = threadIdx.x; w < 2u * N; w += blockDim.x) {
                const size_t at = (size_t)(w / N) * PW + (size_t)pr_lo * N + w % N;
                wr[at] = own[at];
            }
        } else {
            for (uint32_t w = threadIdx.x; w < (uint32_t)CW; w += blockDim.x) wr[w] = own[w];
        }
        return;
    }
    const uint32_t M = 2u * N * T.r;
    const uint32_t am = wide_modswitch(A.ct_in[(size_t)T.ct * A.ct_stride + i], T.q_in, M);
    // per-prime constants by selection (no private arrays: those would be placed in LDS)
    auto mod = [&](int pr) { return ModQ{pr ? A.Q[1] : A.Q[0], pr ? A.qn[1] : A.qn[0]}; };

    // y'' = round(centred(D) / 2^sg) + goff per coefficient of parts a (0) and b
    // (1), D = Phi(c) ACC_j - ACC_j (joined from its two residues with two primes)
    const uint64_t half = (A.Qw - 1) / 2;
    Y y[2][E];
    auto digit_fields = [&](int key) {
        const uint32_t c = key == 0 ? (M - am) % M : am;
        const WideRow w = wide_row(c, T.r, T.comp, N);
        const uint32_t *src = A.acc_rd + T.acc_off + (size_t)w.src * CW;
#pragma unroll
        for (int part = 0; part < 2; part++)
#pragma unroll
            for (int k = 0; k < E; k++) {
                const uint32_t idx = G::LANES * k + L;
                const uint32_t *o = own + part * PW, *s = src + part * PW;
                const uint32_t d0 = sub_q(wide_rot_load(s, idx, w, N, A.Q[0]), o[idx], A.Q[0]);
                if constexpr (NPR == 1) {
                    int32_t xc = d0 > (uint32_t)half ? (int32_t)(d0 - A.Q[0]) : (int32_t)d0;
                    if (A.sg) xc = (xc + (1 << (A.sg - 1))) >> A.sg;
                    y[part][k] = (uint32_t)xc + (uint32_t)A.goff;
                } else {
                    const uint32_t d1 = sub_q(wide_rot_load(s + N, idx, w, N, A.Q[1]), o[N + idx], A.Q[1]);
                    // x = d0 + Q0 ((d1 - d0) Q0^-1 mod Q1), in [0, Q0 Q1)
                    const uint32_t kk = mont_mul(d1 + A.crt_cq - d0, A.crt_inv, mod(1));
                    const uint64_t x = d0 + (uint64_t)A.Q[0] * kk;
                    int64_t xc = x > half ? (int64_t)(x - A.Qw) : (int64_t)x;
                    if (A.sg) xc = (xc + (1ll << (A.sg - 1))) >> A.sg;
                    y[part][k] = (uint64_t)xc + A.goff;
                }
            }
    };
    // NTT-domain output of one prime from the digit-offset correction
    auto start = [&](int pr, uint32_t (&out)[2][E]) {
        const uint32_t *corr = A.bsk_corr + ((size_t)i * NPR + pr) * 2 * N + L * E;
#pragma unroll
        for (int part = 0; part < 2; part++)
#pragma unroll
            for (int k = 0; k < E; k++) out[part][k] = grp == 0 ? corr[part * N + k] : 0u;  // once per component
    };
    // out += the digits of y times BSK_{i,key} for one prime (eq. def:gsw)
    auto mac = [&](int pr, int key, uint32_t (&out)[2][E], bool from_lds = false) {
        const uint32_t *Kp = A.bsk + (((size_t)i * KEYS + key) * NPR + pr) * (2 * A.l * 2 * N);
        // with two digit groups both run the same number of NTTs (their relayouts meet at
        // the same workgroup barriers): a group without a digit left transforms zeros
        for (uint32_t u0 = 0; u0 < A.l; u0 += DG) {
            __asm__ volatile("" ::: "memory");
            const uint32_t u = u0 + (uint32_t)grp;
            const bool real = DG == 1 || u < A.l;
            const uint32_t sh = real ? u * A.log2B : 0u;
            const Y mask = !real ? (Y)0 : (u + 1 == A.l ? ~(Y)0 : (Y)(((Y)1 << A.log2B) - 1));
            if constexpr (ONE_AT_A_TIME) {
                // one digit polynomial at a time (16 waves leave 128 registers per lane):
                // the digit of b meets rows u, then the digit of a rows l + u
#pragma unroll
                for (int part = 1; part >= 0; part--) {
                    __asm__ volatile("" ::: "memory");
                    uint32_t pd[1][E];
#pragma unroll
                    for (int k = 0; k < E; k++) {
                        const Y yv = from_lds ? (Y)ylds[(part * E + k) * G::LANES + L] : y[part][k];
                        pd[0][k] = (uint32_t)((yv >> sh) & mask);
                    }
                    ntt_fwd<N, 1, W, PRIO, DS>(pd, slot, pr ? A.twf1 : A.twf0, L, mod(pr), slot2, &par);
                    const size_t row = part == 1 ? (size_t)u : (size_t)(A.l + u);
                    const uint32_t *k_a = Kp + (row * 2 + 0) * N + L * E;
                    const uint32_t *k_b = Kp + (row * 2 + 1) * N + L * E;
#pragma unroll
                    for (int k = 0; k < E; k++) {
                        out[0][k] = add_q(out[0][k], redc((uint64_t)pd[0][k] * k_a[k], mod(pr)), mod(pr).Q);
                        out[1][k] = add_q(out[1][k], redc((uint64_t)pd[0][k] * k_b[k], mod(pr)), mod(pr).Q);
                    }
                }
                continue;
            }
            uint32_t pd[2][E];
#pragma unroll
            for (int k = 0; k < E; k++) {
                const Y ya = from_lds ? (Y)ylds[k * G::LANES + L] : y[0][k];
                const Y yb = from_lds ? (Y)ylds[(E + k) * G::LANES + L] : y[1][k];
                pd[0][k] = (uint32_t)((yb >> sh) & mask);  // digit of b meets rows u
                pd[1][k] = (uint32_t)((ya >> sh) & mask);  // digit of a meets rows l + u
            }
            ntt_fwd<N, 2, W, PRIO, DS>(pd, slot, pr ? A.twf1 : A.twf0, L, mod(pr), slot2, &par);
            if (!real) continue;
            const uint32_t *kb_a = Kp + ((size_t)u * 2 + 0) * N + L * E;
            const uint32_t *kb_b = Kp + ((size_t)u * 2 + 1) * N + L * E;
            const uint32_t *ka_a = Kp + ((size_t)(A.l + u) * 2 + 0) * N + L * E;
            const uint32_t *ka_b = Kp + ((size_t)(A.l + u) * 2 + 1) * N + L * E;
#pragma unroll
            for (int k = 0; k < E; k++) {
                const uint64_t xa = (uint64_t)pd[0][k] * kb_a[k] + (uint64_t)pd[1][k] * ka_a[k];
                const uint64_t xb = (uint64_t)pd[0][k] * kb_b[k] + (uint64_t)pd[1][k] * ka_b[k];
                out[0][k] = add_q(out[0][k], redc(xa, mod(pr)), mod(pr).Q);
                out[1][k] = add_q(out[1][k], redc(xb, mod(pr)), mod(pr).Q);
            }
        }
    };
    // inverse NTT, ACC_j + product, store to the other buffer
    auto finish = [&](int pr, uint32_t (&out)[2][E]) {
        __asm__ volatile("" ::: "memory");
        if constexpr (DG == 2) {
            // group g hands its product of part 1 - g to the other group through its
            // own exchange slot and finishes part g
            uint32_t *const theirs = reinterpret_cast<uint32_t *>(lds64 + (1 - grp) * GS64);
            __syncthreads();  // every relayout of the forward NTTs is done
#pragma unroll
            for (int k = 0; k < E; k++) slot[k * G::LANES + L] = grp == 0 ? out[1][k] : out[0][k];
            __syncthreads();
            uint32_t o1[1][E];
#pragma unroll
            for (int k = 0; k < E; k++)
                o1[0][k] = add_q(grp == 0 ? out[0][k] : out[1][k], theirs[k * G::LANES + L], mod(pr).Q);
            __syncthreads();  // both slots read before the inverse relayouts reuse them
            ntt_inv<N, 1, W, PRIO, DS>(o1, slot, pr ? A.twi1 : A.twi0, L, mod(pr), slot2, &par);
#pragma unroll
            for (int k = 0; k < E; k++) {
                const uint32_t idx = G::LANES * k + L;
                const size_t at = (size_t)grp * PW + pr * N + idx;
                wr[at] = add_q(o1[0][k], own[at], mod(pr).Q);
            }
            return;
        }
        ntt_inv<N, 2, W, PRIO, DS>(out, slot, pr ? A.twi1 : A.twi0, L, mod(pr), slot2, &par);
#pragma unroll
        for (int part = 0; part < 2; part++)
#pragma unroll
            for (int k = 0; k < E; k++) {
                const uint32_t idx = G::LANES * k + L;
                const size_t at = (size_t)part * PW + pr * N + idx;
                wr[at] = add_q(out[part][k], own[at], mod(pr).Q);
            }
    };
    if constexpr (KEYS == 1) {
        // one prime at a time: only one prime's outputs are live
        digit_fields(0);
#pragma unroll
        for (int pr = pr_lo; pr < pr_hi; pr++) {
            uint32_t out[2][E];
            start(pr, out);
            mac(pr, 0, out);
            finish(pr, out);
        }
    } else if constexpr (Y_LDS) {
        // key 0's fields to LDS, key 1's stay in registers across both primes
        digit_fields(0);
#pragma unroll
        for (int part = 0; part < 2; part++)
#pragma unroll
            for (int k = 0; k < E; k++) ylds[(part * E + k) * G::LANES + L] = y[part][k];
        digit_fields(1);
#pragma unroll
        for (int pr = pr_lo; pr < pr_hi; pr++) {
            uint32_t out[2][E];
            start(pr, out);
            mac(pr, 1, out);
            mac(pr, 0, out, true);
            finish(pr, out);
        }
    } else {
        // one prime at a time as well; each key's digit fields are formed again
        // for the second prime (cheaper than keeping both primes' outputs live)
#pragma unroll
        for (int pr = pr_lo; pr < pr_hi; pr++) {
            uint32_t out[2][E];
            start(pr, out);
            for (int key = 0; key < 2; key++) {
                digit_fields(key);
                mac(pr, key, out);
            }
            finish(pr, out);
        }
    }
}

__device__ __forceinline__ uint64_t wide_join(uint32_t d0, uint32_t d1, const WideArgs &A)
{
    const ModQ m1{A.Q[1], A.qn[1]};
    return d0 + (uint64_t)A.Q[0] * mont_mul(d1 + A.crt_cq - d0, A.crt_inv, m1);
}

// Extraction of component 0 (eq. equ-sam-extr); with two primes then
// round(x Q0 / Q_w) = floor((2 x + Q1) / (2 Q1)) mod Q0 for each coefficient.
template <int N, int NPR>
__global__ __launch_bounds__(256) void k_wide_extract(WideArgs A, const uint64_t *__restrict__ acc_off,
                                                      uint32_t *__restrict__ ext)
{
    const uint32_t *acc = A.acc_rd + acc_off[blockIdx.x];
    uint32_t *o = ext + (size_t)blockIdx.x * (N + 1);
    for (uint32_t k = threadIdx.x; k <= (uint32_t)N; k += blockDim.x) {
        if constexpr (NPR == 1) {
            uint32_t v;
            if (k == N) v = acc[N];  // b_0
            else if (k == 0) v = acc[0];
            else v = acc[N - k] ? A.Q[0] - acc[N - k] : 0u;  // -a_{N-k}
            o[k] = v;
        } else {
            const uint64_t den = 2ull * A.Q[1];
            uint64_t x;
            if (k == N) {
                x = wide_join(acc[2 * N], acc[3 * N], A);  // b_0
            } else {
                const uint32_t src = k ? N - k : 0;
                x = wide_join(acc[src], acc[N + src], A);
                if (k && x) x = A.Qw - x;  // -a_{N-k}
            }
            o[k] = (uint32_t)(((2 * x + A.Q[1]) / den) % A.Q[0]);
        }
    }
}

// The accumulator as uint64 values: component j of a task -> [part][N] at the
// same word offset (a component is 4N words in both layouts).  One prime needs
// no such kernel: its accumulator layout is the output layout.
template <int N>
__global__ __launch_bounds__(256) void k_wide_export(WideArgs A, uint32_t *__restrict__ out)
{
    const WideTask T = A.tasks[blockIdx.x];
    const size_t base = T.acc_off + (size_t)T.comp * 4 * N;
    const uint32_t *acc = A.acc_rd + base;
    for (uint32_t t = threadIdx.x; t < 2u * N; t += blockDim.x) {
        const uint32_t part = t / N, idx = t % N;
        const uint64_t x = wide_join(acc[part * 2 * N + idx], acc[part * 2 * N + N + idx], A);
        out[base + 2 * t] = (uint32_t)x;
        out[base + 2 * t + 1] = (uint32_t)(x >> 32);
    }
}

// ------------------------------------------------------------------ split rings
//
// A ring of N = M NS coefficients (NS = 8192, M = 2, 4, 8: the TFHE-shaped rings
// of 16384 to 65536) is too large for one workgroup.  Its negacyclic NTT is the
// standard Cooley-Tukey network (bit-reversed output, the host's order): the
// first log2 M stages mix the M sub-rings {h NS, ..., (h + 1) NS - 1}, after which
// sub-ring h is an NTT of NS points whose stage with m' groups uses the full
// table's twiddles psi^bitrev(M m' + h m' + i') (twf_sub).  The inverse mirrors
// it.  So one CMux step is three launches: digits + mixing stages (column by
// column), the sub-ring NTTs + product + inverse sub-ring stages (one
// workgroup per sub-ring, as k_wide_step), and the inverse mixing stages +
// accumulation (column by column).

// Stage 1 of a split CMux step: for column j (positions j + h NS of the M
// sub-rings) the difference D = Phi(c) ACC_j - ACC_j, its digit fields, and per
// digit polynomial the Cooley-Tukey stages with m = 1, ..., M/2 groups.
template <int M, int KEYS>
__global__ __launch_bounds__(256) void k_split_digits(WideArgs A)
{
    constexpr uint32_t NS = SPLIT_NS, N = M * NS;
    const uint32_t task = blockIdx.y;
    const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;  // grid.x covers NS columns exactly
    const WideTask T = A.tasks[task];
    const uint32_t i = T.i0 + A.step;
    if (i >= A.n) return;
    const uint32_t Q = A.Q[0];
    const ModQ m{Q, A.qn[0]};
    const uint32_t Mr = 2u * N * T.r;
    const uint32_t am = wide_modswitch(A.ct_in[(size_t)T.ct * A.ct_stride + i], T.q_in, Mr);
    const uint32_t *own = A.acc_rd + T.acc_off + (size_t)T.comp * 2 * N;
    uint32_t *dig = A.dig + (size_t)task * KEYS * A.l * 2 * N + j;
    const uint32_t half = (Q - 1) / 2;
    for (int key = 0; key < KEYS; key++) {
        const uint32_t c = key == 0 ? (Mr - am) % Mr : am;
        const WideRow w = wide_row(c, T.r, T.comp, N);
        const uint32_t *src = A.acc_rd + T.acc_off + (size_t)w.src * 2 * N;
        for (int part = 0; part < 2; part++) {
            uint32_t y[M];
#pragma unroll
            for (int h = 0; h < M; h++) {
                const uint32_t idx = j + h * NS;
                const uint32_t d = sub_q(wide_rot_load(src + part * N, idx, w, N, Q), own[part * N + idx], Q);
                int32_t xc = d > half ? (int32_t)(d - Q) : (int32_t)d;
                if (A.sg) xc = (xc + (1 << (A.sg - 1))) >> A.sg;
                y[h] = (uint32_t)xc + (uint32_t)A.goff;
            }
            for (uint32_t u = 0; u < A.l; u++) {
                const uint32_t sh = u * A.log2B;
                const uint32_t mask = u + 1 == A.l ? ~0u : (1u << A.log2B) - 1;
                uint32_t x[M];
#pragma unroll
                for (int h = 0; h < M; h++) x[h] = (y[h] >> sh) & mask;
#pragma unroll
                for (int mm = 1; mm < M; mm <<= 1) {
                    const int tb = M / (2 * mm);  // pair distance in sub-rings
#pragma unroll
                    for (int g = 0; g < mm; g++) {
                        const uint32_t wt = A.twf0[mm + g];
#pragma unroll
                        for (int hh = 2 * g * tb; hh < 2 * g * tb + tb; hh++) {
                            const uint32_t uu = x[hh], v = mont_mul(x[hh + tb], wt, m);
                            x[hh] = add_q(uu, v, Q);
                            x[hh + tb] = sub_q(uu, v, Q);
                        }
                    }
                }
                uint32_t *o = dig + ((size_t)(key * A.l + u) * 2 + part) * N;
#pragma unroll
                for (int h = 0; h < M; h++) o[h * NS] = x[h];
            }
        }
    }
}

// Stage 2: one workgroup per (task, sub-ring h): the remaining forward stages of
// every digit polynomial, the product with sub-ring h of BSK_i (eq. def:gsw)
// from the digit-offset correction, and the inverse stages within the sub-ring.
template <int KEYS>
__global__ __launch_bounds__(64 * SPLIT_WAVES) __attribute__((amdgpu_waves_per_eu(2))) void k_split_sub(WideArgs A)
{
    constexpr int NS = (int)SPLIT_NS, W = SPLIT_WAVES;
    using G = Geo<NS, W>;
    constexpr int E = G::E;
    // a second exchange slot, so that consecutive relayouts alternate (one barrier each)
    constexpr bool DS = 2 * G::SLOTW * 4 <= 160 * 1024;
    static_assert(G::SLOTW % 2 == 0, "the slot ends on an 8-byte boundary");
    __shared__ uint64_t lds64[G::SLOTW / 2 * (DS ? 2 : 1)];
    uint32_t *const slot = reinterpret_cast<uint32_t *>(lds64);
    uint32_t *const slot2 = slot + G::SLOTW;
    int par = 0;
    const uint32_t M = A.M, N = M * (uint32_t)NS;
    const uint32_t task = blockIdx.x / M, h = blockIdx.x % M;
    const WideTask T = A.tasks[task];
    const uint32_t i = T.i0 + A.step;
    if (i >= A.n) return;
    const int L = threadIdx.x;
    const ModQ m{A.Q[0], A.qn[0]};
    const uint32_t *twf = A.twf_sub + (size_t)h * NS, *twi = A.twi_sub + (size_t)h * NS;
    const uint32_t *dig = A.dig + (size_t)task * KEYS * A.l * 2 * N + (size_t)h * NS;
    uint32_t out[2][E];
    {
        const uint32_t *corr = A.bsk_corr + (size_t)i * 2 * N + (size_t)h * NS + L * E;
#pragma unroll
        for (int part = 0; part < 2; part++)
#pragma unroll
            for (int k = 0; k < E; k++) out[part][k] = corr[part * N + k];
    }
    for (int key = 0; key < KEYS; key++) {
        const uint32_t *Kp = A.bsk + ((size_t)i * KEYS + key) * (2 * A.l * 2 * N) + (size_t)h * NS + L * E;
        for (uint32_t u = 0; u < A.l; u++) {
            __asm__ volatile("" ::: "memory");
            const uint32_t *db = dig + ((size_t)(key * A.l + u) * 2 + 1) * N;  // digit of b meets rows u
            const uint32_t *da = dig + ((size_t)(key * A.l + u) * 2 + 0) * N;  // digit of a meets rows l + u
            uint32_t pd[2][E];
#pragma unroll
            for (int k = 0; k < E; k++) {
                pd[0][k] = db[G::LANES * k + L];
                pd[1][k] = da[G::LANES * k + L];
            }
            ntt_fwd<NS, 2, W, false, DS>(pd, slot, twf, L, m, slot2, &par);
            const uint32_t *kb_a = Kp + ((size_t)u * 2 + 0) * N;
            const uint32_t *kb_b = Kp + ((size_t)u * 2 + 1) * N;
            const uint32_t *ka_a = Kp + ((size_t)(A.l + u) * 2 + 0) * N;
            const uint32_t *ka_b = Kp + ((size_t)(A.l + u) * 2 + 1) * N;
#pragma unroll
            for (int k = 0; k < E; k++) {
                const uint64_t xa = (uint64_t)pd[0][k] * kb_a[k] + (uint64_t)pd[1][k] * ka_a[k];
                const uint64_t xb = (uint64_t)pd[0][k] * kb_b[k] + (uint64_t)pd[1][k] * ka_b[k];
                out[0][k] = add_q(out[0][k], redc(xa, m), m.Q);
                out[1][k] = add_q(out[1][k], redc(xb, m), m.Q);
            }
        }
    }
    __asm__ volatile("" ::: "memory");
    ntt_inv<NS, 2, W, false, DS>(out, slot, twi, L, m, slot2, &par);
    uint32_t *ob = A.outb + (size_t)task * 2 * N + (size_t)h * NS;
#pragma unroll
    for (int part = 0; part < 2; part++)
#pragma unroll
        for (int k = 0; k < E; k++) ob[(size_t)part * N + G::LANES * k + L] = out[part][k];
}

// Stage 3: for column j the Gentleman-Sande stages with m = M/2, ..., 1 groups,
// then ACC_j + product into the other buffer; a task past step n - 1 copies.
template <int M>
__global__ __launch_bounds__(256) void k_split_post(WideArgs A)
{
    constexpr uint32_t NS = SPLIT_NS, N = M * NS;
    const uint32_t task = blockIdx.y;
    const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    const WideTask T = A.tasks[task];
    const uint32_t i = T.i0 + A.step;
    const uint32_t *own = A.acc_rd + T.acc_off + (size_t)T.comp * 2 * N;
    uint32_t *wr = A.acc_wr + T.acc_off + (size_t)T.comp * 2 * N;
    const uint32_t Q = A.Q[0];
    if (i >= A.n) {
#pragma unroll
        for (int part = 0; part < 2; part++)
#pragma unroll
            for (int h = 0; h < M; h++) wr[part * N + j + h * NS] = own[part * N + j + h * NS];
        return;
    }
    const ModQ m{Q, A.qn[0]};
    const uint32_t *ob = A.outb + (size_t)task * 2 * N + j;
#pragma unroll
    for (int part = 0; part < 2; part++) {
        uint32_t x[M];
#pragma unroll
        for (int h = 0; h < M; h++) x[h] = ob[part * N + h * NS];
#pragma unroll
        for (int mm = M / 2; mm >= 1; mm >>= 1) {
            const int tb = M / (2 * mm);
#pragma unroll
            for (int g = 0; g < mm; g++) {
                const uint32_t wt = A.twi0[mm + g];
#pragma unroll
                for (int hh = 2 * g * tb; hh < 2 * g * tb + tb; hh++) {
                    const uint32_t uu = x[hh], v = x[hh + tb];
                    x[hh] = add_q(uu, v, Q);
                    x[hh + tb] = mont_mul(sub_q(uu, v, Q), wt, m);
                }
            }
        }
#pragma unroll
        for (int h = 0; h < M; h++) {
            const uint32_t idx = part * N + j + h * NS;
            wr[idx] = add_q(own[idx], x[h], Q);
        }
    }
}

// ------------------------------------------------------------------ launchers

// Two primes: N <= 4096 (the second prime is 1 mod 2^13); one prime: up to 16384.
#define WIDE_DISPATCH(N_, NPR_, CALL)                 \
    if (NPR_ == 2) {                                  \
        switch (N_) {                                 \
        case 256: CALL(256, 2); break;                \
        case 512: CALL(512, 2); break;                \
        case 1024: CALL(1024, 2); break;              \
        case 2048: CALL(2048, 2); break;              \
        case 4096: CALL(4096, 2); break;              \
        default: break;                               \
        }                                             \
    } else {                                          \
        switch (N_) {                                 \
        case 256: CALL(256, 1); break;                \
        case 512: CALL(512, 1); break;                \
        case 1024: CALL(1024, 1); break;              \
        case 2048: CALL(2048, 1); break;              \
        case 4096: CALL(4096, 1); break;              \
        case 8192: CALL(8192, 1); break;              \
        case 16384: CALL(16384, 1); break;            \
        default: break;                               \
        }                                             \
    }

// Rings above 16384 (one prime): only the per-coefficient kernels exist at that size.
#define BIG_DISPATCH(N_, CALL)          \
    switch (N_) {                       \
    case 32768: CALL(32768, 1); break;  \
    case 65536: CALL(65536, 1); break;  \
    default: break;                     \
    }

void launch_wide_init(uint32_t N, int npr, const WideArgs &A, uint32_t num_tasks, hipStream_t st)
{
#define C_(n, p) hipLaunchKernelGGL((k_wide_init<n, p>), dim3(num_tasks), dim3(256), 0, st, A)
    if (N > 16384 && npr == 1) {
        BIG_DISPATCH(N, C_)
    } else {
        WIDE_DISPATCH(N, npr, C_)
    }
#undef C_
}

// One CMux-step launch with one workgroup per component and prime (two primes only),
// of dg digit groups (two: N = 1024 and 2048).
template <int n, int p, int dg = 1>
static void ps_launch(uint32_t keys, const WideArgs &A, uint32_t num_tasks, hipStream_t st)
{
    if constexpr (p == 2 && (dg == 1 || n == 1024 || n == 2048)) {
        const dim3 grid(2 * num_tasks), block(64 * wide_wpp(n) * dg);
        if (keys == 2) hipLaunchKernelGGL((k_wide_step<n, 2, 2, wide_wpp(n), dg, true>), grid, block, 0, st, A);
        else hipLaunchKernelGGL((k_wide_step<n, 1, 2, wide_wpp(n), dg, true>), grid, block, 0, st, A);
    }
}

void launch_wide_step(uint32_t N, int npr, uint32_t keys, const WideArgs &A, uint32_t num_tasks, hipStream_t st,
                      int wpp, int dg, bool ps)
{
    if (ps && npr == 2) {
        if (dg == 2 && N == 1024) ps_launch<1024, 2, 2>(keys, A, num_tasks, st);
        else if (dg == 2 && N == 2048) ps_launch<2048, 2, 2>(keys, A, num_tasks, st);
        else {
#define P_(n, p) ps_launch<n, p>(keys, A, num_tasks, st)
            WIDE_DISPATCH(N, 2, P_)
#undef P_
        }
        return;
    }
    if (dg == 2 && npr == 1 && N == 1024 && wpp == 4) {
        if (keys == 2) hipLaunchKernelGGL((k_wide_step<1024, 2, 1, 4, 2>), dim3(num_tasks), dim3(512), 0, st, A);
        else hipLaunchKernelGGL((k_wide_step<1024, 1, 1, 4, 2>), dim3(num_tasks), dim3(512), 0, st, A);
        return;
    }
    if (npr == 1 && wpp > 0 && wpp != wide_wpp((int)N)) {
        // twice the waves per component (N = 512, 1024; one prime): the step's work
        // on more SIMDs of each component's compute unit
#define L_(n, w)                                                                                                \
    if (keys == 2) hipLaunchKernelGGL((k_wide_step<n, 2, 1, w>), dim3(num_tasks), dim3(64 * w), 0, st, A); \
    else hipLaunchKernelGGL((k_wide_step<n, 1, 1, w>), dim3(num_tasks), dim3(64 * w), 0, st, A)
        if (N == 1024 && wpp == 4) L_(1024, 4);
        else if (N == 512 && wpp == 2) L_(512, 2);
#undef L_
        return;
    }
#define C_(n, p)                                                                                                   \
    if (keys == 2) hipLaunchKernelGGL((k_wide_step<n, 2, p>), dim3(num_tasks), dim3(64 * wide_wpp(n)), 0, st, A); \
    else hipLaunchKernelGGL((k_wide_step<n, 1, p>), dim3(num_tasks), dim3(64 * wide_wpp(n)), 0, st, A)
    WIDE_DISPATCH(N, npr, C_)
#undef C_
}

void launch_wide_extract(uint32_t N, int npr, const WideArgs &A, const uint64_t *acc_off, size_t count,
                         uint32_t *ext, hipStream_t st)
{
#define C_(n, p) hipLaunchKernelGGL((k_wide_extract<n, p>), dim3((uint32_t)count), dim3(256), 0, st, A, acc_off, ext)
    if (N > 16384 && npr == 1) {
        BIG_DISPATCH(N, C_)
    } else {
        WIDE_DISPATCH(N, npr, C_)
    }
#undef C_
}

void launch_split_step(uint32_t N, uint32_t keys, const WideArgs &A, uint32_t num_tasks, hipStream_t st)
{
    const uint32_t M = N / SPLIT_NS;
    const dim3 cols(SPLIT_NS / 256, num_tasks);
#define D_(mm)                                                                                           \
    if (keys == 2) hipLaunchKernelGGL((k_split_digits<mm, 2>), cols, dim3(256), 0, st, A);            \
    else hipLaunchKernelGGL((k_split_digits<mm, 1>), cols, dim3(256), 0, st, A);                       \
    if (keys == 2) hipLaunchKernelGGL(k_split_sub<2>, dim3(num_tasks * mm), dim3(64 * SPLIT_WAVES), 0, st, A); \
    else hipLaunchKernelGGL(k_split_sub<1>, dim3(num_tasks * mm), dim3(64 * SPLIT_WAVES), 0, st, A);            \
    hipLaunchKernelGGL((k_split_post<mm>), cols, dim3(256), 0, st, A)
    switch (M) {
    case 2: D_(2); break;
    case 4: D_(4); break;
    case 8: D_(8); break;
    default: break;
    }
#undef D_
}

bool split_supports_n(uint32_t N) { return N == 16384 || N == 32768 || N == 65536; }

void launch_wide_export(uint32_t N, const WideArgs &A, uint32_t num_tasks, uint32_t *out, hipStream_t st)
{
#define C_(n, p) hipLaunchKernelGGL(k_wide_export<n>, dim3(num_tasks), dim3(256), 0, st, A, out)
    WIDE_DISPATCH(N, 2, C_)
#undef C_
}

#undef WIDE_DISPATCH
#undef BIG_DISPATCH

int wide_waves_per_poly(uint32_t N) { return wide_wpp((int)N); }

bool wide_supports_wpp(uint32_t N, int npr, int wpp)
{
    return wpp == wide_wpp((int)N) || (npr == 1 && ((N == 1024 && wpp == 4) || (N == 512 && wpp == 2)));
}

bool wide_supports_dg(uint32_t N, int npr, int wpp) { return N == 1024 && npr == 1 && wpp == 4; }

bool wide_supports_ps(uint32_t N, int npr, int dg) { return npr == 2 && wide_supports_n(N, 2) && (dg == 1 || N == 1024 || N == 2048); }

bool wide_supports_n(uint32_t N, int npr)
{
    if (N < 256 || N > (npr == 2 ? 4096u : 65536u)) return false;
    return (N & (N - 1)) == 0;
}

}  // namespace dev
}  // namespace mm
