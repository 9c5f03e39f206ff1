// Device-side building blocks shared by the kernels: exact arithmetic mod Q
// (Q odd, Q < 2^31), the negacyclic NTT held in registers, and the external
// product of one RLWE pair by one bootstrapping-key row block.
//
// Data layout of one degree-N polynomial: it is spread over WPP waves (by
// default 1 up to N = 1024 and N / 1024 above) that act as one set of LANES =
// 64 WPP virtual lanes, each holding E = N / LANES coefficients.  The NTT runs
// in NPH phases; in phase p virtual lane L and register k hold coefficient
//     idx_p(L, k) = ((L >> R_p) << (R_p + LE)) | (k << R_p) | (L & (2^R_p - 1)),
// R_p = max(0, LL - p * LE), LE = log2 E, LL = log2 LANES.  Phase 0 (R = LL)
// is the natural layout idx = LANES k + L used for coefficient-domain work
// (rotation, decomposition, accumulation); the last phase (R = 0) is
// idx = E L + k, in which the NTT output is consumed pointwise.  Butterflies
// whose two inputs differ in a register bit are done in registers; between
// phases the lanes swap layout through an LDS slot (the wave's own when
// WPP = 1, shared by the WPP waves otherwise, with workgroup barriers).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace mm {
namespace dev {

constexpr int ilog2(int x) { return x <= 1 ? 0 : 1 + ilog2(x / 2); }

// Waves per polynomial by default: one up to N = 1024, N / 1024 above (16
// coefficients per lane); a kernel may spread a polynomial over more waves.
constexpr int default_wpp(int N) { return N > 1024 ? N / 1024 : 1; }

template <int N, int W = default_wpp(N)>
struct Geo {
    static constexpr int WPP = W;  // waves per polynomial
    static constexpr int LANES = 64 * WPP;
    static constexpr int LL = ilog2(LANES);
    static constexpr int E = N / LANES;
    static constexpr int LE = ilog2(E);
    static constexpr int LOGN = ilog2(N);
    static constexpr int NPH = 1 + (LL + LE - 1) / LE;
    static constexpr int PAD = N / 16;            // one pad word per 16
    static constexpr int POLYW = N + PAD;         // words of one swizzled poly in LDS
    static constexpr int SLOTW = 2 * POLYW;       // an exchange slot: two polys
    __host__ __device__ static constexpr int R(int p) { return LL - p * LE < 0 ? 0 : LL - p * LE; }
    // highest idx bit whose butterflies run in phase p
    __host__ __device__ static constexpr int HI(int p) { return p == 0 ? LOGN - 1 : R(p - 1) - 1; }
    static_assert(N == LANES * E && E >= 4 && E <= 16 && WPP <= 16,
                  "device path supports N in {256, 512, ..., 16384}");
};

// LDS word address of coefficient idx: one pad word per 16 keeps all phase
// layouts (strides 1, 2^R_p and E between neighbouring lanes) free of bank conflicts.
__host__ __device__ constexpr int swz(int idx) { return idx + (idx >> 4); }

template <int N, int W = default_wpp(N)>
__host__ __device__ constexpr int idx_of(int p, int L, int k)
{
    using G = Geo<N, W>;
    const int R = G::R(p);
    return ((L >> R) << (R + G::LE)) | (k << R) | (L & ((1 << R) - 1));
}

// swz(idx_of(p, L, k)) = swz_base(p, L) + swz_off(R_p, k): the register index k
// only adds a constant (its bits sit between the lane's high and low bits and,
// below bit 4, never carry past it), so a relayout needs one address register
// per side and immediate offsets for the E registers.
template <int N, int W = default_wpp(N)>
__host__ __device__ constexpr int swz_base(int p, int L)
{
    using G = Geo<N, W>;
    const int R = G::R(p);
    const int H = (L >> R) << (R + G::LE), Lo = L & ((1 << R) - 1);
    return H + (H >> 4) + Lo + (R >= 4 ? (Lo >> 4) : 0);
}

__host__ __device__ constexpr int swz_off(int R, int k) { return (k << R) + (R >= 4 ? k << (R - 4) : k >> (4 - R)); }

// Every phase, lane and register of a geometry obeys the split above.
template <int N, int W = default_wpp(N)>
constexpr bool swz_split_holds()
{
    using G = Geo<N, W>;
    for (int p = 0; p < G::NPH; p++)
        for (int L = 0; L < G::LANES; L++)
            for (int k = 0; k < G::E; k++)
                if (swz(idx_of<N, W>(p, L, k)) != swz_base<N, W>(p, L) + swz_off(G::R(p), k)) return false;
    return true;
}

struct ModQ {
    uint32_t Q;   // odd modulus < 2^31
    uint32_t qn;  // -Q^{-1} mod 2^32
};

__device__ __forceinline__ uint32_t add_q(uint32_t a, uint32_t b, uint32_t Q)
{
    const uint32_t s = a + b;  // a, b < Q < 2^31
    return min(s, s - Q);
}

__device__ __forceinline__ uint32_t sub_q(uint32_t a, uint32_t b, uint32_t Q)
{
    const uint32_t d = a - b;  // wraps when a < b; then d + Q is the answer and smaller
    return min(d, d + Q);
}

// Montgomery reduction of x < 2^32 Q: x 2^-32 mod Q in [0, Q).
__device__ __forceinline__ uint32_t redc(uint64_t x, const ModQ &m)
{
    const uint32_t q = (uint32_t)x * m.qn;
    const uint32_t t = (uint32_t)((x + (uint64_t)q * m.Q) >> 32);  // < 2Q
    return min(t, t - m.Q);
}

// a * w 2^-32 mod Q for a < 2^32, w < Q (w held in Montgomery form w 2^32).
__device__ __forceinline__ uint32_t mont_mul(uint32_t a, uint32_t w, const ModQ &m)
{
    return redc((uint64_t)a * w, m);
}

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Barrier between the lanes that share a polynomial: the wave itself, or the
// whole workgroup when a polynomial spans several waves.
template <int N, int W = default_wpp(N)>
__device__ __forceinline__ void poly_sync()
{
    if constexpr (W == 1) wave_sync();
    else __syncthreads();
}

// Move NP polys from the layout of phase `from` to that of phase `to`
// through the LDS slot (NP <= 2).  Lf and Lt are the (virtual) lanes by which
// the two phases address their layouts.
//
// PRIO: the wave drops its issue priority for the LDS round trip and raises it
// again for the butterflies that follow, so that of the waves sharing a SIMD
// the ones with arithmetic ready issue first; the VALU is the bound.  Where a
// relayout is wave-private (one wave per polynomial) this gains (1.8 % on the
// 4096-ciphertext batch at N = 1024); where relayouts end at workgroup
// barriers it loses (4-5 % at N = 4096), since the barrier then waits for the
// waves held back, hence the default.
//
// SYNC_BEFORE = false drops the barrier that keeps the writes from overtaking the
// previous relayout's reads; valid only when consecutive relayouts alternate
// between two slots (then the previous user of this slot is two relayouts back,
// and every wave finished reading it before it wrote for the relayout in between,
// whose barrier this wave has passed).
template <int N, int NP, int W = default_wpp(N), bool PRIO = (W == 1), bool SYNC_BEFORE = true>
__device__ __forceinline__ void relayout(uint32_t (&x)[NP][(Geo<N, W>::E)], uint32_t *slot, int Lf, int Lt,
                                         int from, int to)
{
    using G = Geo<N, W>;
    static_assert(swz_split_holds<N, W>(), "LDS address split");
    uint32_t *sf = slot + swz_base<N, W>(from, Lf), *st = slot + swz_base<N, W>(to, Lt);
    if constexpr (PRIO) __builtin_amdgcn_s_setprio(0);
    if constexpr (SYNC_BEFORE) poly_sync<N, W>();
#pragma unroll
    for (int q = 0; q < NP; q++)
#pragma unroll
        for (int k = 0; k < G::E; k++) sf[q * G::POLYW + swz_off(G::R(from), k)] = x[q][k];
    poly_sync<N, W>();
#pragma unroll
    for (int q = 0; q < NP; q++)
#pragma unroll
        for (int k = 0; k < G::E; k++) x[q][k] = st[q * G::POLYW + swz_off(G::R(to), k)];
    if constexpr (PRIO) __builtin_amdgcn_s_setprio(1);
}

// One relayout through `slot`, or, with DS, through slot and slot2 in turn (par
// counts the relayouts since the last workgroup barrier), dropping the barrier
// before the writes.
template <int N, int NP, int W, bool PRIO, bool DS>
__device__ __forceinline__ void relayout_ds(uint32_t (&x)[NP][(Geo<N, W>::E)], uint32_t *slot, uint32_t *slot2,
                                            int *par, int Lf, int Lt, int from, int to)
{
    if constexpr (DS) {
        uint32_t *s = (*par & 1) ? slot2 : slot;
        *par ^= 1;
        relayout<N, NP, W, PRIO, false>(x, s, Lf, Lt, from, to);
    } else {
        relayout<N, NP, W, PRIO>(x, slot, Lf, Lt, from, to);
    }
}

// Lane-swap exchange (PL) between the last two NTT phases.  Where one wave
// holds a polynomial and the next-to-last phase has R = 2 (N = 256 and 1024),
// the two layouts differ only in which holds idx bits 0, 1 (lanes) and which
// the two idx bits above the registers' (registers).  With PL the next-to-last
// phase runs on the virtual lane pl_lane(L), which puts idx bits 0, 1 on lane
// bits 4, 5, so the exchange is two wavefront lane swaps: v_permlane16_swap
// across lane bit 4 and v_permlane32_swap across lane bit 5, each exchanging
// one register bit for the lane bit in one instruction per register pair,
// instead of an LDS round trip.  Afterwards physical register k holds virtual
// register pl_reg(k) of the last phase, whose lane is pl_lane(L) as well.
template <int N, int W>
constexpr bool pl_ok()
{
    using G = Geo<N, W>;
    return W == 1 && G::NPH >= 3 && G::R(G::NPH - 2) == 2;
}

__host__ __device__ constexpr int pl_lane(int L) { return ((L >> 4) & 3) | ((L & 15) << 2); }

// an involution: swaps the register bits {LE-2, LE-1} with {0, 1}, keeping the order
template <int LE>
__host__ __device__ constexpr int pl_reg(int k)
{
    return (k >> (LE - 2)) | ((k & ((1 << (LE - 2)) - 1)) << 2);
}

template <int N, int W, bool PL>
__device__ __forceinline__ int phase_lane(int p, int L)
{
    if constexpr (PL) return p >= Geo<N, W>::NPH - 2 ? pl_lane(L) : L;
    else return L;
}

// physical register of virtual register k in phase p
template <int N, int W, bool PL>
__host__ __device__ constexpr int phase_reg(int p, int k)
{
    return (PL && p == Geo<N, W>::NPH - 1) ? pl_reg<Geo<N, W>::LE>(k) : k;
}

template <int E, int NP>
__device__ __forceinline__ void lane_swap_45(uint32_t (&x)[NP][E])
{
    constexpr int LE = ilog2(E), b4 = 1 << (LE - 2), b5 = 1 << (LE - 1);
#pragma unroll
    for (int q = 0; q < NP; q++)
#pragma unroll
        for (int k0 = 0; k0 < E; k0++) {
            if (k0 & b4) continue;
            const auto r = __builtin_amdgcn_permlane16_swap(x[q][k0], x[q][k0 | b4], false, false);
            x[q][k0] = r[0];
            x[q][k0 | b4] = r[1];
        }
#pragma unroll
    for (int q = 0; q < NP; q++)
#pragma unroll
        for (int k0 = 0; k0 < E; k0++) {
            if (k0 & b5) continue;
            const auto r = __builtin_amdgcn_permlane32_swap(x[q][k0], x[q][k0 | b5], false, false);
            x[q][k0] = r[0];
            x[q][k0 | b5] = r[1];
        }
}

// Forward negacyclic NTT (Cooley-Tukey, merged psi powers, natural order in,
// bit-reversed order out) of NP polys held in phase-0 layout; returns them in
// the last phase's layout, reduced to [0, Q) (inputs in [0, Q)).
// twf[k] = psi^bitrev(k) 2^32 mod Q.
// The butterflies of NTT phase p for one polynomial (forward: Cooley-Tukey,
// merged psi powers) and, for p > 0, the reduction of the values the previous
// phase left unreduced that are not multiplicands of this phase's first stage.
template <int N, int W, bool PL>
__device__ __forceinline__ void fwd_phase(uint32_t (&x)[(Geo<N, W>::E)], int p, const uint32_t *twf, int L,
                                          const ModQ &m)
{
    using G = Geo<N, W>;
    const int R = G::R(p);
    const int Lp = phase_lane<N, W, PL>(p, L);
    if (p > 0) {
        const int kt = G::HI(p) - R;
#pragma unroll
        for (int k = 0; k < G::E; k++)
            if (!((k >> kt) & 1)) {
                uint32_t &v = x[phase_reg<N, W, PL>(p, k)];
                v = min(v, v - m.Q);
            }
    }
    const int Lhi = (p == 0) ? 0 : (Lp >> R);
#pragma unroll
    for (int b = G::HI(p); b >= R; b--) {
        const int kb = b - R, s = G::LOGN - 1 - b;
#pragma unroll
        for (int k0 = 0; k0 < G::E; k0++) {
            if (k0 & (1 << kb)) continue;
            const int k1 = k0 | (1 << kb);
            const uint32_t w = twf[(1 << s) + ((Lhi << (G::LE - kb - 1)) | (k0 >> (kb + 1)))];
            // Both outputs differ from each other only in bit b, so they agree on bit
            // b - 1: when that bit is 1 both are multiplicands of the next stage, where
            // any 32-bit value is a valid Montgomery input (x w < 2^32 Q), and they
            // stay unreduced in [0, 2Q).  In the last stage of a phase bit b - 1 is a
            // lane bit, so all outputs stay unreduced and the next phase reduces its
            // non-multiplicands after the relayout; the last phase ends reduced.
            const bool lazy = kb > 0 ? ((k0 >> (kb - 1)) & 1) != 0 : p + 1 < G::NPH;
            const int r0 = phase_reg<N, W, PL>(p, k0), r1 = phase_reg<N, W, PL>(p, k1);
            const uint32_t u = x[r0];
            const uint32_t v = mont_mul(x[r1], w, m);
            if (lazy) {
                x[r0] = u + v;
                x[r1] = u - v + m.Q;
            } else {
                x[r0] = add_q(u, v, m.Q);
                x[r1] = sub_q(u, v, m.Q);
            }
        }
    }
}

// Inverse butterflies (Gentleman-Sande) of phase p for one polynomial.
template <int N, int W, bool PL>
__device__ __forceinline__ void inv_phase(uint32_t (&x)[(Geo<N, W>::E)], int p, const uint32_t *twi, int L,
                                          const ModQ &m)
{
    using G = Geo<N, W>;
    const int R = G::R(p);
    const int Lp = phase_lane<N, W, PL>(p, L);
    const int Lhi = (p == 0) ? 0 : (Lp >> R);
#pragma unroll
    for (int b = R; b <= G::HI(p); b++) {
        const int kb = b - R, s = G::LOGN - 1 - b;
#pragma unroll
        for (int k0 = 0; k0 < G::E; k0++) {
            if (k0 & (1 << kb)) continue;
            const int k1 = k0 | (1 << kb);
            const uint32_t w = twi[(1 << s) + ((Lhi << (G::LE - kb - 1)) | (k0 >> (kb + 1)))];
            const int r0 = phase_reg<N, W, PL>(p, k0), r1 = phase_reg<N, W, PL>(p, k1);
            const uint32_t u = x[r0], v = x[r1];
            x[r0] = add_q(u, v, m.Q);
            x[r1] = mont_mul(u - v + m.Q, w, m);
        }
    }
}

// One polynomial's half of a wave-private relayout (one wave per polynomial):
// the writes of its layout in phase `from`, then the reads of phase `to`.  LDS
// operations of one wave complete in order, so the reads see the writes; the
// wave barriers only keep the compiler from reordering them.
template <int N, int W>
__device__ __forceinline__ void swap_layout_1(uint32_t (&x)[(Geo<N, W>::E)], uint32_t *slot, int L, int from, int to)
{
    using G = Geo<N, W>;
    static_assert(W == 1, "wave-private relayout");
    uint32_t *sf = slot + swz_base<N, W>(from, L), *st = slot + swz_base<N, W>(to, L);
    wave_sync();
#pragma unroll
    for (int k = 0; k < G::E; k++) sf[swz_off(G::R(from), k)] = x[k];
    wave_sync();
#pragma unroll
    for (int k = 0; k < G::E; k++) x[k] = st[swz_off(G::R(to), k)];
}

// Forward negacyclic NTT (Cooley-Tukey, merged psi powers, natural order in,
// bit-reversed order out) of NP polys held in phase-0 layout; returns them in
// the last phase's layout, reduced to [0, Q) (inputs in [0, Q)).
// twf[k] = psi^bitrev(k) 2^32 mod Q.
//
// ST (staggered, one wave per polynomial, NP = 2): the two polynomials take
// turns so that each one's relayout is in flight while the other one's
// butterflies run: phase p of poly 0, its writes and the reads of phase p + 1,
// then phase p of poly 1 and its relayout, then phase p + 1 of poly 0, whose
// data has arrived meanwhile.  The same instructions as the lockstep order,
// which waits for every relayout's reads right after issuing them.
template <int N, int NP, int W = default_wpp(N), bool PRIO = (W == 1), bool DS = false, bool PL = false,
          bool ST = false>
__device__ __forceinline__ void ntt_fwd(uint32_t (&x)[NP][(Geo<N, W>::E)], uint32_t *slot, const uint32_t *twf,
                                        int L, const ModQ &m, uint32_t *slot2 = nullptr, int *par = nullptr)
{
    using G = Geo<N, W>;
    static_assert(!PL || pl_ok<N, W>(), "lane-swap exchange needs one wave per polynomial and R = 2 before the last phase");
    static_assert(!ST || (W == 1 && NP == 2 && !PL && !DS), "staggered relayouts: one wave per polynomial, two polys");
    if constexpr (ST) {
#pragma unroll
        for (int p = 0; p < G::NPH; p++)
#pragma unroll
            for (int q = 0; q < NP; q++) {
                fwd_phase<N, W, false>(x[q], p, twf, L, m);
                if (p + 1 < G::NPH) swap_layout_1<N, W>(x[q], slot + q * G::POLYW, L, p, p + 1);
            }
        return;
    }
#pragma unroll
    for (int p = 0; p < G::NPH; p++) {
        const int R = G::R(p);
        const int Lp = phase_lane<N, W, PL>(p, L);
        if (p > 0) {
            if (PL && p == G::NPH - 1) lane_swap_45<G::E, NP>(x);
            else relayout_ds<N, NP, W, PRIO, DS>(x, slot, slot2, par, phase_lane<N, W, PL>(p - 1, L), Lp, p - 1, p);
            // the previous phase left its last stage unreduced; reduce the values
            // that are not multiplicands of this phase's first stage
            const int kt = G::HI(p) - R;
#pragma unroll
            for (int k = 0; k < G::E; k++)
                if (!((k >> kt) & 1))
#pragma unroll
                    for (int q = 0; q < NP; q++) {
                        uint32_t &v = x[q][phase_reg<N, W, PL>(p, k)];
                        v = min(v, v - m.Q);
                    }
        }
        // the polys in lockstep, butterfly by butterfly (lazy outputs as in fwd_phase)
        const int Lhi = (p == 0) ? 0 : (Lp >> R);
#pragma unroll
        for (int b = G::HI(p); b >= R; b--) {
            const int kb = b - R, s = G::LOGN - 1 - b;
#pragma unroll
            for (int k0 = 0; k0 < G::E; k0++) {
                if (k0 & (1 << kb)) continue;
                const int k1 = k0 | (1 << kb);
                const uint32_t w = twf[(1 << s) + ((Lhi << (G::LE - kb - 1)) | (k0 >> (kb + 1)))];
                const bool lazy = kb > 0 ? ((k0 >> (kb - 1)) & 1) != 0 : p + 1 < G::NPH;
                const int r0 = phase_reg<N, W, PL>(p, k0), r1 = phase_reg<N, W, PL>(p, k1);
#pragma unroll
                for (int q = 0; q < NP; q++) {
                    const uint32_t u = x[q][r0];
                    const uint32_t v = mont_mul(x[q][r1], w, m);
                    if (lazy) {
                        x[q][r0] = u + v;
                        x[q][r1] = u - v + m.Q;
                    } else {
                        x[q][r0] = add_q(u, v, m.Q);
                        x[q][r1] = sub_q(u, v, m.Q);
                    }
                }
            }
        }
    }
}

// Inverse negacyclic NTT (Gentleman-Sande, bit-reversed in, natural out),
// without the 1/N factor: polys arrive in the last phase's layout and leave in
// phase-0 layout.  twi[k] = psi^-bitrev(k) 2^32 mod Q.  ST as in ntt_fwd.
template <int N, int NP, int W = default_wpp(N), bool PRIO = (W == 1), bool DS = false, bool PL = false,
          bool ST = false>
__device__ __forceinline__ void ntt_inv(uint32_t (&x)[NP][(Geo<N, W>::E)], uint32_t *slot, const uint32_t *twi,
                                        int L, const ModQ &m, uint32_t *slot2 = nullptr, int *par = nullptr)
{
    using G = Geo<N, W>;
    static_assert(!PL || pl_ok<N, W>(), "lane-swap exchange needs one wave per polynomial and R = 2 before the last phase");
    static_assert(!ST || (W == 1 && NP == 2 && !PL && !DS), "staggered relayouts: one wave per polynomial, two polys");
    if constexpr (ST) {
#pragma unroll
        for (int p = G::NPH - 1; p >= 0; p--)
#pragma unroll
            for (int q = 0; q < NP; q++) {
                inv_phase<N, W, false>(x[q], p, twi, L, m);
                if (p > 0) swap_layout_1<N, W>(x[q], slot + q * G::POLYW, L, p, p - 1);
            }
        return;
    }
#pragma unroll
    for (int p = G::NPH - 1; p >= 0; p--) {
        const int R = G::R(p);
        const int Lp = phase_lane<N, W, PL>(p, L);
        const int Lhi = (p == 0) ? 0 : (Lp >> R);
        // the polys in lockstep, butterfly by butterfly
#pragma unroll
        for (int b = R; b <= G::HI(p); b++) {
            const int kb = b - R, s = G::LOGN - 1 - b;
#pragma unroll
            for (int k0 = 0; k0 < G::E; k0++) {
                if (k0 & (1 << kb)) continue;
                const int k1 = k0 | (1 << kb);
                const uint32_t w = twi[(1 << s) + ((Lhi << (G::LE - kb - 1)) | (k0 >> (kb + 1)))];
                const int r0 = phase_reg<N, W, PL>(p, k0), r1 = phase_reg<N, W, PL>(p, k1);
#pragma unroll
                for (int q = 0; q < NP; q++) {
                    const uint32_t u = x[q][r0], v = x[q][r1];
                    x[q][r0] = add_q(u, v, m.Q);
                    x[q][r1] = mont_mul(u - v + m.Q, w, m);
                }
            }
        }
        if (p > 0) {
            if (PL && p == G::NPH - 1) lane_swap_45<G::E, NP>(x);
            else relayout_ds<N, NP, W, PRIO, DS>(x, slot, slot2, par, Lp, phase_lane<N, W, PL>(p - 1, L), p, p - 1);
        }
    }
}

struct GadgetC {
    uint32_t log2B, l, sg;
    uint32_t off;  // (B/2)(1 + B + ... + B^(l-2)): makes the low l-1 balanced digits unsigned bit fields
};

// y' = round(centred(x) / 2^sg) + off for x in [0, Q]; x = Q is read as 0.
// With the offset, balanced digit u < l-1 is bits [u log2B, (u+1) log2B) of y'
// minus B/2, and the top digit is y' >> ((l-1) log2B) (arithmetic).
__device__ __forceinline__ int32_t gadget_start(uint32_t x, const GadgetC &g, uint32_t Q)
{
    int32_t xc = (x > (Q - 1) / 2) ? (int32_t)(x - Q) : (int32_t)x;
    if (g.sg) xc = (xc + (1 << (g.sg - 1))) >> g.sg;
    return xc + (int32_t)g.off;
}

// Balanced digit u of y' as a residue mod Q.
__device__ __forceinline__ uint32_t gadget_digit(int32_t y, uint32_t u, const GadgetC &g, uint32_t Q)
{
    if (u + 1 == g.l) {
        const int32_t d = y >> (u * g.log2B);
        return d < 0 ? (uint32_t)(d + (int32_t)Q) : (uint32_t)d;
    }
    const uint32_t v = __builtin_amdgcn_ubfe((uint32_t)y, u * g.log2B, g.log2B) - (1u << (g.log2B - 1));
    return min(v, v + Q);  // v < 0 as a signed value -> v + Q
}

// Bit field u of y'' = round(centred(x) / 2^sg) + (B/2)(1 + B + ... + B^(l-1)):
// the balanced digit u plus B/2, in [0, B) below the top and in [0, B] at the
// top (which keeps the final carry), so one extract per digit and no sign fix.
__device__ __forceinline__ uint32_t gadget_field_start(uint32_t x, uint32_t off_all, const GadgetC &g, uint32_t Q)
{
    int32_t xc = (x > (Q - 1) / 2) ? (int32_t)(x - Q) : (int32_t)x;
    if (g.sg) xc = (xc + (1 << (g.sg - 1))) >> g.sg;
    return (uint32_t)xc + off_all;
}

// out += g^{-1}(Da, Db) x K in the NTT domain for one RLWE pair in phase-0
// layout, K the RGSW key block [2l][2][N] in the NTT domain (Montgomery form,
// 1/N folded in): digits of b meet rows u < l, digits of a meet rows l + u
// (eq. def:gsw).  out stays in the last phase's layout.  With OFF the digits
// enter shifted by +B/2 (g.off then holds (B/2)(1 + ... + B^(l-1))) and the
// caller starts out from minus (B/2) sum_rows K.
template <int N, bool OFF = false, int W = default_wpp(N), bool PRIO = (W == 1), bool DS = false, bool PL = false,
          bool ST = false>
__device__ __forceinline__ void ext_mac(const uint32_t (&Da)[(Geo<N, W>::E)], const uint32_t (&Db)[(Geo<N, W>::E)],
                                        const uint32_t *__restrict__ K, uint32_t *slot, const uint32_t *twf, int L,
                                        const ModQ &m, const GadgetC &g, uint32_t (&out)[2][(Geo<N, W>::E)],
                                        uint32_t *slot2 = nullptr, int *par = nullptr)
{
    using G = Geo<N, W>;
    constexpr int E = G::E;
    uint32_t ya[E], yb[E];
#pragma unroll
    for (int k = 0; k < E; k++) {
        if constexpr (OFF) {
            ya[k] = gadget_field_start(Da[k], g.off, g, m.Q);
            yb[k] = gadget_field_start(Db[k], g.off, g, m.Q);
        } else {
            ya[k] = (uint32_t)gadget_start(Da[k], g, m.Q);
            yb[k] = (uint32_t)gadget_start(Db[k], g, m.Q);
        }
    }
    for (uint32_t u = 0; u < g.l; u++) {
        // keep twiddle and key loads inside the iteration (register pressure)
        __asm__ volatile("" ::: "memory");
        uint32_t pd[2][E];
        const uint32_t sh = u * g.log2B, wd = g.log2B + (u + 1 == g.l ? 1u : 0u);
#pragma unroll
        for (int k = 0; k < E; k++) {
            if constexpr (OFF) {
                pd[0][k] = __builtin_amdgcn_ubfe(yb[k], sh, wd);
                pd[1][k] = __builtin_amdgcn_ubfe(ya[k], sh, wd);
            } else {
                pd[0][k] = gadget_digit((int32_t)yb[k], u, g, m.Q);
                pd[1][k] = gadget_digit((int32_t)ya[k], u, g, m.Q);
            }
        }
        ntt_fwd<N, 2, W, PRIO, DS, PL, ST>(pd, slot, twf, L, m, slot2, par);
        // the lane now holds NTT positions E Lk .. E Lk + E - 1 (Lk its lane in the
        // last phase), position E Lk + v in register phase_reg(last, v)
        const int Lk = phase_lane<N, W, PL>(G::NPH - 1, L);
        const uint32_t *kb_a = K + ((size_t)(u)*2 + 0) * N + Lk * E;
        const uint32_t *kb_b = K + ((size_t)(u)*2 + 1) * N + Lk * E;
        const uint32_t *ka_a = K + ((size_t)(g.l + u) * 2 + 0) * N + Lk * E;
        const uint32_t *ka_b = K + ((size_t)(g.l + u) * 2 + 1) * N + Lk * E;
#pragma unroll
        for (int k = 0; k < E; k++) {
            const int v = phase_reg<N, W, PL>(G::NPH - 1, k);  // an involution: also the word of register k
            const uint64_t xa = (uint64_t)pd[0][k] * kb_a[v] + (uint64_t)pd[1][k] * ka_a[v];
            const uint64_t xb = (uint64_t)pd[0][k] * kb_b[v] + (uint64_t)pd[1][k] * ka_b[v];
            out[0][k] = add_q(out[0][k], redc(xa, m), m.Q);
            out[1][k] = add_q(out[1][k], redc(xb, m), m.Q);
        }
    }
}

// out = g^{-1}(Da, Db) x K, coefficient domain, phase-0 layout.
template <int N>
__device__ __forceinline__ void external_product(const uint32_t (&Da)[Geo<N>::E], const uint32_t (&Db)[Geo<N>::E],
                                                 const uint32_t *__restrict__ K, uint32_t *slot,
                                                 const uint32_t *twf, const uint32_t *twi, int L,
                                                 const ModQ &m, const GadgetC &g,
                                                 uint32_t (&out)[2][Geo<N>::E])
{
#pragma unroll
    for (int k = 0; k < Geo<N>::E; k++) out[0][k] = out[1][k] = 0;
    ext_mac<N>(Da, Db, K, slot, twf, L, m, g, out);
    __asm__ volatile("" ::: "memory");
    ntt_inv<N, 2>(out, slot, twi, L, m);
}

}  // namespace dev
}  // namespace mm
