// Kernel argument blocks and launchers (implemented in kernels.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace mm {
namespace dev {

enum : uint32_t {
    TASK_INIT = 1u,     // accumulator starts at Phi(b')(0, V)
    TASK_STORE = 2u,    // write the accumulator to acc_state at the end of the launch
    TASK_EXTRACT = 4u,  // component 0 writes the extracted LWE_N sample when step n is reached
};

// What one wave of a blind-rotation workgroup does.  A group is GW (8 or 4)
// consecutive WaveTasks.  A component slot is WPP consecutive waves (by default
// 1 up to N = 1024, N / 1024 above; 2 in the small-batch schedule) holding the
// same task; the components 0..r-1 of a ciphertext sit on consecutive slots of
// one group.
struct WaveTask {
    int32_t ct;        // ciphertext index, -1 for an idle wave
    uint32_t comp;     // component j
    uint32_t r;        // vector length of the ciphertext's table
    uint32_t tv_off;   // word offset of the table's test vector in the arena
    uint32_t q_in;     // ciphertext modulus
    uint32_t i0;       // first CMux step of this launch
    uint32_t flags;    // TASK_*
    uint32_t steps;    // CMux steps of this task in the launch (0: the launch's step count)
    uint64_t acc_off;  // word offset of the ciphertext's accumulator state (r x 2 x N)
};

struct BrArgs {
    const WaveTask *tasks;
    int num_groups;
    int steps;                 // CMux steps per launch
    const uint32_t *ct_in;     // ciphertexts at their q_in
    uint32_t ct_stride;        // n + 1
    uint32_t n, Q, qn, log2B, l, sg, goff;  // goff: (B/2)(1 + B + ... + B^(l-1))
    uint32_t keys;             // RGSW keys per coordinate (2 for a ternary secret)
    const uint32_t *bsk;       // [n][keys][2l][2][N], NTT domain, x 2^32 / N mod Q
    const uint32_t *bsk_corr;  // [n][2][N]: -(B/2) sum_{key,row} BSK / N, the digit-offset correction
    const uint32_t *twf, *twi; // Montgomery-form twiddles
    const uint32_t *tv;        // test-vector arena
    uint32_t *acc_state;       // accumulators carried between launches
    uint32_t *ext_out;         // [ct][N + 1] extracted samples
};

// One (ciphertext, component) pair of the wide-modulus blind rotation: a
// workgroup of N / LANES... waves owns it for one CMux step.
struct WideTask {
    int32_t ct;        // ciphertext index
    uint32_t comp;     // component j
    uint32_t r;        // vector length of the ciphertext's table
    uint32_t q_in;     // ciphertext modulus
    uint32_t tv_off;   // word offset of the table's test vector ([r][2][N]) in the arena
    uint32_t i0;       // CMux step of the ciphertext at the first launch of a sequence (0 for a batch)
    uint64_t acc_off;  // word offset of the ciphertext's component 0; a component is [2 parts][2 primes][N]
};

// The wide-modulus blind rotation: ring modulus Q_w = Q[0] Q[1], every
// coefficient held as its two residues.
struct WideArgs {
    const WideTask *tasks;
    const uint32_t *ct_in;     // ciphertexts at their q_in
    uint32_t ct_stride;        // n + 1
    uint32_t step;             // launch index within a sequence: a task takes CMux step i = i0 + step
    uint32_t Q[2], qn[2];      // the two primes and -Q^-1 mod 2^32
    uint32_t log2B, l, sg;
    uint32_t crt_cq;           // the smallest multiple of Q[1] that is >= Q[0]
    uint32_t crt_inv;          // Q[0]^-1 mod Q[1], times 2^32 mod Q[1]
    uint32_t n;                // LWE dimension: a task at i >= n carries its accumulator over
    uint64_t Qw, goff;         // Q[0] Q[1]; (B/2)(1 + B + ... + B^(l-1))
    const uint32_t *bsk;       // [n][keys][prime][2l][2][N], NTT domain, x 2^32 / N mod that prime
    const uint32_t *bsk_corr;  // [n][prime][2][N]: the digit-offset correction, summed over keys
    const uint32_t *twf0, *twi0, *twf1, *twi1;
    const uint32_t *tv;        // test-vector arena
    const uint32_t *acc_rd;    // accumulators after step i (read)
    uint32_t *acc_wr;          // accumulators after step i + 1 (written)
    // rings split into M sub-rings of SPLIT_NS coefficients (one prime only):
    uint32_t M;                // sub-rings per ring (0: not split)
    uint32_t *dig;             // digit polynomials after the stages that mix sub-rings, [task][key][u][part][N]
    uint32_t *outb;            // products after the inverse stages within sub-rings, [task][part][N]
    const uint32_t *twf_sub;   // [M][SPLIT_NS]: the forward twiddles of each sub-ring's remaining stages
    const uint32_t *twi_sub;   // [M][SPLIT_NS]: the same for the inverse
};

// Sub-ring size of the split blind rotation: rings of 16384 coefficients and
// more run their NTT stages that mix sub-rings in separate kernels through
// device memory, and every sub-ring of 8192 coefficients in one workgroup.
constexpr uint32_t SPLIT_NS = 8192;

constexpr int KS_CTS_PER_WAVE = 4;
constexpr int KS_TILED_MAX_ROWS = 128;  // l_ks * B_ks handled by the LDS-tiled key switch

// Device layout of the key-switching key: column tiles of 64 output words,
// [i][tile][l_ks B_ks rows][64] (columns past n + 1 hold zeros), so that the
// candidate rows of one coordinate for one tile are one contiguous block.
constexpr int KS_TILE_COLS = 64;

struct KsArgs {
    const uint32_t *lwe_N;  // extracted samples at Q, [*][N + 1]
    const int32_t *rows;    // output row k reads sample rows[k] (null: sample k)
    const uint32_t *ksk;    // [N][col_tiles][l_ks B_ks][64] (tiles of the [N][l_ks][B_ks][n + 1] key)
    uint32_t col_tiles;     // ceil((n + 1) / 64)
    uint64_t *part;         // [splits][count][n + 1] (the tiled kernel writes u32 residues into u64 slots,
                            // the lane kernel unreduced 64-bit sums)
    size_t count;
    uint32_t n, N, Q, log2Bks, l_ks;
};

// Device scratch of the allocation-free key switch: one array per GPU, held
// until the process ends; noalloc_scratch_init returns its device address for
// `device`, which must be the current device (looked up once per device).
constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(64) << 20;
hipError_t noalloc_scratch_init(int device, void **out);

hipError_t init_kernel_attributes();
bool device_supports_n(uint32_t N);  // N in {256, ..., 8192}
int waves_per_poly(uint32_t N);
void launch_lwe_combine(const uint32_t *ct, const uint32_t *tmp, uint32_t *out, size_t count, uint32_t W,
                        const uint32_t *qs, hipStream_t st);
void launch_scatter_rows(const uint32_t *src, uint32_t *dst, const int32_t *rows, size_t count, uint32_t W,
                         hipStream_t st);
// wpp: waves per polynomial (0: one up to N = 1024, N / 1024 above; 2 is also
// available at N = 512 and 1024, see br_supports_wpp).
// ntt: the NTT stage schedule, 0 (every exchange through LDS), 1 (the last
// exchange by wavefront lane swaps; where br_supports_lane_swap(N)) or 2 (LDS
// exchanges, the two polys of an NTT staggered; one wave per polynomial).
void launch_blind_rotate(uint32_t N, const BrArgs &A, int gw, int grid, hipStream_t st, int wpp = 0, int ntt = 0);
bool br_supports_wpp(uint32_t N, int wpp);
bool br_supports_lane_swap(uint32_t N);
// wide modulus: ACC = Phi(b')(0, V) into A.acc_wr; one CMux step (step i0 +
// A.step of each task; a task past step n - 1 copies its component) from
// A.acc_rd into A.acc_wr; extraction of component 0 switched to Q[0]
// (ext[c] from the component at acc_off[c]); the accumulator as uint64 values
// [component][part][N] at the same word offsets.
// npr: primes of the ring modulus (2: the wide modulus Q Q2, N <= 4096; 1: the
// global-accumulator path of the 31-bit modulus, N <= 16384); with one prime the
// accumulator is already in the output layout [component][part][N] (no export).
void launch_wide_init(uint32_t N, int npr, const WideArgs &A, uint32_t num_tasks, hipStream_t st);
// wpp: waves per component workgroup (0: wide_waves_per_poly(N)); with one prime
// also twice that at N = 512 and 1024 (wide_supports_wpp).
// dg = 2 (N = 1024, wpp = 4, one prime): two digit groups of wpp waves per component.
// ps (two primes): one workgroup per component and prime (dg = 2 too: N = 1024, 2048).
void launch_wide_step(uint32_t N, int npr, uint32_t keys, const WideArgs &A, uint32_t num_tasks, hipStream_t st,
                      int wpp = 0, int dg = 1, bool ps = false);
bool wide_supports_wpp(uint32_t N, int npr, int wpp);
bool wide_supports_dg(uint32_t N, int npr, int wpp);  // two digit groups of wpp waves
bool wide_supports_ps(uint32_t N, int npr, int dg = 1);  // one workgroup per prime (of dg digit groups)
void launch_wide_extract(uint32_t N, int npr, const WideArgs &A, const uint64_t *acc_off, size_t count,
                         uint32_t *ext, hipStream_t st);
void launch_wide_export(uint32_t N, const WideArgs &A, uint32_t num_tasks, uint32_t *out, hipStream_t st);
bool wide_supports_n(uint32_t N, int npr);
int wide_waves_per_poly(uint32_t N);  // waves of one k_wide_step workgroup
// The split CMux step (one prime, N = M SPLIT_NS with M in {2, 4, 8}): digits and
// the forward stages that mix sub-rings into A.dig; per (task, sub-ring) the
// remaining forward stages, the product with BSK_i and the inverse stages within
// the sub-ring into A.outb; the inverse stages that mix sub-rings and ACC + product
// into A.acc_wr.  A task past step n - 1 carries its component over.
void launch_split_step(uint32_t N, uint32_t keys, const WideArgs &A, uint32_t num_tasks, hipStream_t st);
bool split_supports_n(uint32_t N);
constexpr int SPLIT_WAVES = (int)SPLIT_NS / 1024;  // waves of one sub-ring workgroup
size_t br_lds_bytes(uint32_t N, int gw, int wpp = 0);
void launch_external_product(uint32_t N, const uint32_t *in, uint32_t *out, size_t count, const uint32_t *K,
                             const uint32_t *twf, const uint32_t *twi, uint32_t Q, uint32_t qn, uint32_t log2B,
                             uint32_t l, uint32_t sg, hipStream_t st);
void launch_negacyclic_mul(uint32_t N, const uint32_t *a, const uint32_t *b, uint32_t *out, size_t count,
                           const uint32_t *twf, const uint32_t *twi, uint32_t Q, uint32_t qn, uint32_t c_fix,
                           hipStream_t st);
void launch_modswitch(const uint32_t *in, uint32_t *out, size_t count, uint32_t q_from, uint32_t q_to,
                      hipStream_t st);
void launch_sample_extract(const uint32_t *rlwe, uint32_t *lwe, size_t count, uint32_t N, uint32_t Q,
                           hipStream_t st);
void launch_keyswitch(const KsArgs &A, uint32_t splits, hipStream_t st);
void launch_keyswitch_tiled(const KsArgs &A, int cpw, uint32_t splits, hipStream_t st);
// one ciphertext per lane, 256 per workgroup, 64 columns (l_ks B_ks <= KS_TILED_MAX_ROWS)
void launch_keyswitch_lanes(const KsArgs &A, uint32_t splits, hipStream_t st);
void launch_ks_finalize(const uint64_t *part, const uint32_t *lwe_N, const int32_t *rows, uint32_t *out, size_t count,
                        uint32_t n,
                        uint32_t N, uint32_t splits, uint32_t Q, const uint32_t *q_out_per_ct, uint32_t q_out,
                        hipStream_t st);

}  // namespace dev
}  // namespace mm
