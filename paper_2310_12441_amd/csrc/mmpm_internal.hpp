// Internal declarations of the BootMMPM library (host side).
#pragma once

#include <cstddef>
#include <cstdint>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <stdexcept>
#include <string>
#include <vector>

#include "mmpm.h"

namespace mm {

// An error that becomes a C status code at the ABI.
struct Error : std::runtime_error {
    int code;
    Error(int c, const std::string &msg) : std::runtime_error(msg), code(c) {}
};

#define MM_REQUIRE(cond, msg)                                    \
    do {                                                         \
        if (!(cond)) throw ::mm::Error(MM_EINVAL, (msg));        \
    } while (0)

// ---------------------------------------------------------------- host Z_Q
inline uint32_t mulmod(uint32_t a, uint32_t b, uint32_t q) { return (uint32_t)((uint64_t)a * b % q); }
inline uint32_t addmod(uint32_t a, uint32_t b, uint32_t q) { uint64_t s = (uint64_t)a + b; return (uint32_t)(s >= q ? s - q : s); }
inline uint32_t submod(uint32_t a, uint32_t b, uint32_t q) { return a >= b ? a - b : a + q - b; }
uint32_t powmod(uint32_t a, uint64_t e, uint32_t q);
bool is_prime(uint32_t q);
void parallel_for(int64_t n, const std::function<void(int64_t)> &fn);
uint32_t bit_length(uint32_t x);
uint32_t bitrev(uint32_t x, uint32_t bits);
// x in [0, Q1 Q2) from its residues mod the primes Q1 and Q2 (Chinese remainders)
uint64_t crt2(uint32_t x1, uint32_t x2, uint32_t Q1, uint32_t Q2);

// Negacyclic NTT tables for Z_Q[x]/(x^N+1): psi a primitive 2N-th root of unity.
// fwd[k] = psi^bitrev(k), inv[k] = psi^-bitrev(k) (k < N), the Cooley-Tukey /
// Gentleman-Sande twiddle order with bit-reversed NTT-domain output.
struct NttTables {
    uint32_t N = 0, Q = 0, psi = 0, n_inv = 0;
    std::vector<uint32_t> fwd, inv;
    void build(uint32_t N, uint32_t Q);
    void forward(uint32_t *a) const;   // natural order in, bit-reversed out
    void inverse(uint32_t *a) const;   // bit-reversed in, natural order out (scaled by 1/N)
};

struct Table {
    uint32_t t, t_out, r, q_in;
    std::vector<uint32_t> V;  // [r][N] scaled test vector, wide: [r][limb][N] (empty for a general table)
    size_t dev_offset = 0;    // word offset in the device test-vector arena
    int g_id = -1, F_id = -1; // general f: the sign table and the extended-f table it runs
};

struct Device;  // device-side state, defined in device.cpp
struct DeviceDeleter {
    void operator()(Device *d) const;
};
struct Server;

}  // namespace mm

struct mm_ctx {
    mm_params p{};
    uint32_t sg = 0;                 // gadget shift: max(0, bits(Q) - l log2_B)
    std::vector<uint32_t> gadget;    // g_u = 2^(sg + u log2_B) mod Q
    std::vector<int32_t> s;          // LWE secret in {0,1} or {-1,0,1}
    std::vector<uint32_t> z;         // RLWE secret (host)
    uint32_t keys = 1;               // RGSW keys per LWE coordinate (2 for a ternary secret)
    bool wide = false;               // Q2 != 0: blind rotation at Q_w = Q Q2, two residues per coefficient
    uint64_t Qw = 0;                 // ring modulus of the blind rotation (Q Q2 or Q)
    std::vector<uint32_t> bsk;       // [n][keys][2l][2][N] coefficient form; wide: [n][keys][limb][2l][2][N]
    std::vector<uint32_t> ksk;       // [N][l_ks][B_ks][n+1]
    mm::NttTables ntt;
    mm::NttTables ntt2;              // tables mod Q2 (wide mode)
    std::vector<mm::Table> tables;
    std::string err;
    std::unique_ptr<mm::Device, mm::DeviceDeleter> dev;
    mm::Server *server = nullptr;
    std::mutex lock;                 // serialises device calls between API and server threads
    ~mm_ctx();
};

namespace mm {

void validate_params(const mm_params &p);
void keygen(mm_ctx &c, const mm_key_draws &d);
void encrypt(const mm_ctx &c, uint32_t q, uint32_t t, const uint32_t *m, size_t count,
             const uint32_t *mask, const int32_t *err, uint32_t *ct);
void decrypt(const mm_ctx &c, uint32_t q, uint32_t t, const uint32_t *ct, size_t count, uint32_t *m);
int table_create(mm_ctx &c, uint32_t t, uint32_t t_out, uint32_t r, uint32_t q_in, const uint32_t *f);
int table_create_general(mm_ctx &c, uint32_t t, uint32_t t_out, uint32_t r, uint32_t q_in, const uint32_t *f);

// device entry points (device.hip)
void device_init(mm_ctx &c, int device);
void device_release(mm_ctx &c);
void run_bootstrap(mm_ctx &c, const int *ids, const uint32_t *ct_in, size_t count, uint32_t *ct_out,
                   uint32_t q_out, uint32_t flags, void *stream);
void run_modswitch(mm_ctx &c, const uint32_t *in, size_t count, uint32_t q_from, uint32_t q_to,
                   uint32_t *out, uint32_t flags, void *stream);
void run_blind_rotate(mm_ctx &c, const int *ids, const uint32_t *ct_in, size_t count, uint32_t steps,
                      uint32_t *acc_out, uint32_t flags, void *stream);
void run_external_product(mm_ctx &c, uint32_t i, const uint32_t *in, size_t count, uint32_t *out,
                          uint32_t flags, void *stream);
void run_sample_extract(mm_ctx &c, const uint32_t *rlwe, size_t count, uint32_t *lwe, uint32_t flags,
                        void *stream);
void run_keyswitch(mm_ctx &c, const uint32_t *lwe_N, size_t count, uint32_t *lwe_n, uint32_t flags,
                   void *stream);
void run_keyswitch_noalloc(mm_ctx &c, const uint32_t *lwe_N, size_t count, uint32_t *lwe_n, void *stream);
void run_negacyclic_mul(mm_ctx &c, const uint32_t *a, const uint32_t *b, size_t count, uint32_t *out,
                        uint32_t flags, void *stream);
int run_autotune(mm_ctx &c, const int *ids, const uint32_t *ct_in, size_t count);
int schedule_count(mm_ctx &c, const int *ids, size_t count);
void set_schedule(mm_ctx &c, const int *ids, size_t count, int choice);
void describe_schedule(mm_ctx &c, const int *ids, size_t count, int choice, int *gw, int *cpw, int *P, int *wpp,
                       int *ks_kernel, int *ntt);
void set_timing(mm_ctx &c, bool on);
void last_timing(mm_ctx &c, float *br_ms, float *ks_ms);

// serving (server.cpp)
Server *server_start(mm_ctx &c, size_t budget, uint32_t chunk);
void server_stop(Server *s);

}  // namespace mm
