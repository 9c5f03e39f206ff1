// Device-side state shared by the batch path (device.cpp) and the serving
// loop (server.cpp).
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <string>
#include <vector>

#include "kernels.hpp"
#include "mmpm_internal.hpp"

namespace mm {

#define HIPC(expr)                                                                                  \
    do {                                                                                            \
        hipError_t e_ = (expr);                                                                     \
        if (e_ != hipSuccess)                                                                       \
            throw ::mm::Error(MM_EDEVICE, std::string(#expr) + " failed: " + hipGetErrorString(e_)); \
    } while (0)

enum WsSlot {
    WS_IN, WS_IN2, WS_OUT, WS_TASKS, WS_EXT, WS_PART, WS_ACC, WS_QOUT, WS_GEN1, WS_GEN2, WS_GENQ,
    WS_ACC2, WS_WOFF,  // wide modulus: second accumulator buffer, per-ciphertext accumulator offsets
    WS_DIG, WS_OUTB,   // split rings: digit polynomials, sub-ring products
    WS_COUNT
};

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
};

struct PinBuf {
    void *p = nullptr;
    size_t bytes = 0;
    hipEvent_t ev = nullptr;  // last stream use of the buffer
};

struct Device {
    int id = -1, num_cu = 0;
    uint32_t qn = 0, c_fix = 0;
    uint32_t *bsk = nullptr, *bsk_corr = nullptr, *ksk = nullptr, *twf = nullptr, *twi = nullptr, *tv = nullptr;
    uint32_t *twf2 = nullptr, *twi2 = nullptr, qn2 = 0;  // second prime of a wide ring modulus
    uint32_t *twf_sub = nullptr, *twi_sub = nullptr;     // split rings: per-sub-ring twiddles
    size_t tv_words = 0, tables_uploaded = 0;
    DevBuf ws[WS_COUNT];
    PinBuf pin[2];
    hipStream_t own = nullptr;
    struct Graph {
        std::string key;
        hipGraphExec_t exec = nullptr;
    };
    std::vector<Graph> graphs;
    std::map<std::string, int> tuned;  // batch shape -> index into the schedule candidates
    int ws_generation = 0;
    void *scratch = nullptr;  // this GPU's fixed scratch array (never freed; see noalloc.hip)
    bool timing = false;
    hipEvent_t tev[3] = {nullptr, nullptr, nullptr};  // before BR, after BR, after key switch

    ~Device()
    {
        hipSetDevice(id);
        hipDeviceSynchronize();
        for (auto &g : graphs)
            if (g.exec) hipGraphExecDestroy(g.exec);
        for (auto &b : ws)
            if (b.p) hipFree(b.p);
        for (auto &b : pin) {
            if (b.p) hipHostFree(b.p);
            if (b.ev) hipEventDestroy(b.ev);
        }
        for (void *p : {(void *)bsk, (void *)bsk_corr, (void *)ksk, (void *)twf, (void *)twi, (void *)tv,
                        (void *)twf2, (void *)twi2, (void *)twf_sub, (void *)twi_sub})
            if (p) hipFree(p);
        for (auto &e : tev)
            if (e) hipEventDestroy(e);
        if (own) hipStreamDestroy(own);
    }
};

Device &ensure_device(mm_ctx &c);
void *ws(Device &d, int slot, size_t bytes);
void *pinned(Device &d, int slot, size_t bytes);
// A key-switch schedule: cpw > 0 selects the LDS-tiled kernel with cpw
// ciphertexts per wave (columns in lanes), cpw = 0 the i-split kernel,
// cpw = KS_LANES the kernel with one ciphertext per lane; P splits the i range.
constexpr int KS_LANES = -1;
struct KsSched {
    int cpw = 0;
    uint32_t P = 1;
};

// A batch schedule: blind-rotation group width (8 or 4 waves; 0 on the
// global-accumulator path), waves per
// component polynomial (0: the ring's default), key switch, and the NTT stage
// schedule (0: every cross-lane exchange through LDS, the two polys of an NTT
// in lockstep; 1: the last exchange by wavefront lane swaps; 2: LDS exchanges
// with the two polys staggered so that one's relayout overlaps the other's
// butterflies; 3, global path only: the ring split into sub-rings of 8192, the
// stages that mix them in separate kernels through device memory).
struct Sched {
    int gw = 8;
    KsSched ks;
    int wpp = 0;
    int ntt = 0;
};

std::vector<dev::WaveTask> pack_tasks(const std::vector<dev::WaveTask> &cts, uint32_t gw, uint32_t wpp,
                                      uint32_t cap = 0);
uint32_t spread_cap(const Device &d, uint64_t comps, uint32_t gw, uint32_t wpp);
KsSched ks_default(const mm_ctx &c, const Device &d, size_t count);
size_t ks_part_words(const mm_ctx &c, const KsSched &k, size_t count);
dev::BrArgs br_args(const mm_ctx &c, const Device &d);
uint32_t ks_splits(const mm_ctx &c, const Device &d, size_t count);
void enqueue_keyswitch(const mm_ctx &c, Device &d, const uint32_t *ext, const int32_t *rows, size_t count,
                       uint32_t *out, const uint32_t *q_out_per_ct, uint32_t q_out, const KsSched &ks, uint64_t *part,
                       hipStream_t st);
// The global-accumulator path: the kernel arguments (tasks, inputs and buffers
// left to the caller) and the number of residues per coefficient (2 with the
// wide modulus, else 1).
dev::WideArgs wide_args(const mm_ctx &c, const Device &d);
int primes_of(const mm_ctx &c);
int light_global_wpp(const mm_ctx &c);  // waves per component of light global-path work (0: the usual)
int light_global_dg(const mm_ctx &c, const Device &d, uint64_t comps);  // digit groups of such work
bool prime_split(const mm_ctx &c, const Device &d, uint64_t comps);     // one workgroup per prime
int prime_split_dg(const mm_ctx &c, const Device &d, uint64_t comps);   // digit groups of those

}  // namespace mm
