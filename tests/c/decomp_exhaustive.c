/* Exhaustive check of the oracle's signed gadget decomposition over every
 * x in [0, Q): each digit but the top one lies in [-B/2, B/2), the top digit
 * in [-B/2, B/2], and the centred x is reconstructed from sum_u d_u 2^(sg+u log2B)
 * within 2^(sg-1) (exactly when sg = 0).  Usage: decomp_exhaustive Q log2B l */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

void orc_decompose(uint32_t Q, uint32_t log2B, uint32_t l, uint32_t x, int32_t *d);
uint32_t orc_gadget_shift(uint32_t Q, uint32_t log2B, uint32_t l);

int main(int argc, char **argv)
{
    if (argc != 4) return 2;
    const uint32_t Q = (uint32_t)strtoul(argv[1], 0, 10);
    const uint32_t lb = (uint32_t)atoi(argv[2]), l = (uint32_t)atoi(argv[3]);
    const uint32_t sg = orc_gadget_shift(Q, lb, l);
    const int64_t B = (int64_t)1 << lb, tol = sg ? ((int64_t)1 << (sg - 1)) : 0;
    long long bad = 0;
    int64_t worst = 0;
#pragma omp parallel for schedule(static) reduction(+ : bad) reduction(max : worst)
    for (int64_t x = 0; x < (int64_t)Q; x++) {
        int32_t d[16];
        orc_decompose(Q, lb, l, (uint32_t)x, d);
        int64_t rec = 0;
        for (uint32_t u = 0; u < l; u++) {
            if (u + 1 < l ? (d[u] < -B / 2 || d[u] >= B / 2) : (d[u] < -B / 2 || d[u] > B / 2)) bad++;
            rec += (int64_t)d[u] * ((int64_t)1 << (sg + u * lb));
        }
        const int64_t xc = x > (int64_t)(Q - 1) / 2 ? x - (int64_t)Q : x;
        int64_t err = xc - rec;
        if (err < 0) err = -err;
        if (err > tol) bad++;
        if (err > worst) worst = err;
    }
    printf("%s Q=%u log2B=%u l=%u sg=%u worst=%lld bad=%lld\n", bad ? "FAIL" : "OK", Q, lb, l, sg,
           (long long)worst, bad);
    return bad ? 1 : 0;
}
