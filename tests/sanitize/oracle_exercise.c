/*
 * Exercises every function of the C oracle on small, ragged and degenerate
 * shapes with exactly sized heap buffers, so that a build with AddressSanitizer
 * and UndefinedBehaviorSanitizer reports any out-of-bounds access, overflow or
 * other undefined behaviour.  Prints "ok" when every call has returned.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "swccl_oracle.h"

static void *xmalloc(size_t n)
{
    void *p = malloc(n ? n : 1);
    if (!p) {
        fprintf(stderr, "out of memory\n");
        exit(2);
    }
    return p;
}

static uint32_t lcg(uint32_t *s)
{
    *s = *s * 1664525u + 1013904223u;
    return *s >> 8;
}

static void labeling(int32_t W, int32_t H, uint32_t *rs)
{
    const int64_t N = (int64_t)W * H;
    uint8_t *in = xmalloc((size_t)N);
    int32_t *lab = xmalloc((size_t)N * 4), *roots = xmalloc((size_t)N * 4), *sizes = xmalloc((size_t)N * 4);
    for (int pct = 0; pct <= 100; pct += 25) {
        for (int64_t i = 0; i < N; ++i) {
            const uint32_t r = lcg(rs) % 100;
            in[i] = (uint8_t)(((int)r < pct) | (((int)(lcg(rs) % 100) < pct) << 1));
        }
        int64_t mx = 0;
        for (int mode = ORC_PERIODIC; mode <= ORC_OPEN; ++mode) {
            const int64_t n = orc_label_bonds(W, H, in, mode, lab);
            if (orc_cluster_sizes(N, lab, roots, sizes, &mx) != n) exit(3);
            (void)orc_cluster_sizes(N, lab, NULL, NULL, NULL);
        }
        const int64_t n = orc_label_sites(W, H, in, lab);
        if (orc_cluster_sizes(N, lab, roots, sizes, &mx) != n) exit(4);
        (void)orc_digest_i32(N, lab);
        (void)orc_digest_u8(N, in);
    }
    free(in);
    free(lab);
    free(roots);
    free(sizes);
}

static void sweeps(int32_t W, int32_t H, int32_t q, double K)
{
    const int64_t N = (int64_t)W * H;
    uint8_t *st = xmalloc((size_t)N), *bonds = xmalloc((size_t)N);
    int32_t *lab = xmalloc((size_t)N * 4);
    int64_t rec[ORC_REC_LEN], recs[3 * ORC_REC_LEN], counts[8];
    const uint64_t T = orc_threshold(K);
    orc_init_states(W, H, q, 0x1105580400000000ull | 7u, 3u, st);
    orc_activate_bonds(W, H, st, T, 11u, 0u, 3u, bonds);
    (void)orc_label_bonds(W, H, bonds, ORC_PERIODIC, lab);
    orc_flip(W, H, q, lab, 11u, 0u, 3u, st);
    (void)orc_satisfied(W, H, q, st, counts);
    orc_sw_sweep(W, H, q, T, 11u, 3u, 1u, st, bonds, lab, rec);
    orc_sw_sweep(W, H, q, T, 11u, 3u, 2u, st, NULL, NULL, NULL);
    orc_sw_run(W, H, q, T, 11u, 3u, 3u, 3, st, recs);
    free(st);
    free(bonds);
    free(lab);
}

/* Every cubic-lattice function on one Lx x Ly x Lz lattice. */
static void cubic(int32_t Lx, int32_t Ly, int32_t Lz, int32_t q, double K, uint32_t *rs)
{
    const int64_t N = (int64_t)Lx * Ly * Lz;
    uint8_t *st = xmalloc((size_t)N), *bonds = xmalloc((size_t)N);
    int32_t *lab = xmalloc((size_t)N * 4);
    int64_t rec[ORC3_REC_LEN], recs[3 * ORC3_REC_LEN], counts[8];
    const uint64_t T = orc_threshold(K);
    orc_init_states(Lx, Ly * Lz, q, 13u, 2u, st);
    orc3_activate_bonds(Lx, Ly, Lz, st, T, 13u, 0u, 2u, bonds);
    for (int64_t i = 0; i < N; ++i) bonds[i] = (uint8_t)(lcg(rs) & 7u);
    (void)orc3_label_bonds(Lx, Ly, Lz, bonds, lab);
    (void)orc3_satisfied(Lx, Ly, Lz, q, st, counts);
    (void)orc3_satisfied(Lx, Ly, Lz, q, st, NULL);
    orc3_sw_sweep(Lx, Ly, Lz, q, T, 13u, 2u, 1u, st, bonds, lab, rec);
    orc3_sw_sweep(Lx, Ly, Lz, q, T, 13u, 2u, 2u, st, NULL, NULL, NULL);
    orc3_sw_run(Lx, Ly, Lz, q, T, 13u, 2u, 3u, 3, st, recs);
    free(st);
    free(bonds);
    free(lab);
}

int main(void)
{
    uint32_t ctr[4] = {0u, 0u, 0u, 0u}, key[2] = {0u, 0u}, out[4];
    orc_philox4x32_10(ctr, key, out);
    ctr[0] = ctr[1] = ctr[2] = ctr[3] = 0xFFFFFFFFu;
    key[0] = key[1] = 0xFFFFFFFFu;
    orc_philox4x32_10(ctr, key, out);
    const double Ks[] = {-1.0, 0.0, 1e-12, 0.5, 1.0050525, 3.0, 50.0, INFINITY};
    for (size_t k = 0; k < sizeof Ks / sizeof Ks[0]; ++k) (void)orc_threshold(Ks[k]);

    uint32_t rs = 12345u;
    const int32_t shapes[][2] = {{1, 1}, {1, 9}, {9, 1}, {2, 2}, {2, 5}, {3, 3}, {7, 4}, {33, 17}, {64, 64}, {130, 66}};
    for (size_t s = 0; s < sizeof shapes / sizeof shapes[0]; ++s) labeling(shapes[s][0], shapes[s][1], &rs);
    const int32_t sw_shapes[][2] = {{2, 2}, {2, 3}, {3, 2}, {5, 7}, {64, 64}, {129, 65}};
    const int32_t qs[] = {2, 3, 8, 9, 255};
    for (size_t s = 0; s < sizeof sw_shapes / sizeof sw_shapes[0]; ++s)
        for (size_t j = 0; j < sizeof qs / sizeof qs[0]; ++j)
            for (size_t k = 0; k < sizeof Ks / sizeof Ks[0]; k += 3)
                sweeps(sw_shapes[s][0], sw_shapes[s][1], qs[j], Ks[k]);
    const int32_t cubes[][3] = {{1, 1, 1}, {1, 1, 5}, {2, 2, 2}, {3, 1, 2}, {5, 4, 3}, {17, 9, 6}, {32, 16, 16}};
    for (size_t s = 0; s < sizeof cubes / sizeof cubes[0]; ++s)
        for (size_t j = 0; j < sizeof qs / sizeof qs[0]; j += 2)
            for (size_t k = 0; k < sizeof Ks / sizeof Ks[0]; k += 2)
                cubic(cubes[s][0], cubes[s][1], cubes[s][2], qs[j], Ks[k], &rs);
    printf("ok\n");
    return 0;
}
