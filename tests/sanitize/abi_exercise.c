/*
 * Drives every entry point of the C ABI that answers before touching the
 * device: workspace and footprint sizes over many shapes (up to the largest
 * accepted lattice and just past it), status strings, thresholds, and every
 * argument error of the lattice, batch, labeling and server calls.  Built with
 * AddressSanitizer and UBSan on the host side of the library; prints "ok" at
 * the end.
 * Returns a non-zero code naming the first unexpected answer.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "swccl.h"

static int fails = 0;
#define EXPECT(cond)                                                  \
    do {                                                              \
        if (!(cond)) {                                                \
            fprintf(stderr, "line %d: %s\n", __LINE__, #cond);        \
            ++fails;                                                  \
        }                                                             \
    } while (0)

static sw_params params(int32_t W, int32_t H, int32_t q, int32_t kind, uint32_t flags)
{
    sw_params p;
    memset(&p, 0, sizeof p);
    p.W = W;
    p.H = H;
    p.q = q;
    p.spin_kind = kind;
    p.K = 1.0;
    p.seed = 1;
    p.flags = flags;
    return p;
}

int main(void)
{
    EXPECT(swccl_abi_version() == SWCCL_ABI_VERSION);
    for (int s = 0; s <= 7; ++s) EXPECT(strcmp(sw_status_string(s), "unknown status") != 0);
    EXPECT(strcmp(sw_status_string(99), "unknown status") == 0);
    EXPECT(sw_last_error() != NULL);
    EXPECT(sw_threshold(0.0) == 0 && sw_threshold(-1.0) == 0 && sw_threshold(INFINITY) == 4294967296ull);
    EXPECT(sw_threshold(NAN) == 0);

    /* sizes: monotone in the lattice, zero exactly for invalid shapes */
    const int32_t sides[] = {1, 2, 3, 63, 64, 65, 127, 128, 129, 1000, 4096, 46340, 46341};
    size_t prev = 0;
    for (size_t i = 0; i < sizeof sides / sizeof sides[0]; ++i) {
        const int32_t L = sides[i];
        const int ok_sw = L >= 2 && L <= 46340, ok_ccl = L <= 46340;
        for (uint32_t f = 0; f < 8; ++f) {
            sw_params p = params(L, L, 3, SW_SPIN_POTTS_U8, f);
            EXPECT((sw_workspace_bytes(&p) > 0) == ok_sw);
        }
        for (int mode = CCL_BONDS_PERIODIC; mode <= CCL_SITES_OPEN; ++mode) {
            const size_t b = ccl_workspace_bytes(L, L, mode);
            EXPECT((b > 0) == ok_ccl);
            if (ok_ccl && mode == CCL_BONDS_PERIODIC) {
                EXPECT(b >= prev);
                prev = b;
            }
        }
        ccl_server_params sp = {CCL_SITES_OPEN, 1, 16, 2};
        EXPECT((ccl_server_footprint(L, L, &sp) > 0) == ok_ccl);
    }
    EXPECT(ccl_workspace_bytes(16, 16, -1) == 0 && ccl_workspace_bytes(16, 16, 3) == 0);
    EXPECT(ccl_workspace_bytes(0, 16, CCL_SITES_OPEN) == 0 && ccl_workspace_bytes(16, -5, CCL_SITES_OPEN) == 0);
    EXPECT(ccl_workspace_bytes(65536, 32768, CCL_SITES_OPEN) == 0);  /* W*H = 2^31 */
    EXPECT(ccl_workspace_bytes(2147483647, 1, CCL_SITES_OPEN) == 0); /* one row below 2^31: tile ids pass 2^31 */
    EXPECT(ccl_workspace_bytes(1 << 22, 1, CCL_SITES_OPEN) > 0);      /* one row of 2^22 pixels */

    /* lattice parameters */
    sw_params bad[] = {params(1, 8, 2, SW_SPIN_ISING_I8, 0), params(8, 8, 1, SW_SPIN_POTTS_U8, 0),
                       params(8, 8, 256, SW_SPIN_POTTS_U8, 0), params(8, 8, 3, SW_SPIN_ISING_I8, 0),
                       params(8, 8, 2, 7, 0), params(8, 8, 2, SW_SPIN_ISING_I8, 1u << 5)};
    for (size_t i = 0; i < sizeof bad / sizeof bad[0]; ++i) EXPECT(sw_workspace_bytes(&bad[i]) == 0);
    sw_params nanK = params(8, 8, 2, SW_SPIN_ISING_I8, 0);
    nanK.K = NAN;
    EXPECT(sw_workspace_bytes(&nanK) == 0);
    EXPECT(sw_workspace_bytes(NULL) == 0);

    sw_params p = params(64, 64, 2, SW_SPIN_ISING_I8, SW_F_SIZES);
    sw_lattice *h = NULL;
    sw_buffers b;
    memset(&b, 0, sizeof b);
    EXPECT(sw_init(NULL, &p, &b, NULL) == SW_ERR_ARG);
    EXPECT(sw_init(&h, &p, NULL, NULL) == SW_ERR_ARG);
    EXPECT(sw_init(&h, &p, &b, NULL) == SW_ERR_ARG); /* no spins */
    b.spins = (void *)0x100000;
    EXPECT(sw_init(&h, &p, &b, NULL) == SW_ERR_ARG); /* sizes without roots/sizes */
    b.roots = (int32_t *)0x200000;
    b.sizes = (int32_t *)0x300000;
    EXPECT(sw_init(&h, &p, &b, NULL) == SW_ERR_WORKSPACE);
    b.workspace = (void *)0x400000;
    b.workspace_bytes = sw_workspace_bytes(&p) - 1;
    EXPECT(sw_init(&h, &p, &b, NULL) == SW_ERR_WORKSPACE);
    b.workspace = (void *)0x400010;
    b.workspace_bytes = sw_workspace_bytes(&p);
    EXPECT(sw_init(&h, &p, &b, NULL) == SW_ERR_WORKSPACE); /* misaligned */
    sw_params big = params(46341, 46341, 2, SW_SPIN_ISING_I8, 0);
    EXPECT(sw_init(&h, &big, &b, NULL) == SW_ERR_SIZE);
    EXPECT(h == NULL);
    EXPECT(sw_sweep(NULL, 1, NULL) == SW_ERR_ARG);
    EXPECT(sw_sweep_phase(NULL, 0, NULL) == SW_ERR_ARG);
    EXPECT(sw_sweep_history(NULL, 1, NULL, NULL) == SW_ERR_ARG);
    EXPECT(sw_observables(NULL, NULL, NULL) == SW_ERR_ARG);
    uint64_t t = 0;
    EXPECT(sw_get_t(NULL, &t) == SW_ERR_ARG && sw_set_t(NULL, 0) == SW_ERR_ARG && sw_destroy(NULL) == SW_ERR_ARG);

    /* labeling */
    int32_t n = 0;
    const uint8_t *in = (const uint8_t *)0x100000;
    int32_t *lab = (int32_t *)0x800000;
    void *ws = (void *)0x1000000;
    const size_t wsb = ccl_workspace_bytes(100, 50, CCL_SITES_OPEN);
    EXPECT(ccl_label(NULL, 100, 50, CCL_SITES_OPEN, lab, NULL, NULL, &n, ws, wsb, NULL) == SW_ERR_ARG);
    EXPECT(ccl_label(in, 100, 50, CCL_SITES_OPEN, NULL, NULL, NULL, &n, ws, wsb, NULL) == SW_ERR_ARG);
    EXPECT(ccl_label(in, 100, 50, 9, lab, NULL, NULL, &n, ws, wsb, NULL) == SW_ERR_ARG);
    EXPECT(ccl_label(in, 100, 50, CCL_SITES_OPEN, lab, lab, NULL, &n, ws, wsb, NULL) == SW_ERR_ARG);
    EXPECT(ccl_label(in, 0, 50, CCL_SITES_OPEN, lab, NULL, NULL, &n, ws, wsb, NULL) == SW_ERR_SIZE);
    EXPECT(ccl_label(in, 100, 50, CCL_SITES_OPEN, (int32_t *)(in + 8), NULL, NULL, &n, ws, wsb, NULL) ==
           SW_ERR_ARG); /* labels overlap the input */
    /* the workspace size covers a call with roots and sizes, which needs all of it */
    EXPECT(ccl_label(in, 100, 50, CCL_SITES_OPEN, lab, lab + 5000, lab + 10000, &n, ws, wsb - 1, NULL) ==
           SW_ERR_WORKSPACE);
    EXPECT(ccl_label(in, 100, 50, CCL_SITES_OPEN, lab, NULL, NULL, &n, ws, 255, NULL) == SW_ERR_WORKSPACE);
    EXPECT(ccl_label(in, 100, 50, CCL_SITES_OPEN, lab, NULL, NULL, &n, NULL, wsb, NULL) == SW_ERR_WORKSPACE);
    EXPECT(ccl_label(in, 100, 50, CCL_SITES_OPEN, lab, NULL, NULL, &n, (char *)ws + 4, wsb, NULL) ==
           SW_ERR_WORKSPACE);

    /* batches: sizes over mixed lattices, errors before anything is enqueued */
    enum { NB = 300 };
    sw_params *bp = malloc(sizeof(sw_params) * NB);
    sw_buffers *bb = calloc(NB, sizeof(sw_buffers));
    for (int j = 0; j < NB; ++j) {
        bp[j] = params(32 << (j % 6), 32 << ((j / 6) % 6), 2, SW_SPIN_ISING_I8, 0);
        bb[j].spins = (void *)(uintptr_t)(0x100000 + 0x1000 * j);
    }
    size_t prevb = 0;
    for (int m = 1; m <= NB; m += 37) {
        const size_t s = swb_workspace_bytes(bp, m);
        EXPECT(s > prevb);
        prevb = s;
    }
    EXPECT(swb_workspace_bytes(bp, 0) == 0 && swb_workspace_bytes(NULL, 3) == 0);
    swb_batch *bh = NULL;
    EXPECT(swb_init(NULL, bp, bb, NB, ws, 1, NULL) == SW_ERR_ARG);
    EXPECT(swb_init(&bh, bp, bb, NB, ws, swb_workspace_bytes(bp, NB) - 1, NULL) == SW_ERR_WORKSPACE);
    bp[7].flags = SW_F_SIZES;
    EXPECT(swb_workspace_bytes(bp, NB) == 0);
    EXPECT(swb_init(&bh, bp, bb, NB, ws, 1u << 30, NULL) == SW_ERR_UNSUPPORTED);
    bp[7].flags = SW_F_REVERSE_TILES;
    EXPECT(swb_init(&bh, bp, bb, NB, ws, 1u << 30, NULL) == SW_ERR_UNSUPPORTED);
    bp[7].flags = 0;
    bb[9].roots = (int32_t *)0x10;
    EXPECT(swb_init(&bh, bp, bb, NB, ws, 1u << 30, NULL) == SW_ERR_ARG);
    EXPECT(bh == NULL);
    EXPECT(swb_sweep(NULL, 1, NULL) == SW_ERR_ARG && swb_sweep_graph(NULL, 1, NULL) == SW_ERR_ARG);
    EXPECT(swb_observables(NULL, 0, NULL, NULL) == SW_ERR_ARG && swb_get_t(NULL, &t) == SW_ERR_ARG);
    EXPECT(swb_destroy(NULL) == SW_ERR_ARG);
    free(bp);
    free(bb);

    /* server */
    ccl_server_params sp = {CCL_SITES_OPEN, 1, 16, 2};
    ccl_server_params badsp[] = {{9, 1, 16, 2}, {CCL_SITES_OPEN, 2, 16, 2}, {CCL_SITES_OPEN, 1, 0, 2},
                                 {CCL_SITES_OPEN, 1, 5000, 2}, {CCL_SITES_OPEN, 1, 16, 0},
                                 {CCL_SITES_OPEN, 1, 16, 65}};
    void *streams[2] = {NULL, NULL};
    ccl_server *sh = NULL;
    for (size_t i = 0; i < sizeof badsp / sizeof badsp[0]; ++i) {
        EXPECT(ccl_server_footprint(64, 64, &badsp[i]) == 0);
        EXPECT(ccl_server_create(&sh, &badsp[i], ws, 1u << 20, streams) == SW_ERR_ARG);
    }
    EXPECT(ccl_server_create(NULL, &sp, ws, 1u << 20, streams) == SW_ERR_ARG);
    EXPECT(ccl_server_create(&sh, &sp, ws, 1u << 20, NULL) == SW_ERR_ARG);
    EXPECT(ccl_server_create(&sh, &sp, (char *)ws + 16, 1u << 20, streams) == SW_ERR_WORKSPACE);
    EXPECT(ccl_server_create(&sh, &sp, ws, 100, streams) == SW_ERR_WORKSPACE);
    EXPECT(sh == NULL);
    int32_t slot = 0;
    uint64_t tag = 0;
    EXPECT(ccl_server_submit(NULL, in, 4, 4, 4, 0, &slot) == SW_ERR_ARG);
    EXPECT(ccl_server_poll(NULL, &slot, &tag, 1, &n) == SW_ERR_ARG);
    EXPECT(ccl_server_result(NULL, 0, NULL, NULL, NULL, NULL) == SW_ERR_ARG);
    EXPECT(ccl_server_release(NULL, 0) == SW_ERR_ARG && ccl_server_destroy(NULL) == SW_ERR_ARG);

    /* cubic lattices: sizes over many shapes (up to the largest accepted
     * classes and past them) and every argument error */
    sw3_params c3;
    memset(&c3, 0, sizeof c3);
    c3.Lx = 64;
    c3.Ly = 32;
    c3.Lz = 16;
    c3.q = 2;
    c3.spin_kind = SW_SPIN_ISING_I8;
    c3.K = 0.44;
    c3.seed = 1;
    const int32_t ext[] = {1, 2, 3, 31, 32, 33, 127, 128, 129, 1024, 2047, 65536};
    for (size_t a = 0; a < sizeof ext / sizeof ext[0]; ++a)
        for (size_t b = 0; b < sizeof ext / sizeof ext[0]; ++b)
            for (size_t c = 0; c < sizeof ext / sizeof ext[0]; ++c) {
                sw3_params q3 = c3;
                q3.Lx = ext[a];
                q3.Ly = ext[b];
                q3.Lz = ext[c];
                const int64_t N = (int64_t)ext[a] * ext[b] * ext[c];
                const size_t w3 = sw3_workspace_bytes(&q3), l3 = ccl3_workspace_bytes(ext[a], ext[b], ext[c]);
                if (N >= ((int64_t)1 << 31)) EXPECT(w3 == 0 && l3 == 0);
                EXPECT((w3 == 0) == (l3 == 0));
                if (w3) EXPECT(w3 > l3 && w3 >= (size_t)N * 3);
            }
    const size_t w3 = sw3_workspace_bytes(&c3);
    EXPECT(w3 > 0);
    sw3_params bad3 = c3;
    bad3.flags = 1;
    EXPECT(sw3_workspace_bytes(&bad3) == 0 && sw3_workspace_bytes(NULL) == 0);
    EXPECT(sw3_sweep(&c3, NULL, 0, 1, NULL, NULL, NULL, ws, w3, NULL) == SW_ERR_ARG);
    EXPECT(sw3_sweep(&c3, (uint8_t *)ws, 0, 1, NULL, NULL, NULL, ws, w3 - 1, NULL) == SW_ERR_WORKSPACE);
    EXPECT(sw3_sweep(&c3, (uint8_t *)ws, UINT32_MAX, 2, NULL, NULL, NULL, ws, w3, NULL) == SW_ERR_STATE);
    EXPECT(sw3_sweep(&bad3, (uint8_t *)ws, 0, 1, NULL, NULL, NULL, ws, w3, NULL) == SW_ERR_ARG);
    EXPECT(sw3_sweep(&c3, (uint8_t *)ws, 0, 0, NULL, NULL, NULL, ws, w3, NULL) == SW_OK);
    EXPECT(sw3_init_spins(&c3, NULL, NULL) == SW_ERR_ARG && sw3_init_spins(NULL, (uint8_t *)ws, NULL) == SW_ERR_ARG);
    const size_t l3 = ccl3_workspace_bytes(64, 32, 16);
    EXPECT(ccl3_label(NULL, 64, 32, 16, (int32_t *)ws, NULL, ws, l3, NULL) == SW_ERR_ARG);
    EXPECT(ccl3_label(in, 64, 32, 16, NULL, NULL, ws, l3, NULL) == SW_ERR_ARG);
    EXPECT(ccl3_label(in, 64, 32, 16, (int32_t *)ws, NULL, ws, l3 - 1, NULL) == SW_ERR_WORKSPACE);
    EXPECT(ccl3_label(in, 0, 32, 16, (int32_t *)ws, NULL, ws, l3, NULL) == SW_ERR_SIZE);

    if (fails) return 1;
    printf("ok\n");
    return 0;
}
