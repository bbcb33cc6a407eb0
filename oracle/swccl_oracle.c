/*
 * swccl_oracle.c -- CPU oracle for the Swendsen-Wang (SW) sweep and for
 * connected-component labeling (CCL) on 2D square lattices.
 *
 * TEST INFRASTRUCTURE ONLY: a plain, single-threaded, obviously-correct
 * reference.  Only tests, the smoke check and the benchmark's CPU-baseline leg
 * call it.  It shares no code with the GPU library.
 *
 * What it follows:
 *   - the Potts Hamiltonian, Sec. II, Eq. potts_hamiltonian;
 *   - the Fortuin-Kasteleyn bond variables and p = 1 - exp(-beta J),
 *     Sec. II, Eqs. fortuin1-fortuin3;
 *   - the three steps of the SW update (activate bonds, identify connected
 *     components, draw a new state per component), Sec. II, enumerated steps;
 *   - union-and-find with roots as set representatives, Sec. II.B.2;
 *   - the few-cluster variant of the Wolff update (Sec. III): the same bond
 *     decomposition, one seed per seed tile, every distinct seeded cluster
 *     flipped with a probability p_flip < 1;
 *   - the same three steps on the simple cubic lattice (the generalisation to
 *     three dimensions that Sec. II names): three bonds per site.
 * Philox4x32-10 follows its published definition (Salmon, Moraes, Dror, Shaw,
 * "Parallel random numbers: as easy as 1, 2, 3", SC'11).
 */
#include "swccl_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ---------------------------------------------------------------- Philox -- */

/* Round multipliers of Philox4x32 (SC'11). */
static const uint32_t PHILOX_M0 = 0xD2511F53u;
static const uint32_t PHILOX_M1 = 0xCD9E8D57u;
/* Key increments ("Weyl" constants): floor(2^32 (golden ratio - 1)) and
 * floor(2^32 (sqrt(3) - 1)). */
static const uint32_t PHILOX_W0 = 0x9E3779B9u;
static const uint32_t PHILOX_W1 = 0xBB67AE85u;

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) { /* the key is bumped between consecutive rounds */
            k0 += PHILOX_W0;
            k1 += PHILOX_W1;
        }
        uint64_t prod0 = (uint64_t)PHILOX_M0 * (uint64_t)c0;
        uint64_t prod1 = (uint64_t)PHILOX_M1 * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(prod0 >> 32), lo0 = (uint32_t)prod0;
        uint32_t hi1 = (uint32_t)(prod1 >> 32), lo1 = (uint32_t)prod1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static void block_for(uint64_t seed, uint32_t word, uint32_t t, uint32_t tag,
                      uint32_t sid, uint32_t out[4])
{
    uint32_t ctr[4] = {word, t, tag, sid};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    orc_philox4x32_10(ctr, key, out);
}

/* Uniform draw of a state in 0..q-1 from one 32-bit word: floor(w * q / 2^32). */
static uint8_t state_from_word(uint32_t w, int32_t q)
{
    return (uint8_t)(((uint64_t)w * (uint64_t)q) >> 32);
}

/* ------------------------------------------------------------- threshold -- */

/* p = 1 - exp(-K) (Sec. II, below Eq. fortuin3; the paper's K is beta*J in
 * the Potts normalisation of Eq. potts_hamiltonian).  A bond between equal
 * spins is active iff a uniform 32-bit r satisfies r < T = floor(p 2^32). */
uint64_t orc_threshold(double K)
{
    if (!(K > 0.0)) return 0;
    double p = -expm1(-K);
    double v = floor(ldexp(p, 32));
    if (v >= 4294967296.0) return 4294967296ull;
    if (v <= 0.0) return 0;
    return (uint64_t)v;
}

/* ----------------------------------------------------------------- init -- */

void orc_init_states(int32_t W, int32_t H, int32_t q, uint64_t seed, uint32_t sid,
                     uint8_t *state)
{
    int64_t N = (int64_t)W * H;
    for (int64_t i = 0; i < N; ++i) {
        uint32_t b[4];
        block_for(seed, (uint32_t)(i >> 2), 0u, ORC_TAG_INIT, sid, b);
        state[i] = state_from_word(b[i & 3], q);
    }
}

/* -------------------------------------------------------------- bonds ---- */

/* Step 1 of the SW update (Sec. II) with the activation rule of Sec. II.A:
 * n_ij = 1 iff s_i = s_j and r < p; otherwise 0. */
void orc_activate_bonds(int32_t W, int32_t H, const uint8_t *state, uint64_t T,
                        uint64_t seed, uint32_t t, uint32_t sid, uint8_t *bonds)
{
    for (int32_t y = 0; y < H; ++y) {
        for (int32_t x = 0; x < W; ++x) {
            int64_t i = (int64_t)y * W + x;
            int64_t right = (int64_t)y * W + (x + 1) % W;
            int64_t down = (int64_t)((y + 1) % H) * W + x;
            uint32_t b[4];
            block_for(seed, (uint32_t)(i >> 1), t, ORC_TAG_BOND, sid, b);
            uint32_t r_right = b[2 * (i & 1)];
            uint32_t r_down = b[2 * (i & 1) + 1];
            int act_right = state[i] == state[right] && (uint64_t)r_right < T;
            int act_down = state[i] == state[down] && (uint64_t)r_down < T;
            bonds[i] = (uint8_t)(act_right | (act_down << 1));
        }
    }
}

/* ---------------------------------------------------------- union-find --- */

/* Root of the tree containing a (Sec. II.B.2: walk up the parent pointers),
 * with path compression afterwards. */
static int32_t uf_find(int32_t *parent, int32_t a)
{
    int32_t root = a;
    while (parent[root] != root) root = parent[root];
    while (parent[a] != root) {
        int32_t next = parent[a];
        parent[a] = root;
        a = next;
    }
    return root;
}

/* Union: the root with the larger index is attached below the smaller one, so
 * that every tree root is the minimum index of its tree. */
static void uf_union(int32_t *parent, int32_t a, int32_t b)
{
    int32_t ra = uf_find(parent, a), rb = uf_find(parent, b);
    if (ra == rb) return;
    if (ra < rb) parent[rb] = ra;
    else parent[ra] = rb;
}

/* Canonical labels: since parent[i] < i for every non-root i, visiting sites in
 * increasing order lets each non-root copy the finished label of its parent. */
static int64_t uf_flatten(int32_t *parent, int64_t N, int32_t *labels)
{
    int64_t n = 0;
    for (int64_t i = 0; i < N; ++i) {
        if (parent[i] == (int32_t)i) {
            labels[i] = (int32_t)i;
            ++n;
        } else {
            labels[i] = labels[parent[i]];
        }
    }
    return n;
}

int64_t orc_label_bonds(int32_t W, int32_t H, const uint8_t *bonds, int32_t mode,
                        int32_t *labels)
{
    int64_t N = (int64_t)W * H;
    int32_t *parent = (int32_t *)malloc((size_t)(N > 0 ? N : 1) * sizeof(int32_t));
    for (int64_t i = 0; i < N; ++i) parent[i] = (int32_t)i;
    for (int32_t y = 0; y < H; ++y) {
        for (int32_t x = 0; x < W; ++x) {
            int32_t i = y * W + x;
            if ((bonds[i] & 1) && (mode == ORC_PERIODIC || x + 1 < W))
                uf_union(parent, i, y * W + (x + 1) % W);
            if ((bonds[i] & 2) && (mode == ORC_PERIODIC || y + 1 < H))
                uf_union(parent, i, ((y + 1) % H) * W + x);
        }
    }
    int64_t n = uf_flatten(parent, N, labels);
    free(parent);
    return n;
}

int64_t orc_label_sites(int32_t W, int32_t H, const uint8_t *occ, int32_t *labels)
{
    int64_t N = (int64_t)W * H;
    int32_t *parent = (int32_t *)malloc((size_t)(N > 0 ? N : 1) * sizeof(int32_t));
    for (int64_t i = 0; i < N; ++i) parent[i] = (int32_t)i;
    for (int32_t y = 0; y < H; ++y) {
        for (int32_t x = 0; x < W; ++x) {
            int32_t i = y * W + x;
            if (!occ[i]) continue;
            if (x + 1 < W && occ[i + 1]) uf_union(parent, i, i + 1);
            if (y + 1 < H && occ[i + W]) uf_union(parent, i, i + W);
        }
    }
    int64_t n = 0;
    for (int64_t i = 0; i < N; ++i) {
        if (!occ[i]) {
            labels[i] = -1;
        } else if (parent[i] == (int32_t)i) {
            labels[i] = (int32_t)i;
            ++n;
        } else {
            labels[i] = labels[parent[i]];
        }
    }
    free(parent);
    return n;
}

int64_t orc_cluster_sizes(int64_t N, const int32_t *labels, int32_t *roots,
                          int32_t *sizes, int64_t *max_size)
{
    int32_t *count = (int32_t *)calloc((size_t)(N > 0 ? N : 1), sizeof(int32_t));
    for (int64_t i = 0; i < N; ++i)
        if (labels[i] >= 0) count[labels[i]]++;
    int64_t n = 0, mx = 0;
    for (int64_t i = 0; i < N; ++i) {
        if (labels[i] == (int32_t)i) {
            if (roots) roots[n] = (int32_t)i;
            if (sizes) sizes[n] = count[i];
            if (count[i] > mx) mx = count[i];
            ++n;
        }
    }
    if (max_size) *max_size = mx;
    free(count);
    return n;
}

/* ----------------------------------------------------------------- flip -- */

/* Step 3 of the SW update (Sec. II; Sec. II.D): each cluster takes one new
 * state, uniform in 0..q-1, drawn from the word indexed by its canonical root r;
 * every site copies the state of its root. */
void orc_flip(int32_t W, int32_t H, int32_t q, const int32_t *labels, uint64_t seed,
              uint32_t t, uint32_t sid, uint8_t *state)
{
    int64_t N = (int64_t)W * H;
    uint8_t *root_state = (uint8_t *)malloc((size_t)(N > 0 ? N : 1));
    for (int64_t r = 0; r < N; ++r) {
        if (labels[r] != (int32_t)r) continue;
        uint32_t b[4];
        block_for(seed, (uint32_t)(r >> 2), t, ORC_TAG_FLIP, sid, b);
        root_state[r] = state_from_word(b[r & 3], q);
    }
    for (int64_t i = 0; i < N; ++i) state[i] = root_state[labels[i]];
    free(root_state);
}

/* --------------------------------------------------------------- digest -- */

/* Check-sum of an array, defined in the header: one Philox block per element,
 * keyed by the element's index and value, summed with 64-bit wrap-around. */
static uint64_t digest_term(uint32_t i, uint32_t v)
{
    const uint32_t ctr[4] = {i, v, ORC_DIGEST_TAG, 0u};
    const uint32_t key[2] = {0u, 0u};
    uint32_t out[4];
    orc_philox4x32_10(ctr, key, out);
    return (uint64_t)out[0] | ((uint64_t)out[1] << 32);
}

uint64_t orc_digest_u8(int64_t N, const uint8_t *a)
{
    uint64_t d = 0;
    for (int64_t i = 0; i < N; ++i) d += digest_term((uint32_t)i, a[i]);
    return d;
}

uint64_t orc_digest_i32(int64_t N, const int32_t *a)
{
    uint64_t d = 0;
    for (int64_t i = 0; i < N; ++i) d += digest_term((uint32_t)i, (uint32_t)a[i]);
    return d;
}

/* ---------------------------------------------------------- observables -- */

/* Number of satisfied bonds, i.e. -H/J of Eq. potts_hamiltonian. */
int64_t orc_satisfied(int32_t W, int32_t H, int32_t q, const uint8_t *state,
                      int64_t counts[8])
{
    int64_t nsat = 0;
    if (counts)
        for (int k = 0; k < 8; ++k) counts[k] = 0;
    for (int32_t y = 0; y < H; ++y) {
        for (int32_t x = 0; x < W; ++x) {
            int64_t i = (int64_t)y * W + x;
            nsat += state[i] == state[(int64_t)y * W + (x + 1) % W];
            nsat += state[i] == state[(int64_t)((y + 1) % H) * W + x];
            if (counts && state[i] < 8 && state[i] < q) counts[state[i]]++;
        }
    }
    return nsat;
}

/* ---------------------------------------------------------------- sweep -- */

void orc_sw_sweep(int32_t W, int32_t H, int32_t q, uint64_t T, uint64_t seed,
                  uint32_t sid, uint32_t t, uint8_t *state, uint8_t *bonds,
                  int32_t *labels, int64_t *rec)
{
    int64_t N = (int64_t)W * H;
    uint8_t *b = bonds ? bonds : (uint8_t *)malloc((size_t)N);
    int32_t *l = labels ? labels : (int32_t *)malloc((size_t)N * sizeof(int32_t));

    orc_activate_bonds(W, H, state, T, seed, t, sid, b);
    int64_t ncl = orc_label_bonds(W, H, b, ORC_PERIODIC, l);
    if (rec) {
        int64_t active = 0;
        for (int64_t i = 0; i < N; ++i) active += (b[i] & 1) + ((b[i] >> 1) & 1);
        int64_t mx = 0;
        orc_cluster_sizes(N, l, NULL, NULL, &mx);
        rec[ORC_REC_ACTIVE] = active;
        rec[ORC_REC_NCLUST] = ncl;
        rec[ORC_REC_MAXCL] = mx;
    }
    orc_flip(W, H, q, l, seed, t, sid, state);
    if (rec) rec[ORC_REC_NSAT] = orc_satisfied(W, H, q, state, rec + ORC_REC_COUNTS);

    if (!bonds) free(b);
    if (!labels) free(l);
}

/* ---------------------------------------------------------- few-cluster -- */

/* floor(p 2^32) for a probability p in [0, 1): an event of probability p
 * happens iff a uniform 32-bit word is below it. */
uint64_t orc_prob_threshold(double p)
{
    if (!(p > 0.0)) return 0;
    double v = floor(ldexp(p, 32));
    if (v >= 4294967295.0) return 4294967295ull;
    return (uint64_t)v;
}

/* The seeds of the few-cluster variant (Sec. III): the lattice is cut into
 * seed tiles of B x B sites (the last column and row of tiles may be
 * narrower), tile j = ty * ceil(W / B) + tx, and each tile draws one site
 * uniformly from its own sites: x from word 0 and y from word 1 of the block
 * (j, t, SEED, sid), each as floor(w * extent / 2^32).  Returns the number of
 * seed tiles; sites[j] receives tile j's seed. */
int64_t orc_few_seeds(int32_t W, int32_t H, int32_t B, uint64_t seed, uint32_t t,
                      uint32_t sid, int32_t *sites)
{
    int32_t ntx = (W + B - 1) / B, nty = (H + B - 1) / B;
    for (int32_t ty = 0; ty < nty; ++ty) {
        for (int32_t tx = 0; tx < ntx; ++tx) {
            int32_t j = ty * ntx + tx;
            int32_t bw = W - tx * B < B ? W - tx * B : B;
            int32_t bh = H - ty * B < B ? H - ty * B : B;
            uint32_t b[4];
            block_for(seed, (uint32_t)j, t, ORC_TAG_SEED, sid, b);
            int32_t x = tx * B + (int32_t)(((uint64_t)b[0] * (uint64_t)bw) >> 32);
            int32_t y = ty * B + (int32_t)(((uint64_t)b[1] * (uint64_t)bh) >> 32);
            sites[j] = y * W + x;
        }
    }
    return (int64_t)ntx * nty;
}

/* One few-cluster sweep t of a q = 2 lattice in place (Sec. III).  Steps 1
 * and 2 are those of the SW update; then every cluster that holds at least
 * one seed is flipped (state -> 1 - state) iff the word of the block
 * (r >> 2, t, FEW, sid) picked by r & 3 is below Tflip, r its canonical root:
 * one draw per distinct cluster, however many seeds it holds.  few (may be
 * NULL) receives the number of distinct seeded clusters and of flipped
 * clusters. */
void orc_few_sweep(int32_t W, int32_t H, uint64_t T, uint64_t Tflip, int32_t B,
                   uint64_t seed, uint32_t sid, uint32_t t, uint8_t *state, uint8_t *bonds,
                   int32_t *labels, int64_t *rec, int64_t *few)
{
    int64_t N = (int64_t)W * H;
    uint8_t *b = bonds ? bonds : (uint8_t *)malloc((size_t)N);
    int32_t *l = labels ? labels : (int32_t *)malloc((size_t)N * sizeof(int32_t));

    orc_activate_bonds(W, H, state, T, seed, t, sid, b);
    int64_t ncl = orc_label_bonds(W, H, b, ORC_PERIODIC, l);
    if (rec) {
        int64_t active = 0;
        for (int64_t i = 0; i < N; ++i) active += (b[i] & 1) + ((b[i] >> 1) & 1);
        int64_t mx = 0;
        orc_cluster_sizes(N, l, NULL, NULL, &mx);
        rec[ORC_REC_ACTIVE] = active;
        rec[ORC_REC_NCLUST] = ncl;
        rec[ORC_REC_MAXCL] = mx;
    }

    int64_t nseed = (int64_t)((W + B - 1) / B) * ((H + B - 1) / B);
    int32_t *sites = (int32_t *)malloc((size_t)nseed * sizeof(int32_t));
    uint8_t *seeded = (uint8_t *)calloc((size_t)N, 1);   /* per canonical root */
    uint8_t *flipped = (uint8_t *)calloc((size_t)N, 1);  /* per canonical root */
    orc_few_seeds(W, H, B, seed, t, sid, sites);
    for (int64_t j = 0; j < nseed; ++j) seeded[l[sites[j]]] = 1;
    int64_t n_seeded = 0, n_flipped = 0;
    for (int64_t r = 0; r < N; ++r) {
        if (!seeded[r]) continue;
        ++n_seeded;
        uint32_t w[4];
        block_for(seed, (uint32_t)(r >> 2), t, ORC_TAG_FEW, sid, w);
        if ((uint64_t)w[r & 3] < Tflip) {
            flipped[r] = 1;
            ++n_flipped;
        }
    }
    for (int64_t i = 0; i < N; ++i)
        if (flipped[l[i]]) state[i] = (uint8_t)(1 - state[i]);
    if (few) {
        few[0] = n_seeded;
        few[1] = n_flipped;
    }
    if (rec) rec[ORC_REC_NSAT] = orc_satisfied(W, H, 2, state, rec + ORC_REC_COUNTS);

    free(sites);
    free(seeded);
    free(flipped);
    if (!bonds) free(b);
    if (!labels) free(l);
}

void orc_sw_run(int32_t W, int32_t H, int32_t q, uint64_t T, uint64_t seed,
                uint32_t sid, uint32_t t0, int32_t n, uint8_t *state, int64_t *rec)
{
    int64_t N = (int64_t)W * H;
    uint8_t *b = (uint8_t *)malloc((size_t)N);
    int32_t *l = (int32_t *)malloc((size_t)N * sizeof(int32_t));
    for (int32_t k = 0; k < n; ++k)
        orc_sw_sweep(W, H, q, T, seed, sid, t0 + (uint32_t)k, state, b, l,
                     rec ? rec + (int64_t)k * ORC_REC_LEN : NULL);
    free(b);
    free(l);
}

/* ------------------------------------------------------- cubic lattices -- */

/* Step 1 on the simple cubic lattice: the bond-activation rule of Sec. II.A
 * applied to the +x, +y and +z bond of every site. */
void orc3_activate_bonds(int32_t Lx, int32_t Ly, int32_t Lz, const uint8_t *state, uint64_t T,
                         uint64_t seed, uint32_t t, uint32_t sid, uint8_t *bonds)
{
    for (int32_t z = 0; z < Lz; ++z) {
        for (int32_t y = 0; y < Ly; ++y) {
            for (int32_t x = 0; x < Lx; ++x) {
                int64_t i = ((int64_t)z * Ly + y) * Lx + x;
                int64_t nx = ((int64_t)z * Ly + y) * Lx + (x + 1) % Lx;
                int64_t ny = ((int64_t)z * Ly + (y + 1) % Ly) * Lx + x;
                int64_t nz = ((int64_t)((z + 1) % Lz) * Ly + y) * Lx + x;
                uint32_t b[4], bz[4];
                block_for(seed, (uint32_t)(i >> 1), t, ORC_TAG_BOND, sid, b);
                block_for(seed, (uint32_t)(i >> 2), t, ORC_TAG_BOND_Z, sid, bz);
                int ax = state[i] == state[nx] && (uint64_t)b[2 * (i & 1)] < T;
                int ay = state[i] == state[ny] && (uint64_t)b[2 * (i & 1) + 1] < T;
                int az = state[i] == state[nz] && (uint64_t)bz[i & 3] < T;
                bonds[i] = (uint8_t)(ax | (ay << 1) | (az << 2));
            }
        }
    }
}

/* Step 2 on the cubic lattice: union-and-find over every active bond
 * (Sec. II.B.2), canonical minimum-index labels. */
int64_t orc3_label_bonds(int32_t Lx, int32_t Ly, int32_t Lz, const uint8_t *bonds, int32_t *labels)
{
    int64_t N = (int64_t)Lx * Ly * Lz;
    int32_t *parent = (int32_t *)malloc((size_t)(N > 0 ? N : 1) * sizeof(int32_t));
    for (int64_t i = 0; i < N; ++i) parent[i] = (int32_t)i;
    for (int32_t z = 0; z < Lz; ++z) {
        for (int32_t y = 0; y < Ly; ++y) {
            for (int32_t x = 0; x < Lx; ++x) {
                int32_t i = (z * Ly + y) * Lx + x;
                if (bonds[i] & 1) uf_union(parent, i, (z * Ly + y) * Lx + (x + 1) % Lx);
                if (bonds[i] & 2) uf_union(parent, i, (z * Ly + (y + 1) % Ly) * Lx + x);
                if (bonds[i] & 4) uf_union(parent, i, (((z + 1) % Lz) * Ly + y) * Lx + x);
            }
        }
    }
    int64_t n = uf_flatten(parent, N, labels);
    free(parent);
    return n;
}

/* -H/J of Eq. potts_hamiltonian on the cubic lattice: satisfied bonds among
 * the 3N nearest-neighbour pairs (each site's +x, +y and +z pair). */
int64_t orc3_satisfied(int32_t Lx, int32_t Ly, int32_t Lz, int32_t q, const uint8_t *state,
                       int64_t counts[8])
{
    int64_t nsat = 0;
    if (counts)
        for (int k = 0; k < 8; ++k) counts[k] = 0;
    for (int32_t z = 0; z < Lz; ++z) {
        for (int32_t y = 0; y < Ly; ++y) {
            for (int32_t x = 0; x < Lx; ++x) {
                int64_t i = ((int64_t)z * Ly + y) * Lx + x;
                nsat += state[i] == state[((int64_t)z * Ly + y) * Lx + (x + 1) % Lx];
                nsat += state[i] == state[((int64_t)z * Ly + (y + 1) % Ly) * Lx + x];
                nsat += state[i] == state[((int64_t)((z + 1) % Lz) * Ly + y) * Lx + x];
                if (counts && state[i] < 8 && state[i] < q) counts[state[i]]++;
            }
        }
    }
    return nsat;
}

void orc3_sw_sweep(int32_t Lx, int32_t Ly, int32_t Lz, int32_t q, uint64_t T, uint64_t seed,
                   uint32_t sid, uint32_t t, uint8_t *state, uint8_t *bonds, int32_t *labels,
                   int64_t *rec)
{
    int64_t N = (int64_t)Lx * Ly * Lz;
    uint8_t *b = bonds ? bonds : (uint8_t *)malloc((size_t)N);
    int32_t *l = labels ? labels : (int32_t *)malloc((size_t)N * sizeof(int32_t));

    orc3_activate_bonds(Lx, Ly, Lz, state, T, seed, t, sid, b);
    int64_t ncl = orc3_label_bonds(Lx, Ly, Lz, b, l);
    if (rec) {
        int64_t active = 0;
        for (int64_t i = 0; i < N; ++i) active += (b[i] & 1) + ((b[i] >> 1) & 1) + ((b[i] >> 2) & 1);
        rec[ORC3_REC_ACTIVE] = active;
        rec[ORC3_REC_NCLUST] = ncl;
    }
    /* step 3 is the square lattice's: one draw per canonical root */
    orc_flip(Lx, Ly * Lz, q, l, seed, t, sid, state);
    if (rec) rec[ORC3_REC_NSAT] = orc3_satisfied(Lx, Ly, Lz, q, state, rec + ORC3_REC_COUNTS);

    if (!bonds) free(b);
    if (!labels) free(l);
}

void orc3_sw_run(int32_t Lx, int32_t Ly, int32_t Lz, int32_t q, uint64_t T, uint64_t seed,
                 uint32_t sid, uint32_t t0, int32_t n, uint8_t *state, int64_t *rec)
{
    int64_t N = (int64_t)Lx * Ly * Lz;
    uint8_t *b = (uint8_t *)malloc((size_t)N);
    int32_t *l = (int32_t *)malloc((size_t)N * sizeof(int32_t));
    for (int32_t k = 0; k < n; ++k)
        orc3_sw_sweep(Lx, Ly, Lz, q, T, seed, sid, t0 + (uint32_t)k, state, b, l,
                      rec ? rec + (int64_t)k * ORC3_REC_LEN : NULL);
    free(b);
    free(l);
}
