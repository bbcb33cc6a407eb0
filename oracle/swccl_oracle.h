/*
 * swccl_oracle.h -- the CPU oracle for the Swendsen-Wang sweep and for
 * connected-component labeling on 2D square lattices.
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, sequential, deliberately slow
 * reference.  Only the test-suite, the smoke check and the CPU-baseline leg of
 * the benchmark may call it; the product path never does.  It shares no code,
 * header, table or helper with the GPU library.
 *
 * Conventions (shared *by definition*, not by code, with the GPU library):
 *   - site index i = y*W + x, x fastest; N = W*H.
 *   - site i owns two bonds: "right" to (x+1 mod W, y) and "down" to
 *     (x, y+1 mod H).  Packed bond byte: bit0 = right, bit1 = down.
 *   - Potts states are stored as 0..q-1 (the paper's 1..q shifted by one).
 *   - Philox4x32-10: key = (lo32(seed), hi32(seed)), counter =
 *     (index word, sweep t, tag, stream id), tags below.
 *   - a bond between equal spins is active iff its 32-bit uniform r satisfies
 *     r < T with T = floor(p * 2^32), p = 1 - exp(-K)  (Sec. II, Eq. fortuin3
 *     and the bond-activation rule of Sec. II.A).
 *   - the canonical label of a cluster is its minimum site index.
 *
 * Each function cites the passage of the paper it follows.
 */
#ifndef SWCCL_ORACLE_H
#define SWCCL_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_TAG_INIT = 0, ORC_TAG_BOND = 1, ORC_TAG_FLIP = 2, ORC_TAG_SEED = 3, ORC_TAG_FEW = 4,
       ORC_TAG_BOND_Z = 5 };
enum { ORC_PERIODIC = 0, ORC_OPEN = 1 };

/* Per-sweep record written by orc_sw_run (one row of ORC_REC_LEN int64). */
enum {
    ORC_REC_ACTIVE = 0,   /* active bonds of the sweep's bond configuration */
    ORC_REC_NCLUST = 1,   /* number of clusters (components)                 */
    ORC_REC_MAXCL = 2,    /* largest cluster size                            */
    ORC_REC_NSAT = 3,     /* satisfied bonds of the spins after the flip     */
    ORC_REC_COUNTS = 4,   /* counts[0..7] of states after the flip           */
    ORC_REC_LEN = 12
};

/* Philox4x32-10 block function (Salmon et al., SC'11). */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* T = floor((1 - exp(-K)) * 2^32), clamped to [0, 2^32]. */
uint64_t orc_threshold(double K);

/* Random initial states 0..q-1 (tag INIT, sweep word 0). */
void orc_init_states(int32_t W, int32_t H, int32_t q, uint64_t seed, uint32_t sid,
                     uint8_t *state);

/* Step 1 of the SW update: packed bond bytes for sweep t. */
void orc_activate_bonds(int32_t W, int32_t H, const uint8_t *state, uint64_t T,
                        uint64_t seed, uint32_t t, uint32_t sid, uint8_t *bonds);

/* Step 2: canonical component labels of a bond configuration.  mode is
 * ORC_PERIODIC or ORC_OPEN (wrap bonds ignored).  Returns the cluster count. */
int64_t orc_label_bonds(int32_t W, int32_t H, const uint8_t *bonds, int32_t mode,
                        int32_t *labels);

/* Labeling of a binary image: 4-connected occupied pixels (occ != 0), open
 * boundaries; background pixels get label -1.  Returns the cluster count. */
int64_t orc_label_sites(int32_t W, int32_t H, const uint8_t *occ, int32_t *labels);

/* Cluster sizes: roots in ascending order and their sizes; labels < 0 are
 * skipped.  roots/sizes may be NULL.  Returns the cluster count and the largest
 * size in *max_size (if not NULL). */
int64_t orc_cluster_sizes(int64_t N, const int32_t *labels, int32_t *roots,
                          int32_t *sizes, int64_t *max_size);

/* Step 3: every cluster takes the state drawn at its canonical root. */
void orc_flip(int32_t W, int32_t H, int32_t q, const int32_t *labels, uint64_t seed,
              uint32_t t, uint32_t sid, uint8_t *state);

/* Satisfied bonds (s_i == s_j over all 2N bonds) and, for k < min(q, 8),
 * counts[k] = number of sites in state k. */
int64_t orc_satisfied(int32_t W, int32_t H, int32_t q, const uint8_t *state,
                      int64_t counts[8]);

/* One SW sweep t in place.  bonds/labels (may be NULL) receive the sweep's
 * bond configuration and canonical labels (both of the pre-flip spins).
 * rec (may be NULL) receives one ORC_REC_LEN record. */
void orc_sw_sweep(int32_t W, int32_t H, int32_t q, uint64_t T, uint64_t seed,
                  uint32_t sid, uint32_t t, uint8_t *state, uint8_t *bonds,
                  int32_t *labels, int64_t *rec);

/* Order-independent digest of an array of N values a_i (a check-sum for
 * comparing large arrays without copying them):
 *   sum over i of lo64(Philox4x32-10(ctr = (i, a_i, ORC_DIGEST_TAG, 0), key = (0, 0)))
 * modulo 2^64, where lo64 = word0 | word1 << 32.  Values are taken as uint32
 * (int32 labels by their two's-complement bits). */
enum { ORC_DIGEST_TAG = 0xD16E57 };
uint64_t orc_digest_u8(int64_t N, const uint8_t *a);
uint64_t orc_digest_i32(int64_t N, const int32_t *a);

/* floor(p 2^32) for p in [0, 1), clamped to [0, 2^32 - 1]. */
uint64_t orc_prob_threshold(double p);
/* Few-cluster variant (Sec. III): one seed per B x B seed tile of sweep t
 * (tag SEED, counter word = tile index).  Returns the tile count. */
int64_t orc_few_seeds(int32_t W, int32_t H, int32_t B, uint64_t seed, uint32_t t,
                      uint32_t sid, int32_t *sites);
/* One few-cluster sweep of a q = 2 lattice: SW bonds and clusters, then every
 * distinct seeded cluster flips iff its root's FEW word is below Tflip.
 * few[0] = distinct seeded clusters, few[1] = flipped clusters (few may be
 * NULL); bonds, labels and rec as for orc_sw_sweep. */
void orc_few_sweep(int32_t W, int32_t H, uint64_t T, uint64_t Tflip, int32_t B,
                   uint64_t seed, uint32_t sid, uint32_t t, uint8_t *state, uint8_t *bonds,
                   int32_t *labels, int64_t *rec, int64_t *few);
/* n sweeps t0..t0+n-1, one record per sweep into rec[n][ORC_REC_LEN]. */
void orc_sw_run(int32_t W, int32_t H, int32_t q, uint64_t T, uint64_t seed,
                uint32_t sid, uint32_t t0, int32_t n, uint8_t *state, int64_t *rec);

/* ---- Simple cubic lattices (the 3D generalisation of Sec. II) ----
 * Lx x Ly x Lz sites, periodic along all three axes, site index
 * i = (z*Ly + y)*Lx + x, N < 2^31.  Site i owns the +x bond to
 * (x+1 mod Lx, y, z), the +y bond to (x, y+1 mod Ly, z) and the +z bond to
 * (x, y, z+1 mod Lz); packed bond byte: bit0 = +x, bit1 = +y, bit2 = +z.
 * The +x and +y words are those of the square lattice at the same index
 * (block(i>>1, t, BOND), words 2(i&1) and 2(i&1)+1); the +z word is
 * block(i>>2, t, BOND_Z)[i&3].  Initial states and cluster draws are those of
 * the square lattice at the same index.  With Lz = 1 the +z bond joins a site
 * to itself, and a sweep equals the square-lattice sweep of Lx x Ly. */
enum {
    ORC3_REC_ACTIVE = 0,  /* active bonds (all three directions)        */
    ORC3_REC_NCLUST = 1,  /* clusters                                   */
    ORC3_REC_NSAT = 2,    /* satisfied bonds of the spins after the flip */
    ORC3_REC_COUNTS = 3,  /* counts[0..7] of states after the flip       */
    ORC3_REC_LEN = 11
};
void orc3_activate_bonds(int32_t Lx, int32_t Ly, int32_t Lz, const uint8_t *state, uint64_t T,
                         uint64_t seed, uint32_t t, uint32_t sid, uint8_t *bonds);
/* Canonical labels of a packed 3D bond configuration (all bonds periodic);
 * returns the cluster count. */
int64_t orc3_label_bonds(int32_t Lx, int32_t Ly, int32_t Lz, const uint8_t *bonds, int32_t *labels);
/* Satisfied bonds over all 3N bonds and, for k < min(q, 8), state counts. */
int64_t orc3_satisfied(int32_t Lx, int32_t Ly, int32_t Lz, int32_t q, const uint8_t *state,
                       int64_t counts[8]);
/* One SW sweep t of the cubic lattice in place; bonds/labels/rec as for
 * orc_sw_sweep (rec: one ORC3_REC_LEN record). */
void orc3_sw_sweep(int32_t Lx, int32_t Ly, int32_t Lz, int32_t q, uint64_t T, uint64_t seed,
                   uint32_t sid, uint32_t t, uint8_t *state, uint8_t *bonds, int32_t *labels,
                   int64_t *rec);
/* n sweeps t0..t0+n-1, one record per sweep into rec[n][ORC3_REC_LEN]. */
void orc3_sw_run(int32_t Lx, int32_t Ly, int32_t Lz, int32_t q, uint64_t T, uint64_t seed,
                 uint32_t sid, uint32_t t0, int32_t n, uint8_t *state, int64_t *rec);

#ifdef __cplusplus
}
#endif
#endif
