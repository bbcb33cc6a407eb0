/*
 * swccl.h -- C ABI of the MI355X (gfx950) Swendsen-Wang / connected-component
 * labeling library (libswccl.so).
 *
 * The library runs one Swendsen-Wang (SW) sweep of a periodic 2D q-state Potts
 * or Ising lattice as three device phases -- bond activation fused with tile
 * labeling, cross-tile merging, and flatten + cluster flip -- and exposes the
 * same labeling kernels as a standalone connected-component labeling call.
 *
 * Model and update (M. Weigel, "Connected component identification and
 * cluster update on GPU", arXiv:1105.5804):
 *   - Potts Hamiltonian, Sec. II, Eq. potts_hamiltonian; q = 2 is the Ising
 *     model.
 *   - Bond variables and p = 1 - exp(-K), Sec. II, Eqs. fortuin1-fortuin3
 *     (K = beta*J in the Potts normalisation; for Ising spins s = +-1 with
 *     H = -J sum s_i s_j pass K = 2*beta*J).
 *   - SW steps 1-3 (activate bonds between equal spins with probability p,
 *     identify connected components, draw one new state per component),
 *     Sec. II enumerated steps; bond activation rule, Sec. II.A; cluster
 *     flipping, Sec. II.D.
 *   - Connected-component labeling as image segmentation / percolation,
 *     Sec. I and Sec. II.
 *
 * Conventions (bit-exact contract; the CPU oracle implements the same
 * definitions independently):
 *   - site index i = y*W + x (x fastest), N = W*H, N < 2^31.
 *   - site i owns the "right" bond to (x+1 mod W, y) and the "down" bond to
 *     (x, y+1 mod H).  Packed bond byte: bit0 = right, bit1 = down.
 *   - random numbers: Philox4x32-10 (Salmon et al., SC'11) with
 *     key = (lo32(seed), hi32(seed)) and counter = (word, t, tag, stream_id).
 *       init  (tag 0): state_i = (w * q) >> 32, w = block(i>>2, 0)[i&3]
 *       bonds (tag 1): block(i>>1, t): right uses word 2(i&1), down 2(i&1)+1
 *       flip  (tag 2): a cluster with canonical root r takes
 *                      (block(r>>2, t)[r&3] * q) >> 32
 *       seed  (tag 3): few-cluster update, seed tile j of edge B (raster
 *                      order, ceil(W/B) per row, narrower at the edges):
 *                      x = tx*B + (w0 * bw) >> 32, y = ty*B + (w1 * bh) >> 32
 *                      with (w0, w1) words 0 and 1 of block(j, t)
 *       few   (tag 4): a seeded cluster with canonical root r flips iff
 *                      block(r>>2, t)[r&3] < floor(p_flip * 2^32)
 *   - a bond between equal spins is active iff its word r < T, with
 *     T = floor((1 - exp(-K)) * 2^32) computed on the host in double.
 *   - the canonical label of a cluster is the minimum site index in it.
 *   - states are stored 0..q-1 (SW_SPIN_POTTS_U8, the paper's 1..q minus one)
 *     or as int8 -1/+1 (SW_SPIN_ISING_I8, q = 2, state 0 <-> -1).
 *
 * Memory and ownership: every device buffer is allocated and owned by the
 * caller; the library allocates no device memory.  Scratch space is the caller's
 * workspace of at least *_workspace_bytes() bytes.  A lattice handle is a small
 * host object created by sw_init and freed by sw_destroy (a batch that ran
 * swb_sweep_graph also holds a capture stream and executable graphs until
 * swb_destroy).
 *
 * Streams: every call enqueues on the given stream (a hipStream_t passed as
 * void*; NULL is the null stream) and returns without waiting, except
 * sw_observables and swb_observables, which wait for the stream, and the
 * server's release and destroy, which wait for their requests.
 *
 * Errors: every entry point returns an sw_status; arguments are checked before
 * anything is enqueued and nothing throws across the ABI.  SW_ERR_DEVICE means
 * a HIP launch or copy failed; sw_last_error() returns its message.
 */
#ifndef SWCCL_H
#define SWCCL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SWCCL_ABI_VERSION 7

typedef int32_t sw_status;
enum {
    SW_OK = 0,
    SW_ERR_ARG = 1,         /* null pointer, bad enum, q out of range, n < 0 */
    SW_ERR_SIZE = 2,        /* W or H < 1 (< 2 for SW), W*H >= 2^31, or a
                               lattice so thin that its tiles' boundary ids
                               (384 per 128 x 64 tile) reach 2^31          */
    SW_ERR_WORKSPACE = 3,   /* workspace missing or smaller than required   */
    SW_ERR_DEVICE = 4,      /* a HIP call failed (see sw_last_error)         */
    SW_ERR_STATE = 5,       /* call out of order, sweep counter would pass
                               32 bits, or no server block or slot free now */
    SW_ERR_UNSUPPORTED = 6, /* combination not supported by the library      */
    SW_ERR_HOST_MEMORY = 7  /* a host-side allocation of the library failed  */
};

/* Spin storage. */
enum { SW_SPIN_ISING_I8 = 0, SW_SPIN_POTTS_U8 = 1 };

/* sw_params.flags */
enum {
    SW_F_KEEP_SPINS = 1u << 0, /* sw_init: do not draw initial spins; use the
                                  caller's (restart from a saved state)       */
    SW_F_SIZES = 1u << 1,      /* every sweep also lists its clusters: roots
                                  (ascending) and sizes into sw_buffers.roots /
                                  .sizes, and the largest size (sw_obs)       */
    SW_F_REVERSE_TILES = 1u << 2, /* a schedule check: the workgroups of the
                                  tile, merge and flip launches visit the
                                  tiles in the reverse order.  Every output is
                                  canonical (minimum-index labels, draws keyed
                                  on the index), so it is identical either
                                  way; batches reject this flag. */
    SW_F_BATCH_FUSED = 1u << 3   /* batches only (on p[0]): sweep with the
                                  fused persistent launch instead of one
                                  launch per phase; the same results.  Single
                                  lattices reject it. */
};

/* Input kinds of ccl_label. */
enum {
    CCL_BONDS_PERIODIC = 0, /* packed bond bytes, bonds wrap around both axes */
    CCL_BONDS_OPEN = 1,     /* packed bond bytes, wrap bonds ignored          */
    CCL_SITES_OPEN = 2      /* binary image (byte != 0 occupied), 4-connected,
                               open boundary; background pixels get label -1 */
};

typedef struct sw_params {
    int32_t W, H;       /* lattice extent, W, H >= 2, W*H < 2^31             */
    int32_t q;          /* number of Potts states, 2..255 (2 for Ising)     */
    int32_t spin_kind;  /* SW_SPIN_ISING_I8 (q must be 2) or SW_SPIN_POTTS_U8 */
    double K;           /* FK coupling: p = 1 - exp(-K); K <= 0 gives p = 0,
                           K = +inf gives p = 1                              */
    uint64_t seed;      /* Philox key                                       */
    uint32_t stream_id; /* fourth counter word: independent replicas        */
    uint32_t flags;     /* SW_F_*                                           */
    int32_t tile_h;     /* tile height of the labeling (tiles are 128 wide):
                           16, 32, 64 or 128, or 0 for the default 64.  The
                           tile size is a free parameter of the paper's
                           local/global split (Sec. II.E, Eqs. optimaltile1-2);
                           results do not depend on it                      */
    int32_t merge_waves; /* merge schedule: tiles per merge workgroup (one
                           wave each), 4, 8 or 16, or 0 for the default 8;
                           results do not depend on it                      */
    double p_flip;      /* few-cluster update only: flip probability of a
                           seeded cluster, 0 <= p_flip < 1                  */
    int32_t few_b;      /* 0: the SW update (every cluster draws a new
                           state).  B >= 1: the few-cluster variant of the
                           Wolff update (Sec. III; q = 2 only, single
                           lattices only): SW bonds and clusters, then one
                           seed per B x B seed tile, and every distinct
                           cluster holding a seed flips (state -> 1 - state)
                           with probability p_flip, one draw per cluster at
                           its canonical root; only flipped sites are
                           written                                          */
    int32_t reserved;   /* must be 0                                        */
} sw_params;

/* Device buffers of one lattice.  All are row-major (i = y*W + x). */
typedef struct sw_buffers {
    void *spins;            /* N bytes (int8 or uint8), read and written     */
    int32_t *labels;        /* N int32 or NULL: canonical labels of the last
                               sweep's bond configuration                   */
    uint8_t *bonds;         /* N bytes or NULL: packed bonds of the last sweep */
    int32_t *roots;         /* N int32 with SW_F_SIZES (else ignored): the last
                               sweep's canonical roots in ascending order, in
                               the first n_clusters entries                 */
    int32_t *sizes;         /* N int32 with SW_F_SIZES: sizes[k] is the size of
                               the cluster rooted at roots[k]               */
    void *workspace;        /* sw_workspace_bytes() bytes, 256-byte aligned  */
    size_t workspace_bytes;
} sw_buffers;

/* Observables; see sw_observables. */
typedef struct sw_obs {
    uint64_t t;              /* sweeps done so far                              */
    uint64_t threshold;      /* T used for bond activation                      */
    int64_t n_sat;           /* satisfied bonds of the current spins (-H/J)     */
    int64_t magnet;          /* Ising: sum of spins; Potts: 0                   */
    int64_t counts[8];       /* sites in state k, k < min(q, 8)                 */
    int64_t n_active_bonds;  /* active bonds of the last sweep (-1: none yet)   */
    int64_t n_clusters;      /* clusters of the last sweep (-1: none yet)       */
    int64_t max_cluster;     /* largest cluster of the last sweep (-1: none yet,
                                or SW_F_SIZES not set)                          */
    /* Order-independent check-sums of the arrays, for comparing runs without
     * copying them: sum over i of lo64(Philox4x32-10(ctr = (i, a_i, 0xD16E57, 0),
     * key = (0, 0))) mod 2^64 with lo64 = word0 | word1 << 32.  a_i is the state
     * 0..q-1 of site i (Ising: +1 -> 1, -1 -> 0), the label bits as uint32, or
     * the bond byte.  Labels / bonds digests are 0 when the buffer is absent or
     * before the first sweep. */
    uint64_t digest_spins;
    uint64_t digest_labels;
    uint64_t digest_bonds;
} sw_obs;

typedef struct sw_lattice sw_lattice;

/* Library and build information. */
int32_t swccl_abi_version(void);
const char *sw_status_string(sw_status s);
/* Message of the last SW_ERR_DEVICE on the calling thread ("" if none). */
const char *sw_last_error(void);

/* T = floor((1 - exp(-K)) * 2^32) clamped to [0, 2^32]: the integer threshold a
 * bond's 32-bit uniform must stay below (Sec. II.A activation rule). */
uint64_t sw_threshold(double K);

/* Workspace bytes needed by a lattice with these parameters, SW_F_SIZES and
 * the few-cluster update's seed marks included (0 if invalid). */
size_t sw_workspace_bytes(const sw_params *p);

/* Create a lattice handle over caller-owned buffers and, unless
 * SW_F_KEEP_SPINS is set, draw the initial spins (t = 0, Philox tag 0): each
 * site independently uniform over the q states, the same law as the state a
 * cluster draws in SW step 3 (Sec. II, enumerated steps).
 * SW_F_SIZES needs b->roots and b->sizes (else SW_ERR_ARG).
 * The handle keeps copies of p and b; the buffers must outlive it.
 * Returns SW_ERR_ARG / SW_ERR_SIZE / SW_ERR_WORKSPACE before enqueuing
 * anything, SW_ERR_HOST_MEMORY if the handle cannot be allocated. */
sw_status sw_init(sw_lattice **out, const sw_params *p, const sw_buffers *b, void *stream);

/* Enqueue n_sweeps SW sweeps t, t+1, ... (Sec. II, steps 1-3).  After the call
 * the spins hold the configuration after the last sweep; labels / bonds (if
 * given) hold that sweep's canonical labels / bond bytes, taken before its
 * flip.  n_sweeps = 0 is a no-op.  With p->few_b > 0 each sweep is a
 * few-cluster update instead (Sec. III): the same bonds and clusters, then
 * the seeded clusters flip as described at sw_params.few_b. */
sw_status sw_sweep(sw_lattice *h, int32_t n_sweeps, void *stream);

/* Per-sweep records of sw_sweep_history (int64 each). */
enum {
    SW_HIST_ACTIVE = 0,  /* active bonds of the sweep                         */
    SW_HIST_NCLUST = 1,  /* clusters of the sweep                             */
    SW_HIST_MAXCL = 2,   /* largest cluster (with SW_F_SIZES), else -1        */
    SW_HIST_NSAT = 3,    /* satisfied bonds of the spins after the flip       */
    SW_HIST_COUNTS = 4,  /* 8 entries: sites in state k after the flip, k < 8 */
    SW_HIST_LEN = 12
};

/* sw_sweep plus one record per sweep into history (device, n_sweeps x
 * SW_HIST_LEN int64, row k for sweep t + k), written on the stream without
 * waiting: a measurement series needs no host round trip per sweep. */
sw_status sw_sweep_history(sw_lattice *h, int32_t n_sweeps, int64_t *history, void *stream);

/* One phase of a sweep, for per-phase timing (Sec. II.E decomposes T_SW into
 * activation + local labeling, consolidation across tiles, and flipping):
 * SW_PHASE_TILE, SW_PHASE_MERGE, SW_PHASE_FLIP in this order make one sweep,
 * identical to sw_sweep(h, 1); t advances after SW_PHASE_FLIP.  A phase out of
 * order returns SW_ERR_STATE; sw_sweep and sw_set_t need the next phase to be
 * SW_PHASE_TILE. */
enum { SW_PHASE_TILE = 0, SW_PHASE_MERGE = 1, SW_PHASE_FLIP = 2 };
sw_status sw_sweep_phase(sw_lattice *h, int32_t phase, void *stream);

/* Measure the current spins (satisfied bonds, state counts, digests) and the
 * last sweep's counters (active bonds, clusters, largest cluster); waits for
 * the stream.  The number of satisfied bonds is -H/J of the Potts Hamiltonian
 * (Sec. II, Eq. potts_hamiltonian); the Ising energy per site follows as
 * -(2 n_sat - 2N)/N and the magnetisation from the state counts.  Active bonds
 * and clusters are those of the last sweep's steps 1 and 2 (Sec. II). */
sw_status sw_observables(sw_lattice *h, sw_obs *out, void *stream);

/* Checkpointing: the full state of a lattice is (spins, t); a restart is
 * sw_init with SW_F_KEEP_SPINS over the saved spins plus sw_set_t. */
sw_status sw_get_t(const sw_lattice *h, uint64_t *t);
sw_status sw_set_t(sw_lattice *h, uint64_t t);

/* Free the host handle (device buffers stay with the caller). */
sw_status sw_destroy(sw_lattice *h);

/* ---- Batches: many independent lattices advanced together (the SW update
 * of Sec. II, steps 1-3, on each lattice).  Lattice j evolves exactly as a
 * single lattice created with p[j] and swept as often would: same spins,
 * bonds, labels and counters.  The lattices share one sweep counter t,
 * starting at 0.  Two engines give the same results:
 *   - by default a sweep is one launch per phase (tile, merge, flatten) over
 *     the tiles of every lattice, a lattice smaller than a tile being one
 *     partial tile;
 *   - with SW_F_BATCH_FUSED on p[0] a sweep is one launch of a persistent
 *     kernel over a work queue: lattices of at most 128 x 64 sites (and at
 *     most 15 x the workgroup's threads, 7680 at the default tile) are swept
 *     whole in one workgroup's LDS; the others are tiled, with their merge
 *     waiting for their own tiles and their flatten for their own merge
 *     (per-lattice counters, no grid-wide barrier), so lattices pipeline
 *     inside the launch.  Each of those waits costs an agent-scope release
 *     and acquire, which on a chip of several XCDs write back and invalidate
 *     L2; the per-phase engine, whose phases meet at kernel boundaries, is
 *     the faster one on MI355X.
 * Every lattice of a batch uses p[0]'s tile_h and merge_waves. */
typedef struct swb_batch swb_batch;

/* Workspace bytes of a batch of n >= 1 lattices (0 if a parameter set is
 * invalid, or asks for SW_F_SIZES or the few-cluster update, which batches do
 * not support). */
size_t swb_workspace_bytes(const sw_params *p, int32_t n);

/* Create a batch over n caller-owned lattices: p[j] and b[j] as for sw_init
 * (b[j].workspace is ignored; b[j].roots and .sizes must be NULL); one
 * 256-byte aligned workspace of swb_workspace_bytes() bytes serves the whole
 * batch.  Draws the initial spins of every lattice without SW_F_KEEP_SPINS.
 * The arrays p and b are copied.  Errors as for sw_init; SW_ERR_UNSUPPORTED
 * for SW_F_SIZES and for few_b != 0. */
sw_status swb_init(swb_batch **out, const sw_params *p, const sw_buffers *b, int32_t n, void *workspace,
                   size_t workspace_bytes, void *stream);

/* Enqueue n_sweeps sweeps of every lattice (asynchronous).  The kernels read
 * the sweep index t from a counter in the workspace, which each sweep
 * advances on the device. */
sw_status swb_sweep(swb_batch *h, int32_t n_sweeps, void *stream);

/* As swb_sweep, but the sweeps are replays of HIP graphs holding the sweeps'
 * kernels (Sec. II steps 1-3 for every lattice of the batch): one graph of
 * eight sweeps, launched once per eight, and one of a single sweep for the
 * rest, each captured on first use on a stream of the library's own; the same
 * trajectory as swb_sweep, and the two may be mixed.  The graph holds
 * no memset nodes.  Errors: SW_ERR_ARG, SW_ERR_STATE (t would pass 2^32 - 1),
 * SW_ERR_DEVICE if capture, instantiation or launch fails (sw_last_error()
 * says which).  Released by swb_destroy. */
sw_status swb_sweep_graph(swb_batch *h, int32_t n_sweeps, void *stream);

/* Observables of lattice j, 0 <= j < n, as sw_observables (max_cluster is
 * always -1); waits for the stream.  SW_ERR_DEVICE if a fused sweep gave up
 * waiting for a lattice's tiles or merge (a broken invariant: the batch's
 * results are then invalid; this bound keeps the launch from hanging). */
sw_status swb_observables(swb_batch *h, int32_t j, sw_obs *out, void *stream);

/* Sweeps done so far; free the host handle. */
sw_status swb_get_t(const swb_batch *h, uint64_t *t);
sw_status swb_destroy(swb_batch *h);

/* Workspace bytes needed by ccl_label for this shape (0 if invalid). */
size_t ccl_workspace_bytes(int32_t W, int32_t H, int32_t mode);

/* As ccl_workspace_bytes, for ccl_label_tiled with tile height tile_h (16,
 * 32, 64, 128, or 0 for the default 64; 0 bytes if invalid). */
size_t ccl_workspace_bytes_tiled(int32_t W, int32_t H, int32_t mode, int32_t tile_h);

/* Connected-component labeling of a bond or site input (steps 2 of the SW
 * update on a given graph; Sec. II.B-II.C solve the same problem).
 *   in          device, N bytes (packed bonds or image, see CCL_*)
 *   labels      device, N int32: canonical labels (min index; -1 background).
 *               Must not alias in.
 *   roots,sizes device, N int32 each, or both NULL: roots in ascending order
 *               and the size of each root's cluster, in the first n entries
 *   n_clusters  device, 1 int32, or NULL: number of clusters n
 * W, H >= 1, W*H < 2^31. */
sw_status ccl_label(const uint8_t *in, int32_t W, int32_t H, int32_t mode, int32_t *labels,
                    int32_t *roots, int32_t *sizes, int32_t *n_clusters, void *workspace,
                    size_t workspace_bytes, void *stream);

/* ccl_label with the tile shape and merge schedule chosen by the caller (an
 * autotuner): tile_h and merge_waves as in sw_params (0: defaults).  The
 * local/global split's tile size trades local work against consolidation
 * work (Sec. II.E, Eqs. optimaltile1-2); the labels do not depend on it.
 * The workspace must hold ccl_workspace_bytes_tiled(W, H, mode, tile_h)
 * bytes.  SW_ERR_ARG for an invalid tile_h or merge_waves, otherwise as
 * ccl_label. */
sw_status ccl_label_tiled(const uint8_t *in, int32_t W, int32_t H, int32_t mode, int32_t tile_h,
                          int32_t merge_waves, int32_t *labels, int32_t *roots, int32_t *sizes,
                          int32_t *n_clusters, void *workspace, size_t workspace_bytes, void *stream);

/* ccl_label without a workspace argument and without any allocation, for
 * callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc).  Its scratch is one
 * static device array of CCL_NOALLOC_SCRATCH_BYTES per GPU, held by the loaded
 * library until the process ends, at an address looked up once per device on
 * that device's first call.  Arguments, outputs and results as ccl_label; the
 * stream must belong to the current device.
 * Limit: a shape whose ccl_workspace_bytes(W, H, mode) (with sizes when roots
 * are requested) exceeds CCL_NOALLOC_SCRATCH_BYTES is refused with
 * SW_ERR_WORKSPACE before anything is enqueued (sw_last_error() gives both
 * sizes); 64 MiB holds an image of 2048 x 2048 with sizes.
 * Every call on one GPU uses the same scratch: calls that overlap on one GPU
 * (different streams, or host threads, without ordering) race and give wrong
 * results; calls on one stream are ordered and safe.  No part of the scratch
 * needs to start at zero.  SW_ERR_DEVICE if the address lookup fails. */
#define CCL_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
sw_status ccl_label_noalloc(const uint8_t *in, int32_t W, int32_t H, int32_t mode, int32_t *labels,
                            int32_t *roots, int32_t *sizes, int32_t *n_clusters, void *stream);

/* ---- Served labeling: requests labeled as they arrive (ccl_label on each),
 * over one caller-owned device arena.  The workload is the image-segmentation
 * use of connected-component labeling that motivates the paper (Sec. I): each
 * request is a binary image (or bond array) whose clusters are identified as
 * in SW step 2 (Sec. II.B-II.C).  An admitted request takes one arena
 * block of ccl_server_footprint() bytes (its input, labels, optional roots
 * and sizes, and labeling workspace), so the number in flight is bounded by
 * memory, not by a fixed slot size; a request that does not fit is refused
 * with SW_ERR_STATE and waits in the caller's queue until blocks are
 * released.  Requests go round-robin to the caller's streams, so copies and
 * labeling of different requests overlap.
 * Continuous batching: a request of at most batch_px pixels (and at most 128
 * tiles of 128 x 64) joins an open batch instead of being labeled at once;
 * ccl_server_flush, or the next ccl_server_poll or release of one of its
 * requests, labels the batch with one launch per phase for all its requests
 * (up to 256 requests and 8192 tiles; a fuller batch is flushed when the next
 * request arrives), so small images share the fixed cost of a launch
 * sequence.  Each request's results are those of ccl_label on it alone.
 * New work goes to an idle stream when there is one (a single request never
 * to the open batch's stream).  A batched image in pinned memory is pulled
 * by a kernel rather than by the copy engines, so it does not queue behind
 * the large copies of other requests.
 * With batching, the front of the arena holds four batch tables per stream,
 * and the server keeps their host copies in pinned host memory (its only
 * allocation besides small host objects).  The server allocates no device
 * memory and is driven from one host thread. */
typedef struct ccl_server ccl_server;
typedef struct ccl_server_params {
    int32_t mode;          /* CCL_* input kind of every request               */
    int32_t sizes;         /* 1: also roots and sizes per request, 0: labels  */
    int32_t max_inflight;  /* requests admitted at once, 1..4096              */
    int32_t n_streams;     /* streams passed to ccl_server_create, 1..64      */
    int32_t batch_px;      /* batch requests of at most this many pixels; 0:
                              label every request on its own at admission   */
} ccl_server_params;

/* Arena bytes one W x H request takes (0 if the shape or p is invalid). */
size_t ccl_server_footprint(int32_t W, int32_t H, const ccl_server_params *p);

/* Create a server over arena (device, 256-byte aligned, arena_bytes) and
 * p->n_streams caller streams (hipStream_t as void*). */
sw_status ccl_server_create(ccl_server **out, const ccl_server_params *p, void *arena, size_t arena_bytes,
                            void *const *streams);

/* Admit one request: copy the W x H image (host memory, row pitch in bytes;
 * pinned memory lets the copy run asynchronously; it must stay unchanged
 * until the request completes) to the arena and enqueue its labeling.
 * *slot identifies the request until it is released.  SW_ERR_STATE: no
 * arena block or request slot is free now (nothing enqueued); SW_ERR_SIZE:
 * the request can never fit or its shape is invalid. */
sw_status ccl_server_submit(ccl_server *s, const uint8_t *image, int32_t W, int32_t H, size_t pitch, uint64_t tag,
                            int32_t *slot);

/* Label the open batch now (asynchronous; no-op without one). */
sw_status ccl_server_flush(ccl_server *s);

/* Completed requests not reported before (non-blocking; flushes the open
 * batch first): up to max pairs
 * (slot, tag) and their number *n.  On SW_ERR_DEVICE *n still counts the
 * pairs written before the request whose event query failed. */
sw_status ccl_server_poll(ccl_server *s, int32_t *slots, uint64_t *tags, int32_t max, int32_t *n);

/* Device pointers of a request's outputs (as ccl_label writes them): labels
 * (W x H), roots and sizes (NULL without sizes) and the cluster count.  Valid
 * until the request is released. */
sw_status ccl_server_result(ccl_server *s, int32_t slot, int32_t **labels, int32_t **roots, int32_t **sizes,
                            int32_t **n_clusters);

/* Return a request's arena block (waits for the request if it still runs). */
sw_status ccl_server_release(ccl_server *s, int32_t slot);

/* Wait for requests still running and free the host object. */
sw_status ccl_server_destroy(ccl_server *s);

/* ---- Simple cubic lattices: the SW sweep in three dimensions.
 *
 * The same three steps (Sec. II) on the periodic Lx x Ly x Lz simple cubic
 * lattice, the generalisation to three dimensions that Sec. II names: six
 * neighbours per site, -H/J = number of satisfied bonds among the 3N
 * nearest-neighbour pairs (Eq. potts_hamiltonian).
 *
 * Conventions (bit-exact, shared by definition with the oracle):
 *   - site index i = (z*Ly + y)*Lx + x (x fastest), N = Lx*Ly*Lz < 2^31.
 *   - site i owns the +x bond to (x+1 mod Lx, y, z), the +y bond to
 *     (x, y+1 mod Ly, z) and the +z bond to (x, y, z+1 mod Lz).  Packed bond
 *     byte: bit0 = +x, bit1 = +y, bit2 = +z.
 *   - the +x and +y words are the square lattice's right and down words at
 *     the same index (block(i>>1, t, tag 1), words 2(i&1) and 2(i&1)+1); the
 *     +z word is word i&3 of block(i>>2, t, tag 5).  Initial states (tag 0),
 *     the activation rule r < T, the canonical (minimum-index) labels and the
 *     per-cluster draw (tag 2) are the square lattice's.  With Lz = 1 the +z
 *     bond joins a site to itself and the sweep follows the Lx x Ly
 *     square-lattice trajectory exactly.
 *
 * The library labels on tiles of 32 x 16 x 16 sites (bonds fused with a
 * union-find in LDS; the clusters touching a tile face get compact ids),
 * merges the ids over the bonds that cross tile faces, then resolves every
 * id, draws one state per cluster and writes the spins (Sec. II.B-II.D). */
typedef struct sw3_params {
    int32_t Lx, Ly, Lz;  /* extents, each >= 1, Lx*Ly*Lz < 2^31           */
    int32_t q;           /* Potts states, 2..255 (2 for Ising)             */
    int32_t spin_kind;   /* SW_SPIN_ISING_I8 (q = 2) or SW_SPIN_POTTS_U8   */
    uint32_t flags;      /* 0 (no flags are defined)                       */
    double K;            /* FK coupling: p = 1 - exp(-K), as sw_params.K   */
    uint64_t seed;       /* Philox key                                     */
    uint32_t stream_id;  /* fourth counter word                            */
    int32_t reserved;    /* 0                                              */
} sw3_params;

/* One per-sweep record of sw3_sweep: int64 fields. */
enum { SW3_REC_ACTIVE = 0, SW3_REC_NCLUST = 1, SW3_REC_NSAT = 2, SW3_REC_COUNTS = 3, SW3_REC_LEN = 11 };

/* Workspace bytes sw3_sweep needs for these parameters (0 if they are
 * invalid).  About 2 bytes per site of codes, 1 of bonds and 8 per tile
 * boundary site of ids. */
size_t sw3_workspace_bytes(const sw3_params *p);

/* Initial states of the N sites (device, N bytes, stored as spin_kind says):
 * the square lattice's init draws at the same site index (Sec. II step 3
 * applied to a random start).  Errors: SW_ERR_ARG (null spins, bad
 * parameters), SW_ERR_SIZE (extents). */
sw_status sw3_init_spins(const sw3_params *p, uint8_t *spins, void *stream);

/* n >= 0 SW sweeps t0 .. t0+n-1 of the cubic lattice, in place on `spins`
 * (device, N bytes, stored as spin_kind says).  Optional device outputs
 * (NULL to skip): `bonds` (N bytes) receives the packed bonds and `labels`
 * (N int32) the canonical labels of the last sweep (both of its spins before
 * the flip); `records` (n x SW3_REC_LEN int64) one record per sweep: active
 * bonds, clusters, then satisfied bonds and state counts 0..7 of the spins
 * after the flip.  `workspace` (device, 256-byte aligned, at least
 * sw3_workspace_bytes) is scratch; its contents need not be kept between
 * calls.  Errors: SW_ERR_ARG, SW_ERR_SIZE, SW_ERR_WORKSPACE, SW_ERR_STATE
 * (t0 + n passes 2^32), SW_ERR_DEVICE. */
sw_status sw3_sweep(const sw3_params *p, uint8_t *spins, uint32_t t0, int32_t n, uint8_t *bonds, int32_t *labels,
                    int64_t *records, void *workspace, size_t workspace_bytes, void *stream);

/* Workspace bytes ccl3_label needs for an Lx x Ly x Lz lattice (0 if the
 * shape is invalid). */
size_t ccl3_workspace_bytes(int32_t Lx, int32_t Ly, int32_t Lz);

/* Connected-component labeling of given bonds on the periodic simple cubic
 * lattice: the cluster identification of the SW update (Sec. II.B-II.C,
 * three dimensions), e.g. for bond percolation.  `bonds` (device, N bytes):
 * bit0 +x, bit1 +y, bit2 +z of each site as for sw3_sweep, wrapping along all
 * three axes; higher bits are ignored.  `labels` (device, N int32) receives
 * the canonical labels (each site's cluster's minimum site index);
 * `n_clusters` (device, one int32, or NULL) the number of clusters.
 * `workspace` (device, 256-byte aligned, at least ccl3_workspace_bytes) is
 * scratch.  Errors: SW_ERR_ARG (null bonds or labels), SW_ERR_SIZE,
 * SW_ERR_WORKSPACE, SW_ERR_DEVICE. */
sw_status ccl3_label(const uint8_t *bonds, int32_t Lx, int32_t Ly, int32_t Lz, int32_t *labels, int32_t *n_clusters,
                     void *workspace, size_t workspace_bytes, void *stream);

#ifdef __cplusplus
}
#endif
#endif
