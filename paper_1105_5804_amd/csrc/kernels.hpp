// kernels.hpp -- gfx950 kernels of one Swendsen-Wang sweep and of connected-
// component labeling on a 2D square lattice.
//
// A sweep is three launches (Sec. II: T_SW = T_activate + T_identify + T_flip,
// with T_identify = T_local + T_global):
//
//   k_tile    one workgroup per 128x64 tile.  Bond activation (Sec. II.A) fused
//             with tile labeling (Sec. II.B): each lane of a 64-lane wave owns
//             two sites of a tile row; the row's bonds become 128-bit masks by
//             wave ballots, right bonds turn into row runs (each site's run
//             start from a DPP max-scan over the lanes), and down bonds join
//             runs by a lock-free union-find over run starts in LDS, fed from
//             compacted per-wave lists of vertical contacts.
//             Clusters that touch the tile border are claimed by their border
//             sites and get a compact boundary id; every site's result is a
//             16-bit code (boundary id, or CAP + the slot of its interior root).
//   k_merge   tile consolidation (Sec. II.C) in one pass: every active bond
//             that crosses a tile edge, the periodic wrap included, unites two
//             boundary ids in a global union-find over the compact id space
//             (CAS linking of the larger-key root under the smaller one).  Only
//             ~2(TW+TH) ids per tile exist, so this structure stays small and
//             cache resident.
//   k_flatten resolves every boundary id to its root, whose key is the
//             cluster's minimum site index (the canonical label), draws one new
//             state per cluster from that root (Sec. II.D) and writes spins
//             and, optionally, labels.
//
// Labeling-only inputs (packed bond bytes or binary images) reuse the same
// three kernels with a different bond source.  The few-cluster update
// (Sec. III) labels with the same tile and merge launches, marks the clusters
// that hold a seed in k_seed and flips only those in k_flatten<M_FEW>.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "philox.hpp"
#include "uf.hpp"

namespace swccl {

constexpr int TW = 128;               // tile width: a wave covers a tile row, 2 sites per lane
constexpr int RPW = 8;                // tile rows per wave
constexpr int WLIST = RPW * TW;       // per-wave work list capacity (one entry per site at most)
constexpr int TLIST = 3 * TW;         // k_tile's per-wave lists: a row adds at most TW entries, a
                                      // fuller list is worked off first (keeps the LDS per wave small)
constexpr uint16_t ID_NONE = 0xFFFF;
constexpr uint16_t CODE_BG = 0xFFFF;

// Tile shapes: TW x TH sites, one wave per RPW rows, so a tile is worked by
// TH / RPW waves.  Per tile there are CAP boundary ids (at least the border
// sites), EDGE edge entries (top row, bottom row, left column, right column)
// and XW words of crossing bits (the right edge's rows, XR words of 64, then
// the bottom edge's even and odd columns).
template <int TH_>
struct Tile {
    static constexpr int TH = TH_;
    static constexpr int TSITES = TW * TH;
    static constexpr int CAP = 2 * (TW + TH);
    static constexpr int EDGE = 2 * TW + 2 * TH;
    static constexpr int XR = (TH + 63) / 64;
    static constexpr int XW = XR + 2;
    static constexpr int NWAVE = TH / RPW;
    static constexpr int NT = 64 * NWAVE;
    static_assert(TH % RPW == 0 && TH >= 2 * RPW && TH <= 128, "tile heights 16, 32, 64, 128");
    static_assert(CAP + TSITES < 0xFFFE, "codes are 16-bit");
};
constexpr int TH_DEFAULT = 64;        // the shape the library uses unless told otherwise

// Kernels that do not depend on the tile shape run 512-thread workgroups.
constexpr int NT = 512;
constexpr int NWAVE = NT / 64;

// The one-tile lattices that k_small sweeps whole in LDS: W <= 128, H <= 64.
constexpr int SMALL_W = 128, SMALL_H = 64, SMALL_SITES = SMALL_W * SMALL_H;

enum : uint32_t { TAG_INIT = 0, TAG_BOND = 1, TAG_FLIP = 2, TAG_SEED = 3, TAG_FEW = 4 };
// M_FEW is a flatten mode only: the few-cluster update labels with M_SW's
// tile and merge kernels and flips in k_flatten<M_FEW>.
enum Mode : int { M_SW = 0, M_BONDS_PERIODIC = 1, M_BONDS_OPEN = 2, M_SITES = 3, M_FEW = 4 };

// Observable counters (unsigned 64-bit, two's complement for signed values).
enum { ST_ACTIVE = 0, ST_NCLUST = 1, ST_NSAT = 2, ST_MAGNET = 3, ST_COUNTS = 4, ST_DIGEST = 12, ST_LEN = 16 };

struct Grid {
    int W, H, ntx, nty, ntiles;
    int rev;  // visit the tiles in reverse order (single lattices only; a schedule check)
};

// One lattice of a batched launch (many independent lattices swept by one
// launch per phase): its shape, buffers and random-number parameters, and the
// first of its tiles in the batch's tile arrays.
struct LatticeDesc {
    Grid g;
    int32_t tile0;
    uint8_t *spins;
    uint8_t *bonds;    // packed bonds of the sweep, or nullptr
    int32_t *labels;   // canonical labels, or nullptr
    uint32_t tm1, tany, k0, k1, sid, q;
    int32_t ising;
    int32_t nmerge;    // fused sweeps: merge groups of the lattice (0 if swept whole in LDS)
};

// How a batched launch finds the lattice of a tile.  Tile-indexed arrays
// (codes, ids, edges, ...) are concatenated over the batch and indexed by the
// batch tile; geometry uses the tile's index inside its lattice.
struct Batch {
    const LatticeDesc *lat;
    const int32_t *lat_of_tile;  // batch tile -> lattice
    const uint32_t *t;           // the batch's sweep counter, read on the device (graph replays)
    int32_t tile_base, ntiles;   // this launch covers tiles [tile_base, tile_base + ntiles)
};

// Shared device helpers (XCD placement, lane masks, union-find in LDS and
// over global ids, wave reductions) are in uf.hpp.

// ----------------------------------------------------------------- init ----

// Initial states: state_i = (w q) >> 32 with w = Philox(i>>2, 0, INIT, sid)[i&3].
__global__ __launch_bounds__(NT) void k_init(uint8_t *spins, int64_t N, uint32_t q, int ising,
                                             uint32_t k0, uint32_t k1, uint32_t sid)
{
    const int64_t w = static_cast<int64_t>(blockIdx.x) * NT + threadIdx.x;
    const int64_t base = w * 4;
    if (base >= N) return;
    const U4 b = philox4x32_10(static_cast<uint32_t>(w), 0u, TAG_INIT, sid, k0, k1);
    const uint32_t words[4] = {b.v0, b.v1, b.v2, b.v3};
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        if (base + j < N) {
            const uint32_t st = draw_state(words[j], q);
            spins[base + j] = ising ? static_cast<uint8_t>(2 * st - 1) : static_cast<uint8_t>(st);
        }
    }
}

__global__ void k_zero_u64(unsigned long long *p, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

__global__ void k_zero_i32(int32_t *p, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

// Copy n bytes from host memory the device can read (pinned) into device
// memory, in the compute queue: a small request's image and a batch's table
// then never wait behind large copies queued on the copy engines.  4 bytes a
// thread (byte loads: the source need not be aligned).
__global__ __launch_bounds__(NT) void k_pull(uint8_t *dst, const uint8_t *src, int64_t n)
{
    const int64_t i = (static_cast<int64_t>(blockIdx.x) * NT + threadIdx.x) * 4;
#pragma unroll
    for (int j = 0; j < 4; ++j)
        if (i + j < n) dst[i + j] = src[i + j];
}

__global__ void k_iota_i32(int32_t *p, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = i;
}

// Advance a device-side sweep counter (the last launch of a batched sweep).
__global__ void k_bump_u32(uint32_t *p)
{
    if (threadIdx.x == 0) p[0] += 1u;
}

// ----------------------------------------------------------------- tile ----

struct TileArgs {
    Grid g;
    const uint8_t *in;        // spins (M_SW), packed bonds or image bytes
    uint8_t *bonds_out;       // M_SW: packed bonds of this sweep, or nullptr
    uint16_t *codes;          // [ntiles][TSITES]
    int32_t *gkey;            // [ntiles][CAP]
    int32_t *gparent;         // [ntiles][CAP]
    int32_t *gsize;           // [ntiles][CAP] or nullptr (zeroed here when given)
    uint16_t *edges;          // [ntiles][EDGE]
    uint64_t *xbits;          // [ntiles][XW]
    int32_t *nb;              // [ntiles]
    int32_t *tile_act;        // [ntiles]: active bonds owned by the tile (M_SW)
    uint32_t tm1;             // M_SW: a bond is active iff its word r <= tm1 ...
    uint32_t tany;            // ... and tany (threshold T > 0); tm1 = T - 1
    uint32_t k0, k1, t, sid;
    Batch b;                  // batched launches only
    uint32_t rk[20];          // single-lattice sweeps: the Philox key schedule of (k0, k1), round r in
                              // rk[2r], rk[2r + 1]
};

// A tile row as two wave ballots: lane L owns sites 2L and 2L+1, bit L of `e`
// belongs to site 2L and bit L of `o` to site 2L+1.  The masks stay in scalar
// registers; the natural-order shift s -> s+1 is (o << 1, e).
struct EO {
    uint64_t e, o;
};

__device__ __forceinline__ EO eo_and(EO a, EO b) { return EO{a.e & b.e, a.o & b.o}; }
__device__ __forceinline__ EO eo_andnot(EO a, EO b) { return EO{a.e & ~b.e, a.o & ~b.o}; }
__device__ __forceinline__ EO eo_shift1(EO m) { return EO{m.o << 1, m.e}; }

// Set bits of m at lanes below the calling lane.
__device__ __forceinline__ int lanes_below(uint64_t m)
{
    return static_cast<int>(__builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(m >> 32),
                                                      __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(m), 0u)));
}

// Append the sites set in m (row starting at slot `base`) to a wave list in
// ascending order, as slot << SH; n is the wave-uniform list length.
template <int SH = 0>
__device__ __forceinline__ void eo_append(uint16_t *list, int &n, EO m, int lane, int base)
{
    const int r0 = n + lanes_below(m.e) + lanes_below(m.o);
    const int b0 = lane_bit(m.e, lane) ? 1 : 0;
    if (b0) list[r0] = static_cast<uint16_t>((base + 2 * lane) << SH);
    if (lane_bit(m.o, lane)) list[r0 + b0] = static_cast<uint16_t>((base + 2 * lane + 1) << SH);
    n += __popcll(m.e) + __popcll(m.o);
}

// Wave-uniform copy of a mask read from LDS.
__device__ __forceinline__ uint64_t uniform64(uint64_t v)
{
    const uint32_t lo = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(v));
    const uint32_t hi = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(v >> 32));
    return (static_cast<uint64_t>(hi) << 32) | lo;
}
__device__ __forceinline__ EO uniform_eo(EO m) { return EO{uniform64(m.e), uniform64(m.o)}; }
// A pointer the caller knows to be wave-uniform, as a scalar value.
template <typename T>
__device__ __forceinline__ T *uniform_ptr(T *p)
{
    return reinterpret_cast<T *>(static_cast<uintptr_t>(uniform64(static_cast<uint64_t>(reinterpret_cast<uintptr_t>(p)))));
}

// Root of x (a byte offset, as the tile kernel's parents) once all unions are
// done; a claimed root (negative entry) is a root.
__device__ __forceinline__ int lroot(int *P, int x)
{
    for (;;) {
        const int p = lds_ld(lds_entry<true>(P, x));
        if (p == x || p < 0) return x;
        x = p;
    }
}

// Border position t of a tile in the layout of the edge arrays: top row,
// bottom row, left column, right column.  Returns the slot, or -1 if the
// position lies outside a ragged tile.
template <int TH>
__device__ __forceinline__ int border_slot(int t, int tw, int th)
{
    if (t < TW) return t < tw ? t : -1;
    if (t < 2 * TW) return (t - TW) < tw ? (th - 1) * TW + (t - TW) : -1;
    if (t < 2 * TW + TH) return (t - 2 * TW) < th ? (t - 2 * TW) * TW : -1;
    return (t - 2 * TW - TH) < th ? (t - 2 * TW - TH) * TW + tw - 1 : -1;
}

// Claimed roots: P[root] = CLAIMING while the id is allocated, then
// -(k + 2) for boundary id k.
constexpr int CLAIMING = -1;

// Lane masks: bit L describes lane L (uicmp yields the mask of one compare).
constexpr int CMP_EQ = 32, CMP_NE = 33, CMP_ULT = 36, CMP_ULE = 37;
__device__ __forceinline__ uint64_t lanes_eq(uint32_t x, uint32_t y) { return __builtin_amdgcn_uicmp(x, y, CMP_EQ); }
__device__ __forceinline__ uint64_t lanes_ne(uint32_t x, uint32_t y) { return __builtin_amdgcn_uicmp(x, y, CMP_NE); }
__device__ __forceinline__ uint64_t lanes_lt(uint32_t x, uint32_t y) { return __builtin_amdgcn_uicmp(x, y, CMP_ULT); }
__device__ __forceinline__ uint64_t lanes_le(uint32_t x, uint32_t y) { return __builtin_amdgcn_uicmp(x, y, CMP_ULE); }

// Maximum of v over the lanes below the calling one (0 for lane 0), v >= 0:
// an inclusive max-scan by row shifts and row broadcasts, then a shift by one
// lane.  Out-of-row sources read 0, the identity; rows outside a broadcast's
// row mask keep their value.
__device__ __forceinline__ int wave_max_below(int v)
{
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x111, 0xF, 0xF, false));  // row_shr:1
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x112, 0xF, 0xF, false));  // row_shr:2
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x114, 0xF, 0xF, false));  // row_shr:4
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x118, 0xF, 0xF, false));  // row_shr:8
    // The row broadcasts write only the rows in their masks (1 and 3, then 2
    // and 3) and leave the others as they are: with the destination as the
    // second source that is one max per step (the compiler emits a copy, a
    // broadcast and a max).  s_nop 1 gives each DPP read of a just-written
    // register its two wait states.
    int out;
    asm("s_nop 1\n\t"
        "v_max_i32_dpp %0, %0, %0 row_bcast:15 row_mask:0xa bank_mask:0xf\n\t"
        "s_nop 1\n\t"
        "v_max_i32_dpp %0, %0, %0 row_bcast:31 row_mask:0xc bank_mask:0xf\n\t"
        "s_nop 1\n\t"
        "v_mov_b32_dpp %1, %0 wave_shr:1 row_mask:0xf bank_mask:0xf bound_ctrl:1"  // lane 0 reads 0
        : "+v"(v), "=v"(out));
    return out;
}

// LDS of the tile phase.  The image mode's extra occupancy masks are paid
// for by slightly shorter lists, so every mode stays under 40 KB per 64 rows.
template <int MODE, int TH_>
struct TileSmem {
    static constexpr int TH = TH_, TSITES = TW * TH, NWAVE = TH / RPW;
    static constexpr int TL = MODE == M_SITES ? (TH < 64 ? TLIST - 16 : TLIST - 8) : TLIST;
    int P[TSITES];                     // union-find parent per site slot, as 4 x slot
    EO Rm[TH];                         // in-tile right bonds per row
    EO Om[MODE == M_SITES ? TH : 1];   // occupied sites per row (images)
    uint16_t wl[NWAVE][TL];            // per-wave work list (contacts, then run starts)
    unsigned long long xr_w[NWAVE];    // right crossing bonds of each wave's rows (bit ly % 64)
    EO xd_s;                           // bottom crossing bonds
    int nb_s;
    int act_w[NWAVE];
};

// A batched launch's tile: take the lattice's shape, buffers and keys from
// its descriptor; lt is the tile's index inside its lattice.
__device__ __forceinline__ void load_batch_tile(TileArgs &a, int tile, int &lt)
{
    const LatticeDesc &L = a.b.lat[a.b.lat_of_tile[tile]];
    a.g = L.g;
    a.in = L.spins;
    a.bonds_out = L.bonds;
    a.tm1 = L.tm1;
    a.tany = L.tany;
    a.k0 = L.k0;
    a.k1 = L.k1;
    a.sid = L.sid;
    a.t = *a.b.t;
    lt = tile - L.tile0;
}

// The kernel's own TileArgs in the kernel-argument segment, behind an opaque
// copy of the segment pointer: a field read through it is a scalar load at
// that point, so output pointers used only at the end of the tile phase are
// not held in scalar registers across it (which would spill some).
typedef const __attribute__((address_space(4))) TileArgs KernTileArgs;
__device__ __forceinline__ KernTileArgs *kernel_tile_args()
{
    KernTileArgs *k = (KernTileArgs *)__builtin_amdgcn_kernarg_segment_ptr();
    asm volatile("" : "+s"(k));
    return k;
}

// The tile phase of one tile: `tile` indexes the tile arrays, `lt` is the
// tile inside its lattice (they differ in batches).  Uses every thread of a
// Tile<TH>::NT-thread workgroup; ends with the workgroup's writes issued.
// With KARG the launch's only argument is the TileArgs `a` came from, and the
// output pointers are re-read from it where they are used; with RKEYS (a
// single-lattice sweep) so is the bond generator's key schedule, row by row
// (scalar loads in place of 18 scalar adds per row).
template <int MODE, bool EVENW, int TH_, bool KARG = false, bool RKEYS = false>
__device__ __forceinline__ void tile_body(TileArgs a, const int tile, const int lt, TileSmem<MODE, TH_> &sm)
{
    using S = Tile<TH_>;
    constexpr int TH = S::TH, TSITES = S::TSITES, CAP = S::CAP, EDGE = S::EDGE, XR = S::XR, XW = S::XW;
    constexpr int NT = S::NT, NWAVE = S::NWAVE;
    constexpr bool NEED_DOWN = MODE == M_SW || MODE == M_SITES;  // bonds from two rows
    constexpr bool NEED_HALO = MODE == M_SW || MODE == M_SITES;  // column right of the tile
    constexpr int TL = TileSmem<MODE, TH_>::TL;
    int *P = sm.P;
    EO *Rm = sm.Rm;
    EO *Om = sm.Om;
    auto &wl = sm.wl;
    unsigned long long *xr_w = sm.xr_w;
    EO &xd_s = sm.xd_s;
    int &nb_s = sm.nb_s;
    int *act_w = sm.act_w;
    const int W = a.g.W, H = a.g.H;
    const int tx = lt % a.g.ntx, ty = lt / a.g.ntx;
    const int gx0 = tx * TW, gy0 = ty * TH;
    const int tw = min(TW, W - gx0), th = min(TH, H - gy0);
    const int lane = threadIdx.x & 63, wave = wave_id();
    const int lx0 = 2 * lane, lx1 = lx0 + 1, x4 = 4 * lx0;
    const bool v0 = lx0 < tw, v1 = lx1 < tw;
    const int hx = (gx0 + tw == W) ? 0 : gx0 + tw;  // column right of the tile
    const bool right_is_wrap = (gx0 + tw == W);
    const bool bottom_is_wrap = (gy0 + th == H);
    const int ly0 = wave * RPW;
    const int nr = max(0, min(RPW, th - ly0));  // tile rows owned by this wave
    uint16_t *mylist = wl[wave];
    // Unite the n contacts of the wave's list (contact c joins slots c and
    // c + TW; the list holds their byte offsets).  Lane L takes contacts L, L+64, ...; a lane whose union is done
    // takes its next contact at once, so one deep union does not hold up the
    // other lanes of its round.
    auto unite_list = [&](int n) {
        wave_lds_fence();
        int i = lane, a = 0, b = 0;
        if (i < n) {
            const int c = mylist[i];  // byte offset of the upper site
            a = lds_ld(lds_entry<true>(P, c));
            b = lds_ld(lds_entry<true>(P, c + 4 * TW));
        }
        while (i < n) {
            int done;
            unite_step<true, true>(P, a, b, done);
            if (done) {
                i += 64;
                if (i < n) {
                    const int c = mylist[i];
                    a = lds_ld(lds_entry<true>(P, c));
                    b = lds_ld(lds_entry<true>(P, c + 4 * TW));
                }
            }
        }
        wave_lds_fence();
    };
    // wave-uniform lane masks
    const EO valid = EO{lanes_lt(lx0, tw), lanes_lt(lx1, tw)};

    if (threadIdx.x == 0) nb_s = 0;  // first used after the barrier closing phase A

    // ---- A0: issue every load of the wave's rows (and the row below) up front,
    // branch-free within the wave: invalid lanes read a clamped valid address.
    // pr[r] holds the bytes of sites lx0 (bits 0-7) and lx1 (bits 8-15).
    const int col = gx0 + (v0 ? lx0 : 0);
    uint32_t pr[RPW + 1];
    uint32_t hl[RPW];
#pragma unroll
    for (int r = 0; r <= RPW; ++r) {
        pr[r] = 0;
        if (r < RPW) hl[r] = 0;
        if (nr > 0 && (r < nr || (NEED_DOWN && r == nr))) {
            int gy = gy0 + ly0 + r;
            if (gy == H) gy = 0;  // ly0 + r <= th, so at most one wrap
            const uint8_t *row = a.in + static_cast<int64_t>(gy) * W;
            if constexpr (EVENW) {
                pr[r] = *reinterpret_cast<const uint16_t *>(row + col);
            } else {
                pr[r] = static_cast<uint32_t>(row[col]) | (static_cast<uint32_t>(row[col + (v1 ? 1 : 0)]) << 8);
            }
            if (NEED_HALO && r < nr) hl[r] = row[hx];  // same byte for every lane
        }
    }

    // ---- A1: bonds as lane masks, row masks, run-start parents, and the
    // vertical contacts of the previous row pair.  Site s repeats the contact
    // of s-1 when s-1 has a down bond and both rows continue from s-1 to s:
    // one union per contact segment suffices.
    unsigned long long xr = 0;
    int nact = 0;  // at most 2 * TSITES
    int ncon = 0;
    EO prevR = EO{0ull, 0ull}, prevD = EO{0ull, 0ull};
#pragma unroll
    for (int r = 0; r < RPW; ++r) {
        if (r >= nr) break;
        const int ly = ly0 + r;
        const int gy = gy0 + ly;
        const uint32_t cur = pr[r], dn = pr[r + 1];
        // lane masks are recomputed per row (one compare each) instead of
        // being held in scalar registers across the unrolled rows, where
        // they would spill
        uint32_t twr = static_cast<uint32_t>(tw);
        int lane_r = lane;
        asm volatile("" : "+s"(twr), "+v"(lane_r));
        const uint64_t V0 = lanes_lt(lx0, twr), V1 = lanes_lt(lx1, twr);
        const uint64_t L0 = lanes_eq(lx0, twr - 1), L1 = lanes_eq(lx1, twr - 1);
        uint64_t mR0, mR1, mD0, mD1, O0 = V0, O1 = V1;

        if constexpr (MODE == M_SW) {
            const uint32_t s0 = cur & 0xFFu, s1 = (cur >> 8) & 0xFFu;
            const uint32_t d0 = dn & 0xFFu, d1 = (dn >> 8) & 0xFFu;
            const uint32_t nxt = from_next_lane(s0);
            const uint32_t sr0 = (!EVENW && lx0 == static_cast<int>(twr) - 1) ? hl[r] : s1;
            const uint32_t sr1 = (lx1 == static_cast<int>(twr) - 1) ? hl[r] : nxt;
            const int64_t i0 = static_cast<int64_t>(gy) * W + gx0 + lx0;
            uint32_t r0R, r0D, r1R, r1D;
            // the key schedule is recomputed per row (scalar adds) rather than
            // held in 20 scalar registers across the unrolled row loop
            uint32_t k0 = __builtin_amdgcn_readfirstlane(a.k0), k1 = __builtin_amdgcn_readfirstlane(a.k1);
            asm volatile("" : "+s"(k0), "+s"(k1));
            U4 blk;
            if constexpr (RKEYS) {
                blk = philox4x32_10_rk(static_cast<uint32_t>(i0 >> 1), a.t, TAG_BOND, a.sid, kernel_tile_args()->rk);
            } else {
                blk = philox4x32_10(static_cast<uint32_t>(i0 >> 1), a.t, TAG_BOND, a.sid, k0, k1);
            }
            if (EVENW || (i0 & 1) == 0) {  // the pair (i0, i0+1) shares one block
                r0R = blk.v0;
                r0D = blk.v1;
                r1R = blk.v2;
                r1D = blk.v3;
            } else {  // odd row start (odd W): i0 is the second site of its block
                r0R = blk.v2;
                r0D = blk.v3;
                const U4 b2 = philox4x32_10(static_cast<uint32_t>((i0 + 1) >> 1), a.t, TAG_BOND, a.sid,
                                            k0, k1);
                r1R = b2.v0;
                r1D = b2.v1;
            }
            // uniform flags are re-read per row as well (held across rows
            // as lane masks, they too would spill)
            uint32_t tany = __builtin_amdgcn_readfirstlane(a.tany);
            uint8_t *bonds_out = uniform_ptr(a.bonds_out);
            asm volatile("" : "+s"(tany), "+s"(bonds_out));
            const uint64_t on0 = tany ? V0 : 0ull, on1 = tany ? V1 : 0ull;
            mR0 = lanes_eq(s0, sr0) & lanes_le(r0R, a.tm1) & on0;
            mD0 = lanes_eq(s0, d0) & lanes_le(r0D, a.tm1) & on0;
            mR1 = lanes_eq(s1, sr1) & lanes_le(r1R, a.tm1) & on1;
            mD1 = lanes_eq(s1, d1) & lanes_le(r1D, a.tm1) & on1;
            if (bonds_out) {
                const uint32_t b0 = lane_bit(mR0, lane) | (lane_bit(mD0, lane) << 1);
                const uint32_t b1 = lane_bit(mR1, lane) | (lane_bit(mD1, lane) << 1);
                const bool w0 = lx0 < static_cast<int>(twr), w1 = lx1 < static_cast<int>(twr);
                if (w1 && (EVENW || !(i0 & 1))) {
                    *reinterpret_cast<uint16_t *>(bonds_out + i0) = static_cast<uint16_t>(b0 | (b1 << 8));
                } else {
                    if (w0) bonds_out[i0] = static_cast<uint8_t>(b0);
                    if (w1) bonds_out[i0 + 1] = static_cast<uint8_t>(b1);
                }
            }
            nact += __popcll(mR0) + __popcll(mD0) + __popcll(mR1) + __popcll(mD1);  // 32-bit sums
        } else if constexpr (MODE == M_BONDS_PERIODIC || MODE == M_BONDS_OPEN) {
            mR0 = lanes_ne(cur & 0x001u, 0u) & V0;
            mD0 = lanes_ne(cur & 0x002u, 0u) & V0;
            mR1 = lanes_ne(cur & 0x100u, 0u) & V1;
            mD1 = lanes_ne(cur & 0x200u, 0u) & V1;
            if (MODE == M_BONDS_OPEN) {
                if (right_is_wrap) {
                    mR0 &= ~L0;
                    mR1 &= ~L1;
                }
                if (bottom_is_wrap && ly == th - 1) mD0 = mD1 = 0ull;
            }
        } else {  // M_SITES: 4-connected occupied pixels, open boundary
            O0 = lanes_ne(cur & 0x00FFu, 0u) & V0;
            O1 = lanes_ne(cur & 0xFF00u, 0u) & V1;
            const uint64_t below_occ = (gy + 1 < H) ? ~0ull : 0ull;
            const uint64_t Dn0 = lanes_ne(dn & 0x00FFu, 0u) & below_occ;
            const uint64_t Dn1 = lanes_ne(dn & 0xFF00u, 0u) & below_occ;
            const uint64_t Hh = (!right_is_wrap && hl[r] != 0) ? ~0ull : 0ull;  // hl is lane-uniform
            mR0 = O0 & ((O1 & ~L0) | (Hh & L0));
            mR1 = O1 & (((O0 >> 1) & ~L1) | (Hh & L1));
            mD0 = O0 & Dn0;
            mD1 = O1 & Dn1;
        }

        // Crossing bonds leave the tile: the last column's right bond and the
        // last row's down bonds.  They are merged by k_merge.
        if ((mR0 & L0) | (mR1 & L1)) xr |= 1ull << (ly & 63);
        const EO R = EO{mR0 & ~L0, mR1 & ~L1};
        // the last tile row's down bonds cross the tile; selected on a uniform
        // condition so the masks stay in scalar registers
        const bool last = ly == th - 1;
        const EO D = last ? EO{0ull, 0ull} : EO{mD0, mD1};
        if (lane_r == 0) {
            if (last) xd_s = EO{mD0, mD1};
            Rm[ly] = R;
            if constexpr (MODE == M_SITES) Om[ly] = EO{O0, O1};
        }
        const int base = ly * TW;
        // Run starts: site 2L starts a run unless bond 2L-1 -> 2L is present,
        // site 2L+1 unless bond 2L -> 2L+1 is; the run start of 2L is the last
        // start at or before it (a max-scan over the lanes below).
        // Scanned in byte offsets within the row (x4 = 4 lx0); lane 0's even
        // site always starts a run, so every other lane finds a start below.
        const bool e_start = lane_bit(~(R.o << 1), lane);
        const bool o_start = lane_bit(~R.e, lane);
        const int below4 = wave_max_below(o_start ? x4 + 8 : (e_start ? x4 + 4 : 0));
        const int rs0 = e_start ? x4 : below4 - 4;
        const int rs1 = o_start ? x4 + 4 : rs0;
        *reinterpret_cast<int2 *>(&P[base + lx0]) = make_int2(4 * base + rs0, 4 * base + rs1);
        if (r > 0) {
            // contacts between this wave's own rows: a full list is united at
            // once (only rows this wave has initialised are involved)
            if (ncon > TL - TW) {
                unite_list(ncon);
                ncon = 0;
            }
            const EO X = eo_and(eo_and(prevD, prevR), R);
            eo_append<2>(mylist, ncon, eo_andnot(prevD, eo_shift1(X)), lane, base - TW);
        }
        prevR = R;
        prevD = D;
    }
    if (lane == 0) {
        xr_w[wave] = xr;
        act_w[wave] = nact;
    }
    __syncthreads();

    // ---- B: contacts with the next wave's first row, then all unions ----
    if (nr > 0 && ly0 + nr < th) {
        if (ncon > TL - TW) {
            unite_list(ncon);
            ncon = 0;
        }
        const EO Rn = uniform_eo(Rm[ly0 + nr]);
        const EO X = eo_and(eo_and(prevD, prevR), Rn);
        eo_append<2>(mylist, ncon, eo_andnot(prevD, eo_shift1(X)), lane, (ly0 + nr - 1) * TW);
    }
    unite_list(ncon);
    __syncthreads();

    // Occupancy of a tile slot: images keep per-row masks, every site of a
    // bond input is a lattice site.
    auto occupied = [&](int slot) {
        if constexpr (MODE == M_SITES) {
            const EO O = Om[slot >> 7];
            const int x = slot & (TW - 1);
            return (((x & 1) ? O.o : O.e) >> (x >> 1) & 1ull) != 0;
        } else {
            return true;
        }
    };

    // ---- C: the clusters that touch the tile border are claimed (one
    // thread per border position), then, after a barrier, every linked run
    // start gets its cluster's final code, stored in its own entry as
    // -(code + 2): the boundary id of a claimed root, else CAP + the root's
    // slot (a claimed root's entry already reads -(id + 2)).  Lane L walks
    // run starts L, L+64, ... of the wave's list up to the first entry that is
    // negative (a claimed root, or a run start another lane has finished:
    // either way the cluster's code) or its own (an unclaimed root); a lane
    // whose walk is done takes its next run start at once.  Only linked run
    // starts (entry neither their own nor negative) are listed.
    auto compress_list = [&](int n) {
        wave_lds_fence();
        int i = lane, s0 = 0, x = 0;
        if (i < n) s0 = x = mylist[i];
        while (i < n) {
            const int p = lds_ld(lds_entry<true>(P, x));
            if (p >= 0 && p != x) {
                x = p;
            } else {
                lds_st(lds_entry<true>(P, s0), p < 0 ? p : -(CAP + (x >> 2)) - 2);
                i += 64;
                if (i < n) s0 = x = mylist[i];
            }
        }
        wave_lds_fence();
    };
    int32_t *gkey = a.gkey, *gparent = a.gparent, *gsize = a.gsize;
    if constexpr (KARG) {
        KernTileArgs *ka = kernel_tile_args();
        gkey = ka->gkey;
        gparent = ka->gparent;
        gsize = ka->gsize;
    }
    for (int t = threadIdx.x; t < EDGE; t += NT) {
        const int slot = border_slot<TH>(t, tw, th);
        if (slot < 0 || !occupied(slot)) continue;
        const int root4 = lroot(P, 4 * slot), root = root4 >> 2;
        int expect = root4;
        if (__hip_atomic_compare_exchange_strong(lds_entry<true>(P, root4), &expect, CLAIMING, __ATOMIC_RELAXED,
                                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)) {
            const int k = atomicAdd(&nb_s, 1);
            lds_st(lds_entry<true>(P, root4), -(k + 2));
            const int id = tile * CAP + k;
            gkey[id] = (gy0 + (root >> 7)) * W + gx0 + (root & (TW - 1));
            gparent[id] = id;
            if (gsize) gsize[id] = 0;
        }
    }
    __syncthreads();
    int nrs = 0;
    // The entries of the wave's sites are read up front (the loads overlap);
    // a flush of the list only rewrites linked run starts of this wave.
    int2 ppr[RPW];
#pragma unroll
    for (int r = 0; r < RPW; ++r)
        ppr[r] = r < nr ? *reinterpret_cast<const int2 *>(&P[(ly0 + r) * TW + lx0]) : make_int2(0, 0);
#pragma unroll
    for (int r = 0; r < RPW; ++r) {
        if (r >= nr) break;
        const int ly = ly0 + r;
        const int base = ly * TW;
        if (nrs > TL - TW) {
            compress_list(nrs);
            nrs = 0;
        }
        const EO R = uniform_eo(Rm[ly]);
        EO O = valid;
        if constexpr (MODE == M_SITES) O = uniform_eo(Om[ly]);
        const int2 pp = ppr[r];
        const EO linked = EO{lanes_ne(static_cast<uint32_t>(pp.x), static_cast<uint32_t>(4 * (base + lx0))) &
                                 lanes_lt(static_cast<uint32_t>(pp.x), 0x80000000u),
                             lanes_ne(static_cast<uint32_t>(pp.y), static_cast<uint32_t>(4 * (base + lx0 + 1))) &
                                 lanes_lt(static_cast<uint32_t>(pp.y), 0x80000000u)};
        eo_append<2>(mylist, nrs, eo_and(eo_andnot(O, eo_shift1(R)), linked), lane, base);
    }
    compress_list(nrs);
    __syncthreads();

    // ---- E: per-site codes (boundary id of a claimed root, else CAP + the
    // root's slot), edge ids, crossing bits.  A site's code is one step past
    // its entry: a run start holds its code (or, an unclaimed root, its own
    // offset), any other site its run start's offset.
    auto code_of = [&](int x, int p) {  // x a slot, p = P[x] (byte offsets)
        x *= 4;
        if (p >= 0 && p != x) p = *lds_entry<true>(P, p);
        return p < 0 ? static_cast<uint32_t>(-p - 2) : static_cast<uint32_t>(CAP + (p >> 2));
    };
    uint16_t *codes = a.codes, *edges = a.edges;
    uint64_t *xbits = a.xbits;
    int32_t *nbp = a.nb, *tile_act = a.tile_act;
    if constexpr (KARG) {
        KernTileArgs *ka = kernel_tile_args();
        codes = ka->codes;
        edges = ka->edges;
        xbits = ka->xbits;
        nbp = ka->nb;
        tile_act = ka->tile_act;
    }
    uint32_t *codes32 = reinterpret_cast<uint32_t *>(codes + static_cast<int64_t>(tile) * TSITES);
    // unrolled: the rows' lookup chains are independent, so their LDS loads overlap
#pragma unroll
    for (int r = 0; r < RPW; ++r) {
        if (r >= nr) break;
        const int ly = ly0 + r;
        EO O = valid;
        if constexpr (MODE == M_SITES) O = Om[ly];
        const int base = ly * TW;
        const int2 pp = *reinterpret_cast<const int2 *>(&P[base + lx0]);
        const uint32_t code0 = lane_bit(O.e, lane) ? code_of(base + lx0, pp.x) : CODE_BG;
        const uint32_t code1 = lane_bit(O.o, lane) ? code_of(base + lx0 + 1, pp.y) : CODE_BG;
        codes32[(base + lx0) >> 1] = code0 | (code1 << 16);
    }
    uint16_t *edg = edges + static_cast<int64_t>(tile) * EDGE;
    for (int t = threadIdx.x; t < EDGE; t += NT) {
        const int slot = border_slot<TH>(t, tw, th);
        uint16_t eid = ID_NONE;
        if (slot >= 0 && occupied(slot)) eid = static_cast<uint16_t>(code_of(slot, P[slot]));
        edg[t] = eid;
    }
    if (threadIdx.x == 0) {
        uint64_t *xb = xbits + static_cast<int64_t>(tile) * XW;
        int act = 0;
#pragma unroll
        for (int j = 0; j < XR; ++j) {
            unsigned long long xrt = 0;  // rows 64 j ... 64 j + 63: the waves (64 / RPW of them) holding them
            for (int w = j * (64 / RPW); w < min(NWAVE, (j + 1) * (64 / RPW)); ++w) xrt |= xr_w[w];
            xb[j] = xrt;
        }
        for (int w = 0; w < NWAVE; ++w) act += act_w[w];
        xb[XR] = xd_s.e;      // bottom crossing bonds of even columns
        xb[XR + 1] = xd_s.o;  // ... and of odd columns
        nbp[tile] = nb_s;
        if (MODE == M_SW && tile_act) tile_act[tile] = act;
    }
}

// 8 waves per SIMD (four 128 x 64 workgroups per CU): the LDS use stays
// under 40 KB per 64 rows and the registers are held to what 8 waves allow
// (some scalar registers spill to vector lanes; the extra latency hiding is
// worth more).
template <int MODE, bool EVENW, bool BATCH, int TH_>
__global__ __launch_bounds__(Tile<TH_>::NT) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_tile(TileArgs a)
{
    __shared__ TileSmem<MODE, TH_> sm;
    int tile, lt;  // tile in the arrays, tile inside its lattice
    if constexpr (BATCH) {
        tile = a.b.tile_base + xcd_remap(blockIdx.x, a.b.ntiles);
        load_batch_tile(a, tile, lt);
    } else {
        tile = lt = xcd_remap(blockIdx.x, a.g.ntiles);
        if (a.g.rev) tile = lt = a.g.ntiles - 1 - tile;
    }
    tile_body<MODE, EVENW, TH_, true, !BATCH && MODE == M_SW>(a, tile, lt, sm);
}

// ---------------------------------------------------------------- merge ----

struct MergeArgs {
    Grid g;
    const uint16_t *edges;
    const uint64_t *xbits;
    const int32_t *gkey;
    int32_t *gparent;
    Batch b;                  // batched launches only
};

// A wave per tile: its lanes walk the bonds crossing the tile's right edge
// (TH rows, 64 per pass) and bottom edge (TW columns, two passes).
// Consecutive crossing bonds that join the same pair of boundary ids are
// skipped.  The workgroup size (tiles per workgroup, one wave each) is the
// merge schedule's free parameter; it is read from blockDim.
// The merge of one tile by the calling wave (`tile` indexes the tile arrays).
template <bool BATCH, int TH_>
__device__ __forceinline__ void merge_tile(MergeArgs a, const int tile)
{
    using S = Tile<TH_>;
    constexpr int TH = S::TH, CAP = S::CAP, EDGE = S::EDGE, XR = S::XR, XW = S::XW;
    const int lane = threadIdx.x & 63;
    int tile0 = 0;  // first tile of the lattice in the arrays
    if constexpr (BATCH) {
        const LatticeDesc &L = a.b.lat[a.b.lat_of_tile[tile]];
        a.g = L.g;
        tile0 = L.tile0;
    }
    const int lt = tile - tile0;
    const int tx = lt % a.g.ntx, ty = lt / a.g.ntx;
    const int tw = min(TW, a.g.W - tx * TW), th = min(TH, a.g.H - ty * TH);
    const uint16_t *e = a.edges + static_cast<int64_t>(tile) * EDGE;
    const uint64_t *xb = a.xbits + static_cast<int64_t>(tile) * XW;
    const int ntR = tile0 + ty * a.g.ntx + (tx + 1 == a.g.ntx ? 0 : tx + 1);
    const int ntD = tile0 + (ty + 1 == a.g.nty ? 0 : ty + 1) * a.g.ntx + tx;
    const uint16_t *eR = a.edges + static_cast<int64_t>(ntR) * EDGE;
    const uint16_t *eD = a.edges + static_cast<int64_t>(ntD) * EDGE;
    uint64_t xr[XR];
#pragma unroll
    for (int j = 0; j < XR; ++j) xr[j] = xb[j];
    const uint64_t xde = xb[XR], xdo = xb[XR + 1];  // bottom crossing bonds, even / odd columns
    auto xr_bit = [&](int y) { return (xr[y >> 6] >> (y & 63)) & 1ull; };
    auto xd_bit = [&](int x) { return (((x & 1) ? xdo : xde) >> (x >> 1)) & 1ull; };
    // Passes of 64 lanes: the right edge (TH rows), then the bottom edge in
    // two halves (TW columns).  Every edge entry a lane needs, and the one
    // before it (for skipping repeats), is loaded up front; all lie inside
    // the tiles' edge arrays.
    constexpr int RP = (TH + 63) / 64;  // passes over the right edge
    const uint16_t *er = e + 2 * TW + TH, *el = eR + 2 * TW, *eb = e + TW;
    uint16_t r_a[RP], r_b[RP], r_ap[RP], r_bp[RP];
#pragma unroll
    for (int j = 0; j < RP; ++j) {
        const int y = min(64 * j + lane, TH - 1), ym = max(y - 1, 0);
        r_a[j] = er[y];
        r_b[j] = el[y];
        r_ap[j] = er[ym];
        r_bp[j] = el[ym];
    }
    const int lm = max(lane - 1, 0);
    const uint16_t b1_a = eb[lane], b1_b = eD[lane], b1_ap = eb[lm], b1_bp = eD[lm];
    const uint16_t b2_a = eb[64 + lane], b2_b = eD[64 + lane], b2_ap = eb[63 + lane], b2_bp = eD[63 + lane];
    // Both ends of a crossing bond are border sites, whose codes are boundary
    // ids (< CAP); the bound keeps any other entry from addressing memory
    // outside the tiles' tables.
    auto ids = [](uint16_t u, uint16_t v) { return u < CAP && v < CAP; };
#pragma unroll
    for (int j = 0; j < RP; ++j) {
        const int y = 64 * j + lane;
        if (y < th && xr_bit(y) && !(y > 0 && xr_bit(y - 1) && r_ap[j] == r_a[j] && r_bp[j] == r_b[j]) &&
            ids(r_a[j], r_b[j]))
            gunite(a.gparent, a.gkey, tile * CAP + r_a[j], ntR * CAP + r_b[j]);
    }
    if (lane < tw && xd_bit(lane) && !(lane > 0 && xd_bit(lane - 1) && b1_ap == b1_a && b1_bp == b1_b) &&
        ids(b1_a, b1_b))
        gunite(a.gparent, a.gkey, tile * CAP + b1_a, ntD * CAP + b1_b);
    const int x2 = 64 + lane;
    if (x2 < tw && xd_bit(x2) && !(xd_bit(x2 - 1) && b2_ap == b2_a && b2_bp == b2_b) && ids(b2_a, b2_b))
        gunite(a.gparent, a.gkey, tile * CAP + b2_a, ntD * CAP + b2_b);
}

template <bool BATCH, int TH_>
__global__ __launch_bounds__(1024) void k_merge(MergeArgs a)
{
    int tile = blockIdx.x * static_cast<int>(blockDim.x >> 6) + wave_id();
    if constexpr (BATCH) {
        if (tile >= a.b.ntiles) return;
        tile += a.b.tile_base;
    } else {
        if (tile >= a.g.ntiles) return;
        if (a.g.rev) tile = a.g.ntiles - 1 - tile;
    }
    merge_tile<BATCH, TH_>(a, tile);
}

// -------------------------------------------------------------- flatten ----

struct FlatArgs {
    Grid g;
    const uint16_t *codes;
    const int32_t *gkey;
    int32_t *gparent;
    const int32_t *nb;
    uint8_t *spins;           // M_SW: written
    int32_t *labels;          // canonical labels or nullptr
    int32_t *tile_ncl;        // [ntiles]: clusters whose canonical root lies in the tile
    // cluster sizes (nullptr when not requested)
    int32_t *gsize;           // [ntiles][CAP]
    int32_t *row_count;       // [H][ntx]: roots per (row, tile column)
    int32_t *rl_slot;         // [ntiles][TSITES]: root slots in raster order
    int32_t *rl_size;         // size, or -(root id + 1) for boundary clusters
    uint32_t q, k0, k1, t, sid;
    int ising;
    Batch b;                  // batched launches only
    // few-cluster flips (M_FEW)
    const uint32_t *sel;      // [ntiles][CAP]: == stamp at the root id of a seeded boundary cluster
    uint32_t *seedmap;        // [ntiles][TSITES / 32]: interior roots that hold a seed (cleared here)
    uint32_t stamp;           // this sweep's mark (t + 1)
    uint32_t tflip;           // a seeded cluster flips iff its FEW word is below this
};

// The seed of seed tile j (Sec. III, few-cluster variant): the lattice is cut
// into few_b x few_b seed tiles (narrower at the right and bottom edges), j in
// raster order, and each draws one of its own sites from the block
// (j, t, SEED, sid): x from word 0, y from word 1, each floor(w * extent / 2^32).
__device__ __forceinline__ void seed_site(int j, int W, int H, int B, int ntx, uint32_t t, uint32_t sid, uint32_t k0,
                                          uint32_t k1, int &x, int &y)
{
    const int tx = j % ntx, ty = j / ntx;
    const uint32_t bw = static_cast<uint32_t>(min(B, W - tx * B)), bh = static_cast<uint32_t>(min(B, H - ty * B));
    const U4 b = philox4x32_10(static_cast<uint32_t>(j), t, TAG_SEED, sid, k0, k1);
    x = tx * B + static_cast<int>((static_cast<uint64_t>(b.v0) * bw) >> 32);
    y = ty * B + static_cast<int>((static_cast<uint64_t>(b.v1) * bh) >> 32);
}

// Whether the seeded cluster with canonical root R flips (one draw per
// distinct cluster, Sec. III).
__device__ __forceinline__ bool few_flips(uint32_t R, const FlatArgs &a)
{
    const U4 b = philox4x32_10(R >> 2, a.t, TAG_FEW, a.sid, a.k0, a.k1);
    return pick(b, R & 3u) < a.tflip;
}

// Spin byte <-> state 0..q-1 (Ising bytes are -1 / +1 for states 0 / 1).
__device__ __forceinline__ uint32_t state_of_byte(uint32_t v, int ising) { return ising ? (v == 1u ? 1u : 0u) : v; }

// Clusters that hold a seed: one thread per seed tile finds the code of its
// seed's site.  A boundary cluster is marked at its root id with this sweep's
// stamp; an interior cluster by the bit of its root slot in its tile's seed
// map, which the flatten of that tile reads and clears.
struct SeedArgs {
    Grid g;
    const uint16_t *codes;
    const int32_t *gparent;
    uint32_t *sel;
    uint32_t *seedmap;
    uint32_t stamp, t, sid, k0, k1;
    int few_b, few_ntx, nseed;
};

template <int TH_>
__global__ __launch_bounds__(NT) void k_seed(SeedArgs a)
{
    using S = Tile<TH_>;
    const int j = static_cast<int>(blockIdx.x) * NT + static_cast<int>(threadIdx.x);
    if (j >= a.nseed) return;
    int x, y;
    seed_site(j, a.g.W, a.g.H, a.few_b, a.few_ntx, a.t, a.sid, a.k0, a.k1, x, y);
    const int lt = (y / S::TH) * a.g.ntx + x / TW;
    const int slot = (y % S::TH) * TW + x % TW;
    const uint32_t code = a.codes[static_cast<int64_t>(lt) * S::TSITES + slot];
    if (code < static_cast<uint32_t>(S::CAP)) {
        a.sel[gfind(a.gparent, lt * S::CAP + static_cast<int>(code))] = a.stamp;
    } else {
        const uint32_t root = code - S::CAP;
        atomicOr(&a.seedmap[static_cast<int64_t>(lt) * (S::TSITES / 32) + (root >> 5)], 1u << (root & 31u));
    }
}

// New state of the cluster whose canonical root is R (Sec. II.D: one uniform
// draw per cluster, here taken at the minimum site index).
__device__ __forceinline__ uint8_t flip_state(uint32_t R, const FlatArgs &a)
{
    const U4 b = philox4x32_10(R >> 2, a.t, TAG_FLIP, a.sid, a.k0, a.k1);
    return static_cast<uint8_t>(draw_state(pick(b, R & 3u), a.q));
}

// LDS of the flatten phase.
template <int MODE, bool SIZES, int TH_>
struct FlatSmem {
    static constexpr int TH = TH_, TSITES = TW * TH, CAP = 2 * (TW + TH), NWAVE = TH / RPW;
    uint8_t ST[MODE == M_SW || MODE == M_FEW ? CAP + TSITES : 1];  // new state per code (boundary id or
                                                                    // CAP + slot); M_FEW: FEW_KEEP = no change
    int32_t Rb[CAP];                              // canonical root (site index) per boundary id
    int32_t Gid[CAP];                             // root id per boundary id
    uint16_t rl[NWAVE][WLIST];                    // interior roots of each wave's rows
    int ncl_w[NWAVE];
    int32_t Ci[SIZES ? TSITES : 1];               // sizes of interior clusters
    int32_t Cb[SIZES ? CAP : 1];                  // per-tile part of boundary clusters
    int32_t rowc[TH + 1];
    uint32_t seedw_s[MODE == M_FEW ? NWAVE : 1][32];  // M_FEW: seed-map words of each wave's rows
};

__device__ __forceinline__ void load_batch_flat(FlatArgs &a, int tile, int &lt)
{
    const LatticeDesc &L = a.b.lat[a.b.lat_of_tile[tile]];
    a.g = L.g;
    a.spins = L.spins;
    a.labels = L.labels;
    a.q = L.q;
    a.k0 = L.k0;
    a.k1 = L.k1;
    a.sid = L.sid;
    a.ising = L.ising;
    a.t = *a.b.t;
    lt = tile - L.tile0;
}

constexpr uint8_t FEW_KEEP = 0xFF;

// The flatten + flip of one tile (`tile` in the arrays, `lt` inside its
// lattice), by a Tile<TH>::NT-thread workgroup.  M_FEW flips only the seeded
// clusters whose draw says so and writes only their sites.
template <int MODE, bool SIZES, int TH_>
__device__ __forceinline__ void flatten_body(FlatArgs a, const int tile, const int lt, FlatSmem<MODE, SIZES, TH_> &sm)
{
    using S = Tile<TH_>;
    constexpr int TH = S::TH, TSITES = S::TSITES, CAP = S::CAP, NT = S::NT, NWAVE = S::NWAVE;
    constexpr int BPT = (CAP + NT - 1) / NT;  // boundary ids per thread
    constexpr int NCODE = CAP + TSITES;
    uint8_t *ST = sm.ST;
    int32_t *Rb = sm.Rb, *Gid = sm.Gid;
    auto &rl = sm.rl;
    int *ncl_w = sm.ncl_w;
    int32_t *Ci = sm.Ci, *Cb = sm.Cb, *rowc = sm.rowc;
    const int W = a.g.W;
    const int tx = lt % a.g.ntx, ty = lt / a.g.ntx;
    const int gx0 = tx * TW, gy0 = ty * TH;
    const int tw = min(TW, W - gx0), th = min(TH, a.g.H - gy0);
    const int lane = threadIdx.x & 63, wave = wave_id();
    const int lx0 = 2 * lane;
    const int ly0 = wave * RPW;
    const int nr = max(0, min(RPW, th - ly0));
    const int nbt = a.nb[tile];
    // each boundary id's parent and key (ids threadIdx.x + j NT), issued with
    // the count's loads (entries past nb are read, not used); a root's key is
    // its cluster's canonical label
    int broot[BPT], bR[BPT];
#pragma unroll
    for (int j = 0; j < BPT; ++j) {
        const int k = static_cast<int>(threadIdx.x) + j * NT;
        broot[j] = bR[j] = 0;
        if (k < CAP) {
            broot[j] = a.gparent[tile * CAP + k];
            bR[j] = a.gkey[tile * CAP + k];
        }
    }

    if constexpr (SIZES) {
        // the scan's closing slot and the largest-size slot after the
        // per-(row, tile column) counts start at zero (no other block writes them)
        if (lt == 0 && threadIdx.x < 2) a.row_count[static_cast<int64_t>(a.g.H) * a.g.ntx + threadIdx.x] = 0;
        for (int k = threadIdx.x; k < TSITES; k += NT) Ci[k] = 0;
        for (int k = threadIdx.x; k < CAP; k += NT) Cb[k] = 0;
    }
    // M_FEW: the seed-map words of this wave's rows (RPW * TW / 32 = 32 of
    // them, word l in lane l), cleared for the next sweep
    uint32_t seedw = 0;
    if constexpr (MODE == M_FEW) {
        static_assert(RPW * TW / 32 == 32, "one seed-map word per lane of the lower half");
        if (lane < 32) {
            uint32_t *w = a.seedmap + static_cast<int64_t>(tile) * (TSITES / 32) + ly0 * (TW / 32) + lane;
            seedw = *w;
            if (seedw) *w = 0u;
        }
    }
    uint32_t cc[RPW];
    const uint32_t *codes32 = reinterpret_cast<const uint32_t *>(a.codes + static_cast<int64_t>(tile) * TSITES);
#pragma unroll
    for (int r = 0; r < RPW; ++r) cc[r] = r < nr ? codes32[((ly0 + r) * TW + lx0) >> 1] : 0xFFFFFFFFu;

    // interior roots (code = CAP + own slot) of the wave's rows, compacted
    int nroot = 0;
    uint16_t *mylist = rl[wave];
#pragma unroll
    for (int r = 0; r < RPW; ++r) {
        if (r >= nr) break;  // unrolled: cc[] stays indexed by constants
        const int base = (ly0 + r) * TW;
        const EO m = EO{lanes_eq(cc[r] & 0xFFFFu, static_cast<uint32_t>(CAP + base + lx0)),
                        lanes_eq(cc[r] >> 16, static_cast<uint32_t>(CAP + base + lx0 + 1))};
        eo_append(mylist, nroot, m, lane, base);
    }
    wave_lds_fence();
    if constexpr (MODE == M_SW) {
        for (int i = lane; i < nroot; i += 64) {
            const int slot = mylist[i];
            ST[CAP + slot] = flip_state(static_cast<uint32_t>((gy0 + (slot >> 7)) * W + gx0 + (slot & (TW - 1))), a);
        }
    } else if constexpr (MODE == M_FEW) {
        // a seeded interior cluster that flips takes the other state of its
        // root (every site of a cluster has the same spin); the interior roots
        // of the wave's list lie in its own rows, whose seed-map words the
        // wave keeps in its own LDS words; a seeded root's spin is loaded
        // ahead of the draw
        uint32_t *myseed = sm.seedw_s[wave];
        if (lane < 32) myseed[lane] = seedw;
        wave_lds_fence();
        for (int i = lane; i < nroot; i += 64) {
            const int slot = mylist[i];
            const uint32_t R = static_cast<uint32_t>((gy0 + (slot >> 7)) * W + gx0 + (slot & (TW - 1)));
            const uint32_t word = myseed[(slot >> 5) - ly0 * (TW / 32)];
            const bool seeded = (word >> (slot & 31)) & 1u;
            uint32_t old = 0;
            if (seeded) old = a.spins[R];
            uint8_t v = FEW_KEEP;
            if (seeded && few_flips(R, a)) v = static_cast<uint8_t>(1u - state_of_byte(old, a.ising));
            ST[CAP + slot] = v;
        }
    }
    // boundary ids: the root and its key (the cluster's minimum site index),
    // loaded at the start
    int nbr = 0;
#pragma unroll
    for (int j = 0; j < BPT; ++j) {
        const int k = static_cast<int>(threadIdx.x) + j * NT;
        if (k < nbt) {
            const int id = tile * CAP + k;
            int r = broot[j], key = bR[j];
            uint32_t old = 0;
            if constexpr (MODE == M_FEW) old = a.spins[bR[j]];  // the id's own tile-local root, in this tile
            if (r != id) {  // below a root (the merge keeps trees shallow): walk up, take the root's key
                r = gfind(a.gparent, r);
                key = a.gkey[r];
            }
            Rb[k] = key;
            Gid[k] = r;
            nbr += r == id;
            if constexpr (MODE == M_SW) ST[k] = flip_state(static_cast<uint32_t>(key), a);
            if constexpr (MODE == M_FEW) {
                // seeded iff its root carries this sweep's mark; the old state
                // was read at the id's own tile-local root (a site of this
                // tile, not yet written)
                uint8_t v = FEW_KEEP;
                if (a.sel[r] == a.stamp && few_flips(static_cast<uint32_t>(key), a))
                    v = static_cast<uint8_t>(1u - state_of_byte(old, a.ising));
                ST[k] = v;
            }
        }
    }
    {
        const unsigned long long s = wave_sum(static_cast<unsigned long long>(nbr));
        if (lane == 0) ncl_w[wave] = static_cast<int>(s) + nroot;
    }
    __syncthreads();
    if (threadIdx.x == 0 && a.tile_ncl) {
        int n = 0;
        for (int w = 0; w < NWAVE; ++w) n += ncl_w[w];
        a.tile_ncl[tile] = n;
    }

    const bool v0 = lx0 < tw, v1 = lx0 + 1 < tw;
#pragma unroll
    for (int r = 0; r < RPW; ++r) {
        if (r >= nr) break;
        const int ly = ly0 + r;
        const int64_t i0 = static_cast<int64_t>(gy0 + ly) * W + gx0 + lx0;
        const uint32_t c0 = cc[r] & 0xFFFFu, c1 = cc[r] >> 16;
        if constexpr (MODE == M_SW) {
            // sites past a ragged tile edge carry CODE_BG: clamp the lookup, never store
            const uint32_t st0 = ST[min(c0, static_cast<uint32_t>(NCODE - 1))];
            const uint32_t st1 = ST[min(c1, static_cast<uint32_t>(NCODE - 1))];
            const uint32_t b0 = a.ising ? (2u * st0 - 1u) & 0xFFu : st0;
            const uint32_t b1 = a.ising ? (2u * st1 - 1u) & 0xFFu : st1;
            if (v1 && !(i0 & 1)) {
                *reinterpret_cast<uint16_t *>(a.spins + i0) = static_cast<uint16_t>(b0 | (b1 << 8));
            } else {
                if (v0) a.spins[i0] = static_cast<uint8_t>(b0);
                if (v1) a.spins[i0 + 1] = static_cast<uint8_t>(b1);
            }
        } else if constexpr (MODE == M_FEW) {
            // only the sites of flipping clusters are written
            const uint32_t st0 = ST[min(c0, static_cast<uint32_t>(NCODE - 1))];
            const uint32_t st1 = ST[min(c1, static_cast<uint32_t>(NCODE - 1))];
            const bool f0 = v0 && st0 != FEW_KEEP, f1 = v1 && st1 != FEW_KEEP;
            const uint32_t b0 = a.ising ? (2u * st0 - 1u) & 0xFFu : st0;
            const uint32_t b1 = a.ising ? (2u * st1 - 1u) & 0xFFu : st1;
            if (f0 && f1 && !(i0 & 1)) {
                *reinterpret_cast<uint16_t *>(a.spins + i0) = static_cast<uint16_t>(b0 | (b1 << 8));
            } else {
                if (f0) a.spins[i0] = static_cast<uint8_t>(b0);
                if (f1) a.spins[i0 + 1] = static_cast<uint8_t>(b1);
            }
        }
        if (a.labels) {
            int32_t R[2];
            const uint32_t cs[2] = {c0, c1};
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const uint32_t c = cs[j];
                const int slot = static_cast<int>(c) - CAP;
                R[j] = c == CODE_BG ? -1
                     : c < static_cast<uint32_t>(CAP) ? Rb[c]
                                                       : (gy0 + (slot >> 7)) * W + gx0 + (slot & (TW - 1));
            }
            if (v1 && !(i0 & 1)) {
                *reinterpret_cast<int2 *>(a.labels + i0) = make_int2(R[0], R[1]);
            } else {
                if (v0) a.labels[i0] = R[0];
                if (v1) a.labels[i0 + 1] = R[1];
            }
        }
        if constexpr (SIZES) {
            if (v0 && c0 != CODE_BG) atomicAdd(c0 < static_cast<uint32_t>(CAP) ? &Cb[c0] : &Ci[c0 - CAP], 1);
            if (v1 && c1 != CODE_BG) atomicAdd(c1 < static_cast<uint32_t>(CAP) ? &Cb[c1] : &Ci[c1 - CAP], 1);
        }
    }

    if constexpr (SIZES) {
        __syncthreads();
        // boundary clusters: add this tile's part at the global root id
        for (int k = threadIdx.x; k < nbt; k += NT)
            if (Cb[k]) __hip_atomic_fetch_add(&a.gsize[Gid[k]], Cb[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        // canonical roots of this tile in raster order: per-row counts, then positions
        EO rm[RPW];
#pragma unroll
        for (int r = 0; r < RPW; ++r) {
            rm[r] = EO{0ull, 0ull};
            if (r >= nr) continue;
            const int ly = ly0 + r;
            const int base = ly * TW;
            bool isr[2];
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const int s = lx0 + j;
                const uint32_t code = (cc[r] >> (16 * j)) & 0xFFFFu;
                const int32_t self = (gy0 + ly) * W + gx0 + s;
                isr[j] = s < tw && code != CODE_BG &&
                         ((code == static_cast<uint32_t>(CAP + base + s)) ||
                          (code < static_cast<uint32_t>(CAP) && Gid[code] == tile * CAP + static_cast<int>(code) &&
                           Rb[code] == self));
            }
            rm[r] = EO{__ballot(isr[0]), __ballot(isr[1])};
            if (lane == 0) {
                const int n = __popcll(rm[r].e) + __popcll(rm[r].o);
                rowc[ly] = n;
                a.row_count[static_cast<int64_t>(gy0 + ly) * a.g.ntx + tx] = n;
            }
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            int acc = 0;
            for (int ly = 0; ly < th; ++ly) {
                const int n = rowc[ly];
                rowc[ly] = acc;
                acc += n;
            }
            rowc[th] = acc;
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < RPW; ++r) {
            if (r >= nr) break;
            const int ly = ly0 + r;
            const int base = ly * TW;
            // ascending site order within the row: even sites below 2L+j, odd sites below
            const int below = lanes_below(rm[r].e) + lanes_below(rm[r].o);
            const int be = lane_bit(rm[r].e, lane) ? 1 : 0;
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                if (!lane_bit(j ? rm[r].o : rm[r].e, lane)) continue;
                const int s = lx0 + j;
                const int pos = rowc[ly] + below + (j ? be : 0);
                const uint32_t code = (cc[r] >> (16 * j)) & 0xFFFFu;
                const int64_t o = static_cast<int64_t>(tile) * TSITES + pos;
                a.rl_slot[o] = base + s;
                a.rl_size[o] = (code < static_cast<uint32_t>(CAP)) ? -(tile * CAP + static_cast<int>(code) + 1)
                                                                   : Ci[base + s];
            }
        }
    }
}

template <int MODE, bool SIZES, bool BATCH, int TH_>
__global__ __launch_bounds__(Tile<TH_>::NT) void k_flatten(FlatArgs a)
{
    __shared__ FlatSmem<MODE, SIZES, TH_> sm;
    int tile, lt;  // tile in the arrays, tile inside its lattice
    if constexpr (BATCH) {
        tile = a.b.tile_base + xcd_remap(blockIdx.x, a.b.ntiles);
        load_batch_flat(a, tile, lt);
    } else {
        tile = lt = xcd_remap(blockIdx.x, a.g.ntiles);
        if (a.g.rev) tile = lt = a.g.ntiles - 1 - tile;
    }
    flatten_body<MODE, SIZES, TH_>(a, tile, lt, sm);
}

// Sum of n per-tile int32 counters into *out64 and/or *out32 (one atomic per
// workgroup; both outputs are cleared by the caller).
__global__ __launch_bounds__(NT) void k_reduce_tiles(const int32_t *v, int n, unsigned long long *out64,
                                                      int32_t *out32)
{
    __shared__ unsigned long long red[NWAVE];
    unsigned long long acc = 0;
    for (int i = blockIdx.x * NT + threadIdx.x; i < n; i += gridDim.x * NT) acc += static_cast<unsigned>(v[i]);
    acc = wave_sum(acc);
    const int lane = threadIdx.x & 63, wave = wave_id();
    if (lane == 0) red[wave] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int w = 0; w < NWAVE; ++w) t += red[w];
        if (out64) add_stat(out64, t);
        if (out32 && t) atomicAdd(out32, static_cast<int32_t>(t));
    }
}

// ------------------------------------------------------------ root list ----

// Exclusive scan of n int32 values in blocks of SCAN_ITEMS; block totals go to
// `totals` (scanned by the next level).
constexpr int SCAN_ITEMS = NT * 8;

__global__ __launch_bounds__(NT) void k_scan_block(const int32_t *in, int32_t *out, int64_t n, int32_t *totals)
{
    __shared__ int32_t part[NT];
    const int64_t base = static_cast<int64_t>(blockIdx.x) * SCAN_ITEMS + threadIdx.x * 8;
    int32_t v[8];
    int32_t sum = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        v[j] = (base + j < n) ? in[base + j] : 0;
        sum += v[j];
    }
    part[threadIdx.x] = sum;
    __syncthreads();
    for (int off = 1; off < NT; off <<= 1) {
        const int32_t add = (static_cast<int>(threadIdx.x) >= off) ? part[threadIdx.x - off] : 0;
        __syncthreads();
        part[threadIdx.x] += add;
        __syncthreads();
    }
    int32_t acc = part[threadIdx.x] - sum;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        if (base + j < n) out[base + j] = acc;
        acc += v[j];
    }
    if (threadIdx.x == NT - 1 && totals) totals[blockIdx.x] = part[NT - 1];
}

__global__ __launch_bounds__(NT) void k_scan_add(int32_t *out, int64_t n, const int32_t *offs)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * NT + threadIdx.x;
    if (i < n) out[i] += offs[i / SCAN_ITEMS];
}

struct EmitArgs {
    Grid g;
    const int32_t *row_off;   // [H*ntx + 1] exclusive offsets
    const int32_t *rl_slot;
    const int32_t *rl_size;
    const int32_t *gsize;
    int32_t *roots;
    int32_t *sizes;
    int32_t *max_size;        // largest size (atomic max), or nullptr
    int32_t *n_clusters;      // the number of clusters (the offsets' total), or nullptr
};

// Write each tile's roots (ascending site index within a row) at their global
// positions; boundary clusters take their size from the global root id.
template <int TH_>
__device__ __forceinline__ void emit_body(const EmitArgs &a, const int tile)
{
    constexpr int TH = Tile<TH_>::TH, TSITES = Tile<TH_>::TSITES;
    __shared__ int32_t rstart[TH + 1];
    const int tx = tile % a.g.ntx, ty = tile / a.g.ntx;
    const int gx0 = tx * TW, gy0 = ty * TH;
    const int th = min(TH, a.g.H - gy0);
    if (threadIdx.x == 0) {
        int acc = 0;
        for (int ly = 0; ly < th; ++ly) {
            const int64_t ix = static_cast<int64_t>(gy0 + ly) * a.g.ntx + tx;
            rstart[ly] = acc;
            acc += a.row_off[ix + 1] - a.row_off[ix];
        }
        rstart[th] = acc;
    }
    __syncthreads();
    const int n = rstart[th];
    int mx = 0;
    for (int j = threadIdx.x; j < n; j += NT) {
        const int64_t o = static_cast<int64_t>(tile) * TSITES + j;
        const int slot = a.rl_slot[o];
        const int ly = slot >> 7;
        const int pos = a.row_off[static_cast<int64_t>(gy0 + ly) * a.g.ntx + tx] + (j - rstart[ly]);
        const int sz = a.rl_size[o];
        const int size = sz >= 0 ? sz : a.gsize[-sz - 1];
        a.roots[pos] = (gy0 + ly) * a.g.W + gx0 + (slot & (TW - 1));
        a.sizes[pos] = size;
        mx = max(mx, size);
    }
    if (a.max_size) {
        mx = wave_max(mx);
        if ((threadIdx.x & 63) == 0 && mx > 0) atomicMax(a.max_size, mx);
    }
    if (a.n_clusters && tile == 0 && threadIdx.x == 0)
        *a.n_clusters = a.row_off[static_cast<int64_t>(a.g.H) * a.g.ntx];
}

template <int TH_>
__global__ __launch_bounds__(NT) void k_emit(EmitArgs a)
{
    emit_body<TH_>(a, xcd_remap(blockIdx.x, a.g.ntiles));
}

// ------------------------------------------------------- small lattices ---
//
// A lattice of one tile (W <= SMALL_W, H <= SMALL_H) is swept entirely inside one
// workgroup: spins and union-find parents stay in LDS for all n sweeps of one
// launch, so a sweep costs neither launches nor an
// HBM round trip (a 64 x 64 lattice is launch-latency bound otherwise).  The
// bonds, canonical labels and new states are those of the tiled path; every
// bond, wrap bonds included, is a union inside the workgroup.

// Per-sweep record of sw_sweep_history: active bonds, clusters, largest cluster
// (-1: not measured), satisfied bonds and state counts of the new spins.
enum { HIST_ACTIVE = 0, HIST_NCLUST = 1, HIST_MAXCL = 2, HIST_NSAT = 3, HIST_COUNTS = 4, HIST_LEN = 12 };

struct SmallArgs {
    int W, H;
    uint8_t *spins;       // read at the start, written at the end
    uint8_t *bonds_out;   // packed bonds of the last sweep, or nullptr
    int32_t *labels;      // canonical labels of the last sweep, or nullptr
    int64_t *hist;        // [n][HIST_LEN] per-sweep records, or nullptr
    int32_t *tile_act;    // [1]: active bonds of the last sweep
    int32_t *tile_ncl;    // [1]: clusters of the last sweep
    uint32_t tm1, tany, k0, k1, sid, q, t0;
    int ising, n;
};

// Row of site i < 2^13 in a lattice of width W <= 128: the float quotient is
// at least 0.5 / W away from the next integer, far above its rounding error.
__device__ __forceinline__ int small_row(int i, float inv_w) { return static_cast<int>((i + 0.5f) * inv_w); }

constexpr int SMALL_NT = 1024;  // 16 waves: more LDS round trips in flight on the one CU

// LDS of a lattice swept whole by an NT_-thread workgroup (at most SITES sites).
template <int NT_, int SITES>
struct SmallSmem {
    int P[SITES];
    uint8_t S[SITES];  // states 0..q-1
    unsigned long long red[NT_ / 64][3];
};

// All a.n sweeps of a lattice of at most SITES sites (W <= SMALL_W, H <=
// SMALL_H) in one NT_-thread workgroup.
template <int NT_, int SITES>
__device__ __forceinline__ void small_body(const SmallArgs &a, SmallSmem<NT_, SITES> &sm)
{
    constexpr int NT = NT_, NWAVE = NT_ / 64, TSITES = SITES;
    constexpr int PAIRS_PER_THREAD = (TSITES / 2 + NT - 1) / NT;  // site pairs 2p, 2p+1 with p = tid + NT m
    static_assert(PAIRS_PER_THREAD <= 8, "a thread's bonds fit one 32-bit mask");
    int *P = sm.P;
    uint8_t *S = sm.S;
    auto &red = sm.red;
    static_assert(2 * TSITES < (1 << 16), "per-workgroup counters fit 16-bit fields");
    const int W = a.W, H = a.H, N = W * H;
    const float inv_w = 1.0f / static_cast<float>(W);
    const int lane = threadIdx.x & 63, wave = wave_id();
    auto right_of = [&](int i) {
        const int y = small_row(i, inv_w), x = i - y * W;
        return y * W + (x + 1 == W ? 0 : x + 1);
    };
    auto down_of = [&](int i) {
        const int y = small_row(i, inv_w);
        return y + 1 == H ? i - y * W : i + W;
    };
    for (int i = threadIdx.x; i < N; i += NT) {
        const uint32_t b = a.spins[i];
        S[i] = static_cast<uint8_t>(a.ising ? (b == 1u ? 1u : 0u) : b);
    }
    __syncthreads();
    // Counters of a sweep's new spins (satisfied bonds, state counts) are
    // taken during the next sweep's bond pass, which compares every
    // neighbour pair anyway; those of the last sweep by one pass at the end.
    // They are reduced as 16-bit fields, four to a word: no total of a
    // workgroup exceeds 2 x 8192 (the bonds of a full tile).
    auto reduce_record = [&](unsigned long long act, unsigned long long ncl, unsigned long long nsat,
                             const unsigned long long (&cnt)[8]) {
        unsigned long long pk[3] = {act | (ncl << 16) | (nsat << 32) | (cnt[0] << 48),
                                    cnt[1] | (cnt[2] << 16) | (cnt[3] << 32) | (cnt[4] << 48),
                                    cnt[5] | (cnt[6] << 16) | (cnt[7] << 32)};
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const unsigned long long w = wave_sum(pk[k]);
            if (lane == 0) red[wave][k] = w;
        }
    };
    // after a barrier: thread k < 11 writes field k of the record of `sweep`
    auto write_record = [&](int sweep, bool last) {
        if (threadIdx.x >= 11) return;
        const int k = threadIdx.x;
        unsigned long long sum = 0;
        for (int w = 0; w < NWAVE; ++w) sum += red[w][k >> 2];
        const unsigned long long tot = (sum >> (16 * (k & 3))) & 0xFFFFull;
        if (a.hist) {
            int64_t *row = a.hist + static_cast<int64_t>(sweep) * HIST_LEN;
            const int col = k == 0 ? HIST_ACTIVE : k == 1 ? HIST_NCLUST : k == 2 ? HIST_NSAT : HIST_COUNTS + k - 3;
            row[col] = static_cast<int64_t>(tot);
            if (k == 0) row[HIST_MAXCL] = -1;
        }
        if (last && k == 0) a.tile_act[0] = static_cast<int32_t>(tot);
        if (last && k == 1) a.tile_ncl[0] = static_cast<int32_t>(tot);
    };
    unsigned long long prev_act = 0, prev_ncl = 0;
    for (int sweep = 0; sweep < a.n; ++sweep) {
        const uint32_t t = a.t0 + static_cast<uint32_t>(sweep);
        const bool last = sweep + 1 == a.n;
        for (int i = threadIdx.x; i < N; i += NT) P[i] = i;
        // bonds of the thread's site pairs (one Philox block per pair): bit
        // 4m + 2j + k of `bonds` is bond k (0 right, 1 down) of site 2p + j
        uint32_t bonds = 0;
        unsigned long long nsat = 0, cnt[8] = {0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
        for (int m = 0; m < PAIRS_PER_THREAD; ++m) {
            const int p = threadIdx.x + NT * m;
            if (2 * p >= N) break;
            const U4 blk = philox4x32_10(static_cast<uint32_t>(p), t, TAG_BOND, a.sid, a.k0, a.k1);
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const int i = 2 * p + j;
                if (i >= N) break;
                const uint32_t wr = j ? blk.v2 : blk.v0, wd = j ? blk.v3 : blk.v1;
                const uint32_t si = S[i];
                const bool er = si == S[right_of(i)], ed = si == S[down_of(i)];
                if (a.hist) {
                    nsat += static_cast<unsigned>(er) + static_cast<unsigned>(ed);
#pragma unroll
                    for (int k = 0; k < 8; ++k) cnt[k] += si == static_cast<uint32_t>(k) ? 1u : 0u;
                }
                const bool br = a.tany && er && wr <= a.tm1;
                const bool bd = a.tany && ed && wd <= a.tm1;
                bonds |= (br ? 1u : 0u) << (4 * m + 2 * j);
                bonds |= (bd ? 1u : 0u) << (4 * m + 2 * j + 1);
                if (last && a.bonds_out) a.bonds_out[i] = static_cast<uint8_t>((br ? 1 : 0) | (bd ? 2 : 0));
            }
        }
        const unsigned long long act = static_cast<unsigned>(__popc(bonds));
        if (sweep > 0 && a.hist) reduce_record(prev_act, prev_ncl, nsat, cnt);  // the previous sweep's record
        __syncthreads();
        if (sweep > 0 && a.hist) write_record(sweep - 1, false);
        // unions of the thread's active bonds, one flat loop: a finished union
        // takes the next bond at once
        {
            uint32_t todo = bonds;
            int u = 0, v = 0, busy = 0;
            while (busy || todo) {
                if (!busy) {
                    const int b = __ffs(todo) - 1;
                    todo &= todo - 1;
                    const int i = 2 * (threadIdx.x + NT * (b >> 2)) + ((b >> 1) & 1);
                    u = i;
                    v = (b & 1) ? down_of(i) : right_of(i);
                    busy = 1;
                }
                int done;
                unite_step(P, u, v, done);
                busy = !done;
            }
        }
        __syncthreads();
        // Every site to its root (replacing parents by ancestors on the way),
        // then the new state of its cluster: the draw at the canonical root
        // (one uniform per cluster), which each site evaluates itself; with
        // roots spread over the lanes a wave would pay for every draw anyway,
        // and no table of new states (nor its barrier) is needed.
        unsigned long long ncl = 0;
        for (int i = threadIdx.x; i < N; i += NT) {
            int x = i, px = lds_ld(&P[x]);
            while (px != x) {
                x = px;
                px = lds_ld(&P[x]);
            }
            if (x != i) lds_st(&P[i], x);
            ncl += x == i ? 1u : 0u;
            const U4 b = philox4x32_10(static_cast<uint32_t>(x) >> 2, t, TAG_FLIP, a.sid, a.k0, a.k1);
            S[i] = static_cast<uint8_t>(draw_state(pick(b, static_cast<uint32_t>(x) & 3u), a.q));
            if (last && a.labels) a.labels[i] = x;
        }
        __syncthreads();
        prev_act = act;
        prev_ncl = ncl;
    }
    {
        // the last sweep's record, from the final spins
        unsigned long long nsat = 0, cnt[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        for (int i = threadIdx.x; i < N; i += NT) {
            const uint32_t si = S[i];
            nsat += static_cast<unsigned>(si == S[right_of(i)]) + static_cast<unsigned>(si == S[down_of(i)]);
#pragma unroll
            for (int k = 0; k < 8; ++k) cnt[k] += si == static_cast<uint32_t>(k) ? 1u : 0u;
        }
        reduce_record(prev_act, prev_ncl, nsat, cnt);
        __syncthreads();
        write_record(a.n - 1, true);
    }
    for (int i = threadIdx.x; i < N; i += NT) {
        const uint32_t st = S[i];
        a.spins[i] = static_cast<uint8_t>(a.ising ? 2u * st - 1u : st);
    }
}

__global__ __launch_bounds__(SMALL_NT) void k_small(SmallArgs a)
{
    __shared__ SmallSmem<SMALL_NT, SMALL_SITES> sm;
    small_body<SMALL_NT, SMALL_SITES>(a, sm);
}

// One per-sweep record from the observable slots (after k_observe and the
// per-tile reductions of the sweep).
__global__ void k_hist_row(const unsigned long long *st, const int32_t *max_size, int64_t *row)
{
    const int k = threadIdx.x;
    if (k >= HIST_LEN) return;
    int64_t v;
    if (k == HIST_ACTIVE) v = static_cast<int64_t>(st[ST_ACTIVE]);
    else if (k == HIST_NCLUST) v = static_cast<int64_t>(st[ST_NCLUST]);
    else if (k == HIST_MAXCL) v = max_size ? static_cast<int64_t>(*max_size) : -1;
    else if (k == HIST_NSAT) v = static_cast<int64_t>(st[ST_NSAT]);
    else v = static_cast<int64_t>(st[ST_COUNTS + k - HIST_COUNTS]);
    row[k] = v;
}

// --------------------------------------------------------------- digest ---

// Check-sum of an array: the sum over i of the low 64 bits of the Philox block
// at counter (i, a_i, DIGEST_TAG, 0) under the zero key, modulo 2^64.  The sum
// is order-independent, so the grid-stride partial sums may add in any order.
constexpr uint32_t DIGEST_TAG = 0xD16E57u;
enum { DIG_U8 = 0, DIG_ISING_I8 = 1, DIG_I32 = 2 };  // a_i: byte, Ising state (+1 -> 1), int32 bits

template <int KIND>
__global__ __launch_bounds__(NT) void k_digest(const void *v, int64_t n, unsigned long long *out)
{
    __shared__ unsigned long long red[NWAVE];
    unsigned long long acc = 0;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * NT + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * NT) {
        uint32_t x;
        if constexpr (KIND == DIG_I32) {
            x = static_cast<const uint32_t *>(v)[i];
        } else {
            const uint32_t b = static_cast<const uint8_t *>(v)[i];
            x = KIND == DIG_ISING_I8 ? (b == 1u ? 1u : 0u) : b;
        }
        const U4 r = philox4x32_10(static_cast<uint32_t>(i), x, DIGEST_TAG, 0u, 0u, 0u);
        acc += static_cast<unsigned long long>(r.v0) | (static_cast<unsigned long long>(r.v1) << 32);
    }
    acc = wave_sum(acc);
    const int lane = threadIdx.x & 63, wave = wave_id();
    if (lane == 0) red[wave] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int w = 0; w < NWAVE; ++w) t += red[w];
        add_stat(out, t);
    }
}

// ----------------------------------------------------------- observables ---

// Satisfied bonds, magnetisation (Ising) and state counts of the spins
// (Eq. potts_hamiltonian: -H/J = number of satisfied bonds).  Blocks take whole
// rows; a thread takes 4 consecutive sites per step.  State counts go to
// packed 16-bit counters (states 0-3 and 4-7), flushed after every row.
__global__ __launch_bounds__(NT) void k_observe(const uint8_t *s, int W, int H, uint32_t q, int ising,
                                                unsigned long long *out)
{
    __shared__ unsigned long long red[NWAVE][10];
    unsigned long long nsat = 0, cnt[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int y = blockIdx.x; y < H; y += gridDim.x) {
        const uint8_t *row = s + static_cast<int64_t>(y) * W;
        const uint8_t *dwn = s + static_cast<int64_t>(y + 1 == H ? 0 : y + 1) * W;
        uint64_t h03 = 0, h47 = 0;
        int steps = 0;  // a 16-bit field takes at most 4 per step: flushed every 8192 steps
        for (int x = threadIdx.x * 4; x < W; x += NT * 4) {
            if (++steps == 8192) {
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    cnt[k] += (h03 >> (16 * k)) & 0xFFFFull;
                    cnt[k + 4] += (h47 >> (16 * k)) & 0xFFFFull;
                }
                h03 = h47 = 0;
                steps = 0;
            }
            uint32_t v[5], d[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int xj = min(x + j, W - 1);
                v[j] = row[xj];
                d[j] = dwn[xj];
            }
            v[4] = row[x + 4 < W ? x + 4 : (x + 4 == W ? 0 : W - 1)];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                if (x + j >= W) break;
                const uint32_t vr = (x + j + 1 == W) ? row[0] : v[j + 1];
                nsat += (v[j] == vr) + (v[j] == d[j]);
                const uint32_t st = ising ? (v[j] == 1u ? 1u : 0u) : v[j];
                if (st < 4) h03 += 1ull << (16 * st);
                else if (st < 8) h47 += 1ull << (16 * (st - 4));
            }
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            cnt[k] += (h03 >> (16 * k)) & 0xFFFFull;
            cnt[k + 4] += (h47 >> (16 * k)) & 0xFFFFull;
        }
    }
    const int lane = threadIdx.x & 63, wave = wave_id();
    unsigned long long vals[10];
    vals[0] = nsat;
    vals[1] = 0;
    for (int k = 0; k < 8; ++k) vals[2 + k] = cnt[k];
    for (int k = 0; k < 10; ++k) {
        const unsigned long long w = wave_sum(vals[k]);
        if (lane == 0) red[wave][k] = w;
    }
    __syncthreads();
    // the magnetisation of the Ising case follows from the counts on the host
    if (threadIdx.x < 10 && threadIdx.x != 1) {
        unsigned long long t = 0;
        for (int w = 0; w < NWAVE; ++w) t += red[w][threadIdx.x];
        const int slot = threadIdx.x == 0 ? ST_NSAT : ST_COUNTS + threadIdx.x - 2;
        add_stat(&out[slot], t);
    }
    (void)q;
}

// ------------------------------------------------ batched labeling requests --
//
// Many labeling requests (the served workload) in one launch per phase: each
// request keeps its input, outputs and per-tile arrays in its own memory; the
// launch's workgroups find their request through a tile -> request table, and
// index the request's arrays with the tile's index inside the request.

struct ReqDesc {
    Grid g;
    int32_t tile0;            // first tile of the request in the launch
    const uint8_t *in;
    int32_t *labels, *roots, *sizes, *n_clusters;  // roots / sizes nullptr without sizes
    uint16_t *codes, *edges;
    int32_t *gkey, *gparent, *gsize, *nb, *tile_ncl;
    uint64_t *xbits;
    int32_t *row_count, *row_off, *rl_slot, *rl_size;  // with sizes
};

struct ReqBatch {
    const ReqDesc *req;
    const int32_t *req_of_tile;  // launch tile -> request
    int32_t ntiles;              // tiles of all requests
};

__device__ __forceinline__ const ReqDesc &req_of(const ReqBatch &rb, int t, int &lt)
{
    const ReqDesc &R = rb.req[rb.req_of_tile[t]];
    lt = t - R.tile0;
    return R;
}

template <int MODE, int TH_>
__global__ __launch_bounds__(Tile<TH_>::NT) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_tile_reqs(ReqBatch rb)
{
    __shared__ TileSmem<MODE, TH_> sm;
    int lt;
    const ReqDesc &R = req_of(rb, xcd_remap(blockIdx.x, rb.ntiles), lt);
    TileArgs a{};
    a.g = R.g;
    a.in = R.in;
    a.codes = R.codes;
    a.gkey = R.gkey;
    a.gparent = R.gparent;
    a.gsize = R.gsize;
    a.edges = R.edges;
    a.xbits = R.xbits;
    a.nb = R.nb;
    // any width: the odd-width form of the row loads serves even widths too
    tile_body<MODE, false, TH_>(a, lt, lt, sm);
}

template <int TH_>
__global__ __launch_bounds__(1024) void k_merge_reqs(ReqBatch rb)
{
    const int t = blockIdx.x * static_cast<int>(blockDim.x >> 6) + wave_id();
    if (t >= rb.ntiles) return;
    int lt;
    const ReqDesc &R = req_of(rb, t, lt);
    MergeArgs m{};
    m.g = R.g;
    m.edges = R.edges;
    m.xbits = R.xbits;
    m.gkey = R.gkey;
    m.gparent = R.gparent;
    merge_tile<false, TH_>(m, lt);
}

template <bool SIZES, int TH_>
__global__ __launch_bounds__(Tile<TH_>::NT) void k_flatten_reqs(ReqBatch rb)
{
    __shared__ FlatSmem<M_BONDS_PERIODIC, SIZES, TH_> sm;
    int lt;
    const ReqDesc &R = req_of(rb, xcd_remap(blockIdx.x, rb.ntiles), lt);
    FlatArgs f{};
    f.g = R.g;
    f.codes = R.codes;
    f.gkey = R.gkey;
    f.gparent = R.gparent;
    f.nb = R.nb;
    f.labels = R.labels;
    f.tile_ncl = R.tile_ncl;
    f.gsize = R.gsize;
    f.row_count = R.row_count;
    f.rl_slot = R.rl_slot;
    f.rl_size = R.rl_size;
    flatten_body<M_BONDS_PERIODIC, SIZES, TH_>(f, lt, lt, sm);
}

template <int TH_>
__global__ __launch_bounds__(NT) void k_emit_reqs(ReqBatch rb)
{
    int lt;
    const ReqDesc &R = req_of(rb, xcd_remap(blockIdx.x, rb.ntiles), lt);
    EmitArgs e{};
    e.g = R.g;
    e.row_off = R.row_off;
    e.rl_slot = R.rl_slot;
    e.rl_size = R.rl_size;
    e.gsize = R.gsize;
    e.roots = R.roots;
    e.sizes = R.sizes;
    e.max_size = nullptr;
    e.n_clusters = R.n_clusters;
    emit_body<TH_>(e, lt);
}

// One workgroup per request: with sizes, the exclusive scan of the request's
// per-(row, tile column) root counts (and their total, the cluster count,
// which the emit writes); without, the cluster count as the sum of its tiles'.
template <bool SIZES>
__global__ __launch_bounds__(NT) void k_scan_reqs(const ReqDesc *req)
{
    const ReqDesc &R = req[blockIdx.x];
    __shared__ int32_t part[NT];
    if constexpr (SIZES) {
        const int64_t n = static_cast<int64_t>(R.g.H) * R.g.ntx + 1;  // the closing slot is 0
        int32_t carry = 0;
        for (int64_t b0 = 0; b0 < n; b0 += SCAN_ITEMS) {
            const int64_t base = b0 + static_cast<int64_t>(threadIdx.x) * 8;
            int32_t v[8], sum = 0;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                v[j] = (base + j < n) ? R.row_count[base + j] : 0;
                sum += v[j];
            }
            part[threadIdx.x] = sum;
            __syncthreads();
            for (int off = 1; off < NT; off <<= 1) {
                const int32_t add = (static_cast<int>(threadIdx.x) >= off) ? part[threadIdx.x - off] : 0;
                __syncthreads();
                part[threadIdx.x] += add;
                __syncthreads();
            }
            int32_t acc = carry + part[threadIdx.x] - sum;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                if (base + j < n) R.row_off[base + j] = acc;
                acc += v[j];
            }
            carry += part[NT - 1];
            __syncthreads();
        }
    } else {
        int32_t acc = 0;
        for (int k = threadIdx.x; k < R.g.ntiles; k += NT) acc += R.tile_ncl[k];
        part[threadIdx.x] = acc;
        __syncthreads();
        for (int off = NT / 2; off > 0; off >>= 1) {
            if (static_cast<int>(threadIdx.x) < off) part[threadIdx.x] += part[threadIdx.x + off];
            __syncthreads();
        }
        if (threadIdx.x == 0 && R.n_clusters) *R.n_clusters = part[0];
    }
}

// ------------------------------------------------------ fused batch sweep ---
//
// One launch per sweep of a whole batch of independent lattices.  Workgroups
// take work items from a queue (a ticket counter) in a fixed order:
//   1. lattices small enough to be swept whole in one workgroup's LDS,
//   2. tiles of the other lattices (bond activation + tile labeling),
//   3. merge groups (up to NWAVE tiles of one lattice, a wave each),
//   4. tiles again (flatten + flip),
// with the tiled lattices in the same order in 2-4.  A merge group waits
// until every tile of its lattice is done, a flatten until every merge group
// of its lattice is done.  Items are handed out in queue order, so every item
// a workgroup waits for was taken earlier by a workgroup that is running and
// itself waits only on items taken before that: the launch needs neither a
// co-resident grid nor a grid-wide barrier, and lattices pipeline (one
// lattice's flatten runs while another's tiles are still labeled).
//
// The counters only grow: every launch takes exactly n_items + gridDim.x
// tickets (each workgroup ends on its first ticket past the items), adds
// ntiles / nmerge to a lattice's counters and gridDim.x to the exit count, so
// a launch finds its place from its first ticket and needs no reset (graph
// replays hold no memset nodes).  The last workgroup to leave advances the
// sweep counter t that the next launch reads.

constexpr unsigned long long FUSED_SPIN_LIMIT = 1ull << 24;  // dependency polls before giving up

struct FusedArgs {
    TileArgs ta;                     // tile arrays and the batch tables (ta.b)
    MergeArgs ma;
    FlatArgs fa;
    const int32_t *small_lat;        // [n_small] lattice of each whole-in-LDS item
    const int32_t *ftile;            // [n_tiles] batch tile of each tile / flatten item
    const int2 *mgroup;              // [n_mgroups] (first batch tile, number of tiles)
    unsigned long long *ticket;      // queue position
    unsigned long long *tiles_done;  // [nlat] tile items finished
    unsigned long long *merge_done;  // [nlat] merge groups finished
    unsigned long long *exit_ctr;    // workgroups finished
    uint32_t *t;                     // sweep counter (the same word as ta.b.t)
    int32_t *fault;                  // set when a dependency wait gave up (results invalid)
    int32_t n_small, n_tiles, n_mgroups;
};

// Thread 0 waits until *p >= target with an acquire at agent scope; the
// workgroup barrier then passes what it acquired on to the other waves.  On a
// chip of several XCDs an agent-scope acquire invalidates the CU's L1 and the
// XCD's L2, so it is taken once per item, by one thread.
__device__ __forceinline__ void fused_wait(const unsigned long long *p, unsigned long long target, int32_t *fault)
{
    if (threadIdx.x == 0) {
        for (unsigned long long k = 0;; ++k) {
            if (__hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) >= target) break;
            if (k == FUSED_SPIN_LIMIT) {
                // a bounded wait: a broken invariant ends the launch instead of hanging it
                __hip_atomic_store(fault, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                break;
            }
            __builtin_amdgcn_s_sleep(2);
        }
    }
    __syncthreads();
}

// The workgroup barrier orders every wave's writes before thread 0's
// agent-scope release, which publishes them with the count (a release writes
// the XCD's L2 back, so it too is issued once per item).
__device__ __forceinline__ void fused_signal(unsigned long long *p)
{
    __syncthreads();
    if (threadIdx.x == 0) __hip_atomic_fetch_add(p, 1ull, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// Lattices swept whole in LDS by a fused launch: at most this many sites (and
// W <= SMALL_W, H <= SMALL_H), so their LDS (5 bytes a site) fits the tile
// phase's budget per workgroup.
template <int NT_>
struct FusedSmall {
    static constexpr int SITES = NT_ * 15 < 7680 ? NT_ * 15 : 7680;
};

template <int TH_>
__global__ __launch_bounds__(Tile<TH_>::NT) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_batch_fused(FusedArgs a)
{
    using S = Tile<TH_>;
    constexpr int NT = S::NT, NWAVE = S::NWAVE, SMALL = FusedSmall<NT>::SITES;
    __shared__ union {
        TileSmem<M_SW, TH_> tile;
        FlatSmem<M_SW, false, TH_> flat;
        SmallSmem<NT, SMALL> small;
    } sm;
    __shared__ unsigned long long ticket_s;
    const uint32_t t = *a.t;  // every workgroup reads it before the last one leaves and advances it
    const long long n_items = static_cast<long long>(a.n_small) + 2ll * a.n_tiles + a.n_mgroups;
    const unsigned long long per_launch = static_cast<unsigned long long>(n_items) + gridDim.x;
    unsigned long long base = 0, launch = 0;
    for (bool first = true;; first = false) {
        if (threadIdx.x == 0) ticket_s = __hip_atomic_fetch_add(a.ticket, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        const unsigned long long tk = uniform64(ticket_s);  // wave-uniform: the item's loads are scalar
        __syncthreads();
        if (first) {
            launch = tk / per_launch;
            base = launch * per_launch;
        }
        long long item = static_cast<long long>(tk - base);
        if (item >= n_items) break;
        if (item < a.n_small) {
            const int j = __builtin_amdgcn_readfirstlane(a.small_lat[item]);
            const LatticeDesc &L = a.ta.b.lat[j];
            SmallArgs s{};
            s.W = L.g.W;
            s.H = L.g.H;
            s.spins = L.spins;
            s.bonds_out = L.bonds;
            s.labels = L.labels;
            s.hist = nullptr;
            s.tile_act = a.ta.tile_act + L.tile0;
            s.tile_ncl = a.fa.tile_ncl + L.tile0;
            s.tm1 = L.tm1;
            s.tany = L.tany;
            s.k0 = L.k0;
            s.k1 = L.k1;
            s.sid = L.sid;
            s.q = L.q;
            s.t0 = t;
            s.ising = L.ising;
            s.n = 1;
            small_body<NT, SMALL>(s, sm.small);
            __syncthreads();  // the LDS is reused by the next item
            continue;
        }
        item -= a.n_small;
        if (item < a.n_tiles) {
            const int tile = __builtin_amdgcn_readfirstlane(a.ftile[item]);
            TileArgs ta = a.ta;
            int lt;
            load_batch_tile(ta, tile, lt);
            if (ta.g.W % 2 == 0)
                tile_body<M_SW, true, TH_>(ta, tile, lt, sm.tile);
            else
                tile_body<M_SW, false, TH_>(ta, tile, lt, sm.tile);
            fused_signal(&a.tiles_done[a.ta.b.lat_of_tile[tile]]);
            continue;
        }
        item -= a.n_tiles;
        if (item < a.n_mgroups) {
            const int2 g2 = a.mgroup[item];
            const int2 grp = make_int2(__builtin_amdgcn_readfirstlane(g2.x), __builtin_amdgcn_readfirstlane(g2.y));
            const int j = a.ta.b.lat_of_tile[grp.x];
            const LatticeDesc &L = a.ta.b.lat[j];
            fused_wait(&a.tiles_done[j], (launch + 1) * static_cast<unsigned long long>(L.g.ntiles), a.fault);
            const int w = wave_id();
            if (w < grp.y) merge_tile<true, TH_>(a.ma, grp.x + w);
            fused_signal(&a.merge_done[j]);
            continue;
        }
        item -= a.n_mgroups;
        {
            const int tile = __builtin_amdgcn_readfirstlane(a.ftile[item]);
            const int j = a.ta.b.lat_of_tile[tile];
            fused_wait(&a.merge_done[j], (launch + 1) * static_cast<unsigned long long>(a.ta.b.lat[j].nmerge),
                       a.fault);
            FlatArgs fa = a.fa;
            int lt;
            load_batch_flat(fa, tile, lt);
            flatten_body<M_SW, false, TH_>(fa, tile, lt, sm.flat);
            __syncthreads();  // the LDS is reused by the next item
        }
    }
    (void)NWAVE;
    if (threadIdx.x == 0) {
        __threadfence();
        const unsigned long long left = __hip_atomic_fetch_add(a.exit_ctr, 1ull, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) + 1;
        if (left % gridDim.x == 0) __hip_atomic_store(a.t, t + 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

}  // namespace swccl
