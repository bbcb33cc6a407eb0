// kernels.hpp -- gfx950 kernels of one Swendsen-Wang sweep and of connected-
// component labeling on a 2D square lattice.
//
// A sweep is three launches (Sec. II: T_SW = T_activate + T_identify + T_flip,
// with T_identify = T_local + T_global):
//
//   k_tile    one workgroup per 128x32 tile.  Bond activation (Sec. II.A) fused
//             with tile labeling (Sec. II.B): the bonds of a tile row are
//             ballots of the 64-lane wave; right bonds become row runs by bit
//             scans of the ballot mask; down bonds join runs by a lock-free
//             union-find with path halving in LDS.  Clusters that touch the
//             tile border get a compact boundary id; every site's result is a
//             16-bit code (boundary id, or CAP + the slot of its interior root).
//   k_merge   tile consolidation (Sec. II.C) in one pass: every active bond
//             that crosses a tile edge, the periodic wrap included, unites two
//             boundary ids in a global union-find over the compact id space
//             (CAS linking of the larger-key root under the smaller one, path
//             halving).  Only ~2(TW+TH) ids per tile exist, so this structure
//             stays small and cache resident.
//   k_flatten resolves every boundary id to its root, whose key is the
//             cluster's minimum site index (the canonical label), draws one new
//             state per cluster from that root (Sec. II.D) and writes spins
//             and, optionally, labels.
//
// Labeling-only inputs (packed bond bytes or binary images) reuse the same
// three kernels with a different bond source.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "philox.hpp"

namespace swccl {

constexpr int TW = 128;               // tile width: a wave covers a tile row, 2 sites per lane
constexpr int TH = 32;                // tile height
constexpr int TSITES = TW * TH;       // sites per tile
constexpr int CAP = 2 * (TW + TH);    // boundary ids per tile (>= border sites)
constexpr int EDGE = 2 * TW + 2 * TH; // edge id entries per tile: top, bottom, left, right
constexpr int XW = 4;                 // crossing-bond words per tile: right rows, bottom cols (2)
constexpr int NT = 256;               // threads per workgroup
constexpr int NWAVE = NT / 64;
constexpr int RPW = TH / NWAVE;       // tile rows per wave
constexpr uint16_t ID_NONE = 0xFFFF;
constexpr uint16_t ID_MARK = 0xFFFE;
constexpr uint16_t CODE_BG = 0xFFFF;
static_assert(TH <= 64, "right-edge crossing bits are one 64-bit word");
static_assert(CAP + TSITES < 0xFFFE, "codes are 16-bit");
static_assert(TW == 128, "a tile row is one wave of 64 lanes x 2 sites");

enum : uint32_t { TAG_INIT = 0, TAG_BOND = 1, TAG_FLIP = 2 };
enum Mode : int { M_SW = 0, M_BONDS_PERIODIC = 1, M_BONDS_OPEN = 2, M_SITES = 3 };

// Per-sweep counters (unsigned 64-bit, two's complement for signed values).
enum { ST_ACTIVE = 0, ST_NCLUST = 1, ST_NSAT = 2, ST_MAGNET = 3, ST_COUNTS = 4, ST_LEN = 16 };

struct Grid {
    int W, H, ntx, nty, ntiles;
};

// ---------------------------------------------------------------- helpers --

// Workgroups are dealt round-robin to the 8 XCDs.  Give each XCD one
// contiguous range of tiles so that tiles sharing halo lines share an L2.
__device__ __forceinline__ int xcd_remap(int b, int n)
{
    const int xcd = b & 7, local = b >> 3;
    const int q = n >> 3, r = n & 7;
    return xcd * q + min(xcd, r) + local;
}

// Spread the low 32 bits of x to the even bit positions of a 64-bit word.
__device__ __forceinline__ uint64_t spread32(uint64_t x)
{
    x &= 0xFFFFFFFFull;
    x = (x | (x << 16)) & 0x0000FFFF0000FFFFull;
    x = (x | (x << 8)) & 0x00FF00FF00FF00FFull;
    x = (x | (x << 4)) & 0x0F0F0F0F0F0F0F0Full;
    x = (x | (x << 2)) & 0x3333333333333333ull;
    x = (x | (x << 1)) & 0x5555555555555555ull;
    return x;
}

struct M128 {
    uint64_t lo, hi;
};

// Lane L owns sites 2L and 2L+1 of a 128-site row: the ballots of the even
// and odd sites interleave into the row's site mask.
__device__ __forceinline__ M128 interleave(uint64_t ev, uint64_t od)
{
    return M128{spread32(ev) | (spread32(od) << 1), spread32(ev >> 32) | (spread32(od >> 32) << 1)};
}

__device__ __forceinline__ bool bit128(const M128 &m, int s)
{
    return s < 64 ? ((m.lo >> s) & 1ull) : ((m.hi >> (s - 64)) & 1ull);
}

// Start of the row run containing site s: one past the highest j < s whose
// bond j -> j+1 is absent (bit j of R clear), or 0.
__device__ __forceinline__ int run_start(const M128 &R, int s)
{
    if (s < 64) {
        const uint64_t z = ~R.lo & ((1ull << s) - 1ull);
        return z ? 64 - __builtin_clzll(z) : 0;
    }
    const uint64_t z = ~R.hi & ((1ull << (s - 64)) - 1ull);
    if (z) return 128 - __builtin_clzll(z);
    if (!((R.lo >> 63) & 1ull)) return 64;
    const uint64_t z0 = ~R.lo & 0x7FFFFFFFFFFFFFFFull;
    return z0 ? 64 - __builtin_clzll(z0) : 0;
}

// ---- LDS union-find (workgroup scope) ----
__device__ __forceinline__ int lds_ld(int *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void lds_st(int *p, int v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Root of x with path halving.  Parents only ever move to ancestors, and a
// root is only changed by the CAS in lunite, so concurrent halving is safe.
__device__ __forceinline__ int lfind(int *P, int x)
{
    for (;;) {
        const int p = lds_ld(&P[x]);
        if (p == x) return x;
        const int g = lds_ld(&P[p]);
        if (g == p) return p;
        lds_st(&P[x], g);
        x = g;
    }
}

// Union: the larger root index is linked below the smaller, so every root is
// the minimum (local, hence global) index of its tree.
__device__ __forceinline__ void lunite(int *P, int a, int b)
{
    for (;;) {
        a = lfind(P, a);
        b = lfind(P, b);
        if (a == b) return;
        if (a < b) {
            const int t = a;
            a = b;
            b = t;
        }
        int expect = a;
        if (__hip_atomic_compare_exchange_strong(&P[a], &expect, b, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_WORKGROUP))
            return;
    }
}

// ---- global union-find over boundary ids (agent scope: 8 XCDs, 8 L2s) ----
__device__ __forceinline__ int g_ld(int *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void g_st(int *p, int v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int gfind(int *G, int x)
{
    for (;;) {
        const int p = g_ld(&G[x]);
        if (p == x) return x;
        const int g = g_ld(&G[p]);
        if (g == p) return p;
        g_st(&G[x], g);
        x = g;
    }
}

// Keys are the global site indices of the tile-local roots; linking the root
// with the larger key below the smaller one makes every final root's key the
// minimum site index of its cluster.
__device__ __forceinline__ void gunite(int *G, const int *key, int a, int b)
{
    for (;;) {
        a = gfind(G, a);
        b = gfind(G, b);
        if (a == b) return;
        if (key[a] < key[b]) {
            const int t = a;
            a = b;
            b = t;
        }
        int expect = a;
        if (__hip_atomic_compare_exchange_strong(&G[a], &expect, b, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT))
            return;
    }
}

__device__ __forceinline__ unsigned long long wave_sum(unsigned long long v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off);
    return v;
}

__device__ __forceinline__ void add_stat(unsigned long long *p, unsigned long long v)
{
    if (v) __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

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
    uint64_t T;
    uint32_t k0, k1, t, sid;
};

template <int MODE>
__global__ __launch_bounds__(NT) void k_tile(TileArgs a)
{
    constexpr bool NEED_DOWN = MODE == M_SW || MODE == M_SITES;  // bonds from two rows
    constexpr bool NEED_HALO = MODE == M_SW || MODE == M_SITES;  // column right of the tile
    __shared__ int P[TSITES];
    __shared__ uint16_t ID[TSITES];
    __shared__ M128 Rm[TH];  // in-tile right bonds per row
    __shared__ M128 Dm[TH];  // in-tile down bonds per row
    __shared__ M128 Om[TH];  // occupied sites per row (all valid sites unless M_SITES)
    __shared__ unsigned long long xr_w[NWAVE];  // right crossing bonds, per wave's rows
    __shared__ M128 xd_s;
    __shared__ int nb_s;
    __shared__ int act_w[NWAVE];

    const int W = a.g.W, H = a.g.H;
    const int tile = xcd_remap(blockIdx.x, a.g.ntiles);
    const int tx = tile % a.g.ntx, ty = tile / a.g.ntx;
    const int gx0 = tx * TW, gy0 = ty * TH;
    const int tw = min(TW, W - gx0), th = min(TH, H - gy0);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int lx0 = 2 * lane, lx1 = lx0 + 1;
    const bool v0 = lx0 < tw, v1 = lx1 < tw;
    const bool last0 = lx0 == tw - 1, last1 = lx1 == tw - 1;
    const int hx = (gx0 + tw == W) ? 0 : gx0 + tw;  // column right of the tile
    const bool right_is_wrap = (gx0 + tw == W);
    const bool bottom_is_wrap = (gy0 + th == H);
    const int ly0 = wave * RPW;
    const int nr = max(0, min(RPW, th - ly0));  // tile rows owned by this wave

    if (threadIdx.x == 0) nb_s = 0;  // first used after the barrier closing phase A

    // ---- A0: issue every load of the wave's rows (and the row below) up front.
    // pr[r] holds the bytes of sites lx0 (bits 0-7) and lx1 (bits 8-15).
    uint32_t pr[RPW + 1];
    uint8_t hl[RPW];
#pragma unroll
    for (int r = 0; r <= RPW; ++r) {
        pr[r] = 0;
        if (r < RPW) hl[r] = 0;
        const bool want = nr > 0 && (r < nr || (NEED_DOWN && r == nr));
        if (want) {
            int gy = gy0 + ly0 + r;
            if (gy == H) gy = 0;  // ly0 + r <= th, so at most one wrap
            const int64_t rowb = static_cast<int64_t>(gy) * W;
            const int64_t i0 = rowb + gx0 + lx0;
            if (v1 && !(i0 & 1)) {
                pr[r] = *reinterpret_cast<const uint16_t *>(a.in + i0);
            } else {
                if (v0) pr[r] = a.in[i0];
                if (v1) pr[r] |= static_cast<uint32_t>(a.in[i0 + 1]) << 8;
            }
            if (NEED_HALO && r < nr && (last0 || last1)) hl[r] = a.in[rowb + hx];
        }
    }

    // ---- A1: bonds of each row, row masks, row-run parents ----
    unsigned long long nact = 0, xr = 0;
#pragma unroll
    for (int r = 0; r < RPW; ++r) {
        if (r >= nr) break;
        const int ly = ly0 + r;
        const int gy = gy0 + ly;
        const int64_t rowb = static_cast<int64_t>(gy) * W;
        const int64_t i0 = rowb + gx0 + lx0;
        const uint32_t cur = pr[r], dn = pr[r + 1];
        bool bR0 = false, bR1 = false, bD0 = false, bD1 = false, o0 = v0, o1 = v1;

        if constexpr (MODE == M_SW) {
            const uint32_t s0 = cur & 0xFFu, s1 = (cur >> 8) & 0xFFu;
            const uint32_t d0 = dn & 0xFFu, d1 = (dn >> 8) & 0xFFu;
            const uint32_t nxt = static_cast<uint32_t>(__shfl_down(static_cast<int>(s0), 1));
            const uint32_t sr0 = last0 ? hl[r] : s1;
            const uint32_t sr1 = last1 ? hl[r] : nxt;
            uint32_t r0R, r0D, r1R, r1D;
            const U4 blk = philox4x32_10(static_cast<uint32_t>(i0 >> 1), a.t, TAG_BOND, a.sid, a.k0, a.k1);
            if ((rowb & 1) == 0) {  // the pair (i0, i0+1) shares one block
                r0R = blk.v0;
                r0D = blk.v1;
                r1R = blk.v2;
                r1D = blk.v3;
            } else {  // odd row start (odd W): i0 is the second site of its block
                r0R = blk.v2;
                r0D = blk.v3;
                const U4 b2 = philox4x32_10(static_cast<uint32_t>((i0 + 1) >> 1), a.t, TAG_BOND, a.sid,
                                            a.k0, a.k1);
                r1R = b2.v0;
                r1D = b2.v1;
            }
            bR0 = v0 && s0 == sr0 && static_cast<uint64_t>(r0R) < a.T;
            bD0 = v0 && s0 == d0 && static_cast<uint64_t>(r0D) < a.T;
            bR1 = v1 && s1 == sr1 && static_cast<uint64_t>(r1R) < a.T;
            bD1 = v1 && s1 == d1 && static_cast<uint64_t>(r1D) < a.T;
            if (a.bonds_out) {
                if (v0) a.bonds_out[i0] = static_cast<uint8_t>(bR0 | (bD0 << 1));
                if (v1) a.bonds_out[i0 + 1] = static_cast<uint8_t>(bR1 | (bD1 << 1));
            }
            nact += static_cast<unsigned>(bR0) + bD0 + bR1 + bD1;
        } else if constexpr (MODE == M_BONDS_PERIODIC || MODE == M_BONDS_OPEN) {
            bR0 = cur & 1u;
            bD0 = (cur >> 1) & 1u;
            bR1 = (cur >> 8) & 1u;
            bD1 = (cur >> 9) & 1u;
            if (MODE == M_BONDS_OPEN) {
                if (right_is_wrap) {
                    bR0 = bR0 && !last0;
                    bR1 = bR1 && !last1;
                }
                if (bottom_is_wrap && ly == th - 1) bD0 = bD1 = false;
            }
        } else {  // M_SITES: 4-connected occupied pixels, open boundary
            o0 = v0 && (cur & 0xFFu) != 0;
            o1 = v1 && (cur & 0xFF00u) != 0;
            const bool has_down = gy + 1 < H;
            const bool d0 = has_down && (dn & 0xFFu) != 0;
            const bool d1 = has_down && (dn & 0xFF00u) != 0;
            const bool nxt = __shfl_down(static_cast<int>(o0), 1) != 0;
            const bool halo = !right_is_wrap && hl[r] != 0;
            bR0 = o0 && (last0 ? halo : o1);
            bR1 = o1 && (last1 ? halo : nxt);
            bD0 = o0 && d0;
            bD1 = o1 && d1;
        }

        // Crossing bonds leave the tile: the last column's right bond and the
        // last row's down bonds.  They are merged by k_merge.
        const bool cross = (last0 && bR0) || (last1 && bR1);
        if (__ballot(cross)) xr |= 1ull << ly;
        const M128 Rrow = interleave(__ballot(bR0 && !last0), __ballot(bR1 && !last1));
        M128 Drow = M128{0ull, 0ull};
        const M128 Dall = interleave(__ballot(bD0), __ballot(bD1));
        if (ly == th - 1) {
            if (lane == 0) xd_s = Dall;
        } else {
            Drow = Dall;
        }
        const M128 Orow = interleave(__ballot(o0), __ballot(o1));
        if (lane == 0) {
            Rm[ly] = Rrow;
            Dm[ly] = Drow;
            Om[ly] = Orow;
        }
        const int base = ly * TW;
        P[base + lx0] = base + (v0 ? run_start(Rrow, lx0) : lx0);
        P[base + lx1] = base + (v1 ? run_start(Rrow, lx1) : lx1);
        ID[base + lx0] = ID_NONE;
        ID[base + lx1] = ID_NONE;
    }
    if (lane == 0) xr_w[wave] = xr;
    if constexpr (MODE == M_SW) {
        const unsigned long long s = wave_sum(nact);
        if (lane == 0) act_w[wave] = static_cast<int>(s);
    }
    __syncthreads();

    // ---- B: down bonds join row runs; one union per vertical contact ----
    for (int r = 0; r < RPW; ++r) {
        const int ly = ly0 + r;
        if (ly + 1 >= th) break;
        const M128 D = Dm[ly], Ra = Rm[ly], Rb = Rm[ly + 1];
        // Site s repeats the contact of s-1 when s-1 has a down bond and both
        // rows continue from s-1 to s.
        const M128 X = M128{D.lo & Ra.lo & Rb.lo, D.hi & Ra.hi & Rb.hi};
        const M128 Xs = M128{X.lo << 1, (X.hi << 1) | (X.lo >> 63)};
        const M128 F = M128{D.lo & ~Xs.lo, D.hi & ~Xs.hi};
        const int base = ly * TW;
        if (bit128(F, lx0)) lunite(P, base + lx0, base + TW + lx0);
        if (bit128(F, lx1)) lunite(P, base + lx1, base + TW + lx1);
    }
    __syncthreads();

    // ---- C: full path compression ----
    for (int r = 0; r < nr; ++r) {
        const int base = (ly0 + r) * TW;
        if (v0) lds_st(&P[base + lx0], lfind(P, base + lx0));
        if (v1) lds_st(&P[base + lx1], lfind(P, base + lx1));
    }
    __syncthreads();

    // ---- D: mark roots of clusters that touch the tile border ----
    for (int r = 0; r < nr; ++r) {
        const int ly = ly0 + r;
        const M128 O = Om[ly];
        const int base = ly * TW;
        const bool edge_row = (ly == 0) || (ly == th - 1);
        if (v0 && bit128(O, lx0) && (edge_row || lx0 == 0 || last0)) ID[P[base + lx0]] = ID_MARK;
        if (v1 && bit128(O, lx1) && (edge_row || last1)) ID[P[base + lx1]] = ID_MARK;
    }
    __syncthreads();

    // ---- E: compact boundary ids ----
    for (int r = 0; r < nr; ++r) {
        const int ly = ly0 + r;
        const int base = ly * TW;
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int s = lx0 + j;
            const bool isb = (s < tw) && P[base + s] == base + s && ID[base + s] == ID_MARK;
            const uint64_t m = __ballot(isb);
            if (m) {
                int first = 0;
                if (lane == 0) first = atomicAdd(&nb_s, __popcll(m));
                first = __shfl(first, 0);
                if (isb) {
                    const int k = first + __popcll(m & ((1ull << lane) - 1ull));
                    ID[base + s] = static_cast<uint16_t>(k);
                    const int id = tile * CAP + k;
                    a.gkey[id] = (gy0 + ly) * W + gx0 + s;
                    a.gparent[id] = id;
                    if (a.gsize) a.gsize[id] = 0;
                }
            }
        }
    }
    __syncthreads();

    // ---- F: codes, edge ids, crossing bits ----
    uint32_t *codes32 = reinterpret_cast<uint32_t *>(a.codes + static_cast<int64_t>(tile) * TSITES);
    uint16_t *edg = a.edges + static_cast<int64_t>(tile) * EDGE;
    for (int r = 0; r < nr; ++r) {
        const int ly = ly0 + r;
        const M128 O = Om[ly];
        const int base = ly * TW;
        uint16_t c[2];
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int s = lx0 + j;
            uint16_t code = CODE_BG, eid = ID_NONE;
            if (s < tw && bit128(O, s)) {
                const int root = P[base + s];
                const uint16_t k = ID[root];
                eid = k;
                code = (k != ID_NONE) ? k : static_cast<uint16_t>(CAP + root);
            }
            c[j] = code;
            if (s < tw) {
                if (ly == 0) edg[s] = eid;
                if (ly == th - 1) edg[TW + s] = eid;
                if (s == 0) edg[2 * TW + ly] = eid;
                if (s == tw - 1) edg[2 * TW + TH + ly] = eid;
            }
        }
        codes32[(base + lx0) >> 1] = static_cast<uint32_t>(c[0]) | (static_cast<uint32_t>(c[1]) << 16);
    }
    if (threadIdx.x == 0) {
        uint64_t *xb = a.xbits + static_cast<int64_t>(tile) * XW;
        unsigned long long xrt = 0;
        for (int w = 0; w < NWAVE; ++w) xrt |= xr_w[w];
        xb[0] = xrt;
        xb[1] = th > 0 ? xd_s.lo : 0ull;
        xb[2] = th > 0 ? xd_s.hi : 0ull;
        a.nb[tile] = nb_s;
        if (MODE == M_SW && a.tile_act) a.tile_act[tile] = act_w[0] + act_w[1] + act_w[2] + act_w[3];
    }
}

// ---------------------------------------------------------------- merge ----

struct MergeArgs {
    Grid g;
    const uint16_t *edges;
    const uint64_t *xbits;
    const int32_t *gkey;
    int32_t *gparent;
};

// One thread per bond crossing the right edge (TH rows) or the bottom edge
// (TW columns) of a tile; consecutive crossing bonds that join the same pair
// of boundary ids are skipped.
__global__ __launch_bounds__(NT) void k_merge(MergeArgs a)
{
    const int tile = xcd_remap(blockIdx.x, a.g.ntiles);
    const int tx = tile % a.g.ntx, ty = tile / a.g.ntx;
    const int tw = min(TW, a.g.W - tx * TW), th = min(TH, a.g.H - ty * TH);
    const int j = threadIdx.x;
    const uint16_t *e = a.edges + static_cast<int64_t>(tile) * EDGE;
    if (j < TH) {
        if (j >= th) return;
        const uint64_t xr = a.xbits[static_cast<int64_t>(tile) * XW];
        if (!((xr >> j) & 1ull)) return;
        const int nt = ty * a.g.ntx + (tx + 1 == a.g.ntx ? 0 : tx + 1);
        const uint16_t *en = a.edges + static_cast<int64_t>(nt) * EDGE;
        const uint16_t ka = e[2 * TW + TH + j], kb = en[2 * TW + j];
        if (j > 0 && ((xr >> (j - 1)) & 1ull) && e[2 * TW + TH + j - 1] == ka && en[2 * TW + j - 1] == kb) return;
        gunite(a.gparent, a.gkey, tile * CAP + ka, nt * CAP + kb);
    } else if (j < TH + TW) {
        const int x = j - TH;
        if (x >= tw) return;
        const uint64_t *xb = a.xbits + static_cast<int64_t>(tile) * XW + 1;
        if (!((xb[x >> 6] >> (x & 63)) & 1ull)) return;
        const int nt = (ty + 1 == a.g.nty ? 0 : ty + 1) * a.g.ntx + tx;
        const uint16_t *en = a.edges + static_cast<int64_t>(nt) * EDGE;
        const uint16_t ka = e[TW + x], kb = en[x];
        if (x > 0 && ((xb[(x - 1) >> 6] >> ((x - 1) & 63)) & 1ull) && e[TW + x - 1] == ka && en[x - 1] == kb)
            return;
        gunite(a.gparent, a.gkey, tile * CAP + ka, nt * CAP + kb);
    }
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
};

// New state of the cluster whose canonical root is R (Sec. II.D: one uniform
// draw per cluster, here taken at the minimum site index).
__device__ __forceinline__ uint8_t flip_state(uint32_t R, const FlatArgs &a)
{
    const U4 b = philox4x32_10(R >> 2, a.t, TAG_FLIP, a.sid, a.k0, a.k1);
    return static_cast<uint8_t>(draw_state(pick(b, R & 3u), a.q));
}

template <int MODE, bool SIZES>
__global__ __launch_bounds__(NT) void k_flatten(FlatArgs a)
{
    __shared__ int32_t Rb[CAP];     // canonical root (site index) per boundary id
    __shared__ int32_t Gid[CAP];    // root id per boundary id
    __shared__ uint8_t Sb[CAP];     // new state per boundary id
    __shared__ uint8_t Si[TSITES];  // new state per interior root slot
    __shared__ uint16_t rlist[TSITES];  // interior root slots
    __shared__ int nroot_s;
    __shared__ int ncl_w[NWAVE];
    __shared__ int32_t Ci[SIZES ? TSITES : 1];  // sizes of interior clusters
    __shared__ int32_t Cb[SIZES ? CAP : 1];     // per-tile part of boundary clusters
    __shared__ int32_t rowc[TH + 1];

    const int W = a.g.W;
    const int tile = xcd_remap(blockIdx.x, a.g.ntiles);
    const int tx = tile % a.g.ntx, ty = tile / a.g.ntx;
    const int gx0 = tx * TW, gy0 = ty * TH;
    const int tw = min(TW, W - gx0), th = min(TH, a.g.H - gy0);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int lx0 = 2 * lane;
    const int ly0 = wave * RPW;
    const int nr = max(0, min(RPW, th - ly0));
    const int nbt = a.nb[tile];

    if (threadIdx.x == 0) nroot_s = 0;
    if constexpr (SIZES) {
        for (int k = threadIdx.x; k < TSITES; k += NT) Ci[k] = 0;
        for (int k = threadIdx.x; k < CAP; k += NT) Cb[k] = 0;
    }
    uint32_t cc[RPW];
    const uint32_t *codes32 = reinterpret_cast<const uint32_t *>(a.codes + static_cast<int64_t>(tile) * TSITES);
#pragma unroll
    for (int r = 0; r < RPW; ++r) cc[r] = r < nr ? codes32[((ly0 + r) * TW + lx0) >> 1] : 0xFFFFFFFFu;
    __syncthreads();

    // interior roots (code = CAP + own slot) into a compact list
#pragma unroll
    for (int r = 0; r < RPW; ++r) {
        if (r >= nr) break;
        const int base = (ly0 + r) * TW;
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int s = lx0 + j;
            const uint32_t code = (cc[r] >> (16 * j)) & 0xFFFFu;
            const bool isr = s < tw && code == static_cast<uint32_t>(CAP + base + s);
            const uint64_t m = __ballot(isr);
            if (m) {
                int first = 0;
                if (lane == 0) first = atomicAdd(&nroot_s, __popcll(m));
                first = __shfl(first, 0);
                if (isr) rlist[first + __popcll(m & ((1ull << lane) - 1ull))] = static_cast<uint16_t>(base + s);
            }
        }
    }

    // boundary ids: resolve to the global root; the root's key is the
    // cluster's minimum site index
    int nbr = 0;
    for (int k = threadIdx.x; k < nbt; k += NT) {
        const int id = tile * CAP + k;
        const int root = gfind(a.gparent, id);
        const int R = a.gkey[root];
        Rb[k] = R;
        Gid[k] = root;
        nbr += root == id;
        if constexpr (MODE == M_SW) Sb[k] = flip_state(static_cast<uint32_t>(R), a);
    }
    {
        const unsigned long long s = wave_sum(static_cast<unsigned long long>(nbr));
        if (lane == 0) ncl_w[wave] = static_cast<int>(s);
    }
    __syncthreads();
    const int nroot = nroot_s;
    if constexpr (MODE == M_SW) {
        for (int j = threadIdx.x; j < nroot; j += NT) {
            const int slot = rlist[j];
            Si[slot] = flip_state(static_cast<uint32_t>((gy0 + (slot >> 7)) * W + gx0 + (slot & (TW - 1))), a);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0 && a.tile_ncl) a.tile_ncl[tile] = nroot + ncl_w[0] + ncl_w[1] + ncl_w[2] + ncl_w[3];

#pragma unroll
    for (int r = 0; r < RPW; ++r) {
        if (r >= nr) break;
        const int ly = ly0 + r;
        const int base = ly * TW;
        const int64_t i0 = static_cast<int64_t>(gy0 + ly) * W + gx0 + lx0;
        int32_t R[2];
        uint32_t st[2] = {0u, 0u};
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const uint32_t code = (cc[r] >> (16 * j)) & 0xFFFFu;
            if (code == CODE_BG) {
                R[j] = -1;
            } else if (code < static_cast<uint32_t>(CAP)) {
                R[j] = Rb[code];
                if constexpr (MODE == M_SW) st[j] = Sb[code];
                if constexpr (SIZES) {
                    if (lx0 + j < tw) atomicAdd(&Cb[code], 1);
                }
            } else {
                const int slot = static_cast<int>(code) - CAP;
                R[j] = (gy0 + (slot >> 7)) * W + gx0 + (slot & (TW - 1));
                if constexpr (MODE == M_SW) st[j] = Si[slot];
                if constexpr (SIZES) {
                    if (lx0 + j < tw) atomicAdd(&Ci[slot], 1);
                }
            }
        }
        const bool v0 = lx0 < tw, v1 = lx0 + 1 < tw;
        if (a.labels) {
            if (v1 && !(i0 & 1)) {
                *reinterpret_cast<int2 *>(a.labels + i0) = make_int2(R[0], R[1]);
            } else {
                if (v0) a.labels[i0] = R[0];
                if (v1) a.labels[i0 + 1] = R[1];
            }
        }
        if constexpr (MODE == M_SW) {
            const uint32_t b0 = a.ising ? (2u * st[0] - 1u) & 0xFFu : st[0];
            const uint32_t b1 = a.ising ? (2u * st[1] - 1u) & 0xFFu : st[1];
            if (v1 && !(i0 & 1)) {
                *reinterpret_cast<uint16_t *>(a.spins + i0) = static_cast<uint16_t>(b0 | (b1 << 8));
            } else {
                if (v0) a.spins[i0] = static_cast<uint8_t>(b0);
                if (v1) a.spins[i0 + 1] = static_cast<uint8_t>(b1);
            }
        }
    }

    if constexpr (SIZES) {
        __syncthreads();
        // boundary clusters: add this tile's part at the global root id
        for (int k = threadIdx.x; k < nbt; k += NT)
            if (Cb[k]) __hip_atomic_fetch_add(&a.gsize[Gid[k]], Cb[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        // roots of this tile in raster order: per-row counts, then positions
        M128 rm[RPW];
#pragma unroll
        for (int r = 0; r < RPW; ++r) {
            rm[r] = M128{0ull, 0ull};
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
            rm[r] = interleave(__ballot(isr[0]), __ballot(isr[1]));
            if (lane == 0) {
                const int n = __popcll(rm[r].lo) + __popcll(rm[r].hi);
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
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const int s = lx0 + j;
                if (!bit128(rm[r], s)) continue;
                const int below = (s < 64) ? __popcll(rm[r].lo & ((1ull << s) - 1ull))
                                           : __popcll(rm[r].lo) + __popcll(rm[r].hi & ((1ull << (s - 64)) - 1ull));
                const int pos = rowc[ly] + below;
                const uint32_t code = (cc[r] >> (16 * j)) & 0xFFFFu;
                const int64_t o = static_cast<int64_t>(tile) * TSITES + pos;
                a.rl_slot[o] = base + s;
                a.rl_size[o] = (code < static_cast<uint32_t>(CAP)) ? -(tile * CAP + static_cast<int>(code) + 1)
                                                                   : Ci[base + s];
            }
        }
    }
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
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) red[wave] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned long long t = red[0] + red[1] + red[2] + red[3];
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
        const int32_t add = (threadIdx.x >= off) ? part[threadIdx.x - off] : 0;
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
};

// Write each tile's roots (ascending site index within a row) at their global
// positions; boundary clusters take their size from the global root id.
__global__ __launch_bounds__(NT) void k_emit(EmitArgs a)
{
    __shared__ int32_t rstart[TH + 1];
    const int tile = xcd_remap(blockIdx.x, a.g.ntiles);
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
    for (int j = threadIdx.x; j < n; j += NT) {
        const int64_t o = static_cast<int64_t>(tile) * TSITES + j;
        const int slot = a.rl_slot[o];
        const int ly = slot >> 7;
        const int pos = a.row_off[static_cast<int64_t>(gy0 + ly) * a.g.ntx + tx] + (j - rstart[ly]);
        const int sz = a.rl_size[o];
        a.roots[pos] = (gy0 + ly) * a.g.W + gx0 + (slot & (TW - 1));
        a.sizes[pos] = sz >= 0 ? sz : a.gsize[-sz - 1];
    }
}

// ----------------------------------------------------------- observables ---

// Satisfied bonds, magnetisation (Ising) and state counts of the spins
// (Eq. potts_hamiltonian: -H/J = number of satisfied bonds).
__global__ __launch_bounds__(NT) void k_observe(const uint8_t *s, int W, int H, uint32_t q, int ising,
                                                unsigned long long *out)
{
    __shared__ unsigned long long red[NWAVE][10];
    const int64_t N = static_cast<int64_t>(W) * H;
    unsigned long long nsat = 0, cnt[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    long long mag = 0;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * NT + threadIdx.x; i < N;
         i += static_cast<int64_t>(gridDim.x) * NT) {
        const int x = static_cast<int>(i % W);
        const int64_t y = i / W;
        const uint8_t v = s[i];
        const uint8_t vr = s[y * W + (x + 1 == W ? 0 : x + 1)];
        const uint8_t vd = s[(y + 1 == H ? 0 : y + 1) * static_cast<int64_t>(W) + x];
        nsat += (v == vr) + (v == vd);
        if (ising) {
            mag += static_cast<int8_t>(v);
            cnt[v == 1 ? 1 : 0]++;
        } else if (v < 8) {
            cnt[v]++;
        }
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    unsigned long long vals[10];
    vals[0] = nsat;
    vals[1] = static_cast<unsigned long long>(mag);
    for (int k = 0; k < 8; ++k) vals[2 + k] = cnt[k];
    for (int k = 0; k < 10; ++k) {
        const unsigned long long w = wave_sum(vals[k]);
        if (lane == 0) red[wave][k] = w;
    }
    __syncthreads();
    if (threadIdx.x < 10) {
        unsigned long long t = 0;
        for (int w = 0; w < NWAVE; ++w) t += red[w][threadIdx.x];
        const int slot = threadIdx.x == 0 ? ST_NSAT : threadIdx.x == 1 ? ST_MAGNET : ST_COUNTS + threadIdx.x - 2;
        __hip_atomic_fetch_add(&out[slot], t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    (void)q;
}

}  // namespace swccl
