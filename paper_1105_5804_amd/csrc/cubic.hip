// cubic.hip -- the SW sweep on the periodic simple cubic lattice: the same
// three steps as on the square lattice (Sec. II), generalised to three
// dimensions, and the host side of the sw3_* calls of include/swccl.h.
//
// A sweep is four launches:
//
//   k3_tile     one 512-thread workgroup per 32 x 16 x 16 tile (the shape of
//               8192 sites with the fewest face sites and crossing bonds);
//               two sites per lane, a wave-wide step covering four tile rows,
//               each wave eight steps.
//               Bond activation of the +x, +y and +z bonds (Sec. II.A) fused
//               with a lock-free union-find in LDS over the bonds that stay in
//               the tile (Sec. II.B.2); the clusters touching any tile face
//               are claimed and get compact ids; every site gets a 16-bit code
//               (its cluster's id, or CAP + the slot of its interior root).
//   k3_merge    every active bond that leaves a tile through its +x, +y or +z
//               face (periodic wraps included) unites two ids in the global
//               union-find (Sec. II.C).  Roots are linked by a fixed random
//               priority of the ids rather than by key: on the cubic lattice
//               at criticality key-ordered links build trees too deep to walk
//               for the ~10^7 ids of a sweep.
//   k3_resolve  every id pointed at its root, and the cluster's minimum site
//               index (its canonical label) gathered at the root's key;
//   k3_flatten  one draw per cluster at that index (Sec. II.D): the tile's ids
//               and its interior roots, then every site's new state (and
//               optionally label) from its code.
//
// With per-sweep records, k3_observe counts the satisfied bonds and states of
// the new spins and k3_record moves the counters into the record.
//
// ccl3_label runs the same tile, merge, resolve and flatten kernels on given
// bond bytes (LABEL = true): no spins, no draws, labels out.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "../../include/swccl.h"
#include "internal.hpp"
#include "philox.hpp"
#include "uf.hpp"

namespace swccl {
namespace cubic {

constexpr int CX = 32, CY = 16, CZ = 16;                      // tile extent (x fastest)
constexpr int PLANE = CX * CY;                                 // sites of a tile z-plane
constexpr int CSITES = PLANE * CZ;                             // sites per tile
constexpr int CAP = CSITES - (CX - 2) * (CY - 2) * (CZ - 2);   // sites on a face of a full tile
// Lanes: two sites each, so a wave-wide step covers 128 sites, RPI tile rows
// of CX sites; the tile's CY * CZ rows are dealt to NW3 waves, RW rows (ITER
// steps) each.  Row R of a tile is (ly, lz) = (R mod CY, R / CY).
constexpr int NW3 = 8;                                         // waves per tile workgroup
constexpr int NT3 = 64 * NW3;
constexpr int LPR = CX / 2;                                    // lanes per tile row
constexpr int RPI = 64 / LPR;                                  // tile rows per step
constexpr int RW = CY * CZ / NW3;                              // tile rows per wave
constexpr int ITER = RW / RPI;                                 // steps per wave
static_assert(CSITES == 128 * NW3 * ITER && ITER == 8, "eight steps of 128 sites per wave");
static_assert(CY % (2 * RPI) == 0 && RW % (2 * RPI) == 0, "steps pair up inside a z-plane");
constexpr int MT = 256;                                        // merge workgroup
constexpr int RT = 64;                                         // resolve workgroup: one wave per tile
constexpr int MSEEN = 1024;                                    // merge: pair-dedup slots per face
constexpr int FX = CY * CZ, FY = CX * CZ, FZ = CX * CY;        // sites of the +x, +y, +z faces
constexpr uint32_t TAG_BOND = 1, TAG_FLIP = 2, TAG_BOND_Z = 5;
constexpr int CLAIMING = -1;
constexpr uint16_t CODE_NONE = 0xFFFF;
static_assert(CAP + CSITES < CODE_NONE, "codes are 16-bit");
static_assert(CAP < (1 << 15), "merge list entries hold two ids in 15 bits each");
static_assert(ITER * 8 <= 64, "a lane's bonds fit one 64-bit mask");

// Counters of a sweep, in the order of the record fields.
enum { S3_ACTIVE = 0, S3_NCLUST = 1, S3_NSAT = 2, S3_COUNTS = 3, S3_LEN = 11 };

struct Geo3 {
    int Lx, Ly, Lz;
    int ntx, nty, ntz, ntiles;
};

// Tile of a workgroup and its extent (ragged at the +x, +y, +z ends).
struct TileOf {
    int tile, gx0, gy0, gz0, tw, th, td;
};
__device__ __forceinline__ TileOf tile_of(const Geo3 &g, int tile)
{
    const int tx = tile % g.ntx, ty = (tile / g.ntx) % g.nty, tz = tile / (g.ntx * g.nty);
    TileOf t;
    t.tile = tile;
    t.gx0 = tx * CX;
    t.gy0 = ty * CY;
    t.gz0 = tz * CZ;
    t.tw = min(CX, g.Lx - t.gx0);
    t.th = min(CY, g.Ly - t.gy0);
    t.td = min(CZ, g.Lz - t.gz0);
    return t;
}

// Site index of tile slot s = (lz CY + ly) CX + lx.
__device__ __forceinline__ int32_t site_of(const Geo3 &g, const TileOf &t, int s)
{
    const int lz = s / PLANE, ly = (s / CX) % CY, lx = s % CX;
    return static_cast<int32_t>((static_cast<int64_t>(t.gz0 + lz) * g.Ly + t.gy0 + ly) * g.Lx + t.gx0 + lx);
}

// Value of x held by the other lane of the calling lane's pair (2m <-> 2m + 1;
// DPP quad permutation 1, 0, 3, 2).
__device__ __forceinline__ uint32_t swap_pair_lanes(uint32_t x)
{
    return static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(x), 0xB1, 0xF, 0xF, false));
}

struct Tile3Args {
    Geo3 g;
    const uint8_t *spins;
    uint8_t *bonds;           // [N] packed bonds of the sweep (bit0 +x, bit1 +y, bit2 +z)
    uint16_t *codes;          // [ntiles][CSITES]
    uint16_t *xface;          // [ntiles][2][FX]: codes of the x = 0 sites, then of the x = tw - 1 sites | +x bond << 15
    int32_t *gkey, *gparent;  // [ntiles][CAP]
    int32_t *nb;              // [ntiles]: ids of the tile
    int32_t *tile_act;        // [ntiles]: active bonds owned by the tile
    uint32_t tm1, tany;       // a bond is active iff its word r <= tm1 and tany (T > 0; tm1 = T - 1)
    uint32_t k0, k1, t, sid;
};

// LABEL: the bonds are given (a.bonds is read, never written); otherwise they
// are drawn from the spins and written.
template <bool LABEL>
__global__ __launch_bounds__(NT3) void k3_tile(Tile3Args a)
{
    __shared__ int P[CSITES];
    __shared__ int nb_s;
    __shared__ unsigned act_w[NW3];
    const Geo3 g = a.g;
    const TileOf T = tile_of(g, xcd_remap(blockIdx.x, g.ntiles));
    const int lane = threadIdx.x & 63, w = wave_id();
    const int sub = lane / LPR, lx0 = 2 * (lane % LPR);  // the lane's row in a step, its first site
    // the lane's tile row at step it, and whether that row lies in the tile
    auto row_of = [&](int it) { return w * RW + it * RPI + sub; };
    auto row_in = [&](int R) { return R % CY < T.th && R / CY < T.td; };
    if (threadIdx.x == 0) nb_s = 0;
    for (int k = threadIdx.x; k < CSITES; k += NT3) P[k] = k;

    // Bonds of the lane's two sites at each step; bit 8 it + 4 j + d of
    // `inside` is bond d (0 +x, 1 +y, 2 +z) of site lx0 + j of the step's row
    // when it stays in the tile (the others cross a face and are merged by
    // k3_merge from the bond array).  Site indices fit 32 bits.
    uint64_t inside = 0;
    uint32_t xbit = 0;  // bit 2 it + j: the +x bond of site lx0 + j of the step's row
    unsigned act = 0;
    const uint32_t Lx = static_cast<uint32_t>(g.Lx), Ly = static_cast<uint32_t>(g.Ly), Lz = static_cast<uint32_t>(g.Lz);
    // a tile full along y and z: every row of every step lies in it, the
    // lane's rows are its first one plus uniform offsets (a wave owns whole
    // z-planes, RW a multiple of CY)
    static_assert(RW % CY == 0, "a wave owns whole z-planes");
    const bool full = T.th == CY && T.td == CZ;
    const uint32_t row_first = ((static_cast<uint32_t>(T.gz0 + w * (RW / CY))) * Ly + static_cast<uint32_t>(T.gy0 + sub)) * Lx;
    const bool ywrap_at_last = static_cast<uint32_t>(T.gy0 + CY) == Ly, zwrap_at_last = static_cast<uint32_t>(T.gz0 + CZ) == Lz;
    // lanes past a ragged edge read a valid column and store nothing
    const uint32_t xs0 = static_cast<uint32_t>(T.gx0 + min(lx0, T.tw - 1));
    const uint32_t xs1 = static_cast<uint32_t>(T.gx0 + min(lx0 + 1, T.tw - 1));
    const uint32_t xn0 = xs0 + 1u == Lx ? 0u : xs0 + 1u, xn1 = xs1 + 1u == Lx ? 0u : xs1 + 1u;
    const bool even_lx = (Lx & 1u) == 0u;
    // with Lx a multiple of 4 every row starts at a multiple of 4, so the two
    // lanes of a pair share one +z block per row: in a tile full along y and
    // z each draws the block of one of two consecutive steps' rows and the
    // halves are swapped between the pair
    const bool zpairs = (Lx & 3u) == 0u && T.th == CY && T.td == CZ;
    const bool odd_lane = (lane & 1) != 0;
    uint32_t zpend0 = 0, zpend1 = 0;  // +z words of the next step's row, drawn with this one
#pragma unroll
    for (int it = 0; it < ITER; ++it) {
        const int R = row_of(it), ly = R % CY, lz = R / CY;
        const bool rin = row_in(R);
        const bool v0 = rin && lx0 < T.tw, v1 = rin && lx0 + 1 < T.tw;
        const bool next_in = rin && lx0 + 2 < T.tw;  // the +x neighbour of site lx0 + 1 is the next lane's first
        // rows outside the tile read a valid row and store nothing
        uint32_t row, rowy, rowz;
        if (full) {
            // the lane's first row plus a wave-uniform offset: RPI rows a
            // step, a plane every CY / RPI steps; the +y and +z rows follow
            // by Lx and Lx Ly except across the lattice's own boundary
            row = row_first + static_cast<uint32_t>(((it * RPI) / CY) * Ly + (it * RPI) % CY) * Lx;
            rowy = ywrap_at_last && ly == CY - 1 ? row - (Ly - 1u) * Lx : row + Lx;
            rowz = zwrap_at_last && lz == CZ - 1 ? row - (Lz - 1u) * Ly * Lx : row + Ly * Lx;
        } else {
            const uint32_t gy = static_cast<uint32_t>(T.gy0 + min(ly, T.th - 1));
            const uint32_t gz = static_cast<uint32_t>(T.gz0 + min(lz, T.td - 1));
            const uint32_t yn = gy + 1u == Ly ? 0u : gy + 1u, zn = gz + 1u == Lz ? 0u : gz + 1u;
            row = (gz * Ly + gy) * Lx;
            rowy = (gz * Ly + yn) * Lx;
            rowz = (zn * Ly + gy) * Lx;
        }
        const uint32_t i0 = row + static_cast<uint32_t>(T.gx0 + lx0);
        uint32_t m0 = 0, m1 = 0;
        if constexpr (LABEL) {
            (void)rowy;
            (void)rowz;
            if (even_lx && v1) {  // the pair in one aligned 16-bit load
                const uint32_t c = *reinterpret_cast<const uint16_t *>(a.bonds + i0);
                m0 = c & 7u;
                m1 = (c >> 8) & 7u;
            } else {
                if (v0) m0 = a.bonds[i0] & 7u;
                if (v1) m1 = a.bonds[i0 + 1] & 7u;
            }
        } else {
            uint32_t s0, s1, y0, y1, z0, z1;
            if (even_lx && v1) {  // the pair in one aligned 16-bit load per row (every row starts even)
                const uint32_t c = *reinterpret_cast<const uint16_t *>(a.spins + row + xs0);
                const uint32_t yy = *reinterpret_cast<const uint16_t *>(a.spins + rowy + xs0);
                const uint32_t zz = *reinterpret_cast<const uint16_t *>(a.spins + rowz + xs0);
                s0 = c & 0xFFu;
                s1 = c >> 8;
                y0 = yy & 0xFFu;
                y1 = yy >> 8;
                z0 = zz & 0xFFu;
                z1 = zz >> 8;
            } else {
                s0 = a.spins[row + xs0];
                s1 = a.spins[row + xs1];
                y0 = a.spins[rowy + xs0];
                y1 = a.spins[rowy + xs1];
                z0 = a.spins[rowz + xs0];
                z1 = a.spins[rowz + xs1];
            }
            const uint32_t nxt = from_next_lane(s0);
            const uint32_t x0 = v1 ? s1 : a.spins[row + xn0];
            const uint32_t x1 = next_in ? nxt : a.spins[row + xn1];
            // words: +x and +y from block(i >> 1, BOND) as on the square
            // lattice, +z word i & 3 of block(i >> 2, BOND_Z)
            const uint32_t c0 = i0 >> 1;
            const U4 bk = philox4x32_10(c0, a.t, TAG_BOND, a.sid, a.k0, a.k1);
            uint32_t rx0, ry0, rx1, ry1;
            if ((i0 & 1u) == 0u) {
                rx0 = bk.v0;
                ry0 = bk.v1;
                rx1 = bk.v2;
                ry1 = bk.v3;
            } else {  // odd row start (odd Lx): i0 is the second site of its block
                rx0 = bk.v2;
                ry0 = bk.v3;
                const U4 b2 = philox4x32_10(c0 + 1u, a.t, TAG_BOND, a.sid, a.k0, a.k1);
                rx1 = b2.v0;
                ry1 = b2.v1;
            }
            uint32_t rz0, rz1;
            if (zpairs && (it & 1) == 0) {
                // the even lane draws its pair's block of this row, the odd lane
                // that of the next step's row (RPI rows on, same plane, no wrap)
                const uint32_t pair = static_cast<uint32_t>(T.gx0 + 2 * ((lane % LPR) & ~1));
                const U4 bz = philox4x32_10((odd_lane ? row + RPI * Lx + pair : row + pair) >> 2, a.t, TAG_BOND_Z,
                                            a.sid, a.k0, a.k1);
                const uint32_t ra = swap_pair_lanes(odd_lane ? bz.v0 : bz.v2);
                const uint32_t rb = swap_pair_lanes(odd_lane ? bz.v1 : bz.v3);
                rz0 = odd_lane ? ra : bz.v0;  // this row: words 0, 1 (even lane) or 2, 3 (odd lane)
                rz1 = odd_lane ? rb : bz.v1;
                zpend0 = odd_lane ? bz.v2 : ra;  // the next step's row
                zpend1 = odd_lane ? bz.v3 : rb;
            } else if (zpairs) {
                rz0 = zpend0;
                rz1 = zpend1;
            } else {
                const U4 bz = philox4x32_10(i0 >> 2, a.t, TAG_BOND_Z, a.sid, a.k0, a.k1);
                rz0 = pick(bz, i0 & 3u);
                if (((i0 + 1u) & 3u) != 0u) {
                    rz1 = pick(bz, (i0 + 1u) & 3u);
                } else {  // site i0 + 1 starts the next block
                    rz1 = philox4x32_10((i0 + 1u) >> 2, a.t, TAG_BOND_Z, a.sid, a.k0, a.k1).v0;
                }
            }
            if (v0 && a.tany)
                m0 = (s0 == x0 && rx0 <= a.tm1 ? 1u : 0u) | (s0 == y0 && ry0 <= a.tm1 ? 2u : 0u) |
                     (s0 == z0 && rz0 <= a.tm1 ? 4u : 0u);
            if (v1 && a.tany)
                m1 = (s1 == x1 && rx1 <= a.tm1 ? 1u : 0u) | (s1 == y1 && ry1 <= a.tm1 ? 2u : 0u) |
                     (s1 == z1 && rz1 <= a.tm1 ? 4u : 0u);
            act += __popc(m0) + __popc(m1);
            if ((i0 & 1u) == 0u && v1) {
                *reinterpret_cast<uint16_t *>(a.bonds + i0) = static_cast<uint16_t>(m0 | (m1 << 8));
            } else {
                if (v0) a.bonds[i0] = static_cast<uint8_t>(m0);
                if (v1) a.bonds[i0 + 1] = static_cast<uint8_t>(m1);
            }
        }
        xbit |= ((m0 & 1u) | ((m1 & 1u) << 1)) << (2 * it);
        const uint32_t in_x = (lx0 + 1 < T.tw ? 0x01u : 0u) | (lx0 + 2 < T.tw ? 0x10u : 0u);
        const uint32_t in_y = ly + 1 < T.th ? 0x22u : 0u, in_z = lz + 1 < T.td ? 0x44u : 0u;
        inside |= static_cast<uint64_t>((m0 | (m1 << 4)) & (in_x | in_y | in_z)) << (8 * it);
    }
    __syncthreads();

    // unions of the bonds inside the tile, one flat loop per lane: a finished
    // union takes the lane's next bond at once
    {
        uint64_t todo = inside;
        int u = 0, v = 0, busy = 0;
        while (busy || todo) {
            if (!busy) {
                const int bit = __ffsll(static_cast<unsigned long long>(todo)) - 1;
                todo &= todo - 1;
                const int it = bit >> 3, j = (bit >> 2) & 1, d = bit & 3;
                u = row_of(it) * CX + lx0 + j;
                v = u + (d == 0 ? 1 : d == 1 ? CX : PLANE);
                busy = 1;
            }
            int done;
            unite_step(P, u, v, done);
            busy = !done;
        }
    }
    __syncthreads();

    // Every site's root, walked once (the trees are final after the unions)
    // and kept in registers for the claims and the codes.  Other waves may
    // already be claiming: a claimed root's entry is negative, and the walk
    // ends there too.
    auto root_of = [&](int x) {
        for (;;) {
            const int p = lds_ld(&P[x]);
            if (p == x || p < 0) return x;
            x = p;
        }
    };
    int rt[ITER][2];
#pragma unroll
    for (int it = 0; it < ITER; ++it) {
        const int R = row_of(it);
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            rt[it][j] = 0;
            if (row_in(R) && lx0 + j < T.tw) rt[it][j] = root_of(R * CX + lx0 + j);
        }
    }
    // claims: the root of every cluster that touches a tile face gets an id
#pragma unroll
    for (int it = 0; it < ITER; ++it) {
        const int R = row_of(it), ly = R % CY, lz = R / CY;
        if (!row_in(R)) continue;
        const bool plane_face = ly == 0 || ly == T.th - 1 || lz == 0 || lz == T.td - 1;
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int lx = lx0 + j;
            if (lx >= T.tw || !(plane_face || lx == 0 || lx == T.tw - 1)) continue;
            const int r = rt[it][j];
            int expect = r;
            if (__hip_atomic_compare_exchange_strong(&P[r], &expect, CLAIMING, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_WORKGROUP)) {
                const int k = atomicAdd(&nb_s, 1);
                lds_st(&P[r], -(k + 2));
                const int id = T.tile * CAP + k;
                a.gkey[id] = site_of(g, T, r);
                a.gparent[id] = id;
            }
        }
    }
    __syncthreads();

    // codes: the id of a claimed root (its entry reads -(id + 2)), else CAP +
    // the root's slot
    {
        uint16_t *codes = a.codes + static_cast<int64_t>(T.tile) * CSITES;
#pragma unroll
        for (int it = 0; it < ITER; ++it) {
            const int R = row_of(it);
            if (!row_in(R)) continue;
            const int s = R * CX + lx0;
            uint32_t c[2] = {CODE_NONE, CODE_NONE};
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                if (lx0 + j >= T.tw) continue;
                const int r = rt[it][j];
                const int pr = lds_ld(&P[r]);
                c[j] = pr < 0 ? static_cast<uint32_t>(-pr - 2) : static_cast<uint32_t>(CAP + r);
            }
            *reinterpret_cast<uint32_t *>(codes + s) = c[0] | (c[1] << 16);
            // the x faces again, packed by row (the merge reads them whole);
            // a row's x-face position is its tile row R
            uint16_t *xf = a.xface + static_cast<int64_t>(T.tile) * (2 * FX);
            if (lx0 == 0) xf[R] = static_cast<uint16_t>(c[0]);
            const int jl = T.tw - 1 - lx0;
            if (jl == 0 || jl == 1)
                xf[FX + R] = static_cast<uint16_t>((jl == 0 ? c[0] : c[1]) | (((xbit >> (2 * it + jl)) & 1u) << 15));
        }
    }
    const unsigned long long tot = wave_sum(act);
    if (lane == 0) act_w[w] = static_cast<unsigned>(tot);
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned sum = 0;
        for (int k = 0; k < NW3; ++k) sum += act_w[k];
        a.nb[T.tile] = nb_s;
        a.tile_act[T.tile] = static_cast<int32_t>(sum);
    }
}

struct Merge3Args {
    Geo3 g;
    const uint8_t *bonds;
    const uint16_t *codes;
    const uint16_t *xface;  // as written by k3_tile
    int32_t *gparent;
};

// Fixed random priority of an id: a bijection of the 32-bit integers
// (multiplications by odd constants and xor-shifts), so no two ids tie.
__device__ __forceinline__ uint32_t id_prio(int x)
{
    uint32_t h = static_cast<uint32_t>(x) * 0x9E3779B1u;
    h ^= h >> 16;
    h *= 0x85EBCA6Bu;
    h ^= h >> 13;
    return h;
}

// Union of the trees holding ids a and b: the root of lower priority is
// linked below the other by a device-scope compare-and-swap (randomised
// linking keeps the expected depth logarithmic); a failed swap returns the
// root's new parent, from which the union goes on.  The walks halve their
// paths as in the square-lattice merge.
__device__ __forceinline__ void gunite_prio(int *G, int a, int b)
{
    gfind2(G, a, b);
    for (;;) {
        if (a == b) return;
        if (id_prio(a) > id_prio(b)) {
            const int t = a;
            a = b;
            b = t;
        }
        int expect = a;
        if (__hip_atomic_compare_exchange_strong(&G[a], &expect, b, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT))
            return;
        a = expect;
        gfind2(G, a, b);
    }
}

// Tile consolidation: each active bond leaving the tile through its +x, +y or
// +z face joins the ids of its two ends (both are face sites, hence claimed).
// Every face has one neighbouring tile, so (face, id, id across) names a
// union.  The workgroup first gathers its distinct unions into a list (the
// bond bits of all its face positions loaded at once, then the codes of the
// active ones, duplicates dropped), then works the list off with every lane
// busy: a lane no longer waits for its wave's deepest union at each of its
// face positions.
constexpr int MPOS = (FX + FY + FZ + MT - 1) / MT;  // face positions per merge thread

__global__ __launch_bounds__(MT) void k3_merge(Merge3Args a)
{
    // seen[d][h]: the last pair (ca << 16 | cb) registered across face d in
    // hash slot h = ca mod MSEEN; a lane that gets its own pair back skips it
    // (the lane that registered it lists it; pairs sharing a slot are at
    // worst listed twice)
    __shared__ unsigned int seen[3][MSEEN];
    __shared__ unsigned int list[FX + FY + FZ];  // d << 30 | ca << 15 | cb
    __shared__ int nlist;
    const Geo3 g = a.g;
    const TileOf T = tile_of(g, xcd_remap(blockIdx.x, g.ntiles));
    for (int k = threadIdx.x; k < 3 * MSEEN; k += MT) (&seen[0][0])[k] = 0xFFFFFFFFu;
    if (threadIdx.x == 0) nlist = 0;
    // the neighbouring tile across each face
    const int tx = T.gx0 / CX, ty = T.gy0 / CY, tz = T.gz0 / CZ;
    const int nbr[3] = {(tz * g.nty + ty) * g.ntx + (tx + 1 == g.ntx ? 0 : tx + 1),
                        (tz * g.nty + (ty + 1 == g.nty ? 0 : ty + 1)) * g.ntx + tx,
                        ((tz + 1 == g.ntz ? 0 : tz + 1) * g.nty + ty) * g.ntx + tx};
    // site index and the neighbour's slot of face position f, or -1
    auto face = [&](int f, int &d, int &s1, int &s2) -> int64_t {
        int lx, ly, lz;
        if (f < FX) {
            d = 0;
            lx = T.tw - 1;
            ly = f % CY;
            lz = f / CY;
        } else if (f < FX + FY) {
            d = 1;
            lx = (f - FX) % CX;
            ly = T.th - 1;
            lz = (f - FX) / CX;
        } else {
            d = 2;
            lx = (f - FX - FY) % CX;
            ly = (f - FX - FY) / CX;
            lz = T.td - 1;
        }
        if (f >= FX + FY + FZ || lx >= T.tw || ly >= T.th || lz >= T.td) return -1;
        s1 = (lz * CY + ly) * CX + lx;
        // across the face the neighbour sits at coordinate 0 of that axis
        s2 = d == 0 ? (lz * CY + ly) * CX : d == 1 ? lz * PLANE + lx : ly * CX + lx;
        return (static_cast<int64_t>(T.gz0 + lz) * g.Ly + T.gy0 + ly) * g.Lx + T.gx0 + lx;
    };
    int ca[MPOS], cb[MPOS], dd[MPOS];
    bool act[MPOS];
#pragma unroll
    for (int j = 0; j < MPOS; ++j) {  // every bond bit first (independent loads)
        int s1, s2;
        const int f = j * MT + static_cast<int>(threadIdx.x);
        const int64_t i = face(f, dd[j], s1, s2);
        if (dd[j] == 0) {  // the +x face from the packed x faces: bond bit and code at once
            const uint32_t h = i >= 0 ? a.xface[static_cast<int64_t>(T.tile) * (2 * FX) + FX + f] : 0u;
            act[j] = ((h >> 15) & 1u) != 0u;
            ca[j] = static_cast<int>(h & 0x7FFFu);
            cb[j] = f;
        } else {
            act[j] = i >= 0 && ((a.bonds[i] >> dd[j]) & 1u);
            ca[j] = s1;
            cb[j] = s2;
        }
    }
#pragma unroll
    for (int j = 0; j < MPOS; ++j) {  // then the codes of the active ones
        if (!act[j]) continue;
        if (dd[j] == 0) {
            cb[j] = a.xface[static_cast<int64_t>(nbr[0]) * (2 * FX) + cb[j]];
        } else {
            ca[j] = a.codes[static_cast<int64_t>(T.tile) * CSITES + ca[j]];
            cb[j] = a.codes[static_cast<int64_t>(nbr[dd[j]]) * CSITES + cb[j]];
        }
        if (ca[j] >= CAP || cb[j] >= CAP) act[j] = false;  // face sites always hold ids
    }
    __syncthreads();  // seen and nlist are set
#pragma unroll
    for (int j = 0; j < MPOS; ++j) {
        const int pa = __shfl_up(act[j] ? ca[j] : -1, 1), pb = __shfl_up(cb[j], 1), pd = __shfl_up(dd[j], 1);
        bool keep = act[j] && !((threadIdx.x & 63) != 0 && pa == ca[j] && pb == cb[j] && pd == dd[j]);
        if (keep) {
            const unsigned int key = (static_cast<unsigned int>(ca[j]) << 16) | static_cast<unsigned int>(cb[j]);
            keep = atomicExch(&seen[dd[j]][ca[j] % MSEEN], key) != key;
        }
        if (keep)
            list[atomicAdd(&nlist, 1)] = (static_cast<unsigned int>(dd[j]) << 30) |
                                         (static_cast<unsigned int>(ca[j]) << 15) | static_cast<unsigned int>(cb[j]);
    }
    __syncthreads();
    const int n = nlist;
    for (int k = threadIdx.x; k < n; k += MT) {
        const unsigned int e = list[k];
        const int d = static_cast<int>(e >> 30), ia = static_cast<int>((e >> 15) & 0x7FFFu),
                  ib = static_cast<int>(e & 0x7FFFu);
        gunite_prio(a.gparent, T.tile * CAP + ia, nbr[d] * CAP + ib);
    }
}

struct Flat3Args {
    Geo3 g;
    uint8_t *spins;
    int32_t *labels;  // or nullptr
    const uint16_t *codes;
    const int32_t *gkey;     // a root's key: its cluster's minimum site index
    const int32_t *gparent;  // resolved: every id's entry is its root
    const int32_t *nb;
    int32_t *tile_ncl;       // [ntiles]: clusters whose root lies in the tile
    uint32_t q, ising, k0, k1, t, sid;
};

// New state of the cluster whose canonical root is R: word R & 3 of
// block(R >> 2, t, FLIP), as on the square lattice.
__device__ __forceinline__ uint32_t new_state(uint32_t R, const Flat3Args &a)
{
    const U4 b = philox4x32_10(R >> 2, a.t, TAG_FLIP, a.sid, a.k0, a.k1);
    return draw_state(pick(b, R & 3u), a.q);
}

// Every id of every tile resolved after the merge:
// the id's entry is pointed at its root (the trees are final, so concurrent
// walks stay valid) and the id's key (the minimum site index of its part of
// the cluster) is taken into the root's key by an atomic minimum, issued only
// when the root's key, read first, is larger (a stale read is larger still),
// so the ids of a large cluster do not all contend for its root.  The root's
// key then holds the cluster's minimum site index: its canonical label.
struct Resolve3Args {
    Geo3 g;
    int32_t *gkey;
    int32_t *gparent;
    const int32_t *nb;
};

__global__ __launch_bounds__(RT) void k3_resolve(Resolve3Args a)
{
    // a one-wave workgroup per tile, its lanes over the tile's ids (few idle
    // lanes in the last pass over a tile's few hundred ids)
    const int tile = static_cast<int>(blockIdx.x);
    const int nbt = a.nb[tile];
    for (int k = threadIdx.x; k < nbt; k += RT) {
        const int id = tile * CAP + k;
        int x = id, p = a.gparent[x];
        while (p != x) {
            x = p;
            p = a.gparent[x];
        }
        if (x == id) continue;
        a.gparent[id] = x;
        const int32_t key = a.gkey[id];  // not a root: its key never changes
        if (key < a.gkey[x]) atomicMin(&a.gkey[x], key);
    }
}

// LABEL: labels only (no draws, spins untouched).
template <bool LABEL>
__global__ __launch_bounds__(NT3) void k3_flatten(Flat3Args a)
{
    __shared__ uint8_t ST[CAP + CSITES];          // new state per code
    __shared__ int32_t Rb[CAP];                   // canonical label per id (labels only)
    __shared__ uint16_t roots[NW3][128 * ITER];   // interior root slots of each wave's rows
    __shared__ unsigned ncl_w[NW3];
    const Geo3 g = a.g;
    const TileOf T = tile_of(g, xcd_remap(blockIdx.x, g.ntiles));
    const int lane = threadIdx.x & 63, w = wave_id();
    const int sub = lane / LPR, lx0 = 2 * (lane % LPR);
    auto row_of = [&](int it) { return w * RW + it * RPI + sub; };
    auto row_in = [&](int R) { return R % CY < T.th && R / CY < T.td; };
    const int nbt = a.nb[T.tile];
    unsigned nbroot = 0;
    for (int k = threadIdx.x; k < nbt; k += NT3) {
        const int id = T.tile * CAP + k;
        const int r = a.gparent[id];  // resolved: the entry is the root
        const int32_t key = a.gkey[r];
        if constexpr (!LABEL) ST[k] = static_cast<uint8_t>(new_state(static_cast<uint32_t>(key), a));
        Rb[k] = key;
        nbroot += r == id ? 1u : 0u;
    }
    // the lane's codes (two per step); the interior roots (code CAP + own
    // slot) of the wave's rows are listed, then draw their states 64 at a time
    const uint16_t *codes = a.codes + static_cast<int64_t>(T.tile) * CSITES;
    uint32_t cc[ITER];
    int nroot = 0;
    uint16_t *mylist = roots[w];
    const uint64_t below = (1ull << lane) - 1ull;
#pragma unroll
    for (int it = 0; it < ITER; ++it) {
        const int R = row_of(it);
        const bool rin = row_in(R);
        const bool v0 = rin && lx0 < T.tw, v1 = rin && lx0 + 1 < T.tw;
        const int s = R * CX + lx0;
        cc[it] = rin ? *reinterpret_cast<const uint32_t *>(codes + s) : 0xFFFFFFFFu;
        const bool r0 = v0 && (cc[it] & 0xFFFFu) == static_cast<uint32_t>(CAP + s);
        const bool r1 = v1 && (cc[it] >> 16) == static_cast<uint32_t>(CAP + s + 1);
        const uint64_t m0 = __ballot(r0), m1 = __ballot(r1);
        const int at = nroot + __popcll(m0 & below) + __popcll(m1 & below);
        if (r0) mylist[at] = static_cast<uint16_t>(s);
        if (r1) mylist[at + (r0 ? 1 : 0)] = static_cast<uint16_t>(s + 1);
        nroot += __popcll(m0) + __popcll(m1);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    if constexpr (!LABEL) {
        for (int k = lane; k < nroot; k += 64) {
            const int s = mylist[k];
            ST[CAP + s] = static_cast<uint8_t>(new_state(static_cast<uint32_t>(site_of(g, T, s)), a));
        }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < ITER; ++it) {
        const int R = row_of(it), ly = R % CY, lz = R / CY;
        if (!row_in(R)) continue;
        const int64_t i0 = (static_cast<int64_t>(T.gz0 + lz) * g.Ly + T.gy0 + ly) * g.Lx + T.gx0 + lx0;
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            if (lx0 + j >= T.tw) continue;
            const uint32_t c = (cc[it] >> (16 * j)) & 0xFFFFu;
            if constexpr (!LABEL) {
                const uint32_t st = ST[c];
                a.spins[i0 + j] = static_cast<uint8_t>(a.ising ? 2u * st - 1u : st);
            }
            if (a.labels)
                a.labels[i0 + j] = c < static_cast<uint32_t>(CAP) ? Rb[c] : site_of(g, T, static_cast<int>(c) - CAP);
        }
    }
    const unsigned long long tot = wave_sum(nbroot);
    if (lane == 0) ncl_w[w] = static_cast<unsigned>(tot) + static_cast<unsigned>(nroot);
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned sum = 0;
        for (int k = 0; k < NW3; ++k) sum += ncl_w[k];
        a.tile_ncl[T.tile] = static_cast<int32_t>(sum);
    }
}

// The sweep's active bonds and clusters from the per-tile counts.
__global__ __launch_bounds__(1024) void k3_reduce_tiles(const int32_t *tile_act, const int32_t *tile_ncl, int ntiles,
                                                        unsigned long long *stats)
{
    __shared__ unsigned long long red[2][16];
    unsigned long long act = 0, ncl = 0;
    for (int t = threadIdx.x; t < ntiles; t += 1024) {
        act += static_cast<unsigned>(tile_act[t]);
        ncl += static_cast<unsigned>(tile_ncl[t]);
    }
    act = wave_sum(act);
    ncl = wave_sum(ncl);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) {
        red[0][w] = act;
        red[1][w] = ncl;
    }
    __syncthreads();
    if (threadIdx.x < 2) {
        unsigned long long v = 0;
        for (int k = 0; k < 16; ++k) v += red[threadIdx.x][k];
        stats[threadIdx.x == 0 ? S3_ACTIVE : S3_NCLUST] = v;
    }
}

// Satisfied bonds among the 3N pairs and state counts 0..7 of the spins
// (-H/J of Eq. potts_hamiltonian on the cubic lattice).
__global__ __launch_bounds__(512) void k3_observe(const uint8_t *spins, Geo3 g, int ising, unsigned long long *stats)
{
    // a wave per row segment of 64 sites, a lane per site: no division per site
    const uint32_t Lx = static_cast<uint32_t>(g.Lx), Ly = static_cast<uint32_t>(g.Ly);
    const uint32_t Lz = static_cast<uint32_t>(g.Lz);
    const uint32_t segs = (Lx + 63u) / 64u;
    const uint32_t nseg = Ly * Lz * segs;
    const uint32_t plane = Lx * Ly;
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t nwaves = gridDim.x * 8u;
    unsigned nsat = 0, cnt[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (uint32_t w = blockIdx.x * 8u + (threadIdx.x >> 6); w < nseg; w += nwaves) {
        const uint32_t row = w / segs, x = (w - row * segs) * 64u + lane;
        if (x >= Lx) continue;
        const uint32_t y = row % Ly, z = row / Ly;
        const uint32_t base = row * Lx;
        const uint32_t ry = y + 1u == Ly ? base - y * Lx : base + Lx;  // the row at y + 1
        const uint32_t rz = z + 1u == Lz ? y * Lx : base + plane;      // the row at z + 1
        const uint32_t s = spins[base + x];
        const uint32_t xn = x + 1u == Lx ? 0u : x + 1u;
        nsat += (s == spins[base + xn] ? 1u : 0u) + (s == spins[ry + x] ? 1u : 0u) + (s == spins[rz + x] ? 1u : 0u);
        const uint32_t st = ising ? (s == 1u ? 1u : 0u) : s;
#pragma unroll
        for (int k = 0; k < 8; ++k) cnt[k] += st == static_cast<uint32_t>(k) ? 1u : 0u;
    }
    // one atomic per counter and workgroup
    __shared__ unsigned long long red[9][8];
    const unsigned long long ns = wave_sum(nsat);
    if (lane == 0) red[0][threadIdx.x >> 6] = ns;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const unsigned long long c = wave_sum(cnt[k]);
        if (lane == 0) red[1 + k][threadIdx.x >> 6] = c;
    }
    __syncthreads();
    if (threadIdx.x < 9) {
        unsigned long long v = 0;
        for (int w = 0; w < 8; ++w) v += red[threadIdx.x][w];
        add_stat(&stats[threadIdx.x == 0 ? S3_NSAT : S3_COUNTS + threadIdx.x - 1], v);
    }
}

// The cluster count of a labeling into the caller's int32.
__global__ void k3_count_out(const unsigned long long *stats, int32_t *n_clusters)
{
    if (threadIdx.x == 0) *n_clusters = static_cast<int32_t>(stats[S3_NCLUST]);
}

// Move the sweep's counters into its record and clear them for the next one.
__global__ void k3_record(unsigned long long *stats, int64_t *row)
{
    const int k = threadIdx.x;
    if (k >= S3_LEN) return;
    if (row) row[k] = static_cast<int64_t>(stats[k]);
    stats[k] = 0ull;
}

}  // namespace cubic
}  // namespace swccl

using namespace swccl;
using namespace swccl::cubic;

namespace {

constexpr size_t ALIGN3 = 256;
size_t up3(size_t v) { return (v + ALIGN3 - 1) / ALIGN3 * ALIGN3; }
int64_t cdiv3(int64_t a, int64_t b) { return (a + b - 1) / b; }

struct Layout3 {
    Geo3 g;
    int64_t N;
    size_t codes, xface, gkey, gparent, nb, tile_act, tile_ncl, stats, bonds, total;
};

// Extents >= 1, N < 2^31, and the ids of all tiles (ntiles x CAP) index
// int32 arrays.
sw_status check_shape3(int32_t Lx, int32_t Ly, int32_t Lz)
{
    if (Lx < 1 || Ly < 1 || Lz < 1) return SW_ERR_SIZE;
    const int64_t N = static_cast<int64_t>(Lx) * Ly * Lz;
    if (N >= (static_cast<int64_t>(1) << 31)) return SW_ERR_SIZE;
    const int64_t nt = cdiv3(Lx, CX) * cdiv3(Ly, CY) * cdiv3(Lz, CZ);
    if (nt * CAP >= (static_cast<int64_t>(1) << 31)) return SW_ERR_SIZE;
    return SW_OK;
}

sw_status check3(const sw3_params *p)
{
    if (!p) return SW_ERR_ARG;
    if (p->q < 2 || p->q > 255) return SW_ERR_ARG;
    if (p->spin_kind != SW_SPIN_ISING_I8 && p->spin_kind != SW_SPIN_POTTS_U8) return SW_ERR_ARG;
    if (p->spin_kind == SW_SPIN_ISING_I8 && p->q != 2) return SW_ERR_ARG;
    if (std::isnan(p->K) || p->flags != 0 || p->reserved != 0) return SW_ERR_ARG;
    return check_shape3(p->Lx, p->Ly, p->Lz);
}

Layout3 layout3(int32_t Lx, int32_t Ly, int32_t Lz, bool own_bonds = true)
{
    Layout3 L{};
    L.g.Lx = Lx;
    L.g.Ly = Ly;
    L.g.Lz = Lz;
    L.g.ntx = static_cast<int>(cdiv3(Lx, CX));
    L.g.nty = static_cast<int>(cdiv3(Ly, CY));
    L.g.ntz = static_cast<int>(cdiv3(Lz, CZ));
    L.g.ntiles = L.g.ntx * L.g.nty * L.g.ntz;
    L.N = static_cast<int64_t>(Lx) * Ly * Lz;
    const size_t nt = static_cast<size_t>(L.g.ntiles);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off += up3(bytes);
        return at;
    };
    L.codes = take(nt * CSITES * sizeof(uint16_t));
    L.xface = take(nt * 2 * FX * sizeof(uint16_t));
    L.gkey = take(nt * CAP * sizeof(int32_t));
    L.gparent = take(nt * CAP * sizeof(int32_t));
    L.nb = take(nt * sizeof(int32_t));
    L.tile_act = take(nt * sizeof(int32_t));
    L.tile_ncl = take(nt * sizeof(int32_t));
    L.stats = take(16 * sizeof(unsigned long long));
    L.bonds = own_bonds ? take(static_cast<size_t>(L.N)) : 0;
    L.total = off;
    return L;
}

Layout3 layout3(const sw3_params *p) { return layout3(p->Lx, p->Ly, p->Lz); }

template <typename T>
T *at3(void *ws, size_t off)
{
    return reinterpret_cast<T *>(static_cast<char *>(ws) + off);
}

}  // namespace

extern "C" {

size_t sw3_workspace_bytes(const sw3_params *p)
{
    if (check3(p) != SW_OK) return 0;
    return layout3(p).total;
}

sw_status sw3_init_spins(const sw3_params *p, uint8_t *spins, void *stream)
{
    const sw_status st = check3(p);
    if (st != SW_OK) return st;
    if (!spins) return SW_ERR_ARG;
    const int64_t N = static_cast<int64_t>(p->Lx) * p->Ly * p->Lz;
    return swccl_internal::init_spins(spins, N, p->q, p->spin_kind == SW_SPIN_ISING_I8, p->seed, p->stream_id,
                                      static_cast<hipStream_t>(stream));
}

size_t ccl3_workspace_bytes(int32_t Lx, int32_t Ly, int32_t Lz)
{
    if (check_shape3(Lx, Ly, Lz) != SW_OK) return 0;
    return layout3(Lx, Ly, Lz, false).total;
}

sw_status ccl3_label(const uint8_t *bonds, int32_t Lx, int32_t Ly, int32_t Lz, int32_t *labels, int32_t *n_clusters,
                     void *workspace, size_t workspace_bytes, void *stream)
{
    const sw_status st = check_shape3(Lx, Ly, Lz);
    if (st != SW_OK) return st;
    if (!bonds || !labels) return SW_ERR_ARG;
    const Layout3 L = layout3(Lx, Ly, Lz, false);
    if (!workspace || workspace_bytes < L.total || reinterpret_cast<uintptr_t>(workspace) % ALIGN3)
        return SW_ERR_WORKSPACE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    unsigned long long *stats = at3<unsigned long long>(workspace, L.stats);
    Tile3Args ta{};
    ta.g = L.g;
    ta.bonds = const_cast<uint8_t *>(bonds);  // LABEL mode only reads them
    ta.codes = at3<uint16_t>(workspace, L.codes);
    ta.xface = at3<uint16_t>(workspace, L.xface);
    ta.gkey = at3<int32_t>(workspace, L.gkey);
    ta.gparent = at3<int32_t>(workspace, L.gparent);
    ta.nb = at3<int32_t>(workspace, L.nb);
    ta.tile_act = at3<int32_t>(workspace, L.tile_act);
    ta.tany = 1u;
    Merge3Args ma{};
    ma.g = L.g;
    ma.bonds = bonds;
    ma.codes = ta.codes;
    ma.xface = ta.xface;
    ma.gparent = ta.gparent;
    Resolve3Args ra{};
    ra.g = L.g;
    ra.gkey = ta.gkey;
    ra.gparent = ta.gparent;
    ra.nb = ta.nb;
    Flat3Args fa{};
    fa.g = L.g;
    fa.labels = labels;
    fa.codes = ta.codes;
    fa.gkey = ta.gkey;
    fa.gparent = ta.gparent;
    fa.nb = ta.nb;
    fa.tile_ncl = at3<int32_t>(workspace, L.tile_ncl);
    const dim3 tiles(static_cast<unsigned>(L.g.ntiles));
    hipLaunchKernelGGL(k3_tile<true>, tiles, dim3(NT3), 0, s, ta);
    hipLaunchKernelGGL(k3_merge, tiles, dim3(MT), 0, s, ma);
    hipLaunchKernelGGL(k3_resolve, tiles, dim3(RT), 0, s, ra);
    hipLaunchKernelGGL(k3_flatten<true>, tiles, dim3(NT3), 0, s, fa);
    if (n_clusters) {
        hipLaunchKernelGGL(k3_reduce_tiles, dim3(1), dim3(1024), 0, s, ta.tile_act, fa.tile_ncl, L.g.ntiles, stats);
        hipLaunchKernelGGL(k3_count_out, dim3(1), dim3(64), 0, s, stats, n_clusters);
    }
    return swccl_internal::device_error(hipGetLastError(), "ccl3_label");
}

sw_status sw3_sweep(const sw3_params *p, uint8_t *spins, uint32_t t0, int32_t n, uint8_t *bonds, int32_t *labels,
                    int64_t *records, void *workspace, size_t workspace_bytes, void *stream)
{
    const sw_status st = check3(p);
    if (st != SW_OK) return st;
    if (!spins || n < 0) return SW_ERR_ARG;
    if (static_cast<uint64_t>(t0) + static_cast<uint64_t>(n) > (static_cast<uint64_t>(1) << 32)) return SW_ERR_STATE;
    const Layout3 L = layout3(p);
    if (!workspace || workspace_bytes < L.total || reinterpret_cast<uintptr_t>(workspace) % ALIGN3)
        return SW_ERR_WORKSPACE;
    if (n == 0) return SW_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const uint64_t T = swccl_internal::bond_threshold(p->K);
    unsigned long long *stats = at3<unsigned long long>(workspace, L.stats);

    Tile3Args ta{};
    ta.g = L.g;
    ta.spins = spins;
    ta.bonds = bonds ? bonds : at3<uint8_t>(workspace, L.bonds);
    ta.codes = at3<uint16_t>(workspace, L.codes);
    ta.xface = at3<uint16_t>(workspace, L.xface);
    ta.gkey = at3<int32_t>(workspace, L.gkey);
    ta.gparent = at3<int32_t>(workspace, L.gparent);
    ta.nb = at3<int32_t>(workspace, L.nb);
    ta.tile_act = at3<int32_t>(workspace, L.tile_act);
    ta.tany = T > 0 ? 1u : 0u;
    ta.tm1 = T > 0 ? static_cast<uint32_t>(T - 1) : 0u;
    ta.k0 = static_cast<uint32_t>(p->seed);
    ta.k1 = static_cast<uint32_t>(p->seed >> 32);
    ta.sid = p->stream_id;

    Merge3Args ma{};
    ma.g = L.g;
    ma.bonds = ta.bonds;
    ma.codes = ta.codes;
    ma.xface = ta.xface;
    ma.gparent = ta.gparent;

    Flat3Args fa{};
    fa.g = L.g;
    fa.spins = spins;
    fa.codes = ta.codes;
    fa.gkey = ta.gkey;
    fa.gparent = ta.gparent;
    fa.nb = ta.nb;
    fa.tile_ncl = at3<int32_t>(workspace, L.tile_ncl);
    fa.q = static_cast<uint32_t>(p->q);
    fa.ising = p->spin_kind == SW_SPIN_ISING_I8 ? 1u : 0u;
    fa.k0 = ta.k0;
    fa.k1 = ta.k1;
    fa.sid = ta.sid;

    Resolve3Args ra{};
    ra.g = L.g;
    ra.gkey = ta.gkey;
    ra.gparent = ta.gparent;
    ra.nb = ta.nb;

    const dim3 tiles(static_cast<unsigned>(L.g.ntiles));
    const int64_t segs = static_cast<int64_t>(L.g.Ly) * L.g.Lz * cdiv3(L.g.Lx, 64);
    const unsigned obs_blocks = static_cast<unsigned>(std::min<int64_t>(cdiv3(segs, 8), 1024));
    hipLaunchKernelGGL(k3_record, dim3(1), dim3(64), 0, s, stats, static_cast<int64_t *>(nullptr));  // clear
    for (int32_t k = 0; k < n; ++k) {
        const uint32_t t = t0 + static_cast<uint32_t>(k);
        ta.t = t;
        fa.t = t;
        fa.labels = k + 1 == n ? labels : nullptr;
        hipLaunchKernelGGL(k3_tile<false>, tiles, dim3(NT3), 0, s, ta);
        hipLaunchKernelGGL(k3_merge, tiles, dim3(MT), 0, s, ma);
        hipLaunchKernelGGL(k3_resolve, tiles, dim3(RT), 0, s, ra);
        hipLaunchKernelGGL(k3_flatten<false>, tiles, dim3(NT3), 0, s, fa);
        if (records) {
            hipLaunchKernelGGL(k3_reduce_tiles, dim3(1), dim3(1024), 0, s, ta.tile_act, fa.tile_ncl, L.g.ntiles, stats);
            hipLaunchKernelGGL(k3_observe, dim3(obs_blocks), dim3(512), 0, s, spins, L.g, static_cast<int>(fa.ising),
                               stats);
            hipLaunchKernelGGL(k3_record, dim3(1), dim3(64), 0, s, stats, records + static_cast<int64_t>(k) * SW3_REC_LEN);
        }
    }
    return swccl_internal::device_error(hipGetLastError(), "sw3_sweep");
}

}  // extern "C"
