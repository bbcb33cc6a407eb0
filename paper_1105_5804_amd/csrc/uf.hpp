// uf.hpp -- device helpers shared by the square- and cubic-lattice kernels:
// XCD-aware workgroup placement, lane masks, the lock-free union-find in LDS
// (Sec. II.B.2) and the global union-find over boundary ids (Sec. II.C), wave
// reductions.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace swccl {

// Workgroups are dealt round-robin to the 8 XCDs.  Give each XCD one
// contiguous range of tiles so that tiles sharing halo lines share an L2.
__device__ __forceinline__ int xcd_remap(int b, int n)
{
    const int xcd = b & 7, local = b >> 3;
    const int q = n >> 3, r = n & 7;
    return xcd * q + min(xcd, r) + local;
}

// Bit `lane` of a wave-uniform mask m, for the calling lane: the mask is used
// as the lane condition directly (no per-lane shift).
__device__ __forceinline__ bool lane_bit(uint64_t m, int lane)
{
    (void)lane;
    return __builtin_amdgcn_inverse_ballot_w64(m);
}


// Value of x held by the next lane (DPP wave shift; the last lane gets 0).
__device__ __forceinline__ uint32_t from_next_lane(uint32_t x)
{
    return static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(x), 0x130, 0xF, 0xF, false));
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

// One step of a union of the trees holding a and b, with a straight-line body
// (nested find/link loops cost more in exec-mask bookkeeping than in LDS
// traffic).  A step climbs both nodes two levels (parent, then grandparent);
// when both are roots the larger is linked below the smaller with an atomic
// min, so every root is the minimum (local, hence global) index of its tree.
// If the larger root had meanwhile been linked elsewhere, the min leaves it
// below its old parent or below the smaller root, and the union goes on with
// that old parent, so no link is lost and every parent stays below its child.
// done is set when the two trees are one.  A lane with nothing to link spends
// its atomic on path halving: min(P[a], grandparent of a) points a at an
// ancestor (entries only ever decrease), which is a no-op when a or its
// parent is a root, so every lane issues the atomic and the step needs no
// branch; the halving keeps the trees shallow for later steps and for the
// compression that follows the unions.
// With BYTES the node values are byte offsets of the entries (4 x index), so
// a value is directly an LDS address.
template <bool BYTES = false>
__device__ __forceinline__ int *lds_entry(int *P, int v)
{
    return BYTES ? reinterpret_cast<int *>(reinterpret_cast<char *>(P) + v) : &P[v];
}

template <bool BYTES = false, bool SAME_PARENT = false>
__device__ __forceinline__ void unite_step(int *P, int &a, int &b, int &done)
{
    const int pa = lds_ld(lds_entry<BYTES>(P, a)), pb = lds_ld(lds_entry<BYTES>(P, b));
    const int ga = lds_ld(lds_entry<BYTES>(P, pa)), gb = lds_ld(lds_entry<BYTES>(P, pb));
    const bool roots = pa == a && pb == b;
    const bool link = roots && a != b;
    const int hi = max(a, b), lo = min(a, b);
    const int old = __hip_atomic_fetch_min(lds_entry<BYTES>(P, link ? hi : a), link ? lo : ga, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_WORKGROUP);
    // with SAME_PARENT a common parent already makes one tree: the union ends
    // a step before both nodes reach the root (whose entry every finished
    // lane would hit; the run-start unions of the tile kernel gain from it,
    // the site unions of the small-lattice kernel do not)
    // bitwise, not short-circuit: the flags stay lane masks (no selects)
    done = static_cast<int>((SAME_PARENT && pa == pb) | (roots & (!link | (old == hi))));
    a = link ? old : ga;
    b = link ? lo : gb;
}

// ---- global union-find over boundary ids ----
//
// Parents only move towards smaller keys, so a stale (older) parent read from
// a non-coherent L2 is still an ancestor: finds may use plain loads.  Every
// change of a root goes through a device-scope CAS; a failed CAS returns the
// node's current parent, from which the union continues.  Keys are the global
// site indices of the tile-local roots, so every final root's key is the
// minimum site index of its cluster.
__device__ __forceinline__ int gfind(const int *G, int x)
{
    for (;;) {
        const int p = G[x];
        if (p == x) return x;
        x = p;
    }
}

// Roots of a and b, both chains walked at once (their loads overlap); the
// body is straight-line, a finished chain just reloads its root.
__device__ __forceinline__ void gfind2(int *G, int &a, int &b)
{
    // path halving: a node passed over is pointed at its grandparent (an
    // ancestor, so concurrent walks stay valid), which keeps the trees of
    // clusters that span many tiles shallow
    int pa = G[a], pb = G[b];
    while (pa != a || pb != b) {
        const int ga = G[pa], gb = G[pb];
        if (ga != pa) G[a] = ga;
        if (gb != pb) G[b] = gb;
        a = ga;
        b = gb;
        pa = G[a];
        pb = G[b];
    }
}

__device__ __forceinline__ void gunite(int *G, const int *key, int a, int b)
{
    gfind2(G, a, b);
    for (;;) {
        if (a == b) return;
        const int ka = key[a], kb = key[b];
        if (ka < kb) {
            const int t = a;
            a = b;
            b = t;
        }
        int expect = a;
        if (__hip_atomic_compare_exchange_strong(&G[a], &expect, b, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT))
            return;
        a = expect;  // a was linked meanwhile: continue from its parent
        gfind2(G, a, b);
    }
}

__device__ __forceinline__ unsigned long long wave_sum(unsigned long long v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off);
    return v;
}

// Index of the calling wave in its workgroup, as a wave-uniform (scalar)
// value: everything derived from it (rows, row pointers, loop bounds) then
// stays in scalar registers and branches on it need no exec masking.
__device__ __forceinline__ int wave_id()
{
    return __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
}

// Maximum over the wave (valid in lane 0).
__device__ __forceinline__ int wave_max(int v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = max(v, __shfl_down(v, off));
    return v;
}

__device__ __forceinline__ void add_stat(unsigned long long *p, unsigned long long v)
{
    if (v) __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Keep the compiler from moving LDS accesses of one wave across this point
// (the DS unit executes one wave's LDS operations in order).
__device__ __forceinline__ void wave_lds_fence()
{
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
}

}  // namespace swccl
