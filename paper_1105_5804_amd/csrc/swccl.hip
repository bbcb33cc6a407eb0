// swccl.hip -- host side of the C ABI declared in include/swccl.h.
//
// Validates arguments, carves the caller's workspace, and enqueues the kernels
// of kernels.hpp on the caller's stream.  Allocates no device memory.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/swccl.h"
#include "internal.hpp"
#include "kernels.hpp"

using namespace swccl;

namespace {

thread_local std::string g_last_error;

constexpr size_t ALIGN = 256;
size_t align_up(size_t v) { return (v + ALIGN - 1) / ALIGN * ALIGN; }
int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Per-tile sizes of a tile shape (the Tile<TH> constants, on the host).
struct TileDims {
    int th, tsites, cap, edge, xw, nt;
};
TileDims dims_of(int th)
{
    return TileDims{th, TW * th, 2 * (TW + th), 2 * TW + 2 * th, (th + 63) / 64 + 2, 64 * (th / RPW)};
}
bool valid_tile_h(int32_t th) { return th == 16 || th == 32 || th == 64 || th == 128; }
bool valid_merge_waves(int32_t mw) { return mw == 4 || mw == 8 || mw == 16; }
constexpr int MERGE_WAVES_DEFAULT = 8;

// Calls f with the tile height as a compile-time constant.
template <typename F>
void with_tile_h(int th, F &&f)
{
    switch (th) {
    case 16: f(std::integral_constant<int, 16>{}); break;
    case 32: f(std::integral_constant<int, 32>{}); break;
    case 128: f(std::integral_constant<int, 128>{}); break;
    default: f(std::integral_constant<int, 64>{}); break;
    }
}

struct Layout {
    Grid g;
    TileDims d;       // tile shape
    int mw;           // merge workgroup: tiles (waves) per workgroup
    bool sizes;
    int64_t nrow;  // H * ntx: entries of the per-(row, tile column) root counts
    size_t codes, gkey, gparent, gsize, edges, xbits, nb, tile_act, tile_ncl, stats;
    size_t row_count, row_off, scan_tmp, rl_slot, rl_size;
    size_t lat_desc, lat_of_tile, t_dev;  // batches only
    size_t small_lat, ftile, mgroup, counters, fault;  // fused batch sweeps
    size_t sel, seedmap;  // few-cluster sweeps: seed marks per root id, seed bits per interior root slot
    bool few;
    size_t total;
};

// Scratch for the multi-level exclusive scan of n values: two arrays of block
// totals per level.
size_t scan_tmp_bytes(int64_t n)
{
    size_t b = 0;
    while (true) {
        const int64_t nb = cdiv(n, SCAN_ITEMS);
        if (nb <= 1) break;
        b += align_up(static_cast<size_t>(nb) * 4) * 2;
        n = nb;
    }
    return b + ALIGN;
}

// N = W H < 2^31, and the boundary ids of all tiles (ntiles x CAP) index int32
// arrays: a very thin lattice has far more tiles than sites / TSITES.
bool valid_shape(int32_t W, int32_t H, int32_t min_side, int th = TH_DEFAULT)
{
    if (W < min_side || H < min_side) return false;
    if (static_cast<int64_t>(W) * H >= (static_cast<int64_t>(1) << 31)) return false;
    return cdiv(W, TW) * cdiv(H, th) * dims_of(th).cap < (static_cast<int64_t>(1) << 31);
}

// Per-tile arrays shared by single lattices and batches; returns the bytes used.
size_t carve_tiles(Layout &L, size_t nt)
{
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off += align_up(bytes);
        return at;
    };
    const TileDims &d = L.d;
    L.codes = take(nt * static_cast<size_t>(d.tsites) * sizeof(uint16_t));
    L.gkey = take(nt * static_cast<size_t>(d.cap) * sizeof(int32_t));
    L.gparent = take(nt * static_cast<size_t>(d.cap) * sizeof(int32_t));
    L.edges = take(nt * static_cast<size_t>(d.edge) * sizeof(uint16_t));
    L.xbits = take(nt * static_cast<size_t>(d.xw) * sizeof(uint64_t));
    L.nb = take(nt * sizeof(int32_t));
    L.tile_act = take(nt * sizeof(int32_t));
    L.tile_ncl = take(nt * sizeof(int32_t));
    L.stats = take(ST_LEN * sizeof(unsigned long long));
    return off;
}

Layout make_layout(int32_t W, int32_t H, bool sizes, int th = TH_DEFAULT, int mw = MERGE_WAVES_DEFAULT,
                   bool few = false)
{
    Layout L{};
    L.d = dims_of(th);
    L.mw = mw;
    L.g.W = W;
    L.g.H = H;
    L.g.ntx = static_cast<int>(cdiv(W, TW));
    L.g.nty = static_cast<int>(cdiv(H, th));
    L.g.ntiles = L.g.ntx * L.g.nty;
    L.sizes = sizes;
    L.nrow = static_cast<int64_t>(H) * L.g.ntx;
    size_t off = carve_tiles(L, static_cast<size_t>(L.g.ntiles));
    const size_t nt = static_cast<size_t>(L.g.ntiles);
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off += align_up(bytes);
        return at;
    };
    if (sizes) {
        L.gsize = take(nt * static_cast<size_t>(L.d.cap) * sizeof(int32_t));
        // per-(row, tile column) root counts, their total, then the largest size
        L.row_count = take(static_cast<size_t>(L.nrow + 2) * sizeof(int32_t));
        L.row_off = take(static_cast<size_t>(L.nrow + 1) * sizeof(int32_t));
        L.scan_tmp = take(scan_tmp_bytes(L.nrow + 1));
        L.rl_slot = take(nt * static_cast<size_t>(L.d.tsites) * sizeof(int32_t));
        L.rl_size = take(nt * static_cast<size_t>(L.d.tsites) * sizeof(int32_t));
    }
    L.few = few;
    if (few) {
        L.sel = take(nt * static_cast<size_t>(L.d.cap) * sizeof(uint32_t));
        L.seedmap = take(nt * static_cast<size_t>(L.d.tsites / 32) * sizeof(uint32_t));
    }
    L.total = off;
    return L;
}

// Workspace of a batch of lattices: the tile arrays over all their tiles,
// then the lattice descriptors and the tile -> lattice table.
Layout make_batch_layout(int64_t ntiles, int32_t nlat, int th, int mw)
{
    Layout L{};
    L.d = dims_of(th);
    L.mw = mw;
    L.g.ntiles = static_cast<int>(ntiles);
    size_t off = carve_tiles(L, static_cast<size_t>(ntiles));
    L.lat_desc = off;
    off += align_up(static_cast<size_t>(nlat) * sizeof(LatticeDesc));
    L.lat_of_tile = off;
    off += align_up(static_cast<size_t>(ntiles) * sizeof(int32_t));
    L.t_dev = off;
    off += align_up(sizeof(uint32_t));
    // fused sweeps: the work-queue tables, then the counters (ticket, exit
    // count, per-lattice tiles and merge groups done) and the fault flag
    L.small_lat = off;
    off += align_up(static_cast<size_t>(nlat) * sizeof(int32_t));
    L.ftile = off;
    off += align_up(static_cast<size_t>(ntiles) * sizeof(int32_t));
    L.mgroup = off;
    off += align_up(static_cast<size_t>(ntiles) * sizeof(int2));
    L.counters = off;
    off += align_up((2 + 2 * static_cast<size_t>(nlat)) * sizeof(unsigned long long));
    L.fault = off;
    off += align_up(sizeof(int32_t));
    L.total = off;
    return L;
}


template <typename T>
T *at(void *ws, size_t off)
{
    return reinterpret_cast<T *>(static_cast<char *>(ws) + off);
}

sw_status device_status(hipError_t e, const char *where)
{
    if (e == hipSuccess) return SW_OK;
    g_last_error = std::string(where) + ": " + hipGetErrorString(e);
    return SW_ERR_DEVICE;
}

sw_status launch_status(const char *where) { return device_status(hipGetLastError(), where); }

// Exclusive scan of n int32 values (in -> out) with block totals in tmp.
void scan_i32(const int32_t *in, int32_t *out, int64_t n, char *tmp, hipStream_t s)
{
    const int64_t nb = cdiv(n, SCAN_ITEMS);
    if (nb <= 1) {
        hipLaunchKernelGGL(k_scan_block, dim3(1), dim3(NT), 0, s, in, out, n, nullptr);
        return;
    }
    int32_t *tot = reinterpret_cast<int32_t *>(tmp);
    int32_t *tot_off = reinterpret_cast<int32_t *>(tmp + align_up(static_cast<size_t>(nb) * 4));
    char *next = tmp + 2 * align_up(static_cast<size_t>(nb) * 4);
    hipLaunchKernelGGL(k_scan_block, dim3(static_cast<unsigned>(nb)), dim3(NT), 0, s, in, out, n, tot);
    scan_i32(tot, tot_off, nb, next, s);
    hipLaunchKernelGGL(k_scan_add, dim3(static_cast<unsigned>(cdiv(n, NT))), dim3(NT), 0, s, out, n, tot_off);
}

TileArgs tile_args(const Layout &L, void *ws, const uint8_t *in)
{
    TileArgs a{};
    a.g = L.g;
    a.in = in;
    a.codes = at<uint16_t>(ws, L.codes);
    a.gkey = at<int32_t>(ws, L.gkey);
    a.gparent = at<int32_t>(ws, L.gparent);
    a.gsize = L.sizes ? at<int32_t>(ws, L.gsize) : nullptr;
    a.edges = at<uint16_t>(ws, L.edges);
    a.xbits = at<uint64_t>(ws, L.xbits);
    a.nb = at<int32_t>(ws, L.nb);
    a.tile_act = at<int32_t>(ws, L.tile_act);
    return a;
}

MergeArgs merge_args(const Layout &L, void *ws)
{
    MergeArgs m{};
    m.g = L.g;
    m.edges = at<uint16_t>(ws, L.edges);
    m.xbits = at<uint64_t>(ws, L.xbits);
    m.gkey = at<int32_t>(ws, L.gkey);
    m.gparent = at<int32_t>(ws, L.gparent);
    return m;
}

// Even W keeps every row start even: one 16-bit load per lane pair.
template <int MODE>
void launch_tile(const Layout &L, const TileArgs &ta, hipStream_t s)
{
    with_tile_h(L.d.th, [&](auto c) {
        constexpr int TH = decltype(c)::value;
        const dim3 grid(static_cast<unsigned>(L.g.ntiles)), block(Tile<TH>::NT);
        if (L.g.W % 2 == 0)
            hipLaunchKernelGGL((k_tile<MODE, true, false, TH>), grid, block, 0, s, ta);
        else
            hipLaunchKernelGGL((k_tile<MODE, false, false, TH>), grid, block, 0, s, ta);
    });
}

// The merge: mw tiles per workgroup, one wave each, over ntiles tiles.
template <bool BATCH>
void launch_merge(const Layout &L, const MergeArgs &ma, int64_t ntiles, hipStream_t s)
{
    const dim3 grid(static_cast<unsigned>(cdiv(ntiles, L.mw))), block(static_cast<unsigned>(64 * L.mw));
    with_tile_h(L.d.th, [&](auto c) {
        constexpr int TH = decltype(c)::value;
        hipLaunchKernelGGL((k_merge<BATCH, TH>), grid, block, 0, s, ma);
    });
}

template <int MODE, bool SIZES, bool BATCH>
void launch_flatten(const Layout &L, const FlatArgs &fa, int64_t ntiles, hipStream_t s)
{
    with_tile_h(L.d.th, [&](auto c) {
        constexpr int TH = decltype(c)::value;
        hipLaunchKernelGGL((k_flatten<MODE, SIZES, BATCH, TH>), dim3(static_cast<unsigned>(ntiles)),
                           dim3(Tile<TH>::NT), 0, s, fa);
    });
}

FlatArgs flat_args(const Layout &L, void *ws)
{
    FlatArgs f{};
    f.g = L.g;
    f.codes = at<uint16_t>(ws, L.codes);
    f.gkey = at<int32_t>(ws, L.gkey);
    f.gparent = at<int32_t>(ws, L.gparent);
    f.nb = at<int32_t>(ws, L.nb);
    f.tile_ncl = at<int32_t>(ws, L.tile_ncl);
    if (L.sizes) {
        f.gsize = at<int32_t>(ws, L.gsize);
        f.row_count = at<int32_t>(ws, L.row_count);
        f.rl_slot = at<int32_t>(ws, L.rl_slot);
        f.rl_size = at<int32_t>(ws, L.rl_size);
    }
    return f;
}

// Roots in ascending order and their sizes from a flatten pass with sizes:
// scan the per-(row, tile column) root counts, then place each tile's roots.
void emit_sizes(const Layout &L, void *ws, const FlatArgs &fa, int32_t *roots, int32_t *sizes, int32_t *max_size,
                int32_t *n_clusters, hipStream_t s)
{
    int32_t *row_off = at<int32_t>(ws, L.row_off);
    scan_i32(fa.row_count, row_off, L.nrow + 1, at<char>(ws, L.scan_tmp), s);
    EmitArgs ea{};
    ea.g = L.g;
    ea.row_off = row_off;
    ea.rl_slot = fa.rl_slot;
    ea.rl_size = fa.rl_size;
    ea.gsize = fa.gsize;
    ea.roots = roots;
    ea.sizes = sizes;
    ea.max_size = max_size;
    ea.n_clusters = n_clusters;
    with_tile_h(L.d.th, [&](auto c) {
        constexpr int TH = decltype(c)::value;
        hipLaunchKernelGGL(k_emit<TH>, dim3(static_cast<unsigned>(L.g.ntiles)), dim3(NT), 0, s, ea);
    });
}

uint64_t threshold_of(double K)
{
    if (!(K > 0.0)) return 0;
    const double p = -std::expm1(-K);
    const double v = std::floor(std::ldexp(p, 32));
    if (v >= 4294967296.0) return 4294967296ull;
    if (v <= 0.0) return 0;
    return static_cast<uint64_t>(v);
}

}  // namespace

struct sw_lattice {
    sw_params p;
    sw_buffers b;
    Layout L;
    uint64_t T;
    uint64_t t;
    bool swept;       // at least one sweep since init / set_t
    bool small_last;  // the last sweep ran in k_small (its counters are in tile 0 alone)
    bool sel_stale;   // few-cluster: the seed marks must be cleared before the next flip
    uint32_t tflip;   // few-cluster: floor(p_flip 2^32)
    int32_t next_phase;  // SW_PHASE_* expected next
};

extern "C" {

int32_t swccl_abi_version(void) { return SWCCL_ABI_VERSION; }

const char *sw_status_string(sw_status s)
{
    switch (s) {
    case SW_OK: return "ok";
    case SW_ERR_ARG: return "invalid argument";
    case SW_ERR_SIZE: return "invalid lattice size";
    case SW_ERR_WORKSPACE: return "workspace missing or too small";
    case SW_ERR_DEVICE: return "device error";
    case SW_ERR_STATE: return "invalid state";
    case SW_ERR_UNSUPPORTED: return "unsupported";
    case SW_ERR_HOST_MEMORY: return "host memory allocation failed";
    default: return "unknown status";
    }
}

const char *sw_last_error(void) { return g_last_error.c_str(); }

uint64_t sw_threshold(double K) { return threshold_of(K); }

static int tile_h_of(const sw_params *p) { return p->tile_h ? p->tile_h : TH_DEFAULT; }
static int merge_waves_of(const sw_params *p) { return p->merge_waves ? p->merge_waves : MERGE_WAVES_DEFAULT; }

static sw_status check_params(const sw_params *p, uint32_t extra_flags = 0)
{
    if (!p) return SW_ERR_ARG;
    if (p->W < 2 || p->H < 2 || static_cast<int64_t>(p->W) * p->H >= (static_cast<int64_t>(1) << 31))
        return SW_ERR_SIZE;
    if (p->q < 2 || p->q > 255) return SW_ERR_ARG;
    if (p->spin_kind != SW_SPIN_ISING_I8 && p->spin_kind != SW_SPIN_POTTS_U8) return SW_ERR_ARG;
    if (p->spin_kind == SW_SPIN_ISING_I8 && p->q != 2) return SW_ERR_ARG;
    if (std::isnan(p->K)) return SW_ERR_ARG;
    if (p->flags & ~(static_cast<uint32_t>(SW_F_KEEP_SPINS | SW_F_SIZES | SW_F_REVERSE_TILES) | extra_flags))
        return SW_ERR_ARG;
    if (p->tile_h != 0 && !valid_tile_h(p->tile_h)) return SW_ERR_ARG;
    if (p->merge_waves != 0 && !valid_merge_waves(p->merge_waves)) return SW_ERR_ARG;
    if (p->reserved != 0 || p->few_b < 0) return SW_ERR_ARG;
    if (p->few_b > 0 && (p->q != 2 || !(p->p_flip >= 0.0 && p->p_flip < 1.0))) return SW_ERR_ARG;
    if (!valid_shape(p->W, p->H, 2, tile_h_of(p))) return SW_ERR_SIZE;
    return SW_OK;
}

// floor(p 2^32) for a probability 0 <= p < 1.
static uint32_t prob_threshold(double p)
{
    if (!(p > 0.0)) return 0;
    const double v = std::floor(std::ldexp(p, 32));
    return v >= 4294967295.0 ? 0xFFFFFFFFu : static_cast<uint32_t>(v);
}

static Layout layout_of(const sw_params *p)
{
    return make_layout(p->W, p->H, (p->flags & SW_F_SIZES) != 0, tile_h_of(p), merge_waves_of(p), p->few_b > 0);
}

size_t sw_workspace_bytes(const sw_params *p)
{
    if (check_params(p) != SW_OK) return 0;
    return layout_of(p).total;
}

sw_status sw_init(sw_lattice **out, const sw_params *p, const sw_buffers *b, void *stream)
{
    if (!out || !b) return SW_ERR_ARG;
    const sw_status ps = check_params(p);
    if (ps != SW_OK) return ps;
    if (!b->spins) return SW_ERR_ARG;
    const bool sizes = (p->flags & SW_F_SIZES) != 0;
    if (sizes && (!b->roots || !b->sizes)) return SW_ERR_ARG;
    const Layout L = layout_of(p);
    if (!b->workspace || b->workspace_bytes < L.total) return SW_ERR_WORKSPACE;
    if (reinterpret_cast<uintptr_t>(b->workspace) % ALIGN) return SW_ERR_WORKSPACE;
    sw_lattice *h = new (std::nothrow) sw_lattice();
    if (!h) return SW_ERR_HOST_MEMORY;
    h->p = *p;
    h->b = *b;
    h->L = L;
    h->L.g.rev = (p->flags & SW_F_REVERSE_TILES) ? 1 : 0;
    h->T = threshold_of(p->K);
    h->t = 0;
    h->swept = false;
    h->sel_stale = L.few;  // the workspace holds anything: clear the marks before the first flip
    h->tflip = prob_threshold(p->p_flip);
    h->next_phase = SW_PHASE_TILE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t N = static_cast<int64_t>(p->W) * p->H;
    if (!(p->flags & SW_F_KEEP_SPINS)) {
        const int64_t nthreads = cdiv(N, 4);
        hipLaunchKernelGGL(k_init, dim3(static_cast<unsigned>(cdiv(nthreads, NT))), dim3(NT), 0, s,
                           static_cast<uint8_t *>(b->spins), N, static_cast<uint32_t>(p->q),
                           p->spin_kind == SW_SPIN_ISING_I8 ? 1 : 0, static_cast<uint32_t>(p->seed),
                           static_cast<uint32_t>(p->seed >> 32), p->stream_id);
        const sw_status st = launch_status("k_init");
        if (st != SW_OK) {
            delete h;
            return st;
        }
    }
    *out = h;
    return SW_OK;
}

// Few-cluster sweeps: one thread per seed tile marks the root id of a seeded
// boundary cluster with t + 1, or the root slot of a seeded interior cluster
// in its tile's seed map (the flatten clears the map as it reads it).  The
// marks are cleared first after init and after sw_set_t (a sweep number may
// then come round again).
static sw_status launch_seeds(sw_lattice *h, hipStream_t s)
{
    const Layout &L = h->L;
    void *ws = h->b.workspace;
    if (h->sel_stale) {
        const int64_t nsel = L.g.ntiles * static_cast<int64_t>(L.d.cap);
        const int64_t nmap = L.g.ntiles * static_cast<int64_t>(L.d.tsites / 32);
        hipLaunchKernelGGL(k_zero_i32, dim3(static_cast<unsigned>(cdiv(nsel, NT))), dim3(NT), 0, s,
                           at<int32_t>(ws, L.sel), static_cast<int>(nsel));
        hipLaunchKernelGGL(k_zero_i32, dim3(static_cast<unsigned>(cdiv(nmap, NT))), dim3(NT), 0, s,
                           at<int32_t>(ws, L.seedmap), static_cast<int>(nmap));
        const sw_status st = launch_status("k_zero_i32");
        if (st != SW_OK) return st;
        h->sel_stale = false;
    }
    SeedArgs sa{};
    sa.g = L.g;
    sa.codes = at<uint16_t>(ws, L.codes);
    sa.gparent = at<int32_t>(ws, L.gparent);
    sa.sel = at<uint32_t>(ws, L.sel);
    sa.seedmap = at<uint32_t>(ws, L.seedmap);
    sa.t = static_cast<uint32_t>(h->t);
    sa.stamp = sa.t + 1u;
    sa.sid = h->p.stream_id;
    sa.k0 = static_cast<uint32_t>(h->p.seed);
    sa.k1 = static_cast<uint32_t>(h->p.seed >> 32);
    sa.few_b = h->p.few_b;
    sa.few_ntx = static_cast<int>(cdiv(h->p.W, h->p.few_b));
    const int64_t nseed = sa.few_ntx * cdiv(h->p.H, h->p.few_b);
    sa.nseed = static_cast<int>(nseed);
    with_tile_h(L.d.th, [&](auto c) {
        constexpr int TH = decltype(c)::value;
        hipLaunchKernelGGL(k_seed<TH>, dim3(static_cast<unsigned>(cdiv(nseed, NT))), dim3(NT), 0, s, sa);
    });
    return launch_status("k_seed");
}

// Enqueue one phase of sweep h->t.
static sw_status launch_phase(sw_lattice *h, int32_t phase, hipStream_t s)
{
    const Layout &L = h->L;
    void *ws = h->b.workspace;
    const uint32_t k0 = static_cast<uint32_t>(h->p.seed), k1 = static_cast<uint32_t>(h->p.seed >> 32);
    const uint32_t t = static_cast<uint32_t>(h->t);
    if (phase == SW_PHASE_TILE) {
        TileArgs ta = tile_args(L, ws, static_cast<const uint8_t *>(h->b.spins));
        ta.bonds_out = h->b.bonds;
        ta.tany = h->T > 0 ? 1u : 0u;
        ta.tm1 = h->T > 0 ? static_cast<uint32_t>(h->T - 1) : 0u;
        ta.k0 = k0;
        ta.k1 = k1;
        for (uint32_t r = 0; r < 10; ++r) {  // Philox's key schedule: the Weyl increments added r times
            ta.rk[2 * r] = k0 + r * 0x9E3779B9u;
            ta.rk[2 * r + 1] = k1 + r * 0xBB67AE85u;
        }
        ta.t = t;
        ta.sid = h->p.stream_id;
        launch_tile<M_SW>(L, ta, s);
        return launch_status("k_tile");
    }
    if (phase == SW_PHASE_MERGE) {
        launch_merge<false>(L, merge_args(L, ws), L.g.ntiles, s);
        return launch_status("k_merge");
    }
    FlatArgs fa = flat_args(L, ws);
    fa.spins = static_cast<uint8_t *>(h->b.spins);
    fa.labels = h->b.labels;
    fa.q = static_cast<uint32_t>(h->p.q);
    fa.k0 = k0;
    fa.k1 = k1;
    fa.t = t;
    fa.sid = h->p.stream_id;
    fa.ising = h->p.spin_kind == SW_SPIN_ISING_I8 ? 1 : 0;
    if (L.few) {
        // few-cluster flip: mark the boundary clusters that hold a seed, then
        // flatten with the seeded clusters' flips
        const sw_status st = launch_seeds(h, s);
        if (st != SW_OK) return st;
        fa.sel = at<uint32_t>(ws, L.sel);
        fa.seedmap = at<uint32_t>(ws, L.seedmap);
        fa.stamp = t + 1u;
        fa.tflip = h->tflip;
        if (!L.sizes) {
            launch_flatten<M_FEW, false, false>(L, fa, L.g.ntiles, s);
            return launch_status("k_flatten");
        }
        launch_flatten<M_FEW, true, false>(L, fa, L.g.ntiles, s);
        emit_sizes(L, ws, fa, h->b.roots, h->b.sizes, fa.row_count + L.nrow + 1, nullptr, s);
        return launch_status("k_flatten");
    }
    if (!L.sizes) {
        launch_flatten<M_SW, false, false>(L, fa, L.g.ntiles, s);
        return launch_status("k_flatten");
    }
    launch_flatten<M_SW, true, false>(L, fa, L.g.ntiles, s);
    emit_sizes(L, ws, fa, h->b.roots, h->b.sizes, fa.row_count + L.nrow + 1, nullptr, s);
    return launch_status("k_flatten");
}

sw_status sw_sweep_phase(sw_lattice *h, int32_t phase, void *stream)
{
    if (!h || phase < SW_PHASE_TILE || phase > SW_PHASE_FLIP) return SW_ERR_ARG;
    if (phase != h->next_phase) return SW_ERR_STATE;
    if (phase == SW_PHASE_TILE && h->t >= 0xFFFFFFFFull) return SW_ERR_STATE;
    const sw_status st = launch_phase(h, phase, static_cast<hipStream_t>(stream));
    if (st != SW_OK) return st;
    if (phase == SW_PHASE_FLIP) {
        h->next_phase = SW_PHASE_TILE;
        h->t += 1;
        h->swept = true;
        h->small_last = false;
    } else {
        h->next_phase = phase + 1;
    }
    return SW_OK;
}

// A lattice of one tile is swept by k_small, all sweeps in one launch (the
// per-phase entry point keeps the tiled path; both give the same results).
static bool small_path(const sw_lattice *h)
{
    return h->p.W <= SMALL_W && h->p.H <= SMALL_H && !h->L.sizes && !h->L.few;
}

static sw_status launch_small(sw_lattice *h, int32_t n, int64_t *hist, hipStream_t s)
{
    const Layout &L = h->L;
    void *ws = h->b.workspace;
    SmallArgs a{};
    a.W = h->p.W;
    a.H = h->p.H;
    a.spins = static_cast<uint8_t *>(h->b.spins);
    a.bonds_out = h->b.bonds;
    a.labels = h->b.labels;
    a.hist = hist;
    a.tile_act = at<int32_t>(ws, L.tile_act);
    a.tile_ncl = at<int32_t>(ws, L.tile_ncl);
    a.tany = h->T > 0 ? 1u : 0u;
    a.tm1 = h->T > 0 ? static_cast<uint32_t>(h->T - 1) : 0u;
    a.k0 = static_cast<uint32_t>(h->p.seed);
    a.k1 = static_cast<uint32_t>(h->p.seed >> 32);
    a.sid = h->p.stream_id;
    a.q = static_cast<uint32_t>(h->p.q);
    a.t0 = static_cast<uint32_t>(h->t);
    a.ising = h->p.spin_kind == SW_SPIN_ISING_I8 ? 1 : 0;
    a.n = n;
    hipLaunchKernelGGL(k_small, dim3(1), dim3(SMALL_NT), 0, s, a);
    return launch_status("k_small");
}

sw_status sw_sweep(sw_lattice *h, int32_t n_sweeps, void *stream)
{
    if (!h || n_sweeps < 0) return SW_ERR_ARG;
    if (h->next_phase != SW_PHASE_TILE) return SW_ERR_STATE;
    if (h->t + static_cast<uint64_t>(n_sweeps) > 0xFFFFFFFFull) return SW_ERR_STATE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (n_sweeps > 0 && small_path(h)) {
        const sw_status st = launch_small(h, n_sweeps, nullptr, s);
        if (st != SW_OK) return st;
        h->t += static_cast<uint64_t>(n_sweeps);
        h->swept = true;
        h->small_last = true;
        return SW_OK;
    }
    for (int32_t n = 0; n < n_sweeps; ++n) {
        for (int32_t ph = SW_PHASE_TILE; ph <= SW_PHASE_FLIP; ++ph) {
            const sw_status st = launch_phase(h, ph, s);
            if (st != SW_OK) return st;
        }
        h->t += 1;
        h->swept = true;
        h->small_last = false;
    }
    return SW_OK;
}

// Observables of one lattice (spins, digests, and the last sweep's per-tile
// counters tile_act / tile_ncl of its ntiles tiles); waits for the stream.
static sw_status measure(const sw_params &p, const sw_buffers &b, bool swept, const int32_t *tile_act,
                         const int32_t *tile_ncl, int ntiles, unsigned long long *obs, const int32_t *max_size_dev,
                         uint64_t T, uint64_t t, sw_obs *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, s, obs, ST_LEN);
    const int64_t N = static_cast<int64_t>(p.W) * p.H;
    const unsigned blocks = static_cast<unsigned>(std::min<int64_t>(p.H, 2048));
    const int ising = p.spin_kind == SW_SPIN_ISING_I8 ? 1 : 0;
    hipLaunchKernelGGL(k_observe, dim3(blocks), dim3(NT), 0, s, static_cast<const uint8_t *>(b.spins), p.W, p.H,
                       static_cast<uint32_t>(p.q), ising, obs);
    if (swept) {
        const unsigned rb = static_cast<unsigned>(std::min<int64_t>(cdiv(ntiles, NT), 64));
        hipLaunchKernelGGL(k_reduce_tiles, dim3(rb), dim3(NT), 0, s, tile_act, ntiles, obs + ST_ACTIVE,
                           static_cast<int32_t *>(nullptr));
        hipLaunchKernelGGL(k_reduce_tiles, dim3(rb), dim3(NT), 0, s, tile_ncl, ntiles, obs + ST_NCLUST,
                           static_cast<int32_t *>(nullptr));
    }
    const unsigned db = static_cast<unsigned>(std::min<int64_t>(cdiv(N, NT), 4096));
    if (ising)
        hipLaunchKernelGGL(k_digest<DIG_ISING_I8>, dim3(db), dim3(NT), 0, s, b.spins, N, obs + ST_DIGEST);
    else
        hipLaunchKernelGGL(k_digest<DIG_U8>, dim3(db), dim3(NT), 0, s, b.spins, N, obs + ST_DIGEST);
    if (swept && b.labels)
        hipLaunchKernelGGL(k_digest<DIG_I32>, dim3(db), dim3(NT), 0, s, b.labels, N, obs + ST_DIGEST + 1);
    if (swept && b.bonds)
        hipLaunchKernelGGL(k_digest<DIG_U8>, dim3(db), dim3(NT), 0, s, b.bonds, N, obs + ST_DIGEST + 2);
    sw_status st = launch_status("observables");
    if (st != SW_OK) return st;
    unsigned long long host[ST_LEN];
    int32_t max_size = -1;
    st = device_status(hipMemcpyAsync(host, obs, sizeof(host), hipMemcpyDeviceToHost, s), "copy observables");
    if (st != SW_OK) return st;
    if (max_size_dev && swept) {
        st = device_status(hipMemcpyAsync(&max_size, max_size_dev, sizeof(max_size), hipMemcpyDeviceToHost, s),
                           "copy max size");
        if (st != SW_OK) return st;
    }
    st = device_status(hipStreamSynchronize(s), "sync");
    if (st != SW_OK) return st;
    std::memset(out, 0, sizeof(*out));
    out->t = t;
    out->threshold = T;
    out->n_sat = static_cast<int64_t>(host[ST_NSAT]);
    for (int k = 0; k < 8; ++k) out->counts[k] = k < p.q ? static_cast<int64_t>(host[ST_COUNTS + k]) : 0;
    out->magnet = ising ? 2 * out->counts[1] - N : 0;
    out->n_active_bonds = swept ? static_cast<int64_t>(host[ST_ACTIVE]) : -1;
    out->n_clusters = swept ? static_cast<int64_t>(host[ST_NCLUST]) : -1;
    out->max_cluster = (max_size_dev && swept) ? max_size : -1;
    out->digest_spins = host[ST_DIGEST];
    out->digest_labels = host[ST_DIGEST + 1];
    out->digest_bonds = host[ST_DIGEST + 2];
    return SW_OK;
}

sw_status sw_observables(sw_lattice *h, sw_obs *out, void *stream)
{
    if (!h || !out) return SW_ERR_ARG;
    const Layout &L = h->L;
    void *ws = h->b.workspace;
    const int32_t *max_dev = L.sizes ? at<int32_t>(ws, L.row_count) + L.nrow + 1 : nullptr;
    return measure(h->p, h->b, h->swept, at<int32_t>(ws, L.tile_act), at<int32_t>(ws, L.tile_ncl),
                   h->small_last ? 1 : L.g.ntiles,
                   at<unsigned long long>(ws, L.stats), max_dev, h->T, h->t, out, static_cast<hipStream_t>(stream));
}

sw_status sw_sweep_history(sw_lattice *h, int32_t n_sweeps, int64_t *history, void *stream)
{
    if (!h || n_sweeps < 0 || (n_sweeps > 0 && !history)) return SW_ERR_ARG;
    if (h->next_phase != SW_PHASE_TILE) return SW_ERR_STATE;
    if (h->t + static_cast<uint64_t>(n_sweeps) > 0xFFFFFFFFull) return SW_ERR_STATE;
    if (n_sweeps == 0) return SW_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (small_path(h)) {
        const sw_status st = launch_small(h, n_sweeps, history, s);
        if (st != SW_OK) return st;
        h->t += static_cast<uint64_t>(n_sweeps);
        h->swept = true;
        h->small_last = true;
        return SW_OK;
    }
    const Layout &L = h->L;
    void *ws = h->b.workspace;
    unsigned long long *obs = at<unsigned long long>(ws, L.stats);
    const int32_t *max_dev = L.sizes ? at<int32_t>(ws, L.row_count) + L.nrow + 1 : nullptr;
    const unsigned blocks = static_cast<unsigned>(std::min<int64_t>(h->p.H, 2048));
    const unsigned rb = static_cast<unsigned>(std::min<int64_t>(cdiv(L.g.ntiles, NT), 64));
    for (int32_t n = 0; n < n_sweeps; ++n) {
        for (int32_t ph = SW_PHASE_TILE; ph <= SW_PHASE_FLIP; ++ph) {
            const sw_status st = launch_phase(h, ph, s);
            if (st != SW_OK) return st;
        }
        h->t += 1;
        h->swept = true;
        h->small_last = false;
        hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, s, obs, ST_LEN);
        hipLaunchKernelGGL(k_observe, dim3(blocks), dim3(NT), 0, s, static_cast<const uint8_t *>(h->b.spins), h->p.W,
                           h->p.H, static_cast<uint32_t>(h->p.q), h->p.spin_kind == SW_SPIN_ISING_I8 ? 1 : 0, obs);
        hipLaunchKernelGGL(k_reduce_tiles, dim3(rb), dim3(NT), 0, s, at<int32_t>(ws, L.tile_act), L.g.ntiles,
                           obs + ST_ACTIVE, static_cast<int32_t *>(nullptr));
        hipLaunchKernelGGL(k_reduce_tiles, dim3(rb), dim3(NT), 0, s, at<int32_t>(ws, L.tile_ncl), L.g.ntiles,
                           obs + ST_NCLUST, static_cast<int32_t *>(nullptr));
        hipLaunchKernelGGL(k_hist_row, dim3(1), dim3(64), 0, s, obs, max_dev, history + static_cast<int64_t>(n) * HIST_LEN);
        const sw_status st = launch_status("sw_sweep_history");
        if (st != SW_OK) return st;
    }
    return SW_OK;
}

sw_status sw_get_t(const sw_lattice *h, uint64_t *t)
{
    if (!h || !t) return SW_ERR_ARG;
    *t = h->t;
    return SW_OK;
}

sw_status sw_set_t(sw_lattice *h, uint64_t t)
{
    if (!h) return SW_ERR_ARG;
    if (t > 0xFFFFFFFFull || h->next_phase != SW_PHASE_TILE) return SW_ERR_STATE;
    h->t = t;
    h->swept = false;
    h->sel_stale = h->L.few;
    return SW_OK;
}

sw_status sw_destroy(sw_lattice *h)
{
    if (!h) return SW_ERR_ARG;
    delete h;
    return SW_OK;
}

size_t ccl_workspace_bytes(int32_t W, int32_t H, int32_t mode)
{
    return ccl_workspace_bytes_tiled(W, H, mode, 0);
}

size_t ccl_workspace_bytes_tiled(int32_t W, int32_t H, int32_t mode, int32_t tile_h)
{
    if (mode < CCL_BONDS_PERIODIC || mode > CCL_SITES_OPEN) return 0;
    if (tile_h != 0 && !valid_tile_h(tile_h)) return 0;
    const int th = tile_h ? tile_h : TH_DEFAULT;
    if (!valid_shape(W, H, 1, th)) return 0;
    return make_layout(W, H, true, th).total;
}

}  // extern "C"

namespace {

// Argument checks of ccl_label (before anything is enqueued).
sw_status ccl_check(const uint8_t *in, int32_t W, int32_t H, int32_t mode, const int32_t *labels,
                    const int32_t *roots, const int32_t *sizes, int th = TH_DEFAULT)
{
    if (!in || !labels) return SW_ERR_ARG;
    if (mode < CCL_BONDS_PERIODIC || mode > CCL_SITES_OPEN) return SW_ERR_ARG;
    if ((roots == nullptr) != (sizes == nullptr)) return SW_ERR_ARG;
    if (!valid_shape(W, H, 1, th)) return SW_ERR_SIZE;
    const int64_t N = static_cast<int64_t>(W) * H;
    const uintptr_t ib = reinterpret_cast<uintptr_t>(in), lb = reinterpret_cast<uintptr_t>(labels);
    if (ib < lb + static_cast<uintptr_t>(N) * 4 && lb < ib + static_cast<uintptr_t>(N)) return SW_ERR_ARG;
    return SW_OK;
}

// The labeling launches over a workspace laid out by L (no entry of it needs
// to start at zero: every word is written before it is read).
sw_status ccl_enqueue(const Layout &L, const uint8_t *in, int32_t mode, int32_t *labels, int32_t *roots,
                      int32_t *sizes, int32_t *n_clusters, void *workspace, hipStream_t s)
{
    const bool want_sizes = roots != nullptr;
    const TileArgs ta = tile_args(L, workspace, in);
    switch (mode) {
    case CCL_BONDS_PERIODIC: launch_tile<M_BONDS_PERIODIC>(L, ta, s); break;
    case CCL_BONDS_OPEN: launch_tile<M_BONDS_OPEN>(L, ta, s); break;
    default: launch_tile<M_SITES>(L, ta, s); break;
    }
    launch_merge<false>(L, merge_args(L, workspace), L.g.ntiles, s);
    FlatArgs fa = flat_args(L, workspace);
    fa.labels = labels;
    if (want_sizes) {
        // the flatten mode only matters for M_SW; all labeling inputs share one
        // path; the emit also writes the cluster count (the offsets' total)
        launch_flatten<M_BONDS_PERIODIC, true, false>(L, fa, L.g.ntiles, s);
        emit_sizes(L, workspace, fa, roots, sizes, nullptr, n_clusters, s);
    } else {
        launch_flatten<M_BONDS_PERIODIC, false, false>(L, fa, L.g.ntiles, s);
    }
    if (n_clusters && !want_sizes) {
        hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, s, n_clusters, 1);
        const unsigned rb = static_cast<unsigned>(std::min<int64_t>(cdiv(L.g.ntiles, NT), 64));
        hipLaunchKernelGGL(k_reduce_tiles, dim3(rb), dim3(NT), 0, s, fa.tile_ncl, L.g.ntiles,
                           static_cast<unsigned long long *>(nullptr), n_clusters);
    }
    return SW_OK;
}

// Scratch of ccl_label_noalloc: one copy per GPU, held from module load until
// the process ends.  Host code never uses the symbol's name as an address (on
// the host it is a stand-in); it uses the device address that
// hipGetSymbolAddress returns, looked up once per device.
static __device__ __align__(256) char scratch[CCL_NOALLOC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[MAX_DEVICES] = {};

// Device address of the current device's scratch (nullptr on failure).
sw_status scratch_of_current_device(void **out)
{
    int dev = -1;
    if (const sw_status st = device_status(hipGetDevice(&dev), "hipGetDevice")) return st;
    if (dev < 0 || dev >= MAX_DEVICES) {
        g_last_error = "device ordinal beyond the library's table";
        return SW_ERR_DEVICE;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        if (const sw_status st = device_status(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "hipGetSymbolAddress"))
            return st;
        if (!ptr || reinterpret_cast<uintptr_t>(ptr) % ALIGN) {
            g_last_error = "static scratch has no usable device address";
            return SW_ERR_DEVICE;
        }
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return SW_OK;
}

}  // namespace

extern "C" {

sw_status ccl_label(const uint8_t *in, int32_t W, int32_t H, int32_t mode, int32_t *labels, int32_t *roots,
                    int32_t *sizes, int32_t *n_clusters, void *workspace, size_t workspace_bytes, void *stream)
{
    return ccl_label_tiled(in, W, H, mode, 0, 0, labels, roots, sizes, n_clusters, workspace, workspace_bytes,
                           stream);
}

sw_status ccl_label_tiled(const uint8_t *in, int32_t W, int32_t H, int32_t mode, int32_t tile_h,
                          int32_t merge_waves, int32_t *labels, int32_t *roots, int32_t *sizes,
                          int32_t *n_clusters, void *workspace, size_t workspace_bytes, void *stream)
{
    if (tile_h != 0 && !valid_tile_h(tile_h)) return SW_ERR_ARG;
    if (merge_waves != 0 && !valid_merge_waves(merge_waves)) return SW_ERR_ARG;
    const int th = tile_h ? tile_h : TH_DEFAULT, mw = merge_waves ? merge_waves : MERGE_WAVES_DEFAULT;
    if (const sw_status st = ccl_check(in, W, H, mode, labels, roots, sizes, th)) return st;
    const Layout L = make_layout(W, H, roots != nullptr, th, mw);
    if (!workspace || workspace_bytes < L.total) return SW_ERR_WORKSPACE;
    if (reinterpret_cast<uintptr_t>(workspace) % ALIGN) return SW_ERR_WORKSPACE;
    ccl_enqueue(L, in, mode, labels, roots, sizes, n_clusters, workspace, static_cast<hipStream_t>(stream));
    return launch_status("ccl_label");
}

sw_status ccl_label_noalloc(const uint8_t *in, int32_t W, int32_t H, int32_t mode, int32_t *labels, int32_t *roots,
                            int32_t *sizes, int32_t *n_clusters, void *stream)
{
    if (const sw_status st = ccl_check(in, W, H, mode, labels, roots, sizes)) return st;
    const Layout L = make_layout(W, H, roots != nullptr);
    if (L.total > CCL_NOALLOC_SCRATCH_BYTES) {
        g_last_error = "ccl_label_noalloc: this shape needs " + std::to_string(L.total) +
                       " bytes of scratch, the static scratch holds " +
                       std::to_string(static_cast<size_t>(CCL_NOALLOC_SCRATCH_BYTES));
        return SW_ERR_WORKSPACE;
    }
    void *ws = nullptr;
    if (const sw_status st = scratch_of_current_device(&ws)) return st;
    ccl_enqueue(L, in, mode, labels, roots, sizes, n_clusters, ws, static_cast<hipStream_t>(stream));
    return launch_status("ccl_label_noalloc");
}

// ------------------------------------------------------------------ batches --

struct swb_batch {
    int32_t n;
    std::vector<sw_params> p;
    std::vector<sw_buffers> b;
    std::vector<uint64_t> T;
    std::vector<LatticeDesc> desc;     // host copies of what the device tables hold
    std::vector<int32_t> lat_of_tile;
    std::vector<uint8_t> small;        // swept whole in LDS by the fused launch
    std::vector<int32_t> small_lat, ftile;  // host copies of the fused work-queue tables
    std::vector<int2> mgroup;
    Layout L;
    void *ws;
    int32_t tiles_even;  // tiles of even-width lattices come first
    bool fused;          // one persistent launch per sweep (else one per phase)
    int32_t grid;        // workgroups of the fused launch
    int32_t n_small, n_ftiles, n_mgroups;
    uint64_t t;          // host mirror of the device sweep counter
    bool swept;
    // GRAPH_CHUNK[k] sweeps captured as one graph (swb_sweep_graph), each
    // made on first use
    hipStream_t cap = nullptr;
    hipGraph_t graph[2] = {nullptr, nullptr};
    hipGraphExec_t exec[2] = {nullptr, nullptr};
};

// The fused launch's work queue: lattices swept whole in LDS, then the tiles
// of the others (largest lattice first), their merge groups (up to one tile
// per wave of a workgroup) and, by the same table, their flattens; and the
// grid: as many workgroups as the device holds at once (more would only wait).
static sw_status build_fused_queue(swb_batch *h)
{
    const Layout &L = h->L;
    const int n = h->n;
    const int wg_threads = L.d.nt, nwave = L.d.th / RPW;
    const int small_sites = std::min(15 * wg_threads, 7680);  // FusedSmall<NT>::SITES
    try {
        h->small.assign(static_cast<size_t>(n), 0);
        std::vector<int32_t> order(static_cast<size_t>(n));
        for (int j = 0; j < n; ++j) order[static_cast<size_t>(j)] = j;
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
            return static_cast<int64_t>(h->p[a].W) * h->p[a].H > static_cast<int64_t>(h->p[b].W) * h->p[b].H;
        });
        for (const int j : order) {
            const sw_params &q = h->p[static_cast<size_t>(j)];
            LatticeDesc &d = h->desc[static_cast<size_t>(j)];
            if (q.W <= SMALL_W && q.H <= SMALL_H && q.W * q.H <= small_sites) {
                h->small[static_cast<size_t>(j)] = 1;
                h->small_lat.push_back(j);
                d.nmerge = 0;
            }
        }
        for (const int j : order) {
            if (h->small[static_cast<size_t>(j)]) continue;
            LatticeDesc &d = h->desc[static_cast<size_t>(j)];
            for (int k = 0; k < d.g.ntiles; ++k) h->ftile.push_back(d.tile0 + k);
            int nm = 0;
            for (int k = 0; k < d.g.ntiles; k += nwave, ++nm)
                h->mgroup.push_back(make_int2(d.tile0 + k, std::min(nwave, d.g.ntiles - k)));
            d.nmerge = nm;
        }
    } catch (const std::bad_alloc &) {
        return SW_ERR_HOST_MEMORY;
    }
    h->n_small = static_cast<int32_t>(h->small_lat.size());
    h->n_ftiles = static_cast<int32_t>(h->ftile.size());
    h->n_mgroups = static_cast<int32_t>(h->mgroup.size());
    int dev = 0, cus = 0, per_cu = 0;
    sw_status st = device_status(hipGetDevice(&dev), "hipGetDevice");
    if (st == SW_OK)
        st = device_status(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev), "CU count");
    if (st == SW_OK) {
        hipError_t e = hipSuccess;
        with_tile_h(L.d.th, [&](auto c) {
            constexpr int TH = decltype(c)::value;
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch_fused<TH>, Tile<TH>::NT, 0);
        });
        st = device_status(e, "fused-sweep occupancy");
    }
    if (st != SW_OK) return st;
    const int64_t items = static_cast<int64_t>(h->n_small) + 2 * static_cast<int64_t>(h->n_ftiles) + h->n_mgroups;
    h->grid = static_cast<int32_t>(std::max<int64_t>(1, std::min<int64_t>(items, static_cast<int64_t>(std::max(per_cu, 1)) * cus)));
    return SW_OK;
}

static sw_status check_batch(const sw_params *p, const sw_buffers *b, int32_t n, int64_t *ntiles)
{
    if (!p || !b || n < 1) return SW_ERR_ARG;
    int64_t nt = 0;
    const int th = tile_h_of(&p[0]);
    for (int32_t j = 0; j < n; ++j) {
        const sw_status st = check_params(&p[j], SW_F_BATCH_FUSED);
        if (st != SW_OK) return st;
        if ((p[j].flags & (SW_F_SIZES | SW_F_REVERSE_TILES)) || p[j].few_b != 0) return SW_ERR_UNSUPPORTED;
        // one tile shape and merge schedule per batch
        if (tile_h_of(&p[j]) != th || merge_waves_of(&p[j]) != merge_waves_of(&p[0])) return SW_ERR_ARG;
        if (!b[j].spins || b[j].roots || b[j].sizes) return SW_ERR_ARG;
        nt += cdiv(p[j].W, TW) * cdiv(p[j].H, th);
    }
    // tile ids times CAP must stay in int32
    if (nt * dims_of(th).cap >= (static_cast<int64_t>(1) << 31)) return SW_ERR_SIZE;
    *ntiles = nt;
    return SW_OK;
}

size_t swb_workspace_bytes(const sw_params *p, int32_t n)
{
    int64_t nt = 0;
    try {
        std::vector<sw_buffers> dummy(n > 0 ? static_cast<size_t>(n) : 0);
        for (auto &d : dummy) d.spins = reinterpret_cast<void *>(1);
        if (n < 1 || check_batch(p, dummy.data(), n, &nt) != SW_OK) return 0;
    } catch (const std::bad_alloc &) {
        return 0;
    }
    return make_batch_layout(nt, n, tile_h_of(&p[0]), merge_waves_of(&p[0])).total;
}

sw_status swb_init(swb_batch **out, const sw_params *p, const sw_buffers *b, int32_t n, void *workspace,
                   size_t workspace_bytes, void *stream)
{
    if (!out) return SW_ERR_ARG;
    int64_t nt = 0;
    const sw_status cs = check_batch(p, b, n, &nt);
    if (cs != SW_OK) return cs;
    const Layout L = make_batch_layout(nt, n, tile_h_of(&p[0]), merge_waves_of(&p[0]));
    if (!workspace || workspace_bytes < L.total) return SW_ERR_WORKSPACE;
    if (reinterpret_cast<uintptr_t>(workspace) % ALIGN) return SW_ERR_WORKSPACE;
    swb_batch *h = new (std::nothrow) swb_batch();
    if (!h) return SW_ERR_HOST_MEMORY;
    h->n = n;
    h->L = L;
    h->ws = workspace;
    h->t = 0;
    h->swept = false;
    try {
        h->p.assign(p, p + n);
        h->b.assign(b, b + n);
        h->T.resize(static_cast<size_t>(n));
        h->desc.resize(static_cast<size_t>(n));
        h->lat_of_tile.resize(static_cast<size_t>(nt));
    } catch (const std::bad_alloc &) {
        delete h;
        return SW_ERR_HOST_MEMORY;
    }
    // even widths first (one tile-kernel launch per width parity)
    int32_t tile = 0;
    for (int parity = 0; parity < 2; ++parity) {
        for (int32_t j = 0; j < n; ++j) {
            if ((p[j].W & 1) != parity) continue;
            LatticeDesc &d = h->desc[static_cast<size_t>(j)];
            d.g.W = p[j].W;
            d.g.H = p[j].H;
            d.g.ntx = static_cast<int>(cdiv(p[j].W, TW));
            d.g.nty = static_cast<int>(cdiv(p[j].H, L.d.th));
            d.g.ntiles = d.g.ntx * d.g.nty;
            d.tile0 = tile;
            d.spins = static_cast<uint8_t *>(b[j].spins);
            d.bonds = b[j].bonds;
            d.labels = b[j].labels;
            const uint64_t T = threshold_of(p[j].K);
            d.tany = T > 0 ? 1u : 0u;
            d.tm1 = T > 0 ? static_cast<uint32_t>(T - 1) : 0u;
            d.k0 = static_cast<uint32_t>(p[j].seed);
            d.k1 = static_cast<uint32_t>(p[j].seed >> 32);
            d.sid = p[j].stream_id;
            d.q = static_cast<uint32_t>(p[j].q);
            d.ising = p[j].spin_kind == SW_SPIN_ISING_I8 ? 1 : 0;
            for (int k = 0; k < d.g.ntiles; ++k) h->lat_of_tile[static_cast<size_t>(tile + k)] = j;
            tile += d.g.ntiles;
        }
        if (parity == 0) h->tiles_even = tile;
    }
    for (int32_t j = 0; j < n; ++j) h->T[static_cast<size_t>(j)] = threshold_of(p[j].K);
    hipStream_t s = static_cast<hipStream_t>(stream);
    h->fused = (p[0].flags & SW_F_BATCH_FUSED) != 0;
    sw_status st = SW_OK;
    if (h->fused) {
        st = build_fused_queue(h);
        if (st != SW_OK) {
            delete h;
            return st;
        }
    }
    st = device_status(hipMemcpyAsync(at<LatticeDesc>(workspace, L.lat_desc), h->desc.data(),
                                                h->desc.size() * sizeof(LatticeDesc), hipMemcpyHostToDevice, s),
                                 "copy lattice table");
    if (st == SW_OK)
        st = device_status(hipMemcpyAsync(at<int32_t>(workspace, L.lat_of_tile), h->lat_of_tile.data(),
                                          h->lat_of_tile.size() * sizeof(int32_t), hipMemcpyHostToDevice, s),
                           "copy tile table");
    if (st == SW_OK) {
        hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, s, at<int32_t>(workspace, L.t_dev), 1);
        st = launch_status("k_zero_i32");
    }
    if (st == SW_OK && h->fused) {
        if (!h->small_lat.empty())
            st = device_status(hipMemcpyAsync(at<int32_t>(workspace, L.small_lat), h->small_lat.data(),
                                              h->small_lat.size() * sizeof(int32_t), hipMemcpyHostToDevice, s),
                               "copy small-lattice table");
        if (st == SW_OK && !h->ftile.empty())
            st = device_status(hipMemcpyAsync(at<int32_t>(workspace, L.ftile), h->ftile.data(),
                                              h->ftile.size() * sizeof(int32_t), hipMemcpyHostToDevice, s),
                               "copy tile-item table");
        if (st == SW_OK && !h->mgroup.empty())
            st = device_status(hipMemcpyAsync(at<int2>(workspace, L.mgroup), h->mgroup.data(),
                                              h->mgroup.size() * sizeof(int2), hipMemcpyHostToDevice, s),
                               "copy merge-group table");
        if (st == SW_OK) {
            const int nc = 2 + 2 * n;
            hipLaunchKernelGGL(k_zero_u64, dim3(static_cast<unsigned>(cdiv(nc, 256))), dim3(256), 0, s,
                               at<unsigned long long>(workspace, L.counters), nc);
            hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, s, at<int32_t>(workspace, L.fault), 1);
            // every boundary-id parent a valid id and every tile's id count 0
            // before the first sweep, so no read in a fused launch can leave
            // the id tables, whatever it sees
            const int nid = static_cast<int>(nt) * L.d.cap;
            hipLaunchKernelGGL(k_iota_i32, dim3(static_cast<unsigned>(cdiv(nid, 256))), dim3(256), 0, s,
                               at<int32_t>(workspace, L.gparent), nid);
            hipLaunchKernelGGL(k_zero_i32, dim3(static_cast<unsigned>(cdiv(nt, 256))), dim3(256), 0, s,
                               at<int32_t>(workspace, L.nb), static_cast<int>(nt));
            st = launch_status("zero fused counters");
        }
    }
    for (int32_t j = 0; j < n && st == SW_OK; ++j) {
        if (p[j].flags & SW_F_KEEP_SPINS) continue;
        const int64_t N = static_cast<int64_t>(p[j].W) * p[j].H;
        hipLaunchKernelGGL(k_init, dim3(static_cast<unsigned>(cdiv(cdiv(N, 4), NT))), dim3(NT), 0, s,
                           static_cast<uint8_t *>(b[j].spins), N, static_cast<uint32_t>(p[j].q),
                           p[j].spin_kind == SW_SPIN_ISING_I8 ? 1 : 0, static_cast<uint32_t>(p[j].seed),
                           static_cast<uint32_t>(p[j].seed >> 32), p[j].stream_id);
        st = launch_status("k_init");
    }
    // the tables are read by later launches on this stream; the host copies stay
    // alive in the handle, so a pageable-copy staging delay is harmless
    if (st != SW_OK) {
        delete h;
        return st;
    }
    *out = h;
    return SW_OK;
}

}  // extern "C"

namespace {

// Enqueue one batched sweep: tile launches (per width parity), merge, flatten,
// and the bump of the device sweep counter the kernels read t from.
void enqueue_batch_sweep(const swb_batch *h, hipStream_t s)
{
    const Layout &L = h->L;
    void *ws = h->ws;
    Batch bt{};
    bt.lat = at<LatticeDesc>(ws, L.lat_desc);
    bt.lat_of_tile = at<int32_t>(ws, L.lat_of_tile);
    bt.t = at<uint32_t>(ws, L.t_dev);
    if (h->fused) {
        FusedArgs fa{};
        fa.ta = tile_args(L, ws, nullptr);
        fa.ta.b = bt;
        fa.ma = merge_args(L, ws);
        fa.ma.b = bt;
        fa.fa = flat_args(L, ws);
        fa.fa.b = bt;
        fa.small_lat = at<int32_t>(ws, L.small_lat);
        fa.ftile = at<int32_t>(ws, L.ftile);
        fa.mgroup = at<int2>(ws, L.mgroup);
        unsigned long long *c = at<unsigned long long>(ws, L.counters);
        fa.ticket = c;
        fa.exit_ctr = c + 1;
        fa.tiles_done = c + 2;
        fa.merge_done = c + 2 + h->n;
        fa.t = at<uint32_t>(ws, L.t_dev);
        fa.fault = at<int32_t>(ws, L.fault);
        fa.n_small = h->n_small;
        fa.n_tiles = h->n_ftiles;
        fa.n_mgroups = h->n_mgroups;
        with_tile_h(L.d.th, [&](auto c2) {
            constexpr int TH = decltype(c2)::value;
            hipLaunchKernelGGL(k_batch_fused<TH>, dim3(static_cast<unsigned>(h->grid)), dim3(Tile<TH>::NT), 0, s,
                               fa);
        });
        return;
    }
    const int32_t total = L.g.ntiles, even = h->tiles_even;
    TileArgs ta = tile_args(L, ws, nullptr);
    ta.b = bt;
    with_tile_h(L.d.th, [&](auto c) {
        constexpr int TH = decltype(c)::value;
        if (even > 0) {
            ta.b.tile_base = 0;
            ta.b.ntiles = even;
            hipLaunchKernelGGL((k_tile<M_SW, true, true, TH>), dim3(static_cast<unsigned>(even)), dim3(Tile<TH>::NT),
                               0, s, ta);
        }
        if (total > even) {
            ta.b.tile_base = even;
            ta.b.ntiles = total - even;
            hipLaunchKernelGGL((k_tile<M_SW, false, true, TH>), dim3(static_cast<unsigned>(total - even)),
                               dim3(Tile<TH>::NT), 0, s, ta);
        }
    });
    MergeArgs ma = merge_args(L, ws);
    ma.b = bt;
    ma.b.tile_base = 0;
    ma.b.ntiles = total;
    launch_merge<true>(L, ma, total, s);
    FlatArgs fa = flat_args(L, ws);
    fa.b = bt;
    fa.b.tile_base = 0;
    fa.b.ntiles = total;
    launch_flatten<M_SW, false, true>(L, fa, total, s);
    hipLaunchKernelGGL(k_bump_u32, dim3(1), dim3(64), 0, s, at<uint32_t>(ws, L.t_dev));
}

void drop_graph(swb_batch *h)
{
    for (int k = 0; k < 2; ++k) {
        if (h->exec[k]) (void)hipGraphExecDestroy(h->exec[k]);
        if (h->graph[k]) (void)hipGraphDestroy(h->graph[k]);
        h->exec[k] = nullptr;
        h->graph[k] = nullptr;
    }
    if (h->cap) (void)hipStreamDestroy(h->cap);
    h->cap = nullptr;
}

// Sweeps per graph: one, and a chunk of eight that pays one graph launch for
// eight sweeps.
constexpr int32_t GRAPH_CHUNK[2] = {1, 8};

// Capture GRAPH_CHUNK[k] sweeps as graph k, on a stream of the library's own:
// capture runs nothing, and the caller's stream may be one that cannot be
// captured.
sw_status capture_graph(swb_batch *h, int k)
{
    sw_status st = SW_OK;
    if (!h->cap) st = device_status(hipStreamCreateWithFlags(&h->cap, hipStreamNonBlocking), "create capture stream");
    if (st == SW_OK) st = device_status(hipStreamBeginCapture(h->cap, hipStreamCaptureModeThreadLocal), "begin capture");
    if (st == SW_OK) {
        for (int32_t i = 0; i < GRAPH_CHUNK[k]; ++i) enqueue_batch_sweep(h, h->cap);
        const hipError_t le = hipGetLastError();
        const hipError_t ee = hipStreamEndCapture(h->cap, &h->graph[k]);
        st = device_status(le != hipSuccess ? le : ee, "capture batched sweep");
    }
    if (st == SW_OK)
        st = device_status(hipGraphInstantiate(&h->exec[k], h->graph[k], nullptr, nullptr, 0),
                           "instantiate batched sweep");
    if (st != SW_OK) drop_graph(h);
    return st;
}

}  // namespace

extern "C" {

sw_status swb_sweep(swb_batch *h, int32_t n_sweeps, void *stream)
{
    if (!h || n_sweeps < 0) return SW_ERR_ARG;
    if (h->t + static_cast<uint64_t>(n_sweeps) > 0xFFFFFFFFull) return SW_ERR_STATE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    for (int32_t k = 0; k < n_sweeps; ++k) {
        enqueue_batch_sweep(h, s);
        const sw_status st = launch_status("swb_sweep");
        if (st != SW_OK) return st;
        h->t += 1;
        h->swept = true;
    }
    return SW_OK;
}

sw_status swb_sweep_graph(swb_batch *h, int32_t n_sweeps, void *stream)
{
    if (!h || n_sweeps < 0) return SW_ERR_ARG;
    if (h->t + static_cast<uint64_t>(n_sweeps) > 0xFFFFFFFFull) return SW_ERR_STATE;
    if (n_sweeps == 0) return SW_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    int32_t left = n_sweeps;
    while (left > 0) {
        const int k = left >= GRAPH_CHUNK[1] ? 1 : 0;
        if (!h->exec[k]) {
            const sw_status st = capture_graph(h, k);
            if (st != SW_OK) return st;
        }
        const sw_status st = device_status(hipGraphLaunch(h->exec[k], s), "launch batched sweep graph");
        if (st != SW_OK) return st;
        h->t += static_cast<uint64_t>(GRAPH_CHUNK[k]);
        h->swept = true;
        left -= GRAPH_CHUNK[k];
    }
    return SW_OK;
}

sw_status swb_observables(swb_batch *h, int32_t j, sw_obs *out, void *stream)
{
    if (!h || !out || j < 0 || j >= h->n) return SW_ERR_ARG;
    const Layout &L = h->L;
    const LatticeDesc &d = h->desc[static_cast<size_t>(j)];
    const bool in_lds = h->fused && h->small[static_cast<size_t>(j)];  // its counters are in its first tile
    hipStream_t s = static_cast<hipStream_t>(stream);
    const sw_status st = measure(h->p[static_cast<size_t>(j)], h->b[static_cast<size_t>(j)], h->swept,
                                 at<int32_t>(h->ws, L.tile_act) + d.tile0, at<int32_t>(h->ws, L.tile_ncl) + d.tile0,
                                 in_lds ? 1 : d.g.ntiles, at<unsigned long long>(h->ws, L.stats), nullptr,
                                 h->T[static_cast<size_t>(j)], h->t, out, s);
    if (st != SW_OK || !h->fused) return st;
    int32_t fault = 0;
    sw_status fs = device_status(hipMemcpyAsync(&fault, at<int32_t>(h->ws, L.fault), sizeof(fault),
                                                hipMemcpyDeviceToHost, s), "copy fault flag");
    if (fs == SW_OK) fs = device_status(hipStreamSynchronize(s), "sync");
    if (fs != SW_OK) return fs;
    if (fault) {
        g_last_error = "fused batch sweep: a dependency wait gave up; the batch's results are invalid";
        return SW_ERR_DEVICE;
    }
    return SW_OK;
}

sw_status swb_get_t(const swb_batch *h, uint64_t *t)
{
    if (!h || !t) return SW_ERR_ARG;
    *t = h->t;
    return SW_OK;
}

sw_status swb_destroy(swb_batch *h)
{
    if (!h) return SW_ERR_ARG;
    drop_graph(h);
    delete h;
    return SW_OK;
}

}  // extern "C"

// ---------------------------------------------- batched labeling requests --

namespace swccl_internal {

int64_t request_tiles(int32_t W, int32_t H) { return cdiv(W, TW) * cdiv(H, TH_DEFAULT); }

sw_status device_error(hipError_t e, const char *where) { return device_status(e, where); }

sw_status init_spins(uint8_t *spins, int64_t N, int32_t q, bool ising, uint64_t seed, uint32_t sid, hipStream_t s)
{
    if (N <= 0) return SW_OK;
    hipLaunchKernelGGL(k_init, dim3(static_cast<unsigned>(cdiv(cdiv(N, 4), NT))), dim3(NT), 0, s, spins, N,
                       static_cast<uint32_t>(q), ising ? 1 : 0, static_cast<uint32_t>(seed),
                       static_cast<uint32_t>(seed >> 32), sid);
    return launch_status("k_init");
}

uint64_t bond_threshold(double K) { return threshold_of(K); }

sw_status pull(void *dst, const void *src_dev, int64_t n, hipStream_t s)
{
    if (n <= 0) return SW_OK;
    hipLaunchKernelGGL(k_pull, dim3(static_cast<unsigned>(cdiv(n, static_cast<int64_t>(NT) * 4))), dim3(NT), 0, s,
                       static_cast<uint8_t *>(dst), static_cast<const uint8_t *>(src_dev), n);
    return launch_status("pull");
}

size_t batch_table_bytes(int32_t n, int64_t ntiles)
{
    return align_up(static_cast<size_t>(n) * sizeof(ReqDesc)) + align_up(static_cast<size_t>(ntiles) * sizeof(int32_t));
}

sw_status label_batch(const LabelRequest *r, int32_t n, int32_t mode, bool sizes, void *table, void *stage,
                      size_t table_bytes, hipStream_t s)
{
    if (n < 1 || !r || !table || !stage) return SW_ERR_ARG;
    int64_t nt = 0;
    for (int32_t k = 0; k < n; ++k) nt += request_tiles(r[k].W, r[k].H);
    const size_t desc_bytes = align_up(static_cast<size_t>(n) * sizeof(ReqDesc));
    const size_t need = batch_table_bytes(n, nt);
    if (need > table_bytes || nt >= (static_cast<int64_t>(1) << 31)) return SW_ERR_WORKSPACE;
    std::memset(stage, 0, need);
    ReqDesc *desc = static_cast<ReqDesc *>(stage);
    int32_t *req_of_tile = reinterpret_cast<int32_t *>(static_cast<char *>(stage) + desc_bytes);
    int32_t tile = 0;
    for (int32_t k = 0; k < n; ++k) {
        const Layout L = make_layout(r[k].W, r[k].H, sizes);
        void *ws = r[k].ws;
        ReqDesc &d = desc[k];
        d.g = L.g;
        d.tile0 = tile;
        d.in = r[k].in;
        d.labels = r[k].labels;
        d.roots = sizes ? r[k].roots : nullptr;
        d.sizes = sizes ? r[k].sizes : nullptr;
        d.n_clusters = r[k].n_clusters;
        d.codes = at<uint16_t>(ws, L.codes);
        d.edges = at<uint16_t>(ws, L.edges);
        d.gkey = at<int32_t>(ws, L.gkey);
        d.gparent = at<int32_t>(ws, L.gparent);
        d.gsize = sizes ? at<int32_t>(ws, L.gsize) : nullptr;
        d.nb = at<int32_t>(ws, L.nb);
        d.tile_ncl = at<int32_t>(ws, L.tile_ncl);
        d.xbits = at<uint64_t>(ws, L.xbits);
        d.row_count = sizes ? at<int32_t>(ws, L.row_count) : nullptr;
        d.row_off = sizes ? at<int32_t>(ws, L.row_off) : nullptr;
        d.rl_slot = sizes ? at<int32_t>(ws, L.rl_slot) : nullptr;
        d.rl_size = sizes ? at<int32_t>(ws, L.rl_size) : nullptr;
        for (int t = 0; t < L.g.ntiles; ++t) req_of_tile[tile + t] = k;
        tile += L.g.ntiles;
    }
    // the table goes over by a kernel that reads the pinned stage: a copy-engine
    // transfer would queue behind the large images other streams copy
    void *dstage = nullptr;
    if (const sw_status st = device_status(hipHostGetDevicePointer(&dstage, stage, 0), "stage device address"))
        return st;
    if (const sw_status st = pull(table, dstage, static_cast<int64_t>(need), s)) return st;
    ReqBatch rb{};
    rb.req = static_cast<const ReqDesc *>(table);
    rb.req_of_tile = reinterpret_cast<const int32_t *>(static_cast<char *>(table) + desc_bytes);
    rb.ntiles = tile;
    constexpr int TH = TH_DEFAULT;
    const dim3 tiles(static_cast<unsigned>(tile));
    switch (mode) {
    case CCL_BONDS_PERIODIC: hipLaunchKernelGGL((k_tile_reqs<M_BONDS_PERIODIC, TH>), tiles, dim3(Tile<TH>::NT), 0, s, rb); break;
    case CCL_BONDS_OPEN: hipLaunchKernelGGL((k_tile_reqs<M_BONDS_OPEN, TH>), tiles, dim3(Tile<TH>::NT), 0, s, rb); break;
    default: hipLaunchKernelGGL((k_tile_reqs<M_SITES, TH>), tiles, dim3(Tile<TH>::NT), 0, s, rb); break;
    }
    constexpr int MW = MERGE_WAVES_DEFAULT;
    hipLaunchKernelGGL(k_merge_reqs<TH>, dim3(static_cast<unsigned>(cdiv(tile, MW))), dim3(64 * MW), 0, s, rb);
    if (sizes) {
        hipLaunchKernelGGL((k_flatten_reqs<true, TH>), tiles, dim3(Tile<TH>::NT), 0, s, rb);
        hipLaunchKernelGGL(k_scan_reqs<true>, dim3(static_cast<unsigned>(n)), dim3(NT), 0, s, rb.req);
        hipLaunchKernelGGL(k_emit_reqs<TH>, tiles, dim3(NT), 0, s, rb);
    } else {
        hipLaunchKernelGGL((k_flatten_reqs<false, TH>), tiles, dim3(Tile<TH>::NT), 0, s, rb);
        hipLaunchKernelGGL(k_scan_reqs<false>, dim3(static_cast<unsigned>(n)), dim3(NT), 0, s, rb.req);
    }
    return launch_status("batched labeling");
}

}  // namespace swccl_internal
