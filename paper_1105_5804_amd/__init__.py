"""Swendsen-Wang cluster updates and connected-component labeling on MI355X.

Thin Python layer over the C ABI of ``libswccl.so`` (``include/swccl.h``):
torch provides device memory and the current HIP stream, every step of the
computation runs in the library's gfx950 kernels.  There is no CPU fallback:
without the built library or a GPU every compute call raises.
"""
from __future__ import annotations

import ctypes
import math

from . import _lib
from ._lib import (  # noqa: F401
    CCL_BONDS_OPEN,
    CCL_BONDS_PERIODIC,
    CCL_SITES_OPEN,
    SW_SPIN_ISING_I8,
    SW_SPIN_POTTS_U8,
    SwccLError,
)

__all__ = [
    "SWLattice",
    "CubicLattice",
    "ccl3_label",
    "SWBatch",
    "ccl_label",
    "ccl_label_noalloc",
    "ccl_workspace_bytes",
    "threshold",
    "ising_K",
    "potts_K",
    "CCL_BONDS_PERIODIC",
    "CCL_BONDS_OPEN",
    "CCL_SITES_OPEN",
]

_MODES = {"bonds_periodic": CCL_BONDS_PERIODIC, "bonds_open": CCL_BONDS_OPEN, "sites_open": CCL_SITES_OPEN}


def threshold(K: float) -> int:
    """Integer bond threshold T = floor((1 - exp(-K)) 2^32) used by the library."""
    return int(_lib.lib().sw_threshold(float(K)))


def ising_K(beta: float, J: float = 1.0) -> float:
    """FK coupling of the +-1 Ising model, H = -J sum s_i s_j: K = 2 beta J."""
    return 2.0 * beta * J


def potts_K(beta: float, J: float = 1.0) -> float:
    """FK coupling of the Potts model, H = -J sum delta(s_i, s_j): K = beta J."""
    return beta * J


BETA_C_ISING = 0.5 * math.log1p(math.sqrt(2.0))
# critical coupling of the 3D Ising model on the simple cubic lattice (from
# the Monte Carlo literature; no closed form is known)
BETA_C_ISING_3D = 0.22165455


def _torch():
    import torch

    if not torch.cuda.is_available():
        raise RuntimeError("swccl needs a ROCm GPU: torch.cuda.is_available() is False")
    return torch


def _stream(torch, stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _workspace(torch, nbytes: int, device):
    """A 256-byte aligned device byte range of at least nbytes (tensor, pointer)."""
    buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
    p = buf.data_ptr()
    return buf, p + ((-p) % 256)


def _obs_dict(o, N: int, q: int, ising: bool) -> dict:
    d = {
        "t": int(o.t),
        "threshold": int(o.threshold),
        "n_sat": int(o.n_sat),
        "magnet": int(o.magnet),
        "counts": [int(c) for c in o.counts][: min(q, 8)],
        "n_active_bonds": int(o.n_active_bonds),
        "n_clusters": int(o.n_clusters),
        "max_cluster": int(o.max_cluster),
        "digest_spins": int(o.digest_spins),
        "digest_labels": int(o.digest_labels),
        "digest_bonds": int(o.digest_bonds),
    }
    if ising:
        d["energy_per_site"] = -(2.0 * d["n_sat"] - 2.0 * N) / N
        d["abs_m"] = abs(d["magnet"]) / N
    else:
        d["energy_per_site"] = -d["n_sat"] / N
    return d


class SWLattice:
    """One periodic W x H lattice advanced by Swendsen-Wang sweeps on the GPU.

    ``spins`` is an (H, W) int8 (Ising, +-1) or uint8 (Potts, 0..q-1) tensor.
    With ``keep_labels`` / ``keep_bonds`` the canonical labels / packed bonds of
    the last sweep are kept in ``labels`` / ``bonds``; with ``sizes`` every sweep
    also lists its clusters (``cluster_sizes()``) and their largest size.
    ``reverse_tiles`` runs the tiles in the reverse order (a schedule check:
    every output is the same).  ``tile_h`` (16, 32, 64, 128; 0 = 64) and
    ``merge_waves`` (4, 8, 16; 0 = 8) choose the tile shape and merge schedule
    (outputs do not depend on them; ``paper_1105_5804_amd.tune`` picks them).
    ``few_b`` > 0 makes every sweep the few-cluster variant of the Wolff
    update (Sec. III, q = 2): the SW bonds and clusters, one seed per
    ``few_b`` x ``few_b`` seed tile, and every distinct seeded cluster flipped
    with probability ``p_flip`` (0 <= p_flip < 1).  The constructor enqueues on
    the current stream; methods given another ``stream`` are ordered only with
    that stream's work (synchronise the two as with any torch side stream).
    """

    def __init__(self, W: int, H: int, q: int = 2, K: float | None = None, seed: int = 0,
                 stream_id: int = 0, ising: bool | None = None, keep_labels: bool = False,
                 keep_bonds: bool = False, sizes: bool = False, spins=None, t: int = 0,
                 device: str = "cuda", reverse_tiles: bool = False, tile_h: int = 0, merge_waves: int = 0,
                 few_b: int = 0, p_flip: float = 0.0):
        torch = _torch()
        L = _lib.lib()
        if ising is None:
            ising = q == 2
        if K is None:
            K = ising_K(BETA_C_ISING) if q == 2 else math.log1p(math.sqrt(q))
        self.W, self.H, self.q, self.K = int(W), int(H), int(q), float(K)
        self.seed, self.stream_id, self.ising = int(seed), int(stream_id), bool(ising)
        self.device = torch.device(device)
        p = _lib.SwParams(self.W, self.H, self.q, _lib.SW_SPIN_ISING_I8 if ising else _lib.SW_SPIN_POTTS_U8,
                          self.K, self.seed & (2**64 - 1), self.stream_id,
                          (_lib.SW_F_SIZES if sizes else 0) | (_lib.SW_F_REVERSE_TILES if reverse_tiles else 0),
                          int(tile_h), int(merge_waves))
        p.few_b, p.p_flip = int(few_b), float(p_flip)
        self.few_b, self.p_flip = int(few_b), float(p_flip)
        self.tile_h, self.merge_waves = int(tile_h) or 64, int(merge_waves) or 8
        ws = L.sw_workspace_bytes(ctypes.byref(p))
        if ws == 0:
            _lib.check(_lib.SW_ERR_ARG if self.W >= 2 and self.H >= 2 else _lib.SW_ERR_SIZE, "sw_workspace_bytes")
        dt = torch.int8 if ising else torch.uint8
        if spins is not None:
            if spins.shape != (self.H, self.W) or spins.dtype != dt or spins.device.type != "cuda":
                raise ValueError(f"spins must be a ({self.H}, {self.W}) {dt} GPU tensor")
            self.spins = spins.contiguous()
            p.flags |= _lib.SW_F_KEEP_SPINS
        else:
            self.spins = torch.empty((self.H, self.W), dtype=dt, device=self.device)
        self.labels = torch.empty((self.H, self.W), dtype=torch.int32, device=self.device) if keep_labels else None
        self.bonds = torch.empty((self.H, self.W), dtype=torch.uint8, device=self.device) if keep_bonds else None
        N = self.W * self.H
        self.roots = torch.empty(N, dtype=torch.int32, device=self.device) if sizes else None
        self.sizes = torch.empty(N, dtype=torch.int32, device=self.device) if sizes else None
        self._ws_buf, ws_ptr = _workspace(torch, ws, self.device)
        self._bufs = _lib.SwBuffers(
            self.spins.data_ptr(),
            self.labels.data_ptr() if self.labels is not None else None,
            self.bonds.data_ptr() if self.bonds is not None else None,
            self.roots.data_ptr() if self.roots is not None else None,
            self.sizes.data_ptr() if self.sizes is not None else None,
            ws_ptr,
            ws,
        )
        self._params = p
        self._h = ctypes.c_void_p()
        _lib.check(L.sw_init(ctypes.byref(self._h), ctypes.byref(p), ctypes.byref(self._bufs),
                             _stream(torch)), "sw_init")
        if t:
            _lib.check(L.sw_set_t(self._h, int(t)), "sw_set_t")

    @property
    def threshold(self) -> int:
        return threshold(self.K)

    @property
    def t(self) -> int:
        v = ctypes.c_uint64()
        _lib.check(_lib.lib().sw_get_t(self._h, ctypes.byref(v)), "sw_get_t")
        return int(v.value)

    @t.setter
    def t(self, value: int) -> None:
        _lib.check(_lib.lib().sw_set_t(self._h, int(value)), "sw_set_t")

    def sweep(self, n: int = 1, stream=None) -> None:
        """Enqueue n sweeps on the current (or given) stream; does not wait."""
        torch = _torch()
        _lib.check(_lib.lib().sw_sweep(self._h, int(n), _stream(torch, stream)), "sw_sweep")

    def sweep_history(self, n: int, stream=None):
        """Enqueue n sweeps and return their per-sweep records, an (n, 12) int64
        device tensor (columns: active bonds, clusters, largest cluster or -1,
        satisfied bonds and counts[8] of the new spins); does not wait."""
        torch = _torch()
        hist = torch.empty((max(int(n), 1), _lib.SW_HIST_LEN), dtype=torch.int64, device=self.device)
        _lib.check(_lib.lib().sw_sweep_history(self._h, int(n), hist.data_ptr(), _stream(torch, stream)),
                   "sw_sweep_history")
        return hist[: int(n)]

    def sweep_phase(self, phase: int, stream=None) -> None:
        """Enqueue one phase (0 tile, 1 merge, 2 flip) of the next sweep."""
        torch = _torch()
        _lib.check(_lib.lib().sw_sweep_phase(self._h, int(phase), _stream(torch, stream)), "sw_sweep_phase")

    def observables(self, stream=None) -> dict:
        """Counters of the current spins and of the last sweep (waits for the stream)."""
        torch = _torch()
        o = _lib.SwObs()
        _lib.check(_lib.lib().sw_observables(self._h, ctypes.byref(o), _stream(torch, stream)), "sw_observables")
        return _obs_dict(o, self.W * self.H, self.q, self.ising)

    def cluster_sizes(self, stream=None):
        """(roots ascending, sizes) of the last sweep's clusters (needs ``sizes=True``;
        waits for the stream)."""
        if self.roots is None:
            raise ValueError("lattice was created without sizes=True")
        n = self.observables(stream)["n_clusters"]
        if n < 0:
            raise ValueError("no sweep yet")
        return self.roots[:n], self.sizes[:n]

    def state(self):
        """(spins copy, t): everything needed to resume bit-exactly."""
        return self.spins.clone(), self.t

    def close(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.lib().sw_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class CubicLattice:
    """One periodic Lx x Ly x Lz simple cubic lattice advanced by SW sweeps.

    ``spins`` is an (Lz, Ly, Lx) int8 (Ising, +-1) or uint8 (Potts, 0..q-1)
    tensor.  With ``keep_labels`` / ``keep_bonds`` the canonical labels /
    packed bonds (bit0 +x, bit1 +y, bit2 +z) of the last sweep of each call
    are kept in ``labels`` / ``bonds``.  ``sweep(n, records=True)`` returns the
    (n, 11) int64 device tensor of per-sweep records (active bonds, clusters,
    satisfied bonds and counts[8] of the new spins).  The host keeps the sweep
    counter ``t``; the calls enqueue on the current (or given) stream and do
    not wait.
    """

    def __init__(self, Lx: int, Ly: int, Lz: int, q: int = 2, K: float | None = None, seed: int = 0,
                 stream_id: int = 0, ising: bool | None = None, keep_labels: bool = False,
                 keep_bonds: bool = False, spins=None, t: int = 0, device: str = "cuda"):
        torch = _torch()
        L = _lib.lib()
        if ising is None:
            ising = q == 2
        if K is None:
            K = ising_K(BETA_C_ISING_3D) if q == 2 else math.log1p(math.sqrt(q))
        self.Lx, self.Ly, self.Lz, self.q, self.K = int(Lx), int(Ly), int(Lz), int(q), float(K)
        self.seed, self.stream_id, self.ising = int(seed), int(stream_id), bool(ising)
        self.device = torch.device(device)
        self._params = _lib.Sw3Params(self.Lx, self.Ly, self.Lz, self.q,
                                      _lib.SW_SPIN_ISING_I8 if ising else _lib.SW_SPIN_POTTS_U8, 0, self.K,
                                      self.seed & (2**64 - 1), self.stream_id, 0)
        ws = L.sw3_workspace_bytes(ctypes.byref(self._params))
        if ws == 0:
            bad_size = min(self.Lx, self.Ly, self.Lz) < 1 or self.Lx * self.Ly * self.Lz >= 2**31
            _lib.check(_lib.SW_ERR_SIZE if bad_size else _lib.SW_ERR_ARG, "sw3_workspace_bytes")
        shape = (self.Lz, self.Ly, self.Lx)
        dt = torch.int8 if ising else torch.uint8
        self._ws_buf, self._ws_ptr = _workspace(torch, ws, self.device)
        self._ws = ws
        self.labels = torch.empty(shape, dtype=torch.int32, device=self.device) if keep_labels else None
        self.bonds = torch.empty(shape, dtype=torch.uint8, device=self.device) if keep_bonds else None
        if spins is not None:
            if tuple(spins.shape) != shape or spins.dtype != dt or spins.device.type != "cuda":
                raise ValueError(f"spins must be a {shape} {dt} GPU tensor")
            self.spins = spins.contiguous()
        else:
            self.spins = torch.empty(shape, dtype=dt, device=self.device)
            _lib.check(L.sw3_init_spins(ctypes.byref(self._params), self.spins.data_ptr(), _stream(torch)),
                       "sw3_init_spins")
        self.t = int(t)

    @property
    def threshold(self) -> int:
        return threshold(self.K)

    def sweep(self, n: int = 1, records: bool = False, stream=None):
        """Enqueue n sweeps t .. t+n-1 and advance t; with ``records`` return
        their (n, 11) int64 device tensor of per-sweep records."""
        torch = _torch()
        rec = None
        if records:
            rec = torch.empty((max(int(n), 1), _lib.SW3_REC_LEN), dtype=torch.int64, device=self.device)
        _lib.check(_lib.lib().sw3_sweep(ctypes.byref(self._params), self.spins.data_ptr(), int(self.t), int(n),
                                        self.bonds.data_ptr() if self.bonds is not None else None,
                                        self.labels.data_ptr() if self.labels is not None else None,
                                        rec.data_ptr() if rec is not None else None, self._ws_ptr, self._ws,
                                        _stream(torch, stream)), "sw3_sweep")
        self.t += int(n)
        return rec[: int(n)] if rec is not None else None


def ccl3_label(bonds, workspace=None, stream=None):
    """Canonical labels of packed cubic bonds: ``bonds`` is an (Lz, Ly, Lx)
    uint8 GPU tensor (bit0 +x, bit1 +y, bit2 +z, periodic).  Returns
    (labels as an (Lz, Ly, Lx) int32 tensor, n_clusters); enqueues on the
    current (or given) stream and waits for it to read the count."""
    torch = _torch()
    if bonds.dim() != 3 or bonds.dtype != torch.uint8 or bonds.device.type != "cuda":
        raise ValueError("bonds must be an (Lz, Ly, Lx) uint8 GPU tensor")
    bonds = bonds.contiguous()
    Lz, Ly, Lx = (int(v) for v in bonds.shape)
    L = _lib.lib()
    ws = L.ccl3_workspace_bytes(Lx, Ly, Lz)
    if ws == 0:
        _lib.check(_lib.SW_ERR_SIZE, "ccl3_workspace_bytes")
    if workspace is None:
        buf, wptr = _workspace(torch, ws, bonds.device)
    else:
        buf, wptr = workspace, workspace.data_ptr()
        if workspace.device.type != "cuda" or workspace.numel() < ws or wptr % 256:
            raise ValueError(f"workspace must be a 256-byte aligned GPU buffer of at least {ws} bytes")
    labels = torch.empty((Lz, Ly, Lx), dtype=torch.int32, device=bonds.device)
    ncl = torch.zeros(1, dtype=torch.int32, device=bonds.device)
    s = stream if stream is not None else torch.cuda.current_stream(bonds.device)
    _lib.check(L.ccl3_label(bonds.data_ptr(), Lx, Ly, Lz, labels.data_ptr(), ncl.data_ptr(), wptr, ws,
                            _stream(torch, s)), "ccl3_label")
    s.synchronize()
    del buf
    return labels, int(ncl.item())


class SWBatch:
    """Many independent lattices advanced together, one launch per sweep phase.

    ``specs`` is a sequence of dicts with keys W, H and optionally q, K, seed,
    stream_id, ising (defaults as in ``SWLattice``).  Lattice j evolves exactly
    as ``SWLattice(**specs[j])`` would.  ``spins[j]`` (and ``labels[j]`` /
    ``bonds[j]`` with ``keep_labels`` / ``keep_bonds``) are its tensors.
    ``tile_h`` / ``merge_waves`` as in ``SWLattice``, one choice per batch.
    A sweep is one launch per phase over all lattices; ``fused=True`` uses one
    launch of the fused persistent kernel instead (lattices of at most 128 x 64
    swept whole in LDS, the others tiled, phases ordered per lattice).
    """

    def __init__(self, specs, keep_labels: bool = False, keep_bonds: bool = False, device: str = "cuda",
                 tile_h: int = 0, merge_waves: int = 0, fused: bool = False):
        torch = _torch()
        L = _lib.lib()
        self.device = torch.device(device)
        n = len(specs)
        if n < 1:
            raise ValueError("a batch needs at least one lattice")
        P = (_lib.SwParams * n)()
        B = (_lib.SwBuffers * n)()
        self.specs, self.spins, self.labels, self.bonds = [], [], [], []
        for j, sp in enumerate(specs):
            W, H = int(sp["W"]), int(sp["H"])
            q = int(sp.get("q", 2))
            ising = bool(sp.get("ising", q == 2))
            K = sp.get("K")
            if K is None:
                K = ising_K(BETA_C_ISING) if q == 2 else math.log1p(math.sqrt(q))
            seed, sid = int(sp.get("seed", 0)), int(sp.get("stream_id", 0))
            self.specs.append(dict(W=W, H=H, q=q, K=float(K), seed=seed, stream_id=sid, ising=ising))
            P[j] = _lib.SwParams(W, H, q, _lib.SW_SPIN_ISING_I8 if ising else _lib.SW_SPIN_POTTS_U8, float(K),
                                 seed & (2**64 - 1), sid, _lib.SW_F_BATCH_FUSED if fused else 0,
                                 int(tile_h), int(merge_waves))
            dt = torch.int8 if ising else torch.uint8
            sp_t = torch.empty((H, W), dtype=dt, device=self.device)
            lab = torch.empty((H, W), dtype=torch.int32, device=self.device) if keep_labels else None
            bnd = torch.empty((H, W), dtype=torch.uint8, device=self.device) if keep_bonds else None
            self.spins.append(sp_t)
            self.labels.append(lab)
            self.bonds.append(bnd)
            B[j] = _lib.SwBuffers(spins=sp_t.data_ptr(), labels=lab.data_ptr() if lab is not None else None,
                                  bonds=bnd.data_ptr() if bnd is not None else None)
        ws = L.swb_workspace_bytes(P, n)
        if ws == 0:
            _lib.check(_lib.SW_ERR_ARG, "swb_workspace_bytes")
        self._ws_buf, ws_ptr = _workspace(torch, ws, self.device)
        self._P, self._B = P, B
        self._h = ctypes.c_void_p()
        _lib.check(L.swb_init(ctypes.byref(self._h), P, B, n, ws_ptr, ws, _stream(torch)), "swb_init")
        self.n = n

    @property
    def t(self) -> int:
        v = ctypes.c_uint64()
        _lib.check(_lib.lib().swb_get_t(self._h, ctypes.byref(v)), "swb_get_t")
        return int(v.value)

    def sweep(self, n: int = 1, stream=None, graph: bool = False) -> None:
        """Enqueue n sweeps of every lattice; does not wait.  With graph=True
        each sweep is one replay of a captured HIP graph (same trajectory)."""
        torch = _torch()
        fn = _lib.lib().swb_sweep_graph if graph else _lib.lib().swb_sweep
        _lib.check(fn(self._h, int(n), _stream(torch, stream)), "swb_sweep_graph" if graph else "swb_sweep")

    def observables(self, j: int, stream=None) -> dict:
        """Counters of lattice j (waits for the stream)."""
        torch = _torch()
        o = _lib.SwObs()
        _lib.check(_lib.lib().swb_observables(self._h, int(j), ctypes.byref(o), _stream(torch, stream)),
                   "swb_observables")
        return _obs_dict(o, self.specs[j]["W"] * self.specs[j]["H"], self.specs[j]["q"], self.specs[j]["ising"])

    def close(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.lib().swb_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def ccl_workspace_bytes(W: int, H: int, mode: str | int = "bonds_periodic", tile_h: int = 0) -> int:
    m = _MODES[mode] if isinstance(mode, str) else int(mode)
    return int(_lib.lib().ccl_workspace_bytes_tiled(int(W), int(H), m, int(tile_h)))


def ccl_label(inp, mode: str | int = "bonds_periodic", sizes: bool = False, workspace=None,
              labels=None, stream=None, tile_h: int = 0, merge_waves: int = 0):
    """Connected-component labels of an (H, W) uint8 GPU tensor.

    mode: "bonds_periodic" / "bonds_open" (packed bonds, bit0 right, bit1 down)
    or "sites_open" (binary image, 4-connected, background label -1).
    Returns labels, or (labels, roots, sizes, n_clusters) when sizes=True;
    roots ascend and sizes[k] belongs to roots[k].  With a ``stream`` other
    than the current one, that stream first waits for the current stream's
    work; with sizes the call waits for ``stream`` (to read the count).
    ``tile_h`` / ``merge_waves`` choose the tile shape and merge schedule as in
    ``SWLattice`` (the labels do not depend on them).
    """
    torch = _torch()
    L = _lib.lib()
    m = _MODES[mode] if isinstance(mode, str) else int(mode)
    if inp.dim() != 2 or inp.dtype != torch.uint8 or inp.device.type != "cuda":
        raise ValueError("input must be a 2D uint8 GPU tensor")
    inp = inp.contiguous()
    H, W = inp.shape
    ws = L.ccl_workspace_bytes_tiled(W, H, m, int(tile_h))
    if ws == 0:
        _lib.check(_lib.SW_ERR_SIZE, "ccl_workspace_bytes")
    made = []  # tensors allocated here, on the current stream
    if workspace is None:
        wbuf, wptr = _workspace(torch, ws, inp.device)
        made.append(wbuf)
    else:
        if workspace.device != inp.device or not workspace.is_contiguous():
            raise ValueError(f"workspace must be a contiguous tensor on {inp.device}")
        wbuf = workspace
        p = workspace.data_ptr()
        wptr = p + ((-p) % 256)
        if workspace.numel() * workspace.element_size() - (wptr - p) < ws:
            raise ValueError("workspace too small")
    if labels is None:
        labels = torch.empty((H, W), dtype=torch.int32, device=inp.device)
        made.append(labels)
    elif (labels.shape != (H, W) or labels.dtype != torch.int32 or labels.device != inp.device
          or not labels.is_contiguous()):
        raise ValueError(f"labels must be a contiguous ({H}, {W}) int32 tensor on {inp.device}")
    ncl = torch.empty(1, dtype=torch.int32, device=inp.device)  # written by the library
    made.append(ncl)
    roots = szs = None
    if sizes:
        roots = torch.empty(H * W, dtype=torch.int32, device=inp.device)
        szs = torch.empty(H * W, dtype=torch.int32, device=inp.device)
        made += [roots, szs]
    cur = torch.cuda.current_stream(inp.device)
    side = stream is not None and stream != cur
    if side:
        # the input's copy (if .contiguous() made one) was enqueued on the current stream
        stream.wait_stream(cur)
        made.append(inp)
    st = L.ccl_label_tiled(inp.data_ptr(), W, H, m, int(tile_h), int(merge_waves), labels.data_ptr(),
                           roots.data_ptr() if sizes else None, szs.data_ptr() if sizes else None,
                           ncl.data_ptr(), wptr, ws, _stream(torch, stream))
    _lib.check(st, "ccl_label")
    if side:
        # memory allocated on the current stream and used on another: the
        # allocator must not hand it out again before that stream's work is done
        for t in made:
            t.record_stream(stream)
    del wbuf
    if not sizes:
        return labels
    if side:
        stream.synchronize()
    n = int(ncl.item())
    return labels, roots[:n], szs[:n], n


def ccl_label_noalloc(inp, labels, n_clusters=None, roots=None, sizes=None,
                      mode: str | int = "bonds_periodic", stream=None) -> None:
    """ccl_label into caller-made outputs with the library's static scratch:
    nothing is allocated (for code under graph capture or loops that must not
    allocate).  ``inp`` (H, W) uint8 and ``labels`` (H, W) int32, contiguous, on
    the current device; ``n_clusters`` one int32 or None; ``roots`` and
    ``sizes`` N int32 each or both None.  Enqueued on ``stream`` (default: the
    current stream) without waiting.  Calls that overlap on one GPU share the
    scratch and race; calls on one stream are safe."""
    torch = _torch()
    L = _lib.lib()
    m = _MODES[mode] if isinstance(mode, str) else int(mode)
    if inp.dim() != 2 or inp.dtype != torch.uint8 or inp.device.type != "cuda" or not inp.is_contiguous():
        raise ValueError("input must be a contiguous 2D uint8 GPU tensor")
    H, W = inp.shape
    if (labels.shape != (H, W) or labels.dtype != torch.int32 or labels.device != inp.device
            or not labels.is_contiguous()):
        raise ValueError(f"labels must be a contiguous ({H}, {W}) int32 tensor on {inp.device}")
    for name, t in (("n_clusters", n_clusters), ("roots", roots), ("sizes", sizes)):
        if t is not None and (t.dtype != torch.int32 or t.device != inp.device or not t.is_contiguous()):
            raise ValueError(f"{name} must be a contiguous int32 tensor on {inp.device}")
    if (roots is None) != (sizes is None):
        raise ValueError("roots and sizes go together")
    if roots is not None and (roots.numel() < H * W or sizes.numel() < H * W):
        raise ValueError("roots and sizes need H * W entries each")
    st = L.ccl_label_noalloc(inp.data_ptr(), W, H, m, labels.data_ptr(),
                             roots.data_ptr() if roots is not None else None,
                             sizes.data_ptr() if sizes is not None else None,
                             n_clusters.data_ptr() if n_clusters is not None else None,
                             _stream(torch, stream))
    _lib.check(st, "ccl_label_noalloc")


from .server import CCLServer  # noqa: E402  (needs the helpers above)

__all__.append("CCLServer")
