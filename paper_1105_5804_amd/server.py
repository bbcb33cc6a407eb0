"""Served connected-component labeling: a thin layer over the ``ccl_server_*``
C ABI (argument marshalling only).

Requests are host images labeled as they arrive.  The library admits a request
when its footprint fits in the device arena (``SW_ERR_STATE`` otherwise: the
request waits here, in submission order), spreads requests over the given
streams, and reports completions through ``poll``.  A request still waiting
for admission can be withdrawn (``cancel``) or dropped after a deadline
(``expire``); an admitted one runs to completion.  A request that can never
be admitted (an invalid shape, or a footprint larger than the arena) is refused
by ``submit``; one the library refuses later for another reason is dropped from
the queue by ``pump`` and reported in ``rejected``.
"""
from __future__ import annotations

import collections
import ctypes
import time

from . import _lib
from . import _MODES, _torch

_STATE = _lib.SW_ERR_STATE


class CCLServer:
    """Label host images (``(H, W)`` uint8 CPU tensors, ideally pinned) on the GPU.

    arena_bytes of device memory hold the requests in flight; ``sizes`` adds
    the sorted roots and sizes of every request's clusters.  Requests of at
    most ``batch_px`` pixels are batched: those admitted between two pumps
    (or polls) are labeled together, one launch per phase for all of them.
    """

    def __init__(self, arena_bytes: int, mode: str | int = "sites_open", sizes: bool = True,
                 max_inflight: int = 256, n_streams: int = 4, device: str = "cuda", batch_px: int = 0):
        torch = _torch()
        L = _lib.lib()
        self.mode = _MODES[mode] if isinstance(mode, str) else int(mode)
        self.sizes = bool(sizes)
        self.params = _lib.CclServerParams(self.mode, 1 if sizes else 0, int(max_inflight), int(n_streams),
                                           int(batch_px))
        self.device = torch.device(device)
        # streams at the default priority
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(n_streams)]
        self._arena = torch.empty(int(arena_bytes) + 256, dtype=torch.uint8, device=self.device)
        base = self._arena.data_ptr()
        self._arena_ptr = base + ((-base) % 256)
        self._arena_off = self._arena_ptr - base
        arr = (ctypes.c_void_p * n_streams)(*[s.cuda_stream for s in self.streams])
        self._h = ctypes.c_void_p()
        _lib.check(L.ccl_server_create(ctypes.byref(self._h), ctypes.byref(self.params), self._arena_ptr,
                                       int(arena_bytes), arr), "ccl_server_create")
        self.arena_bytes = int(arena_bytes)
        self._queue = collections.deque()   # (tag, image, submit time) waiting for admission
        self._inflight = {}                 # slot -> (tag, image, W, H)
        cap = int(max_inflight)
        self.rejected = []                  # (tag, status) dropped from the queue by pump
        self._pslots = (ctypes.c_int32 * cap)()
        self._ptags = (ctypes.c_uint64 * cap)()

    def footprint(self, W: int, H: int) -> int:
        return int(_lib.lib().ccl_server_footprint(int(W), int(H), ctypes.byref(self.params)))

    def _try_submit(self, tag: int, img) -> bool:
        H, W = img.shape
        slot = ctypes.c_int32()
        st = _lib.lib().ccl_server_submit(self._h, img.data_ptr(), W, H, img.stride(0), tag, ctypes.byref(slot))
        if st == _STATE:
            return False
        _lib.check(st, "ccl_server_submit")
        self._inflight[slot.value] = (tag, img, W, H)
        return True

    def submit(self, tag: int, img) -> None:
        """Queue a request; it is admitted at once if the arena has room.
        Raises for a request that could never be admitted (nothing is queued)."""
        if img.dim() != 2 or img.dtype.itemsize != 1 or img.device.type != "cpu" or img.stride(1) != 1:
            raise ValueError("a request is a 2D uint8 CPU tensor with unit column stride")
        H, W = img.shape
        fp = self.footprint(W, H)
        if fp == 0 or fp > self.arena_bytes:
            raise _lib.SwccLError(f"ccl_server_submit: a {W}x{H} request can never be admitted "
                                  f"(footprint {fp} B, arena {self.arena_bytes} B)", _lib.SW_ERR_SIZE)
        if self._queue or not self._try_submit(tag, img):
            self._queue.append((tag, img, time.monotonic()))

    def _flush(self) -> None:
        _lib.check(_lib.lib().ccl_server_flush(self._h), "ccl_server_flush")

    def pump(self) -> list:
        """Admit queued requests, in order, while they fit, then label the open
        batch.  A queued request the library refuses for any reason other than
        lack of room is dropped (so it cannot block the requests behind it);
        returns the tags dropped by this call, which are also appended, with
        their status, to ``rejected``."""
        dropped = []
        while self._queue:
            tag, img, _ = self._queue[0]
            try:
                if not self._try_submit(tag, img):
                    break
            except _lib.SwccLError as e:
                self.rejected.append((tag, e.status))
                dropped.append(tag)
            self._queue.popleft()
        self._flush()
        return dropped

    def cancel(self, tag: int) -> bool:
        """Withdraw the oldest queued request with this tag (True if there was
        one).  An admitted request cannot be withdrawn from the device: poll and
        release it."""
        for k, item in enumerate(self._queue):
            if item[0] == tag:
                del self._queue[k]
                return True
        return False

    def expire(self, max_wait: float, now: float | None = None) -> list:
        """Withdraw the queued requests that have waited more than max_wait
        seconds since their submit (``now`` defaults to time.monotonic());
        returns their tags in queue order."""
        now = time.monotonic() if now is None else now
        gone = [item[0] for item in self._queue if now - item[2] > max_wait]
        if gone:
            self._queue = collections.deque(item for item in self._queue if now - item[2] <= max_wait)
        return gone

    def poll(self) -> list:
        """[(slot, tag)] of requests completed since the last poll (non-blocking)."""
        n = ctypes.c_int32()
        cap = len(self._pslots)
        _lib.check(_lib.lib().ccl_server_poll(self._h, self._pslots, self._ptags, cap, ctypes.byref(n)),
                   "ccl_server_poll")
        return [(int(self._pslots[i]), int(self._ptags[i])) for i in range(n.value)]

    def result(self, slot: int):
        """(labels (H, W), roots, sizes, n) of a completed request as views of the
        arena (valid until release); roots and sizes are None without sizes."""
        torch = _torch()
        ptrs = [ctypes.c_void_p() for _ in range(4)]
        _lib.check(_lib.lib().ccl_server_result(self._h, int(slot), *[ctypes.byref(p) for p in ptrs]),
                   "ccl_server_result")
        _, _, W, H = self._inflight[slot]
        N = W * H

        def view(ptr, count, shape=None):
            off = ptr - self._arena_ptr + self._arena_off
            t = self._arena[off:off + 4 * count].view(torch.int32)
            return t.view(shape) if shape else t

        ncl = int(view(ptrs[3].value, 1).item())
        labels = view(ptrs[0].value, N, (H, W))
        if not self.sizes:
            return labels, None, None, ncl
        return labels, view(ptrs[1].value, ncl), view(ptrs[2].value, ncl), ncl

    def release(self, slot: int) -> None:
        """Return a request's arena block.  Work the caller has enqueued on the
        current stream (e.g. a copy of the result views) finishes before any
        later request can write the block: every server stream waits for it."""
        torch = _torch()
        ev = torch.cuda.Event()
        ev.record(torch.cuda.current_stream(self.device))
        for s in self.streams:
            s.wait_event(ev)
        _lib.check(_lib.lib().ccl_server_release(self._h, int(slot)), "ccl_server_release")
        del self._inflight[slot]

    @property
    def pending(self) -> int:
        return len(self._queue) + len(self._inflight)

    def close(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.lib().ccl_server_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
