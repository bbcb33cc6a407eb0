"""Host logic of the labeling server's admission queue (no device): requests
that do not fit wait in submission order, are admitted by ``pump`` as room
appears, and can be withdrawn (``cancel``) or dropped after a deadline
(``expire``) while they wait.  The device-side admission is replaced by a stub
that admits while a capacity lasts."""
import collections

import pytest

torch = pytest.importorskip("torch")

from paper_1105_5804_amd._lib import SwccLError  # noqa: E402
from paper_1105_5804_amd.server import CCLServer  # noqa: E402


def _server(capacity):
    srv = object.__new__(CCLServer)  # no device: the queue logic only
    srv._queue = collections.deque()
    srv._inflight = {}
    srv.rejected = []
    srv.admitted = []
    srv.room = capacity
    srv.arena_bytes = 1 << 20
    srv.broken = set()  # tags the stub refuses with a status other than "no room"
    srv.footprint = lambda W, H: 64 * W * H if W > 0 and H > 0 else 0

    def try_submit(tag, img):
        if tag in srv.broken:
            raise SwccLError("ccl_server_submit: device error (4)", 4)
        if srv.room == 0:
            return False
        srv.room -= 1
        slot = len(srv.admitted)
        srv.admitted.append(tag)
        srv._inflight[slot] = (tag, img, img.shape[1], img.shape[0])
        return True

    srv._try_submit = try_submit
    srv.flushes = 0

    def flush():
        srv.flushes += 1

    srv._flush = flush
    return srv


def _img(n=4):
    return torch.zeros((n, n), dtype=torch.uint8)


def test_fifo_admission():
    srv = _server(2)
    for t in range(5):
        srv.submit(t, _img())
    assert srv.admitted == [0, 1] and [q[0] for q in srv._queue] == [2, 3, 4]
    assert srv.pending == 5
    srv.room = 1
    srv.pump()
    assert srv.admitted == [0, 1, 2] and srv.flushes == 1  # the batch admitted so far is labeled
    srv.submit(5, _img())  # the queue is not empty: a new request waits behind it
    assert srv.admitted == [0, 1, 2] and [q[0] for q in srv._queue] == [3, 4, 5]
    srv.room = 10
    srv.pump()
    assert srv.admitted == [0, 1, 2, 3, 4, 5] and not srv._queue


def test_cancel_queued_only():
    srv = _server(1)
    for t in (10, 11, 12, 11):
        srv.submit(t, _img())
    assert srv.cancel(10) is False  # admitted: runs to completion
    assert srv.cancel(11) is True
    assert [q[0] for q in srv._queue] == [12, 11]  # the oldest 11 went first
    assert srv.cancel(11) is True and srv.cancel(11) is False
    assert srv.cancel(99) is False
    srv.room = 5
    srv.pump()
    assert srv.admitted == [10, 12]


def test_expire_by_wait():
    srv = _server(0)
    for t in range(4):
        srv.submit(t, _img())
    t0 = srv._queue[0][2]
    stamps = [t0 - 5.0, t0 - 1.0, t0 - 3.0, t0]  # submit times, as if spread out
    srv._queue = collections.deque((q[0], q[1], s) for q, s in zip(srv._queue, stamps))
    assert srv.expire(10.0, now=t0) == []
    assert srv.expire(2.0, now=t0) == [0, 2]
    assert [q[0] for q in srv._queue] == [1, 3]
    assert srv.expire(0.5, now=t0 + 0.25) == [1]
    assert srv.pending == 1
    srv.room = 1
    srv.pump()
    assert srv.admitted == [3] and srv.pending == 1  # admitted requests stay pending until released


def test_submit_rejects_bad_images():
    srv = _server(1)
    for bad in (torch.zeros(4, dtype=torch.uint8), torch.zeros((4, 4), dtype=torch.int32),
                torch.zeros((4, 4), dtype=torch.uint8).t()[:, ::2]):
        with pytest.raises(ValueError):
            srv.submit(0, bad)
    assert srv.admitted == [] and not srv._queue


def test_submit_refuses_requests_that_can_never_fit():
    """A request larger than the arena (or of an invalid shape) is refused at
    submit and never enters the queue, so it cannot block the ones behind it."""
    srv = _server(0)
    srv.submit(1, _img())  # waits: no room now
    with pytest.raises(SwccLError) as e:
        srv.submit(2, _img(200))  # 64 * 200 * 200 B > arena
    assert e.value.status == 2
    with pytest.raises(SwccLError):
        srv.submit(3, torch.zeros((0, 4), dtype=torch.uint8))
    assert [q[0] for q in srv._queue] == [1]
    srv.room = 1
    srv.pump()
    assert srv.admitted == [1] and not srv._queue


def test_pump_drops_a_request_the_library_refuses():
    """A queued request refused for another reason than lack of room is dropped
    and reported; the requests behind it are admitted."""
    srv = _server(0)
    for t in range(4):
        srv.submit(t, _img())
    srv.broken = {1}
    srv.room = 10
    assert srv.pump() == [1]
    assert srv.admitted == [0, 2, 3] and not srv._queue
    assert srv.rejected == [(1, 4)]
