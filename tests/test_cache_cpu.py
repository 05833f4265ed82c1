"""The software-managed device cache (the paper's section "Memory models and software
managed cache") on the host stand-in backend, no GPU: the plain model in
oracle/cache_model.py pinned by a sequence worked by hand from the paper's rules and by
data coherence, then the library held to the model op by op on seeded random sequences,
with real bytes moved through the views."""

import ctypes
import random

import pytest
import torch

from oracle import cache_model as M

KB = 1024


def D():
    from paper_2203_06777_amd import dwf

    return dwf


# Worked by hand from the paper's rules: watermark three 1 KB buffers; an open moves the
# buffer to the front of the use order, the victim is the last buffer with no open view,
# buffers advised as infrequently used go first, a dirty device copy is written back on
# eviction.  Each row: operation, then the expected (state, resident) of A..E ("-" =
# unknown to the cache) and the counters (host->device, device->host, evictions).
E_, CD, AD, CO = M.EMPTY, M.CPU_DIRTY, M.ACC_DIRTY, M.CONSISTENT
HAND = [
    # op                       A          B          C          D          E         h2d d2h ev
    (("open", "A", M.ACC_READ), [(CO, 1), "-", "-", "-", "-"], (1, 0, 0)),
    (("close", "A"), [(CO, 1), "-", "-", "-", "-"], (1, 0, 0)),
    (("open", "B", M.ACC_WRITE), [(CO, 1), (AD, 1), "-", "-", "-"], (2, 0, 0)),
    (("close", "B"), [(CO, 1), (AD, 1), "-", "-", "-"], (2, 0, 0)),
    (("open", "C", M.ACC_READ), [(CO, 1), (AD, 1), (CO, 1), "-", "-"], (3, 0, 0)),
    (("close", "C"), [(CO, 1), (AD, 1), (CO, 1), "-", "-"], (3, 0, 0)),
    # A becomes the most recent without a copy (it is Consistent); order A, C, B
    (("open", "A", M.CPU_READ), [(CO, 1), (AD, 1), (CO, 1), "-", "-"], (3, 0, 0)),
    (("close", "A"), [(CO, 1), (AD, 1), (CO, 1), "-", "-"], (3, 0, 0)),
    # D needs room: B is least recent, written back, its block reused; order D, A, C
    (("open", "D", M.ACC_READ), [(CO, 1), (E_, 0), (CO, 1), (CO, 1), "-"], (4, 1, 1)),
    (("close", "D"), [(CO, 1), (E_, 0), (CO, 1), (CO, 1), "-"], (4, 1, 1)),
    # C advised infrequent: evicted before A and D although D is more recent than A
    (("advise", "C", M.INFREQUENT), [(CO, 1), (E_, 0), (CO, 1), (CO, 1), "-"], (4, 1, 1)),
    (("open", "E", M.ACC_READ), [(CO, 1), (E_, 0), (E_, 0), (CO, 1), (CO, 1)], (5, 1, 2)),
    (("close", "E"), [(CO, 1), (E_, 0), (E_, 0), (CO, 1), (CO, 1)], (5, 1, 2)),
    # A held open (order A, E, D); B needs room: A is skipped, D (least recent) goes
    (("open", "A", M.ACC_WRITE), [(AD, 1), (E_, 0), (E_, 0), (CO, 1), (CO, 1)], (5, 1, 2)),
    (("open", "B", M.ACC_READ), [(AD, 1), (CO, 1), (E_, 0), (E_, 0), (CO, 1)], (6, 1, 3)),
    (("close", "B"), [(AD, 1), (CO, 1), (E_, 0), (E_, 0), (CO, 1)], (6, 1, 3)),
    # host write to A: its newer device data comes back first, then the host copy is newer
    (("open", "A", M.CPU_WRITE), [(CD, 1), (CO, 1), (E_, 0), (E_, 0), (CO, 1)], (6, 2, 3)),
    (("close", "A"), [(CD, 1), (CO, 1), (E_, 0), (E_, 0), (CO, 1)], (6, 2, 3)),
    (("close", "A"), [(CD, 1), (CO, 1), (E_, 0), (E_, 0), (CO, 1)], (6, 2, 3)),
    # the device view of A needs the host data again
    (("open", "A", M.ACC_READ), [(CO, 1), (CO, 1), (E_, 0), (E_, 0), (CO, 1)], (7, 2, 3)),
    (("close", "A"), [(CO, 1), (CO, 1), (E_, 0), (E_, 0), (CO, 1)], (7, 2, 3)),
    # a host write to a buffer without a device copy leaves it Empty
    (("open", "C", M.CPU_WRITE), [(CO, 1), (CO, 1), (E_, 0), (E_, 0), (CO, 1)], (7, 2, 3)),
    (("close", "C"), [(CO, 1), (CO, 1), (E_, 0), (E_, 0), (CO, 1)], (7, 2, 3)),
]
KEYS = "ABCDE"


def _check_model(m, want, counters):
    snap, (h2d, d2h, ev, _) = m.snapshot()
    for k, w in zip(KEYS, want):
        if w == "-":
            assert k not in snap, k
        else:
            assert (snap[k][0], int(snap[k][2])) == w, (k, snap[k], w)
    assert (h2d, d2h, ev) == counters


def _apply_model(m, op):
    if op[0] == "open":
        m.open(op[1], KB, op[2])
    elif op[0] == "close":
        m.close(op[1])
    elif op[0] == "advise":
        m.advise(op[1], op[2])


def test_model_follows_the_hand_worked_sequence():
    m = M.CacheModel(3 * KB)
    for op, want, counters in HAND:
        _apply_model(m, op)
        _check_model(m, want, counters)


def test_model_every_view_sees_the_last_write():
    """Data coherence over random sequences, and the watermark: the model raises if a view
    shows anything but the last version written (a wrong transition, e.g. an eviction that
    drops a dirty copy, or a device view that misses a host write, would)."""
    rng = random.Random(5)
    for trial in range(40):
        m = M.CacheModel(rng.choice([2, 3, 5]) * KB)
        keys = [f"k{i}" for i in range(rng.choice([3, 6, 9]))]
        held = []
        for step in range(300):
            r = rng.random()
            if held and r < 0.2:
                m.close(held.pop(rng.randrange(len(held))))
            elif r < 0.25:
                k = rng.choice(keys)
                if k in m.entries:
                    m.advise(k, rng.choice([M.NORMAL, M.INFREQUENT]))
            else:
                k = rng.choice(keys)
                intent = rng.randrange(4)
                try:
                    m.open(k, KB, intent)
                except MemoryError:
                    assert all(m.entries[x].refs for x in m.order[0] + m.order[1])
                    continue
                if intent == M.ACC_READ and rng.random() < 0.3 and len(held) < 2:
                    held.append(k)  # keep a read view open for a while (pins the buffer)
                else:
                    m.close(k)
            assert m.held <= m.watermark
            assert sum(e.nbytes for e in m.entries.values() if e.resident) <= m.held


class _Lib:
    """The library cache on the host stand-in backend with 1 KB host buffers."""

    def __init__(self, watermark):
        self.c = D().dwf_cache_create(watermark, D().DWF_CACHE_HOST_SIM)
        self.bufs = {}

    def buf(self, k):
        if k not in self.bufs:
            self.bufs[k] = torch.zeros(KB, dtype=torch.uint8)
        return self.bufs[k]

    def apply(self, op):
        if op[0] == "open":
            return D().dwf_cache_open(self.c, self.buf(op[1]), KB, op[2])
        if op[0] == "close":
            return D().dwf_cache_close(self.c, self.buf(op[1]))
        if op[0] == "advise":
            return D().dwf_cache_advise(self.c, self.buf(op[1]), op[2])

    def snapshot(self, keys):
        out = {}
        for k in keys:
            if k in self.bufs:
                try:
                    st, refs, res = D().dwf_cache_query(self.c, self.bufs[k])
                except D().DwfError:
                    continue
                out[k] = (st, refs, res)
        s = D().dwf_cache_get_stats(self.c)
        return out, (s["h2d_count"], s["d2h_count"], s["evictions"], s["held_bytes"])


def test_library_follows_the_hand_worked_sequence():
    lib = _Lib(3 * KB)
    for op, want, counters in HAND:
        lib.apply(op)
        snap, (h2d, d2h, ev, _) = lib.snapshot(KEYS)
        for k, w in zip(KEYS, want):
            if w != "-":
                assert (snap[k][0], int(snap[k][2])) == w, (op, k, snap[k], w)
        assert (h2d, d2h, ev) == counters, op
    D().dwf_cache_destroy(lib.c)


@pytest.mark.parametrize("seed", range(12))
def test_library_matches_the_model_and_moves_the_bytes(seed):
    """Seeded random sequences: after every operation the library's states, open-view
    counts, residency, copy and eviction counters and bytes held equal the model's; every
    write view writes a fresh byte pattern and every view must show the last one."""
    rng = random.Random(100 + seed)
    wm = rng.choice([2, 3, 4]) * KB
    keys = [f"k{i}" for i in range(rng.choice([3, 5, 8]))]
    m = M.CacheModel(wm)
    lib = _Lib(wm)
    last = {k: 0 for k in keys}
    held = []
    for step in range(250):
        r = rng.random()
        if held and r < 0.2:
            k = held.pop(rng.randrange(len(held)))
            m.close(k)
            lib.apply(("close", k))
        elif r < 0.25:
            k, a = rng.choice(keys), rng.choice([M.NORMAL, M.INFREQUENT])
            if k in m.entries:
                m.advise(k, a)
                lib.apply(("advise", k, a))
        else:
            k, intent = rng.choice(keys), rng.randrange(4)
            try:
                m.open(k, KB, intent)
                model_ok = True
            except MemoryError:
                model_ok = False
            if not model_ok:
                with pytest.raises(D().DwfError) as ei:
                    lib.apply(("open", k, intent))
                assert ei.value.code == -2
                continue
            view = lib.apply(("open", k, intent))
            got = ctypes.string_at(view, KB)
            assert got == bytes([last[k] % 251]) * KB, (step, k, intent)
            if intent in (M.ACC_WRITE, M.CPU_WRITE):
                last[k] += 1
                ctypes.memset(view, last[k] % 251, KB)
            if intent == M.ACC_READ and rng.random() < 0.3 and len(held) < 2:
                held.append(k)
            else:
                m.close(k)
                lib.apply(("close", k))
        msnap, mc = m.snapshot()
        lsnap, lc = lib.snapshot(keys)
        assert {k: (s, r_, bool(res)) for k, (s, r_, res) in msnap.items()} == lsnap, step
        assert mc == lc, step
    for k in held:
        lib.apply(("close", k))
    D().dwf_cache_flush(lib.c)
    for k, t in lib.bufs.items():  # after a flush the host buffers hold the last data
        assert bytes(t.numpy()) == bytes([last[k] % 251]) * KB
    D().dwf_cache_destroy(lib.c)


def test_release_and_destroy_write_back():
    c = D().dwf_cache_create(2 * KB, D().DWF_CACHE_HOST_SIM)
    a, b = torch.zeros(KB, dtype=torch.uint8), torch.zeros(KB, dtype=torch.uint8)
    ctypes.memset(D().dwf_cache_open(c, a, KB, D().DWF_ACC_WRITE), 7, KB)
    D().dwf_cache_close(c, a)
    ctypes.memset(D().dwf_cache_open(c, b, KB, D().DWF_ACC_WRITE), 9, KB)
    D().dwf_cache_close(c, b)
    assert int(a[0]) == 0 and int(b[0]) == 0  # still only on the "device"
    D().dwf_cache_release(c, a)
    assert bytes(a.numpy()) == b"\x07" * KB
    with pytest.raises(D().DwfError):
        D().dwf_cache_query(c, a)
    D().dwf_cache_destroy(c)
    assert bytes(b.numpy()) == b"\x09" * KB


def test_errors():
    c = D().dwf_cache_create(2 * KB, D().DWF_CACHE_HOST_SIM)
    a, b, big = (torch.zeros(KB, dtype=torch.uint8), torch.zeros(KB, dtype=torch.uint8),
                 torch.zeros(4 * KB, dtype=torch.uint8))
    err = D().DwfError
    with pytest.raises(err):
        D().dwf_cache_open(c, a, KB, 7)  # intent
    with pytest.raises(err):
        D().dwf_cache_open(c, big, 4 * KB, D().DWF_ACC_READ)  # above the watermark
    with pytest.raises(err):
        D().dwf_cache_close(c, a)  # no view
    D().dwf_cache_open(c, a, KB, D().DWF_ACC_READ)
    with pytest.raises(err):
        D().dwf_cache_open(c, a, 2 * KB, D().DWF_ACC_READ)  # other size
    with pytest.raises(err):
        D().dwf_cache_release(c, a)  # open view
    with pytest.raises(err):
        D().dwf_cache_advise(c, b, 5)
    D().dwf_cache_open(c, b, KB, D().DWF_ACC_READ)
    x = torch.zeros(KB, dtype=torch.uint8)
    with pytest.raises(err) as ei:  # both resident buffers held open
        D().dwf_cache_open(c, x, KB, D().DWF_ACC_READ)
    assert ei.value.code == -2
    with pytest.raises(err):
        D().dwf_cache_destroy(c)  # views open
    for t in (a, b):
        D().dwf_cache_close(c, t)
    D().dwf_cache_open(c, x, KB, D().DWF_ACC_READ)  # now a buffer can be evicted
    D().dwf_cache_close(c, x)
    with pytest.raises(err):
        D().dwf_cache_create(0, D().DWF_CACHE_HOST_SIM)
    with pytest.raises(err):
        D().dwf_cache_create(KB, 9)
    D().dwf_cache_destroy(c)
