"""Plain model of the software-managed device cache (test infrastructure).

Only tests/ use this module.  It follows the paper's description of its
MemoryManager (section "Memory models and software managed cache") step by step,
with plain Python containers and no attention to speed:

* a table of entries keyed by the host buffer, each with its size, whether a
  device copy exists, a count of open views and one of the states Empty,
  CpuDirty, AcceleratorDirty and Consistent;
* opening a view names one of the intents CpuRead, CpuWrite, AcceleratorRead,
  AcceleratorWrite and migrates the whole buffer as the state requires;
* the device bytes held stay below a high watermark; to make room, entries with
  no open view are evicted in least-recently-used order (every access moves an
  entry to the front of the order), entries advised as infrequently used first.

Readings where the paper is silent (each listed in the design notes):
AcceleratorWrite is a read-write view (the host data is copied in first);
CpuWrite of a buffer with a device copy leaves it CpuDirty, of one without a
device copy leaves it Empty; an evicted entry's device block is kept for reuse
by a new entry of the same size and counts against the watermark until it is
freed to make room (other sizes are freed, most recently evicted first, before
any further entry is evicted); a new device copy goes to the front of the order;
changing the advice keeps an entry's recency, at the front of the other class.

The model also tracks data versions (a counter bumped by every write view) on
both sides so tests can check that every view sees the last data written.
"""

CPU_READ, CPU_WRITE, ACC_READ, ACC_WRITE = 0, 1, 2, 3
EMPTY, CPU_DIRTY, ACC_DIRTY, CONSISTENT = 0, 1, 2, 3
NORMAL, INFREQUENT = 0, 1


class Entry:
    def __init__(self, key, nbytes):
        self.key = key
        self.nbytes = nbytes
        self.state = EMPTY
        self.refs = 0
        self.resident = False
        self.advice = NORMAL
        self.host_version = 0  # version of the data in the host buffer
        self.dev_version = None  # version in the device copy (None: no copy)


class CacheModel:
    def __init__(self, watermark):
        self.watermark = watermark
        self.entries = {}
        self.order = {NORMAL: [], INFREQUENT: []}  # index 0 = most recently used
        self.pool = []  # sizes of device blocks kept for reuse, in eviction order
        self.held = 0
        self.h2d = self.d2h = self.evictions = 0
        self.latest = {}  # key -> version of the last data written through any view

    # --- helpers -------------------------------------------------------------
    def _copy_in(self, e):
        e.dev_version = e.host_version
        self.h2d += 1

    def _copy_out(self, e):
        e.host_version = e.dev_version
        self.d2h += 1

    def _evict(self, e):
        if e.state == ACC_DIRTY:
            self._copy_out(e)
        self.order[e.advice].remove(e.key)
        self.pool.append(e.nbytes)
        e.resident = False
        e.dev_version = None
        e.state = EMPTY
        self.evictions += 1

    def _victim(self):
        for adv in (INFREQUENT, NORMAL):
            for key in reversed(self.order[adv]):
                if self.entries[key].refs == 0:
                    return self.entries[key]
        return None

    def _make_resident(self, e):
        while True:
            if e.nbytes in self.pool:
                self.pool.remove(e.nbytes)
                break
            if self.held + e.nbytes <= self.watermark:
                self.held += e.nbytes
                break
            if self.pool:
                self.held -= self.pool.pop()
                continue
            v = self._victim()
            if v is None:
                raise MemoryError("every resident buffer has an open view")
            self._evict(v)
        e.resident = True
        self.order[e.advice].insert(0, e.key)

    def _touch(self, e):
        lst = self.order[e.advice]
        lst.remove(e.key)
        lst.insert(0, e.key)

    # --- the operations ------------------------------------------------------
    def open(self, key, nbytes, intent):
        if key not in self.entries:
            if nbytes > self.watermark:
                raise ValueError("buffer larger than the watermark")
            self.entries[key] = Entry(key, nbytes)
            self.latest.setdefault(key, 0)
        e = self.entries[key]
        if e.nbytes != nbytes:
            raise ValueError("size differs from the registered one")
        if intent in (ACC_READ, ACC_WRITE):
            if not e.resident:
                self._make_resident(e)
                self._copy_in(e)
                e.state = CONSISTENT
            else:
                self._touch(e)
                if e.state == CPU_DIRTY:
                    self._copy_in(e)
                    e.state = CONSISTENT
            if intent == ACC_WRITE:
                e.state = ACC_DIRTY
        else:
            if e.resident:
                self._touch(e)
            if e.state == ACC_DIRTY:
                self._copy_out(e)
                e.state = CONSISTENT
            if intent == CPU_WRITE and e.resident:
                e.state = CPU_DIRTY
        e.refs += 1
        # what the view shows, and the write it may make
        seen = e.dev_version if intent in (ACC_READ, ACC_WRITE) else e.host_version
        if seen != self.latest[key]:
            raise AssertionError(f"view of {key} shows version {seen}, last written {self.latest[key]}")
        if intent in (ACC_WRITE, CPU_WRITE):
            self.latest[key] += 1
            if intent == ACC_WRITE:
                e.dev_version = self.latest[key]
            else:
                e.host_version = self.latest[key]
        return e

    def close(self, key):
        e = self.entries.get(key)
        if e is None or e.refs == 0:
            raise ValueError("no open view")
        e.refs -= 1

    def advise(self, key, advice):
        e = self.entries[key]
        if e.advice == advice:
            return
        if e.resident:
            self.order[e.advice].remove(key)
            self.order[advice].insert(0, key)
        e.advice = advice

    def release(self, key):
        e = self.entries[key]
        if e.refs:
            raise ValueError("open view")
        if e.resident:
            self._evict(e)
            self.evictions -= 1
        del self.entries[key]

    def flush(self):
        for e in self.entries.values():
            if e.state == ACC_DIRTY:
                self._copy_out(e)
                e.state = CONSISTENT

    def snapshot(self):
        """(state, refs, resident) of every entry and the counters."""
        return ({k: (e.state, e.refs, e.resident) for k, e in self.entries.items()},
                (self.h2d, self.d2h, self.evictions, self.held))
