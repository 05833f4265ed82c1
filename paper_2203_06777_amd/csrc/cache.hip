// Software-managed device cache of host buffers (the paper's MemoryManager:
// section "Memory models and software managed cache").
//
// Each host buffer the caller opens becomes an entry, found by its host address
// in a hash table, that holds the device copy (or none), the size, a count of
// open views and one of four states:
//   Empty             no device copy; the host buffer holds the data
//   CpuDirty          device copy present, the host copy is newer
//   AcceleratorDirty  device copy present and newer than the host copy
//   Consistent        both copies equal
// Opening a view names an intent and moves the whole buffer as that intent and
// the state require:
//   AcceleratorRead   Empty/CpuDirty: host -> device, Consistent; otherwise unchanged
//   AcceleratorWrite  Empty/CpuDirty: host -> device; then AcceleratorDirty
//   CpuRead           AcceleratorDirty: device -> host, Consistent; otherwise unchanged
//   CpuWrite          AcceleratorDirty: device -> host; a device copy becomes CpuDirty
// Accelerator intents return the device address, CPU intents the host address.
// The device bytes held stay under a high watermark: before a new device copy is
// made, entries with no open view are evicted (an AcceleratorDirty one is written
// back first) in least-recently-opened order, entries advised as infrequently used
// before all others.  The order is kept in two doubly linked lists (one per advice)
// with the most recent entry at the front: an open moves its entry to the front
// and the victim is the last entry without an open view, so a touch is O(1).
// Device blocks of evicted entries are kept for reuse by a new entry of the same
// size and count against the watermark until they are freed to make room.
//
// Backend DWF_CACHE_HOST_SIM keeps the "device" copies in host memory and copies
// with memcpy: the same policy, testable without a GPU.
#include <cstdlib>
#include <cstring>
#include <list>
#include <unordered_map>
#include <vector>

#include "dwf_common.h"

struct dwf_cache_s {
    struct Entry {
        void *host = nullptr;
        size_t bytes = 0;
        void *dev = nullptr;
        int state = DWF_ST_EMPTY;
        int refs = 0;
        int advice = DWF_ADVISE_NORMAL;
        std::list<Entry *>::iterator pos;  // place in lru[advice] (valid while dev != nullptr)
    };
    size_t watermark = 0;
    int backend = DWF_CACHE_DEVICE;
    int device = 0;
    size_t held = 0;      // device bytes of resident entries and of the free pool
    size_t resident = 0;  // device bytes of resident entries
    std::unordered_map<void *, Entry *> table;
    std::list<Entry *> lru[2];  // front: most recently opened; [DWF_ADVISE_NORMAL], [DWF_ADVISE_INFREQUENT]
    std::vector<std::pair<void *, size_t>> pool;  // device blocks of evicted entries
    dwf_cache_stats st{};
};

namespace dwf {
namespace {

// Makes the cache's device current for the scope of a call (device backend), restoring the
// caller's device after.
struct OnDevice {
    int prev = -1;
    explicit OnDevice(dwf_cache c) {
        if (c->backend == DWF_CACHE_DEVICE && hipGetDevice(&prev) == hipSuccess && prev != c->device)
            (void)hipSetDevice(c->device);
        else
            prev = -1;
    }
    ~OnDevice() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

int dev_alloc(dwf_cache c, void **p, size_t bytes) {
    if (c->backend == DWF_CACHE_HOST_SIM) {
        *p = std::aligned_alloc(256, (bytes + 255) & ~(size_t)255);
        return *p ? DWF_OK : fail(DWF_ENOMEM, "dwf_cache: host stand-in allocation failed");
    }
    OnDevice on(c);
    if (hipMalloc(p, bytes) != hipSuccess) {
        *p = nullptr;
        return fail(DWF_ENOMEM, "dwf_cache: hipMalloc failed below the watermark");
    }
    return DWF_OK;
}

void dev_free(dwf_cache c, void *p) {
    if (c->backend == DWF_CACHE_HOST_SIM) {
        std::free(p);
        return;
    }
    OnDevice on(c);
    (void)hipFree(p);
}

// to_host: device -> host.  Copies are ordered on `st`; sync waits for them.
int copy(dwf_cache c, dwf_cache_s::Entry *e, bool to_host, hipStream_t st) {
    if (c->backend == DWF_CACHE_HOST_SIM) {
        if (to_host) std::memcpy(e->host, e->dev, e->bytes);
        else std::memcpy(e->dev, e->host, e->bytes);
    } else {
        DWF_HIP(hipMemcpyAsync(to_host ? e->host : e->dev, to_host ? e->dev : e->host, e->bytes,
                               to_host ? hipMemcpyDeviceToHost : hipMemcpyHostToDevice, st));
    }
    if (to_host) {
        c->st.d2h_count += 1;
        c->st.d2h_bytes += e->bytes;
    } else {
        c->st.h2d_count += 1;
        c->st.h2d_bytes += e->bytes;
    }
    return DWF_OK;
}

int sync(dwf_cache c, hipStream_t st) {
    if (c->backend == DWF_CACHE_DEVICE) DWF_HIP(hipStreamSynchronize(st));
    return DWF_OK;
}

// Drops e's device copy (written back first when it is the newer one); the block goes to the pool.
int evict(dwf_cache c, dwf_cache_s::Entry *e, hipStream_t st) {
    if (e->state == DWF_ST_ACC_DIRTY) {
        int rc = copy(c, e, true, st);
        if (rc) return rc;
    }
    c->lru[e->advice].erase(e->pos);
    c->pool.emplace_back(e->dev, e->bytes);
    c->resident -= e->bytes;
    e->dev = nullptr;
    e->state = DWF_ST_EMPTY;
    c->st.evictions += 1;
    return DWF_OK;
}

// The eviction victim: the least recently opened entry without an open view, infrequent ones first.
dwf_cache_s::Entry *victim(dwf_cache c) {
    for (int a : {DWF_ADVISE_INFREQUENT, DWF_ADVISE_NORMAL})
        for (auto it = c->lru[a].rbegin(); it != c->lru[a].rend(); ++it)
            if ((*it)->refs == 0) return *it;
    return nullptr;
}

// A device block of `bytes` for e, evicting and freeing until it fits under the watermark.
int make_resident(dwf_cache c, dwf_cache_s::Entry *e, hipStream_t st) {
    const size_t bytes = e->bytes;
    for (;;) {
        for (size_t k = 0; k < c->pool.size(); ++k)
            if (c->pool[k].second == bytes) {  // reuse: ordered after the evicted entry's write-back on st
                e->dev = c->pool[k].first;
                c->pool.erase(c->pool.begin() + (long)k);
                c->resident += bytes;
                return DWF_OK;
            }
        if (c->held + bytes <= c->watermark) break;
        if (!c->pool.empty()) {  // a block of another size: free it (after the copies that use it)
            int rc = sync(c, st);
            if (rc) return rc;
            dev_free(c, c->pool.back().first);
            c->held -= c->pool.back().second;
            c->pool.pop_back();
            continue;
        }
        dwf_cache_s::Entry *v = victim(c);
        if (!v) return fail(DWF_ENOMEM, "dwf_cache: every resident buffer has an open view; raise the watermark");
        int rc = evict(c, v, st);
        if (rc) return rc;
    }
    int rc = dev_alloc(c, &e->dev, bytes);
    if (rc) return rc;
    c->held += bytes;
    c->resident += bytes;
    return DWF_OK;
}

void touch(dwf_cache c, dwf_cache_s::Entry *e) {
    auto &l = c->lru[e->advice];
    l.splice(l.begin(), l, e->pos);
}

}  // namespace
}  // namespace dwf

using namespace dwf;

extern "C" {

int dwf_cache_create(size_t watermark_bytes, int backend, dwf_cache *out) {
    if (!out) return fail(DWF_EINVAL, "dwf_cache_create: out is NULL");
    *out = nullptr;
    if (backend != DWF_CACHE_DEVICE && backend != DWF_CACHE_HOST_SIM)
        return fail(DWF_EINVAL, "dwf_cache_create: unknown backend");
    if (watermark_bytes == 0) return fail(DWF_EINVAL, "dwf_cache_create: the watermark must be positive");
    dwf_cache c = new (std::nothrow) dwf_cache_s;
    if (!c) return fail(DWF_ENOMEM, "dwf_cache_create: out of host memory");
    c->watermark = watermark_bytes;
    c->backend = backend;
    if (backend == DWF_CACHE_DEVICE && hipGetDevice(&c->device) != hipSuccess) {
        delete c;
        return fail(DWF_EHIP, "dwf_cache_create: hipGetDevice failed");
    }
    c->st.watermark = watermark_bytes;
    *out = c;
    return DWF_OK;
}

int dwf_cache_open(dwf_cache c, void *host, size_t bytes, int intent, void **view, void *stream) {
    if (!c || !host || !view) return fail(DWF_EINVAL, "dwf_cache_open: NULL argument");
    if (intent < DWF_CPU_READ || intent > DWF_ACC_WRITE) return fail(DWF_EINVAL, "dwf_cache_open: unknown intent");
    if (bytes == 0) return fail(DWF_EINVAL, "dwf_cache_open: zero-sized buffer");
    const hipStream_t st = (hipStream_t)stream;
    dwf_cache_s::Entry *e;
    auto it = c->table.find(host);
    if (it == c->table.end()) {
        if (bytes > c->watermark) return fail(DWF_EINVAL, "dwf_cache_open: the buffer is larger than the watermark");
        e = new (std::nothrow) dwf_cache_s::Entry;
        if (!e) return fail(DWF_ENOMEM, "dwf_cache_open: out of host memory");
        e->host = host;
        e->bytes = bytes;
        c->table.emplace(host, e);
    } else {
        e = it->second;
        if (e->bytes != bytes) return fail(DWF_EINVAL, "dwf_cache_open: the buffer was opened with another size");
    }
    int rc;
    if (intent == DWF_ACC_READ || intent == DWF_ACC_WRITE) {
        if (!e->dev) {
            if ((rc = make_resident(c, e, st))) return rc;
            e->pos = c->lru[e->advice].insert(c->lru[e->advice].begin(), e);
            e->state = DWF_ST_CPU_DIRTY;  // the new device copy is stale until the copy below lands
            if ((rc = copy(c, e, false, st))) return rc;
            e->state = DWF_ST_CONSISTENT;
        } else {
            touch(c, e);
            if (e->state == DWF_ST_CPU_DIRTY) {
                if ((rc = copy(c, e, false, st))) return rc;
                e->state = DWF_ST_CONSISTENT;
            }
        }
        if (intent == DWF_ACC_WRITE) e->state = DWF_ST_ACC_DIRTY;
        *view = e->dev;
    } else {
        if (e->dev) touch(c, e);
        if (e->state == DWF_ST_ACC_DIRTY) {
            if ((rc = copy(c, e, true, st))) return rc;
            e->state = DWF_ST_CONSISTENT;
        }
        if (intent == DWF_CPU_WRITE && e->dev) e->state = DWF_ST_CPU_DIRTY;
        // the host may touch the buffer as soon as this returns: every copy queued so far is done
        if ((rc = sync(c, st))) return rc;
        *view = e->host;
    }
    e->refs += 1;
    return DWF_OK;
}

int dwf_cache_close(dwf_cache c, void *host) {
    if (!c || !host) return fail(DWF_EINVAL, "dwf_cache_close: NULL argument");
    auto it = c->table.find(host);
    if (it == c->table.end() || it->second->refs == 0)
        return fail(DWF_EINVAL, "dwf_cache_close: no open view of this buffer");
    it->second->refs -= 1;
    return DWF_OK;
}

int dwf_cache_advise(dwf_cache c, void *host, int advice) {
    if (!c || !host) return fail(DWF_EINVAL, "dwf_cache_advise: NULL argument");
    if (advice != DWF_ADVISE_NORMAL && advice != DWF_ADVISE_INFREQUENT)
        return fail(DWF_EINVAL, "dwf_cache_advise: unknown advice");
    auto it = c->table.find(host);
    if (it == c->table.end()) return fail(DWF_EINVAL, "dwf_cache_advise: buffer not known to the cache");
    dwf_cache_s::Entry *e = it->second;
    if (e->advice == advice) return DWF_OK;
    if (e->dev) {  // keeps its recency rank: front of the other list
        c->lru[e->advice].erase(e->pos);
        e->pos = c->lru[advice].insert(c->lru[advice].begin(), e);
    }
    e->advice = advice;
    return DWF_OK;
}

int dwf_cache_release(dwf_cache c, void *host, void *stream) {
    if (!c || !host) return fail(DWF_EINVAL, "dwf_cache_release: NULL argument");
    auto it = c->table.find(host);
    if (it == c->table.end()) return fail(DWF_EINVAL, "dwf_cache_release: buffer not known to the cache");
    dwf_cache_s::Entry *e = it->second;
    if (e->refs) return fail(DWF_EINVAL, "dwf_cache_release: the buffer has an open view");
    const hipStream_t st = (hipStream_t)stream;
    int rc;
    if (e->dev) {
        if ((rc = evict(c, e, st))) return rc;
        c->st.evictions -= 1;  // counted as a release, not as an eviction
    }
    if ((rc = sync(c, st))) return rc;
    c->table.erase(it);
    delete e;
    return DWF_OK;
}

int dwf_cache_flush(dwf_cache c, void *stream) {
    if (!c) return fail(DWF_EINVAL, "dwf_cache_flush: NULL cache");
    const hipStream_t st = (hipStream_t)stream;
    for (auto &kv : c->table) {
        dwf_cache_s::Entry *e = kv.second;
        if (e->state == DWF_ST_ACC_DIRTY) {
            int rc = copy(c, e, true, st);
            if (rc) return rc;
            e->state = DWF_ST_CONSISTENT;
        }
    }
    return sync(c, st);
}

int dwf_cache_query(dwf_cache c, const void *host, int *state, int *refs, int *resident) {
    if (!c || !host) return fail(DWF_EINVAL, "dwf_cache_query: NULL argument");
    auto it = c->table.find(const_cast<void *>(host));
    if (it == c->table.end()) return fail(DWF_EINVAL, "dwf_cache_query: buffer not known to the cache");
    if (state) *state = it->second->state;
    if (refs) *refs = it->second->refs;
    if (resident) *resident = it->second->dev != nullptr;
    return DWF_OK;
}

int dwf_cache_get_stats(dwf_cache c, dwf_cache_stats *out) {
    if (!c || !out) return fail(DWF_EINVAL, "dwf_cache_get_stats: NULL argument");
    c->st.entries = (long long)c->table.size();
    c->st.resident_bytes = c->resident;
    c->st.held_bytes = c->held;
    *out = c->st;
    return DWF_OK;
}

int dwf_cache_destroy(dwf_cache c, void *stream) {
    if (!c) return DWF_OK;
    for (auto &kv : c->table)
        if (kv.second->refs) return fail(DWF_EINVAL, "dwf_cache_destroy: a buffer has an open view");
    int rc = dwf_cache_flush(c, stream);
    if (rc) return rc;
    for (auto &kv : c->table) {
        if (kv.second->dev) dev_free(c, kv.second->dev);
        delete kv.second;
    }
    for (auto &b : c->pool) dev_free(c, b.first);
    delete c;
    return DWF_OK;
}

}  // extern "C"
