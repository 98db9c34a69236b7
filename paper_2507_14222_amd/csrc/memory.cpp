// Device memory of libig: where model buffers and fit scratch come from.
//
// Without a caller allocator, memory comes from a per-device arena: large chunks
// taken from the runtime once and sub-allocated (best fit, freed ranges coalesced
// with their neighbours inside a chunk).  Repeated fits then never return memory
// to the runtime nor ask it for new multi-GB blocks (runtime allocation of such
// blocks after earlier frees stalled the host for up to seconds).  Chunks go back
// only when the arena cannot grow, or when the caller asks (ig_release_memory).
//
// Scratch is stream-ordered on top of that: a freed scratch block keeps an event
// recorded on the freeing stream, and whoever takes the block next makes its own
// stream wait for that event (free when it is the same stream).
//
// With a caller allocator (ig_fit_opts.alloc), every model buffer and every
// scratch block of the call comes from it instead; a model remembers the
// allocator and hands its buffers back to it when it is freed.
#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "common.h"

namespace ig {

namespace {
constexpr int kMaxDev = 64;
constexpr size_t kAlign = 256;
constexpr size_t kChunk = (size_t)1 << 30;   // smallest chunk taken from the runtime

size_t align_up(size_t b, size_t a) { return (b + a - 1) / a * a; }

struct Arena {
    struct Chunk {
        char *base;
        size_t size;
    };
    std::vector<Chunk> chunks;
    std::map<char *, size_t> free_at;               // start -> bytes
    std::multimap<size_t, char *> free_by_size;     // bytes -> start
    std::unordered_map<void *, size_t> live;        // start -> bytes
    size_t reserved = 0, in_use = 0;

    const Chunk *chunk_of(char *p) const {
        for (const Chunk &c : chunks)
            if (p >= c.base && p < c.base + c.size) return &c;
        return nullptr;
    }
    void erase_free(std::map<char *, size_t>::iterator it) {
        auto range = free_by_size.equal_range(it->second);
        for (auto j = range.first; j != range.second; ++j)
            if (j->second == it->first) {
                free_by_size.erase(j);
                break;
            }
        free_at.erase(it);
    }
    void insert_free(char *p, size_t b) {
        free_at[p] = b;
        free_by_size.emplace(b, p);
    }
    // a free range back, merged with free neighbours of the same chunk
    void put(char *p, size_t b) {
        const Chunk *ch = chunk_of(p);
        auto next = free_at.lower_bound(p);
        if (next != free_at.end() && next->first == p + b && next->first < ch->base + ch->size) {
            b += next->second;
            erase_free(next);
        }
        auto it = free_at.lower_bound(p);
        if (it != free_at.begin()) {
            auto prev = std::prev(it);
            if (prev->first + prev->second == p && prev->first >= ch->base) {
                p = prev->first;
                b += prev->second;
                erase_free(prev);
            }
        }
        insert_free(p, b);
    }
    void *take(size_t want) {
        auto it = free_by_size.lower_bound(want);
        if (it == free_by_size.end()) return nullptr;
        char *p = it->second;
        const size_t b = it->first;
        erase_free(free_at.find(p));
        if (b > want) insert_free(p + want, b - want);
        live[p] = want;
        in_use += want;
        return p;
    }
    // chunks that are wholly free go back to the runtime
    void trim() {
        for (size_t i = chunks.size(); i-- > 0;) {
            auto it = free_at.find(chunks[i].base);
            if (it == free_at.end() || it->second != chunks[i].size) continue;
            erase_free(it);
            (void)hipFree(chunks[i].base);
            reserved -= chunks[i].size;
            chunks.erase(chunks.begin() + (ptrdiff_t)i);
        }
    }
};

struct CachedBlock {
    void *p;
    size_t bytes;
    hipEvent_t ev;
};

struct DeviceMemory {
    Arena arena;
    std::vector<CachedBlock> cached;           // freed scratch waiting for reuse
    std::unordered_map<void *, size_t> scratch_live;
    std::vector<hipEvent_t> spare_events;
    size_t cached_bytes = 0;
};

struct Memory {
    std::mutex mu;
    DeviceMemory dev[kMaxDev];
};
Memory &mem() {
    static Memory *m = new Memory();   // never destroyed: frees may run at exit
    return *m;
}

#ifndef IG_SCRATCH_CACHE_GB
#define IG_SCRATCH_CACHE_GB 32
#endif
constexpr size_t kCacheCap = (size_t)IG_SCRATCH_CACHE_GB << 30;   // cached scratch bytes per device

size_t round_scratch(size_t b) {
    if (b <= 4096) return 4096;
    const int lg = 63 - __builtin_clzll((unsigned long long)(b - 1));
    const size_t step = (size_t)1 << (lg - 3);   // eight sizes per power of two
    return (b + step - 1) / step * step;
}

int current_device() {
    int d = 0;
    IG_HIP(hipGetDevice(&d));
    IG_REQUIRE(d >= 0 && d < kMaxDev, IG_E_UNSUPPORTED, "device index above 63");
    return d;
}

void arena_free(DeviceMemory &dm, void *p) {
    auto it = dm.arena.live.find(p);
    if (it == dm.arena.live.end()) return;
    const size_t b = it->second;
    dm.arena.live.erase(it);
    dm.arena.in_use -= b;
    dm.arena.put(static_cast<char *>(p), b);
}

// cached scratch of a device back into its arena (lock held)
void drop_cached(DeviceMemory &dm, size_t keep) {
    std::sort(dm.cached.begin(), dm.cached.end(),
              [](const CachedBlock &x, const CachedBlock &y) { return x.bytes < y.bytes; });
    for (size_t i = dm.cached.size(); i-- > 0 && dm.cached_bytes > keep;) {
        CachedBlock b = dm.cached[i];
        (void)hipEventSynchronize(b.ev);
        dm.spare_events.push_back(b.ev);
        dm.cached_bytes -= b.bytes;
        dm.cached.erase(dm.cached.begin() + (ptrdiff_t)i);
        arena_free(dm, b.p);
    }
}

// arena allocation of `bytes` (lock held): grows by a chunk, or after dropping the
// cached scratch and trimming free chunks, once more
void *arena_alloc(DeviceMemory &dm, size_t bytes) {
    const size_t want = align_up(bytes ? bytes : 1, kAlign);
    if (void *p = dm.arena.take(want)) return p;
    for (int attempt = 0; attempt < 2; ++attempt) {
        if (attempt) {
            drop_cached(dm, 0);
            if (void *p = dm.arena.take(want)) return p;
            dm.arena.trim();
        }
        const size_t size = align_up(std::max(want, kChunk), (size_t)2 << 20);
        void *c = nullptr;
        if (hipMalloc(&c, size) == hipSuccess && c) {
            dm.arena.chunks.push_back({static_cast<char *>(c), size});
            dm.arena.reserved += size;
            dm.arena.insert_free(static_cast<char *>(c), size);
            return dm.arena.take(want);
        }
        (void)hipGetLastError();
    }
    return nullptr;
}

thread_local const ig_allocator *t_user = nullptr;   // the caller allocator of the running call
}  // namespace

UserAllocScope::UserAllocScope(const ig_allocator *a) : prev(t_user) {
    if (a) {
        IG_REQUIRE(a->alloc && a->free, IG_E_INVAL, "allocator without alloc or free");
        t_user = a;
    }
}
UserAllocScope::~UserAllocScope() { t_user = prev; }
const ig_allocator *current_user_allocator() { return t_user; }

void *device_alloc(size_t bytes, hipStream_t s, const ig_allocator *user) {
    if (user) {
        void *p = user->alloc(bytes ? bytes : 1, (void *)s, user->ctx);
        if (!p) throw Error(IG_E_NOMEM, "the caller's allocator returned no memory for " + std::to_string(bytes) +
                                            " bytes");
        return p;
    }
    const int d = current_device();
    Memory &m = mem();
    std::lock_guard<std::mutex> lock(m.mu);
    void *p = arena_alloc(m.dev[d], bytes);
    if (!p) throw Error(IG_E_NOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed");
    return p;
}

void device_free(void *p, int dev, const ig_allocator *user) noexcept {
    if (!p) return;
    if (user) {
        user->free(p, nullptr, user->ctx);
        return;
    }
    if (dev < 0 || dev >= kMaxDev) return;
    Memory &m = mem();
    std::lock_guard<std::mutex> lock(m.mu);
    arena_free(m.dev[dev], p);
}

void *scratch_alloc(size_t bytes, hipStream_t s) {
    if (const ig_allocator *u = t_user) {
        void *p = u->alloc(bytes ? bytes : 1, (void *)s, u->ctx);
        if (!p) throw Error(IG_E_NOMEM, "the caller's allocator returned no scratch of " + std::to_string(bytes) +
                                            " bytes");
        return p;
    }
    const int d = current_device();
    const size_t want = round_scratch(bytes ? bytes : 1);
    Memory &m = mem();
    std::lock_guard<std::mutex> lock(m.mu);
    DeviceMemory &dm = m.dev[d];
    size_t best = SIZE_MAX, bi = 0;
    for (size_t i = 0; i < dm.cached.size(); ++i) {
        const CachedBlock &b = dm.cached[i];
        if (b.bytes >= want && b.bytes <= 2 * want && b.bytes < best) {
            best = b.bytes;
            bi = i;
        }
    }
    if (best != SIZE_MAX) {
        CachedBlock b = dm.cached[bi];
        IG_HIP(hipStreamWaitEvent(s, b.ev, 0));
        dm.cached.erase(dm.cached.begin() + (ptrdiff_t)bi);
        dm.spare_events.push_back(b.ev);
        dm.cached_bytes -= b.bytes;
        dm.scratch_live[b.p] = b.bytes;
        return b.p;
    }
    void *p = arena_alloc(dm, want);
    if (!p) throw Error(IG_E_NOMEM, "device scratch allocation of " + std::to_string(bytes) + " bytes failed");
    dm.scratch_live[p] = align_up(want, kAlign);
    return p;
}

void scratch_free(void *p, hipStream_t s) noexcept {
    if (!p) return;
    if (const ig_allocator *u = t_user) {
        u->free(p, (void *)s, u->ctx);
        return;
    }
    int d = 0;
    if (hipGetDevice(&d) != hipSuccess || d < 0 || d >= kMaxDev) {
        (void)hipGetLastError();
        return;
    }
    Memory &m = mem();
    std::lock_guard<std::mutex> lock(m.mu);
    DeviceMemory &dm = m.dev[d];
    auto it = dm.scratch_live.find(p);
    if (it == dm.scratch_live.end()) return;
    const size_t bytes = it->second;
    dm.scratch_live.erase(it);
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    (void)hipStreamIsCapturing(s, &cap);
    hipEvent_t ev = nullptr;
    if (cap == hipStreamCaptureStatusNone) {
        if (!dm.spare_events.empty()) {
            ev = dm.spare_events.back();
            dm.spare_events.pop_back();
        } else if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
            (void)hipGetLastError();
            ev = nullptr;
        }
    }
    if (!ev || hipEventRecord(ev, s) != hipSuccess) {
        // no event to order a later user after this stream's work: wait here instead
        (void)hipGetLastError();
        if (ev) dm.spare_events.push_back(ev);
        if (cap == hipStreamCaptureStatusNone) (void)hipStreamSynchronize(s);
        arena_free(dm, p);
        return;
    }
    dm.cached.push_back({p, bytes, ev});
    dm.cached_bytes += bytes;
    if (dm.cached_bytes > kCacheCap) drop_cached(dm, kCacheCap / 2);
}

// ------------------------------------------------------------- uploads ----
// Host tables go to the device through a pinned staging ring per device, so that
// the copy is queued on the stream and the host goes on at once (a copy from
// pageable memory returns only when the copy is done, which waits for the work
// queued before it).  Each upload records an event; a range of the ring is taken
// again only after the events of the uploads that used it have completed.
namespace {
constexpr size_t kRing = (size_t)8 << 20;   // bytes per device
constexpr size_t kRingMax = kRing / 4;      // larger uploads are copied directly

struct Pending {
    size_t lo, hi;
    hipEvent_t ev;
};

struct Ring {
    std::mutex mu;
    char *base = nullptr;
    bool failed = false;
    size_t head = 0;
    std::vector<Pending> pending;   // in ring order
    std::vector<hipEvent_t> spare;
};

Ring &ring(int d) {
    static Ring *r = new Ring[kMaxDev];   // never destroyed: uploads may run at exit
    return r[d];
}
}  // namespace

void upload(void *dst, const void *src, size_t bytes, hipStream_t s) {
    if (!bytes) return;
    const int d = current_device();
    Ring &r = ring(d);
    std::unique_lock<std::mutex> lock(r.mu);
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    (void)hipStreamIsCapturing(s, &cap);
    if (!r.base && !r.failed && hipHostMalloc((void **)&r.base, kRing, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        r.base = nullptr;
        r.failed = true;
    }
    if (!r.base || bytes > kRingMax || cap != hipStreamCaptureStatusNone) {
        lock.unlock();
        IG_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s));
        return;
    }
    const size_t want = align_up(bytes, 256);
    size_t lo = r.head;
    if (lo + want > kRing) lo = 0;
    const size_t hi = lo + want;
    // wait for the uploads that used [lo, hi), oldest first
    for (size_t i = 0; i < r.pending.size();) {
        Pending &q = r.pending[i];
        if (q.lo < hi && lo < q.hi) {
            IG_HIP(hipEventSynchronize(q.ev));
            r.spare.push_back(q.ev);
            r.pending.erase(r.pending.begin() + (ptrdiff_t)i);
        } else {
            ++i;
        }
    }
    std::memcpy(r.base + lo, src, bytes);
    IG_HIP(hipMemcpyAsync(dst, r.base + lo, bytes, hipMemcpyHostToDevice, s));
    hipEvent_t ev = nullptr;
    if (!r.spare.empty()) {
        ev = r.spare.back();
        r.spare.pop_back();
    } else {
        IG_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    }
    IG_HIP(hipEventRecord(ev, s));
    r.pending.push_back({lo, hi, ev});
    r.head = hi;
}

void release_memory() {
    const int d = current_device();
    Memory &m = mem();
    std::lock_guard<std::mutex> lock(m.mu);
    drop_cached(m.dev[d], 0);
    m.dev[d].arena.trim();
}

void memory_stats(uint64_t *reserved, uint64_t *in_use, uint64_t *cached) {
    const int d = current_device();
    Memory &m = mem();
    std::lock_guard<std::mutex> lock(m.mu);
    *reserved = m.dev[d].arena.reserved;
    *in_use = m.dev[d].arena.in_use - m.dev[d].cached_bytes;
    *cached = m.dev[d].cached_bytes;
}

}  // namespace ig
