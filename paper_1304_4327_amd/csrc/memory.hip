// Caching device allocator for trees and per-call scratch.
//
// hipMalloc maps fresh memory and hipFree waits for the whole device; the
// runtime's stream-ordered pool avoids the wait but still costs tens of
// microseconds per call.  A build or a search takes a dozen buffers, so the
// library keeps released blocks on a per-device free list and hands them out
// again:
//   * a block released on stream s is recorded with an event on s (blocks
//     released together share one event, counted by reference);
//   * a later request on the same stream takes it at once (stream order puts
//     the new work after everything queued before the release);
//   * a request on another stream first makes its stream wait for the event.
// Blocks stay with the process until knn_release_cached_memory(), or until a
// hipMalloc runs out of memory, which releases the device's cached blocks and
// tries once more.
#include "common.hpp"

#include <map>
#include <mutex>
#include <unordered_map>
#include <vector>

namespace knnx {
namespace {

// an event shared by the blocks of one release
struct SharedEvent {
    hipEvent_t ev = nullptr;
    int refs = 0;
};

struct Block {
    void *p = nullptr;
    size_t bytes = 0;
    int device = 0;
    hipStream_t stream = nullptr;  // stream of the last release
    SharedEvent *ready = nullptr;  // recorded on that stream at release
};

void drop_ref(SharedEvent *&r) {
    if (r && --r->refs == 0) {
        (void)hipEventDestroy(r->ev);
        delete r;
    }
    r = nullptr;
}

constexpr int kMaxDevices = 64;

struct Cache {
    std::mutex mu;
    std::unordered_map<void *, Block> live;                // handed out
    std::multimap<size_t, Block> free_blocks[kMaxDevices];  // by size
};

Cache &cache() {
    static Cache *c = new Cache();  // never destroyed: blocks may be released
                                    // from static destructors of callers
    return *c;
}

size_t round_bytes(size_t b) {
    if (b <= (size_t(1) << 20)) return (b + 511) & ~size_t(511);
    return (b + (size_t(2) << 20) - 1) & ~((size_t(2) << 20) - 1);
}

// frees every cached block of one device; caller holds the lock
hipError_t drain_device(Cache &c, int dev) {
    hipError_t first = hipSuccess;
    for (auto &kv : c.free_blocks[dev]) {
        Block &b = kv.second;
        if (b.ready) {
            hipError_t e = hipEventSynchronize(b.ready->ev);
            if (first == hipSuccess) first = e;
            drop_ref(b.ready);
        }
        hipError_t e = hipFree(b.p);
        if (first == hipSuccess) first = e;
    }
    c.free_blocks[dev].clear();
    return first;
}

}  // namespace

hipError_t dev_alloc(void **out, size_t bytes, hipStream_t s) {
    *out = nullptr;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    const size_t need = round_bytes(bytes == 0 ? 1 : bytes);
    Cache &c = cache();
    std::lock_guard<std::mutex> lock(c.mu);
    auto &fl = c.free_blocks[dev];
    auto it = fl.lower_bound(need);
    // take a cached block unless it is much larger than asked for
    if (it != fl.end() && it->first <= std::max(2 * need, need + (size_t(4) << 20))) {
        Block b = it->second;
        fl.erase(it);
        if (b.ready && b.stream != s) {
            e = hipStreamWaitEvent(s, b.ready->ev, 0);
            if (e != hipSuccess) {
                fl.emplace(b.bytes, b);
                return e;
            }
        }
        drop_ref(b.ready);
        c.live.emplace(b.p, b);
        *out = b.p;
        return hipSuccess;
    }
    void *p = nullptr;
    e = hipMalloc(&p, need);
    if (e == hipErrorOutOfMemory) {
        (void)hipGetLastError();
        (void)drain_device(c, dev);
        e = hipMalloc(&p, need);
    }
    if (e != hipSuccess) return e;
    Block b;
    b.p = p;
    b.bytes = need;
    b.device = dev;
    c.live.emplace(p, b);
    *out = p;
    return hipSuccess;
}

void dev_free_many(void *const *ps, int n, hipStream_t s) {
    Cache &c = cache();
    std::lock_guard<std::mutex> lock(c.mu);
    SharedEvent *ev = nullptr;  // created on the first block that needs it
    bool synced = false;
    for (int i = 0; i < n; ++i) {
        if (!ps[i]) continue;
        auto it = c.live.find(ps[i]);
        if (it == c.live.end()) continue;  // not ours: ignore rather than corrupt the lists
        Block b = it->second;
        c.live.erase(it);
        b.stream = s;
        if (!ev && !synced) {
            int cur = 0;
            const bool switch_dev = hipGetDevice(&cur) == hipSuccess && cur != b.device;
            if (switch_dev) (void)hipSetDevice(b.device);
            ev = new SharedEvent();
            if (hipEventCreateWithFlags(&ev->ev, hipEventDisableTiming) != hipSuccess ||
                hipEventRecord(ev->ev, s) != hipSuccess) {
                // no event: the blocks can only be reused after the stream is idle
                if (ev->ev) (void)hipEventDestroy(ev->ev);
                delete ev;
                ev = nullptr;
                (void)hipStreamSynchronize(s);
                synced = true;
            }
            if (switch_dev) (void)hipSetDevice(cur);
        }
        b.ready = ev;
        if (ev) ++ev->refs;
        c.free_blocks[b.device].emplace(b.bytes, b);
    }
}

void dev_free(void *p, hipStream_t s) { dev_free_many(&p, 1, s); }

hipError_t release_cached() {
    Cache &c = cache();
    std::lock_guard<std::mutex> lock(c.mu);
    int cur = 0;
    hipError_t first = hipGetDevice(&cur);
    for (int dev = 0; dev < kMaxDevices; ++dev) {
        if (c.free_blocks[dev].empty()) continue;
        (void)hipSetDevice(dev);
        hipError_t e = drain_device(c, dev);
        if (first == hipSuccess) first = e;
    }
    (void)hipSetDevice(cur);
    return first;
}

size_t cached_bytes() {
    Cache &c = cache();
    std::lock_guard<std::mutex> lock(c.mu);
    size_t t = 0;
    for (auto &fl : c.free_blocks)
        for (auto &kv : fl) t += kv.first;
    return t;
}

}  // namespace knnx
