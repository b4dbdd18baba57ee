// Device-memory pool behind every library allocation.
//
// A solve request maps tens of GB of device memory (near-field values, grids,
// spectra, Krylov bases).  Mapping that much afresh with hipMalloc after the
// previous request freed it costs 0.2 s to several seconds, depending on what
// the driver still has to clear, which made the setup time of identical
// requests vary by an order of magnitude.  Freed blocks are therefore kept per
// device and handed out again: a request of the same rounded size takes a
// cached block (large requests also take one up to 1/8 larger), so a request
// that repeats an earlier one maps nothing new.  When hipMalloc fails, the
// device's cached blocks are released and the allocation is tried once more.
// Cached blocks beyond half of the device's memory are released at once.
#include <map>
#include <mutex>
#include <unordered_map>

#include "common.h"

namespace sie {
namespace {

struct Block {
    size_t bytes;
    int device;
};

struct Pool {
    std::mutex mu;
    std::unordered_map<void *, Block> live;                  // handed out
    std::map<int, std::multimap<size_t, void *>> cached;     // per device, by size
    std::map<int, size_t> cached_bytes;
    std::map<int, size_t> cap;                               // per device
};

Pool &pool() {
    static Pool *p = new Pool;   // never destroyed: frees may come from static destructors
    return *p;
}

size_t rounded(size_t bytes) {
    if (bytes <= 4096) return 4096;
    const size_t mb2 = size_t(2) << 20;
    if (bytes >= mb2) return (bytes + mb2 - 1) / mb2 * mb2;
    size_t r = 4096;
    while (r < bytes) r <<= 1;
    return r;
}

void release_cached(Pool &P, int dev) {
    auto &c = P.cached[dev];
    for (auto &kv : c) (void)hipFree(kv.second);
    c.clear();
    P.cached_bytes[dev] = 0;
}

thread_local int t_synced = 0;

}  // namespace

PoolSyncedFree::PoolSyncedFree() { ++t_synced; }
PoolSyncedFree::~PoolSyncedFree() { --t_synced; }

void *pool_alloc(size_t bytes) {
    if (!bytes) return nullptr;
    int dev = 0;
    SIE_HIP(hipGetDevice(&dev));
    const size_t r = rounded(bytes);
    Pool &P = pool();
    std::lock_guard<std::mutex> lk(P.mu);
    auto &c = P.cached[dev];
    auto it = c.lower_bound(r);
    if (it != c.end() && (it->first == r || (r >= (size_t(2) << 20) && it->first <= r + r / 8))) {
        void *q = it->second;
        const size_t b = it->first;
        c.erase(it);
        P.cached_bytes[dev] -= b;
        P.live[q] = {b, dev};
        return q;
    }
    void *q = nullptr;
    hipError_t e = hipMalloc(&q, r);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        release_cached(P, dev);
        e = hipMalloc(&q, r);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            throw Error(SIE_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
        }
    }
    P.live[q] = {r, dev};
    return q;
}

void pool_free(void *q) {
    if (!q) return;
    Pool &P = pool();
    Block b;
    {
        std::lock_guard<std::mutex> lk(P.mu);
        auto it = P.live.find(q);
        if (it == P.live.end()) return;
        b = it->second;
        P.live.erase(it);
    }
    int cur = 0;
    (void)hipGetDevice(&cur);
    if (cur != b.device) (void)hipSetDevice(b.device);
    // as hipFree does: work of any stream that may still use the block ends
    // before it can be handed out again (unless the caller has completed it)
    if (!t_synced) (void)hipDeviceSynchronize();
    std::lock_guard<std::mutex> lk(P.mu);
    if (!P.cap.count(b.device)) {
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) != hipSuccess) { (void)hipGetLastError(); tot = 0; }
        P.cap[b.device] = tot / 2;
    }
    if (P.cached_bytes[b.device] + b.bytes > P.cap[b.device]) {
        (void)hipFree(q);
    } else {
        P.cached[b.device].emplace(b.bytes, q);
        P.cached_bytes[b.device] += b.bytes;
    }
    if (cur != b.device) (void)hipSetDevice(cur);
}

size_t pool_cached_bytes(int device) {
    Pool &P = pool();
    std::lock_guard<std::mutex> lk(P.mu);
    auto it = P.cached_bytes.find(device);
    return it == P.cached_bytes.end() ? 0 : it->second;
}

void pool_trim(int device) {
    Pool &P = pool();
    std::lock_guard<std::mutex> lk(P.mu);
    int cur = 0;
    (void)hipGetDevice(&cur);
    if (cur != device) (void)hipSetDevice(device);
    release_cached(P, device);
    if (cur != device) (void)hipSetDevice(cur);
}

}  // namespace sie
