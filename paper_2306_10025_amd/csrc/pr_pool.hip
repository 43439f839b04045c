// Per-device cache of idle device blocks.
//
// Every buffer a handle owns goes through pool_alloc / pool_release.  A block
// released by pr_destroy is kept idle (up to a per-device byte limit) and
// handed to a later request of a close size, so repeated setups on one device
// neither map nor unmap memory: hipFree synchronises the whole device and
// unmaps its pages, which costs far more than the kernels of a small setup.
//
// Sizes round up to a power of two below 1 MiB and to a multiple of 2 MiB
// above; a request reuses an idle block of its own rounded size, or up to one
// eighth larger for multi-MiB blocks.  An idle block holds whatever its last
// owner wrote: no caller may rely on fresh memory being zero (hipMalloc does
// not promise that either).  A block is released only after every stream that
// used it has been synchronised (pr_destroy does that), so a later owner on
// any stream sees it idle.  Pinned host blocks (a handle's few-KB mirror of
// solver scalars) are cached the same way under their own key.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <vector>

#include "pr_internal.h"

namespace {

constexpr size_t kSmall = size_t(1) << 20;
constexpr size_t kGrain = size_t(2) << 20;
constexpr int kHostKey = -1;                        // pinned host blocks
constexpr size_t kHostLimit = size_t(64) << 20;

struct DevCache {
    std::multimap<size_t, void*> idle;   // rounded size -> block
    size_t idle_bytes = 0;
    int64_t reuses = 0;
    int64_t mallocs = 0;
    bool limit_set = false;
    size_t limit = 0;
};

struct Pool {
    std::mutex mu;
    std::map<int, DevCache> dev;
    bool user_limit = false;
    size_t user_limit_bytes = 0;
};

// Never destroyed: at process exit the HIP runtime may already be gone, and
// the driver reclaims the memory anyway.
Pool& pool() {
    static Pool* p = new Pool();
    return *p;
}

size_t round_size(size_t b) {
    if (b <= 256) return 256;
    if (b < kSmall) {
        size_t r = 256;
        while (r < b) r <<= 1;
        return r;
    }
    return (b + kGrain - 1) / kGrain * kGrain;
}

// Idle bytes kept for a key: the user's limit if set (pinned blocks never
// beyond kHostLimit), else one eighth of the device's memory.
size_t limit_of(Pool& P, DevCache& c, int key) {
    if (key == kHostKey) return P.user_limit ? std::min(P.user_limit_bytes, kHostLimit) : kHostLimit;
    if (P.user_limit) return P.user_limit_bytes;
    if (!c.limit_set) {
        hipDeviceProp_t prop;
        size_t total = 0;
        if (hipGetDeviceProperties(&prop, key) == hipSuccess) total = prop.totalGlobalMem;
        else (void)hipGetLastError();
        c.limit = total / 8;
        c.limit_set = true;
    }
    return c.limit;
}

// Removes idle blocks, largest first, until at most `keep` bytes stay idle.
void trim_locked(DevCache& c, size_t keep, std::vector<void*>& out) {
    while (c.idle_bytes > keep && !c.idle.empty()) {
        auto it = std::prev(c.idle.end());
        c.idle_bytes -= it->first;
        out.push_back(it->second);
        c.idle.erase(it);
    }
}

// Frees blocks outside the lock (hipFree synchronises the device).
void free_blocks(const std::vector<void*>& v, bool host) {
    for (void* q : v) (void)(host ? hipHostFree(q) : hipFree(q));
}

hipError_t raw_alloc(bool host, void** p, size_t r) {
    return host ? hipHostMalloc(p, r, hipHostMallocDefault) : hipMalloc(p, r);
}

hipError_t cache_alloc(int key, size_t bytes, void** p, size_t* got) {
    const bool host = key == kHostKey;
    const size_t r = round_size(bytes ? bytes : 1);
    Pool& P = pool();
    {
        std::lock_guard<std::mutex> lk(P.mu);
        DevCache& c = P.dev[key];
        auto it = c.idle.lower_bound(r);
        if (it != c.idle.end() && (it->first == r || (r >= kSmall && it->first - r <= r / 8))) {
            *p = it->second;
            *got = it->first;
            c.idle_bytes -= it->first;
            c.idle.erase(it);
            c.reuses += 1;
            return hipSuccess;
        }
    }
    hipError_t e = raw_alloc(host, p, r);
    if (e == hipErrorOutOfMemory) {
        // the idle blocks of this key may be what is missing
        (void)hipGetLastError();
        std::vector<void*> drop;
        {
            std::lock_guard<std::mutex> lk(P.mu);
            trim_locked(P.dev[key], 0, drop);
        }
        free_blocks(drop, host);
        e = raw_alloc(host, p, r);
    }
    if (e != hipSuccess) {
        *p = nullptr;
        return e;
    }
    *got = r;
    std::lock_guard<std::mutex> lk(P.mu);
    P.dev[key].mallocs += 1;
    return hipSuccess;
}

void cache_release(int key, void* p, size_t got) {
    if (!p) return;
    Pool& P = pool();
    std::vector<void*> drop;
    {
        std::lock_guard<std::mutex> lk(P.mu);
        DevCache& c = P.dev[key];
        const size_t lim = limit_of(P, c, key);
        if (got > lim) {
            drop.push_back(p);
        } else {
            trim_locked(c, lim - got, drop);
            c.idle.emplace(got, p);
            c.idle_bytes += got;
        }
    }
    free_blocks(drop, key == kHostKey);
}

// Trims every key to the limit `keep` (pinned blocks to at most kHostLimit).
void trim_all(size_t keep) {
    Pool& P = pool();
    std::vector<void*> drop, hdrop;
    {
        std::lock_guard<std::mutex> lk(P.mu);
        for (auto& kv : P.dev) {
            const bool host = kv.first == kHostKey;
            trim_locked(kv.second, host ? std::min(keep, kHostLimit) : keep, host ? hdrop : drop);
        }
    }
    free_blocks(drop, false);
    free_blocks(hdrop, true);
}

}  // namespace

hipError_t pool_alloc(int device, size_t bytes, void** p, size_t* got) {
    return cache_alloc(device < 0 ? 0 : device, bytes, p, got);
}

void pool_release(int device, void* p, size_t got) { cache_release(device < 0 ? 0 : device, p, got); }

hipError_t pool_host_alloc(size_t bytes, void** p, size_t* got) { return cache_alloc(kHostKey, bytes, p, got); }

void pool_host_release(void* p, size_t got) { cache_release(kHostKey, p, got); }

int pr_set_memory_cache_limit(int64_t bytes) {
    if (bytes < -1) return pr_fail(nullptr, PR_ERR_INVALID_ARG, "cache limit below -1");
    Pool& P = pool();
    if (bytes == -1) {
        // back to the default: trim each device to its own limit
        std::vector<void*> drop, hdrop;
        {
            std::lock_guard<std::mutex> lk(P.mu);
            P.user_limit = false;
            for (auto& kv : P.dev) {
                const bool host = kv.first == kHostKey;
                trim_locked(kv.second, limit_of(P, kv.second, kv.first), host ? hdrop : drop);
            }
        }
        free_blocks(drop, false);
        free_blocks(hdrop, true);
        return PR_OK;
    }
    {
        std::lock_guard<std::mutex> lk(P.mu);
        P.user_limit = true;
        P.user_limit_bytes = (size_t)bytes;
    }
    trim_all((size_t)bytes);
    return PR_OK;
}

int pr_release_cached_memory(void) {
    trim_all(0);
    return PR_OK;
}

int pr_memory_cache_info(int32_t device, int64_t* info) {
    if (!info) return pr_fail(nullptr, PR_ERR_INVALID_ARG, "null info");
    if (device < -1) return pr_fail(nullptr, PR_ERR_INVALID_ARG, "device below -1");
    Pool& P = pool();
    std::lock_guard<std::mutex> lk(P.mu);
    auto it = P.dev.find(device);
    if (it == P.dev.end()) {
        info[0] = info[1] = info[2] = info[3] = 0;
        return PR_OK;
    }
    const DevCache& c = it->second;
    info[0] = (int64_t)c.idle_bytes;
    info[1] = (int64_t)c.idle.size();
    info[2] = c.reuses;
    info[3] = c.mallocs;
    return PR_OK;
}
