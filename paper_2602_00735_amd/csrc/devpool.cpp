// Process-wide cache of the library's device allocations.
//
// A handle holds a few large buffers (factors, Krylov bases: gigabytes at
// the large configurations) and a few dozen small ones.  Mapping and
// unmapping them with hipMalloc / hipFree for every handle costs a few
// milliseconds per setup/destroy pair, which a caller that sets up one
// handle per problem pays every time.  Released blocks therefore stay
// mapped and serve later requests on the same device whose rounded size
// they match within 1/8 (best fit).  Cached bytes are capped (default: a
// third of the device's memory; ras_pml_set_cache_limit), and a hipMalloc
// that runs out of memory hands the device's cached blocks back to the
// driver and tries once more.
//
// The cache never decides when memory is idle: a caller returns a block
// only after the work that used it has finished (the handle synchronises
// its device first, as hipFree would).
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "devpool.h"
#include "ras_pml.h"

namespace raspml {
namespace {

struct Block {
    void *p;
    size_t bytes;
    int dev;
};

std::mutex g_mu;
std::vector<Block> g_free;                       // cached, idle
std::unordered_map<void *, Block> g_live;        // handed out
size_t g_cached = 0;
long long g_limit = -1;                          // < 0: a third of the device memory

constexpr size_t kSmall = size_t(1) << 20;
constexpr size_t kGrain = size_t(2) << 20;

size_t rounded(size_t b) {
    if (b == 0) b = 1;
    return b <= kSmall ? (b + 511) & ~size_t(511) : (b + kGrain - 1) & ~(kGrain - 1);
}

size_t limit_for(int dev) {
    if (g_limit >= 0) return static_cast<size_t>(g_limit);
    size_t fr = 0, total = 0;
    int cur = 0;
    if (hipGetDevice(&cur) == hipSuccess && cur == dev && hipMemGetInfo(&fr, &total) == hipSuccess)
        return total / 3;
    return size_t(32) << 30;
}

// Hands the idle blocks of `dev` (every device when dev < 0) back to the
// driver; returns the bytes released.
size_t release_idle(int dev) {
    std::vector<Block> out;
    {
        std::lock_guard<std::mutex> g(g_mu);
        auto keep = std::partition(g_free.begin(), g_free.end(),
                                   [&](const Block &b) { return dev >= 0 && b.dev != dev; });
        out.assign(keep, g_free.end());
        g_free.erase(keep, g_free.end());
        for (const Block &b : out) g_cached -= b.bytes;
    }
    size_t n = 0;
    for (const Block &b : out) {
        (void)hipFree(b.p);
        n += b.bytes;
    }
    return n;
}

}  // namespace

hipError_t pool_alloc(void **p, size_t bytes) {
    *p = nullptr;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    const size_t want = rounded(bytes);
    {
        std::lock_guard<std::mutex> g(g_mu);
        int best = -1;
        for (size_t i = 0; i < g_free.size(); ++i) {
            const Block &b = g_free[i];
            if (b.dev != dev || b.bytes < want || b.bytes > want + want / 8) continue;
            if (best < 0 || b.bytes < g_free[best].bytes) best = static_cast<int>(i);
        }
        if (best >= 0) {
            const Block b = g_free[best];
            g_free[best] = g_free.back();
            g_free.pop_back();
            g_cached -= b.bytes;
            g_live[b.p] = b;
            *p = b.p;
            return hipSuccess;
        }
    }
    e = hipMalloc(p, want);
    if (e == hipErrorOutOfMemory) {
        (void)hipGetLastError();
        if (release_idle(dev) > 0) e = hipMalloc(p, want);
    }
    if (e != hipSuccess) {
        *p = nullptr;
        return e;
    }
    std::lock_guard<std::mutex> g(g_mu);
    g_live[*p] = Block{*p, want, dev};
    return hipSuccess;
}

void pool_free(void *p) {
    if (!p) return;
    Block b{};
    {
        std::lock_guard<std::mutex> g(g_mu);
        auto it = g_live.find(p);
        if (it == g_live.end()) return;
        b = it->second;
        g_live.erase(it);
        if (g_cached + b.bytes <= limit_for(b.dev)) {
            g_free.push_back(b);
            g_cached += b.bytes;
            return;
        }
    }
    (void)hipFree(b.p);
}

}  // namespace raspml

extern "C" int ras_pml_empty_cache(long long *released_bytes) {
    const size_t n = raspml::release_idle(-1);
    if (released_bytes) *released_bytes = static_cast<long long>(n);
    return RAS_OK;
}

extern "C" int ras_pml_set_cache_limit(long long bytes) {
    {
        std::lock_guard<std::mutex> g(raspml::g_mu);
        raspml::g_limit = bytes < 0 ? -1 : bytes;
    }
    // Trim what the new limit no longer covers (idle blocks only).
    if (bytes >= 0) {
        std::vector<raspml::Block> out;
        {
            std::lock_guard<std::mutex> g(raspml::g_mu);
            while (!raspml::g_free.empty() && raspml::g_cached > static_cast<size_t>(bytes)) {
                out.push_back(raspml::g_free.back());
                raspml::g_cached -= raspml::g_free.back().bytes;
                raspml::g_free.pop_back();
            }
        }
        for (const auto &b : out) (void)hipFree(b.p);
    }
    return RAS_OK;
}

extern "C" int ras_pml_fill_idle_cache(int byte) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return RAS_EHIP;
    std::lock_guard<std::mutex> g(raspml::g_mu);
    for (const auto &b : raspml::g_free)
        if (b.dev == dev && hipMemset(b.p, byte & 0xff, b.bytes) != hipSuccess) return RAS_EHIP;
    return hipDeviceSynchronize() == hipSuccess ? RAS_OK : RAS_EHIP;
}

extern "C" int ras_pml_cache_info(long long *cached_bytes, long long *live_bytes) {
    std::lock_guard<std::mutex> g(raspml::g_mu);
    if (cached_bytes) *cached_bytes = static_cast<long long>(raspml::g_cached);
    if (live_bytes) {
        size_t n = 0;
        for (const auto &kv : raspml::g_live) n += kv.second.bytes;
        *live_bytes = static_cast<long long>(n);
    }
    return RAS_OK;
}
