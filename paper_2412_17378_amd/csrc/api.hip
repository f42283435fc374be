// Library-wide pieces of the bgs C ABI: error text, version, device queries.
#include <mutex>
#include <string>
#include <vector>

#include "common.h"

namespace bgs {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

bgs_status fail(bgs_status code, const std::string& msg) {
    g_last_error = msg;
    return code;
}

int cu_count() {
    static std::mutex mu;
    static std::vector<int> cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 1;
    std::lock_guard<std::mutex> lock(mu);
    if ((int)cache.size() <= dev) cache.resize(dev + 1, 0);
    if (cache[dev] == 0) {
        int n = 0;
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n < 1) n = 1;
        cache[dev] = n;
    }
    return cache[dev];
}

}  // namespace bgs

extern "C" const char* bgs_last_error(void) { return bgs::g_last_error.c_str(); }

extern "C" const char* bgs_version(void) { return "bgs 0.1 gfx950"; }
