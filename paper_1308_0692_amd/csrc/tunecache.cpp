// On-disk cache of autotuned tile choices (fdlb_set_tune_cache).
//
// One text line per entry, "fdlb-tile-v1 <key> <tile> <tile_alt> <ms>", appended as results
// come in; when the file is read, the last well-formed line of a key wins and lines that do
// not parse are skipped.  A key names everything a choice depends on: the device (architecture
// and marketing name), a hash of the compiled tile shapes, the precision and the problem sizes
// (every member's, for a batch).  A cached tile that no longer fits, or a file that cannot be
// read, sends the caller back to timing the shapes.
#include <cstdio>
#include <cstring>
#include <fstream>
#include <mutex>
#include <sstream>
#include <string>

#include "fdlb_internal.h"

namespace fdlb {

namespace {
std::mutex g_mu;
std::string g_path;  // empty: no cache

uint64_t fnv1a(const void* data, size_t n, uint64_t h = 1469598103934665603ULL) {
    const unsigned char* p = (const unsigned char*)data;
    for (size_t i = 0; i < n; ++i) {
        h ^= p[i];
        h *= 1099511628211ULL;
    }
    return h;
}
}  // namespace

void set_tune_cache_path(const char* path) {
    std::lock_guard<std::mutex> lock(g_mu);
    g_path = path ? path : "";
}

bool tune_cache_enabled() {
    std::lock_guard<std::mutex> lock(g_mu);
    return !g_path.empty();
}

std::string tune_key_prefix() {
    int dev = 0;
    FDLB_HIP(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    FDLB_HIP(hipGetDeviceProperties(&prop, dev));
    uint64_t h = 1469598103934665603ULL;
    for (int prec : {FDLB_FP32, FDLB_FP64})
        for (const TileShape& t : tile_shapes(prec)) h = fnv1a(&t, sizeof(t), h);
    std::ostringstream o;
    std::string name = std::string(prop.gcnArchName) + "/" + prop.name;
    for (char& c : name)
        if (c == ' ' || c == '\t' || c == '\n') c = '_';
    o << name << "/tiles" << std::hex << h;
    return o.str();
}

bool tune_cache_get(const std::string& key, int& tile, int& tile_alt, double& ms) {
    std::lock_guard<std::mutex> lock(g_mu);
    if (g_path.empty()) return false;
    std::ifstream f(g_path);
    if (!f) return false;
    bool found = false;
    std::string line;
    while (std::getline(f, line)) {
        std::istringstream in(line);
        std::string tag, k;
        int t = -1, ta = -1;
        double m = 0;
        if (!(in >> tag >> k >> t >> ta >> m) || tag != "fdlb-tile-v1" || k != key || t < 0 || !(m > 0)) continue;
        std::string rest;
        if (in >> rest) continue;  // trailing garbage: not a line this library wrote
        tile = t;
        tile_alt = ta;
        ms = m;
        found = true;
    }
    return found;
}

void tune_cache_put(const std::string& key, int tile, int tile_alt, double ms) {
    std::lock_guard<std::mutex> lock(g_mu);
    if (g_path.empty()) return;
    std::ofstream f(g_path, std::ios::app);
    if (!f) return;  // an unwritable cache only costs the next tuning
    char buf[64];
    std::snprintf(buf, sizeof(buf), "%.6g", ms);
    f << "fdlb-tile-v1 " << key << ' ' << tile << ' ' << tile_alt << ' ' << buf << '\n';
}

}  // namespace fdlb
