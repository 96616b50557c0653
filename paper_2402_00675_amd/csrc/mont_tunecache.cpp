// Persistent cache of tuned launch shapes: JSON lines in the file named by
// $MONT_TUNE_CACHE, one record per tuning, e.g.
//   {"key": "gfx950:v65538:mul:w32:v2:log2n22", "unroll": 1, "nontemporal": 1, ...}
// Keys start with the device's architecture and the library version, so a
// cache written by another GPU or another build of the library is never
// applied.  A lookup reads the file again (tunings are rare and the file is
// small) and takes the last record with the key.  With no file named, the
// records this process stored are kept in memory instead.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>

#include "mont_common.hpp"
#include "mont_tuneline.hpp"

namespace mont {

static std::mutex g_tc_mu;
static std::map<std::string, TuneRecord> g_tc_mem;

std::string tune_key_prefix()
{
    int dev = 0;
    hipDeviceProp_t p;
    std::string arch = "unknown";
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&p, dev) == hipSuccess) {
        arch = p.gcnArchName;
        const size_t c = arch.find(':');
        if (c != std::string::npos)
            arch.resize(c);
    }
    char v[32];
    snprintf(v, sizeof v, ":v%u:", mont_version());
    return arch + v;
}

bool tune_lookup(const std::string &key, TuneRecord &out)
{
    std::lock_guard<std::mutex> g(g_tc_mu);
    const char *path = std::getenv("MONT_TUNE_CACHE");
    bool found = false;
    if (path && *path) {
        if (FILE *f = std::fopen(path, "r")) {
            char line[1024];
            std::string k;
            TuneRecord r;
            while (std::fgets(line, sizeof line, f))
                if (tune_parse_line(line, k, r) && k == key) {
                    out = r;
                    found = true;
                }
            std::fclose(f);
        }
        return found;  // a named file is the whole cache: its records, nothing remembered from other files
    }
    auto it = g_tc_mem.find(key);
    if (it == g_tc_mem.end())
        return false;
    out = it->second;
    return true;
}

void tune_store(const std::string &key, const TuneRecord &r)
{
    std::lock_guard<std::mutex> g(g_tc_mu);
    g_tc_mem[key] = r;
    const char *path = std::getenv("MONT_TUNE_CACHE");
    if (!path || !*path)
        return;
    FILE *f = std::fopen(path, "a");
    if (!f)
        return;
    std::fputs(tune_format_line(key, r).c_str(), f);
    std::fclose(f);
}

}  // namespace mont
