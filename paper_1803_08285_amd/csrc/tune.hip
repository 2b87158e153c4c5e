// Autotuner for batched plans: a measured search over schedule tunables with an
// on-disk cache.
//
// The search space only changes schedules (tile order, grid sizes, the beam's
// wave-tile shape), never the order of any sum, so every candidate produces
// bitwise the same maps and the tuner may simply keep the fastest.  Results are
// cached in a small JSON file (SGWB_TUNE_CACHE, else $HOME/.cache/sgwb_tune.json)
// keyed by device name, compute-unit count and the plan's job signature; a
// cache hit skips all timing.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <sys/stat.h>
#include <unistd.h>

#include <map>
#include <string>

#include "sgwb_internal.h"

namespace sgwb {

static std::string cache_path()
{
    const char *e = getenv("SGWB_TUNE_CACHE");
    if (e && *e) return e;
    const char *h = getenv("HOME");
    if (!h || !*h) return "";
    std::string dir = std::string(h) + "/.cache";
    mkdir(dir.c_str(), 0755);
    return dir + "/sgwb_tune.json";
}

static std::map<std::string, Tunables> read_cache(const std::string &path)
{
    std::string text;
    FILE *f = path.empty() ? nullptr : fopen(path.c_str(), "r");
    if (!f) return {};
    char buf[4096];
    size_t n;
    while ((n = fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, n);
    fclose(f);
    return parse_cache_text(text);
}

static void write_cache(const std::string &path, const std::map<std::string, Tunables> &m)
{
    if (path.empty()) return;
    const std::string tmp = path + ".tmp" + std::to_string((long)getpid());
    FILE *f = fopen(tmp.c_str(), "w");
    if (!f) return;
    const std::string text = format_cache_text(m);
    const bool ok = fwrite(text.data(), 1, text.size(), f) == text.size();
    if (fclose(f) == 0 && ok)
        rename(tmp.c_str(), path.c_str());
    else
        unlink(tmp.c_str());
}

bool tune_cache_load(const std::string &key, Tunables *t)
{
    const auto m = read_cache(cache_path());
    auto it = m.find(key);
    if (it == m.end()) return false;
    *t = it->second;
    return true;
}

void tune_cache_store(const std::string &key, const Tunables &t)
{
    const std::string path = cache_path();
    auto m = read_cache(path);
    m[key] = t;
    write_cache(path, m);
}

std::string device_key()
{
    int dev = 0, cus = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    hipDeviceProp_t p;
    std::string arch = "unknown";
    if (hipGetDeviceProperties(&p, dev) == hipSuccess) {
        arch = p.gcnArchName;
        const size_t c = arch.find(':');
        if (c != std::string::npos) arch = arch.substr(0, c);
    }
    return arch + ":" + std::to_string(cus);
}

}  // namespace sgwb
