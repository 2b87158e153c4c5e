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
    std::map<std::string, Tunables> m;
    FILE *f = path.empty() ? nullptr : fopen(path.c_str(), "r");
    if (!f) return m;
    char line[4096];
    while (fgets(line, sizeof line, f)) {
        char *q1 = strchr(line, '"');
        if (!q1) continue;
        char *q2 = strchr(q1 + 1, '"');
        if (!q2) continue;
        std::string key(q1 + 1, q2);
        Tunables t;
        // entries without every field (an older format) are left out: a miss retunes
        if (sscanf(q2 + 1,
                   ": {\"x_strip_major\": %d, \"x_grid_per_cu\": %d, \"beam_shape\": %d, \"beam_grid_per_cu\": %d, "
                   "\"xm_per_job\": %d}",
                   &t.x_strip_major, &t.x_grid_per_cu, &t.beam_shape, &t.beam_grid_per_cu, &t.xm_per_job) == 5)
            m[key] = t;
    }
    fclose(f);
    return m;
}

static void write_cache(const std::string &path, const std::map<std::string, Tunables> &m)
{
    if (path.empty()) return;
    const std::string tmp = path + ".tmp" + std::to_string((long)getpid());
    FILE *f = fopen(tmp.c_str(), "w");
    if (!f) return;
    fprintf(f, "{\n");
    size_t i = 0;
    for (const auto &kv : m) {
        fprintf(f,
                "\"%s\": {\"x_strip_major\": %d, \"x_grid_per_cu\": %d, \"beam_shape\": %d, \"beam_grid_per_cu\": %d, "
                "\"xm_per_job\": %d}%s\n",
                kv.first.c_str(), kv.second.x_strip_major, kv.second.x_grid_per_cu, kv.second.beam_shape,
                kv.second.beam_grid_per_cu, kv.second.xm_per_job, ++i < m.size() ? "," : "");
    }
    fprintf(f, "}\n");
    fclose(f);
    rename(tmp.c_str(), path.c_str());
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
