// Schedule tunables of batched plans and their on-disk cache format, free of
// any device code so that it is tested on the CPU (with the address and
// undefined-behaviour sanitizers) as well as used by tune.hip and plan.hip.
//
// The cache is a small JSON object, one entry per line:
//   {
//   "<key>": {"x_strip_major": 1, "x_grid_per_cu": 2, "beam_shape": 1, "beam_grid_per_cu": 4, "xm_per_job": 0, "branches": 0},
//   ...
//   }
// Keys name the device and the plan's job signature (no quotes or newlines in
// them).  Lines that do not parse, or lack a field (an older format), are
// skipped: a miss only means the plan is tuned again.
#pragma once

#include <stdio.h>
#include <string.h>

#include <map>
#include <string>

namespace sgwb {

constexpr int kBeamShape4x4 = 0;
constexpr int kBeamShape2x4 = 1;

struct Tunables {
    int x_strip_major = 1;    // dirty-map tiles: column tiles fastest within a strip
    int x_grid_per_cu = 2;    // persistent dirty-map workgroups per compute unit
    int beam_shape = kBeamShape2x4;
    int beam_grid_per_cu = 4; // persistent beam workgroups per compute unit (0: one per tile group)
    int xm_per_job = 0;       // matrix-core dirty maps: one launch per job instead of one for all
    int branches = 0;         // beams on a second stream of the graph, beside the dirty maps
};

inline bool tunables_valid(const Tunables &t)
{
    return (t.x_strip_major == 0 || t.x_strip_major == 1) && t.x_grid_per_cu >= 1 && t.x_grid_per_cu <= 64 &&
           (t.beam_shape == kBeamShape4x4 || t.beam_shape == kBeamShape2x4) && t.beam_grid_per_cu >= 0 &&
           t.beam_grid_per_cu <= 64 && (t.xm_per_job == 0 || t.xm_per_job == 1) &&
           (t.branches == 0 || t.branches == 1);
}

// Skip spaces and tabs.
inline const char *skip_blanks(const char *p)
{
    while (*p == ' ' || *p == '\t') ++p;
    return p;
}

// Expect the literal `lit` (after blanks); nullptr if it is not there.
inline const char *expect(const char *p, const char *lit)
{
    p = skip_blanks(p);
    const size_t n = strlen(lit);
    return strncmp(p, lit, n) == 0 ? p + n : nullptr;
}

// A decimal integer in [-1e6, 1e6] (after blanks); nullptr if there is none.
inline const char *small_int(const char *p, int *out)
{
    p = skip_blanks(p);
    bool neg = false;
    if (*p == '-' || *p == '+') neg = *p++ == '-';
    if (*p < '0' || *p > '9') return nullptr;
    long v = 0;
    while (*p >= '0' && *p <= '9') {
        v = v * 10 + (*p++ - '0');
        if (v > 1000000) return nullptr;
    }
    *out = (int)(neg ? -v : v);
    return p;
}

// One cache line -> (key, tunables); false if it is not a complete, valid entry.
inline bool parse_cache_line(const char *line, std::string *key, Tunables *t)
{
    const char *q1 = strchr(line, '"');
    if (!q1) return false;
    const char *q2 = strchr(q1 + 1, '"');
    if (!q2 || q2 == q1 + 1) return false;
    Tunables v;
    const struct {
        const char *name;
        int *field;
    } fields[] = {{"\"x_strip_major\":", &v.x_strip_major}, {"\"x_grid_per_cu\":", &v.x_grid_per_cu},
                  {"\"beam_shape\":", &v.beam_shape},       {"\"beam_grid_per_cu\":", &v.beam_grid_per_cu},
                  {"\"xm_per_job\":", &v.xm_per_job},       {"\"branches\":", &v.branches}};
    const char *p = expect(q2 + 1, ":");
    if (p) p = expect(p, "{");
    for (size_t i = 0; p && i < sizeof fields / sizeof fields[0]; ++i) {
        if (i > 0) p = expect(p, ",");
        if (p) p = expect(p, fields[i].name);
        if (p) p = small_int(p, fields[i].field);
    }
    if (p) p = expect(p, "}");
    if (!p || !tunables_valid(v)) return false;
    key->assign(q1 + 1, q2);
    *t = v;
    return true;
}

inline std::map<std::string, Tunables> parse_cache_text(const std::string &text)
{
    std::map<std::string, Tunables> m;
    size_t pos = 0;
    while (pos < text.size()) {
        size_t end = text.find('\n', pos);
        if (end == std::string::npos) end = text.size();
        const std::string line = text.substr(pos, end - pos);
        std::string key;
        Tunables t;
        if (parse_cache_line(line.c_str(), &key, &t)) m[key] = t;
        pos = end + 1;
    }
    return m;
}

inline std::string format_cache_text(const std::map<std::string, Tunables> &m)
{
    std::string out = "{\n";
    size_t i = 0;
    for (const auto &kv : m) {
        char buf[256];
        snprintf(buf, sizeof buf,
                 "\": {\"x_strip_major\": %d, \"x_grid_per_cu\": %d, \"beam_shape\": %d, \"beam_grid_per_cu\": %d, "
                 "\"xm_per_job\": %d, \"branches\": %d}%s\n",
                 kv.second.x_strip_major, kv.second.x_grid_per_cu, kv.second.beam_shape, kv.second.beam_grid_per_cu,
                 kv.second.xm_per_job, kv.second.branches, ++i < m.size() ? "," : "");
        out += "\"" + kv.first + buf;
    }
    out += "}\n";
    return out;
}

}  // namespace sgwb
