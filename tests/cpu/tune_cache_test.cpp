// CPU checks of the batched plans' tuning-cache format (tune_cache.h), built
// with the address and undefined-behaviour sanitizers by
// tests/test_host_policy_cpu.py: a formatted cache parses back to the same
// entries; damaged, truncated, out-of-range or older-format lines are skipped
// without reading out of bounds.
#include <stdio.h>
#include <stdlib.h>

#include <random>
#include <string>

#include "tune_cache.h"

using sgwb::Tunables;

static int failures = 0;
#define CHECK(c)                                                              \
    do {                                                                      \
        if (!(c)) {                                                           \
            fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #c); \
            if (++failures > 20) exit(1);                                     \
        }                                                                     \
    } while (0)

static bool same(const Tunables &a, const Tunables &b)
{
    return a.x_strip_major == b.x_strip_major && a.x_grid_per_cu == b.x_grid_per_cu && a.beam_shape == b.beam_shape &&
           a.beam_grid_per_cu == b.beam_grid_per_cu && a.xm_per_job == b.xm_per_job && a.branches == b.branches;
}

int main()
{
    std::mt19937_64 rng(11);
    // round trip
    for (int rep = 0; rep < 200; ++rep) {
        std::map<std::string, Tunables> m;
        const int n = (int)(rng() % 6);
        for (int i = 0; i < n; ++i) {
            std::string key = "gfx950:256:";
            const int parts = 1 + (int)(rng() % 40);
            for (int k = 0; k < parts; ++k) key += "m" + std::to_string(rng() % 100000) + ".898.853;";
            Tunables t;
            t.x_strip_major = (int)(rng() % 2);
            t.x_grid_per_cu = 1 + (int)(rng() % 8);
            t.beam_shape = (int)(rng() % 2);
            t.beam_grid_per_cu = (int)(rng() % 9);
            t.xm_per_job = (int)(rng() % 2);
            t.branches = (int)(rng() % 2);
            m[key] = t;
        }
        const std::string text = sgwb::format_cache_text(m);
        const auto back = sgwb::parse_cache_text(text);
        CHECK(back.size() == m.size());
        for (const auto &kv : m) {
            auto it = back.find(kv.first);
            CHECK(it != back.end() && same(it->second, kv.second));
        }
        // every prefix of the text parses without reading past its end, and
        // only to entries of the full text
        for (size_t cut = 0; cut < text.size(); cut += 1 + rng() % 37) {
            const auto part = sgwb::parse_cache_text(text.substr(0, cut));
            for (const auto &kv : part) {
                auto it = m.find(kv.first);
                CHECK(it != m.end() && same(it->second, kv.second));
            }
        }
    }
    // damaged lines
    const char *bad[] = {
        "",
        "\"",
        "\"\": {\"x_strip_major\": 1, \"x_grid_per_cu\": 2, \"beam_shape\": 1, \"beam_grid_per_cu\": 4, \"xm_per_job\": 0, \"branches\": 0}",
        "\"k\": {\"x_strip_major\": 1, \"x_grid_per_cu\": 2, \"beam_shape\": 1, \"beam_grid_per_cu\": 4, \"xm_per_job\": 0}",
        "\"k\": {\"x_strip_major\": 7, \"x_grid_per_cu\": 2, \"beam_shape\": 1, \"beam_grid_per_cu\": 4, \"xm_per_job\": 0, \"branches\": 0}",
        "\"k\": {\"x_strip_major\": 1, \"x_grid_per_cu\": -2, \"beam_shape\": 1, \"beam_grid_per_cu\": 4, \"xm_per_job\": 0, \"branches\": 0}",
        "\"k\": {\"x_strip_major\": 1, \"x_grid_per_cu\": 2, \"beam_shape\": 5, \"beam_grid_per_cu\": 4, \"xm_per_job\": 0, \"branches\": 0}",
        "\"k\": {\"x_strip_major\": 1, \"x_grid_per_cu\": 2, \"beam_shape\": 1, \"beam_grid_per_cu\": 4, \"xm_per_job\": 0, \"branches\": 3}",
        "\"k\": {\"x_strip_major\": 1, \"x_grid_per_cu\": 2, \"beam_shape\": 1, \"beam_grid_per_cu\": 4, \"xm_per_job\": 0, \"branches\": 0",
        "\"k\" {\"x_strip_major\": 1}",
        "{",
        "}",
        "\"k\": {\"x_strip_major\": 99999999999999999999, \"x_grid_per_cu\": 2, \"beam_shape\": 1, \"beam_grid_per_cu\": 4, \"xm_per_job\": 0, \"branches\": 0}",
    };
    for (const char *line : bad) {
        std::string key;
        Tunables t;
        CHECK(!sgwb::parse_cache_line(line, &key, &t));
    }
    std::string good = "\"k\": {\"x_strip_major\": 0, \"x_grid_per_cu\": 8, \"beam_shape\": 0, \"beam_grid_per_cu\": 0, "
                       "\"xm_per_job\": 1, \"branches\": 1}";
    {
        std::string key;
        Tunables t;
        CHECK(sgwb::parse_cache_line(good.c_str(), &key, &t) && key == "k" && t.x_grid_per_cu == 8 && t.branches == 1);
    }
    // random bytes never crash the parser
    for (int rep = 0; rep < 2000; ++rep) {
        std::string junk;
        const int len = (int)(rng() % 300);
        for (int i = 0; i < len; ++i) junk += (char)(1 + rng() % 255);
        (void)sgwb::parse_cache_text(junk);
        std::string mixed = good.substr(0, rng() % good.size()) + junk;
        (void)sgwb::parse_cache_text(mixed);
    }
    if (failures) {
        fprintf(stderr, "%d checks failed\n", failures);
        return 1;
    }
    printf("tune cache: all checks passed\n");
    return 0;
}
