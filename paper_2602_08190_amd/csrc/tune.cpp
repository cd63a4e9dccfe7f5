// Tile cache: per-kind tile shapes measured by the autotuner, stored as JSON
//   {"arch": "gfx950", "waves_per_cu": 16,
//    "kinds": {"FOR32": {"unit": 2, "waves_per_block": 4, ...}, ...}}
// Unknown keys are ignored, so the autotuner may add its measurements.
#include <dlfcn.h>

#include <cctype>
#include <cstdlib>
#include <fstream>
#include <map>
#include <sstream>

#include "tune.hpp"

namespace zf {

namespace {
struct Json {
    const std::string &s;
    size_t i = 0;
    explicit Json(const std::string &src) : s(src) {}
    void ws() {
        while (i < s.size() && std::isspace(static_cast<unsigned char>(s[i]))) i++;
    }
    bool eat(char c) {
        ws();
        if (i < s.size() && s[i] == c) {
            i++;
            return true;
        }
        return false;
    }
    std::string str() {
        ws();
        if (i >= s.size() || s[i] != '"') throw 0;
        std::string out;
        for (i++; i < s.size() && s[i] != '"'; i++) {
            if (s[i] == '\\' && i + 1 < s.size()) i++;
            out += s[i];
        }
        if (i >= s.size()) throw 0;
        i++;
        return out;
    }
    // Skip any value; numbers are returned through *num when non-null.
    void value(double *num) {
        ws();
        if (i >= s.size()) throw 0;
        const char c = s[i];
        if (c == '"') {
            str();
        } else if (c == '{') {
            i++;
            if (eat('}')) return;
            do {
                str();
                if (!eat(':')) throw 0;
                value(nullptr);
            } while (eat(','));
            if (!eat('}')) throw 0;
        } else if (c == '[') {
            i++;
            if (eat(']')) return;
            do value(nullptr);
            while (eat(','));
            if (!eat(']')) throw 0;
        } else {
            size_t j = i;
            while (j < s.size() && (std::isalnum(static_cast<unsigned char>(s[j])) || s[j] == '-' ||
                                    s[j] == '+' || s[j] == '.'))
                j++;
            if (j == i) throw 0;
            if (num) *num = std::strtod(s.substr(i, j - i).c_str(), nullptr);
            i = j;
        }
    }
};

const char *kKindNames[K_COUNT] = {"LZ77", "ANS", "RLE64", "RLE32", "SDICT", "DICT128", "DICT64",
                                   "DICT32", "FOR64", "FOR32", "F2I", "PLAIN", "TREE"};

std::string default_cache_path() {
    Dl_info info;
    if (dladdr(reinterpret_cast<void *>(&default_cache_path), &info) && info.dli_fname) {
        std::string p = info.dli_fname;
        const size_t k = p.find_last_of('/');
        return (k == std::string::npos ? std::string(".") : p.substr(0, k)) + "/tune_gfx950.json";
    }
    return "tune_gfx950.json";
}
}  // namespace

const char *kind_name(uint32_t k) { return k < K_COUNT ? kKindNames[k] : "?"; }

TileShape default_tiles() {
    TileShape t;
    for (uint32_t k = 0; k < K_COUNT; k++) {
        t.unit[k] = (k == K_PLAIN) ? 65536u : (k == K_RLE32 || k == K_RLE64 || k == K_TREE) ? 4096u
                    : (k == K_LZ) ? 16u : (k == K_SDICT) ? 4096u : 2u;
        t.wpb[k] = 4;
        // rates for ordering batches when the cache has no measurement
        t.rate_gbps[k] = k == K_LZ ? 600 : k == K_ANS ? 1200 : k == K_SDICT ? 800
                         : (k == K_RLE32 || k == K_RLE64 || k == K_TREE) ? 3000 : 4000;
    }
    t.wpcu = 16;
    return t;
}

bool read_tune_cache(const std::string &path, TileShape &t) {
    std::ifstream f(path);
    if (!f) return false;
    std::stringstream ss;
    ss << f.rdbuf();
    const std::string src = ss.str();
    Json j(src);
    try {
        if (!j.eat('{')) return false;
        if (j.eat('}')) return true;
        do {
            const std::string key = j.str();
            if (!j.eat(':')) return false;
            if (key == "waves_per_cu") {
                double v = 0;
                j.value(&v);
                if (v >= 1 && v <= 32) t.wpcu = uint32_t(v);
            } else if (key == "kinds") {
                if (!j.eat('{')) return false;
                if (!j.eat('}')) {
                    do {
                        const std::string kn = j.str();
                        if (!j.eat(':') || !j.eat('{')) return false;
                        int kind = -1;
                        for (uint32_t k = 0; k < K_COUNT; k++)
                            if (kn == kKindNames[k]) kind = int(k);
                        if (!j.eat('}')) {
                            do {
                                const std::string f2 = j.str();
                                if (!j.eat(':')) return false;
                                double v = 0;
                                j.value(&v);
                                if (kind < 0) continue;
                                if (f2 == "unit" && v >= 1) t.unit[kind] = uint32_t(v);
                                if (f2 == "waves_per_block" && v >= 1 && v <= 16) t.wpb[kind] = uint32_t(v);
                                if (f2 == "plain_GBps" && v > 0) t.rate_gbps[kind] = v;
                            } while (j.eat(','));
                            if (!j.eat('}')) return false;
                        }
                    } while (j.eat(','));
                    if (!j.eat('}')) return false;
                }
            } else {
                j.value(nullptr);
            }
        } while (j.eat(','));
        return j.eat('}');
    } catch (...) {
        return false;
    }
}

TileShape resolve_tiles(const zf_plan_opts &o) {
    TileShape t = default_tiles();
    std::string path;
    if (o.tune_cache) path = o.tune_cache;
    else if (const char *e = std::getenv("ZF_TUNE_CACHE")) path = e;
    else path = default_cache_path();
    if (!path.empty()) read_tune_cache(path, t);
    for (uint32_t k = 0; k < K_COUNT && k < ZF_KIND_COUNT; k++) {
        if (o.tiles[k].unit) t.unit[k] = o.tiles[k].unit;
        if (o.tiles[k].waves_per_block) t.wpb[k] = std::min(16u, o.tiles[k].waves_per_block);
    }
    if (o.waves_per_cu) t.wpcu = std::min(32u, o.waves_per_cu);
    // sane floors: GP units cover at least one window, PLAIN units one vector
    t.unit[K_RLE32] = std::max(64u, t.unit[K_RLE32]);
    t.unit[K_RLE64] = std::max(64u, t.unit[K_RLE64]);
    t.unit[K_TREE] = std::max(64u, t.unit[K_TREE]);
    t.unit[K_PLAIN] = std::max(1024u, t.unit[K_PLAIN]);
    t.unit[K_SDICT] = std::max(256u, t.unit[K_SDICT]);
    // LZ77: output bytes per block, 4, 8 or 16
    t.unit[K_LZ] = t.unit[K_LZ] <= 4 ? 4u : t.unit[K_LZ] <= 8 ? 8u : 16u;
    return t;
}

uint32_t scheduled_unit(uint32_t kind, uint32_t sched, uint32_t tuned) {
    if (sched == 0 || sched > 4) return tuned;
    switch (kind) {
    case K_RLE32:
    case K_RLE64:
    case K_TREE: return 1024u << (sched - 1);         // 1024 .. 8192 elements
    case K_PLAIN: return 16384u << (2 * (sched - 1)); // 16 KiB .. 1 MiB
    case K_LZ:
    case K_SDICT: return tuned;
    default: return 1u << (sched - 1);                 // 1 .. 8 blocks
    }
}

}  // namespace zf
