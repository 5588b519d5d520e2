// Persistent autotuner cache: the per-tile cost fits that qmm_batched_tune
// measures, kept in memory and in a JSON file, keyed by the GPU architecture,
// the encoding the products run in (FP4 codes for p <= 8, centred int8 bytes
// otherwise) and a bucket of the product shape (the larger of m and n: up to
// 128, up to 512, above).  qmm_batched_create reads the file named by the
// environment variable QMM_TUNE_CACHE once per process and looks each product's
// costs up under its own key.
//
// File format (written by tune_cache_save, read back by tune_cache_load):
//   {"version": 1, "entries": [
//     {"arch": "gfx950", "enc": "fp4", "bucket": "le512",
//      "costs": [fixed0, per_stage0, ..., fixed3, per_stage3]}, ...]}
#include <cctype>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "qmm_internal.h"

namespace qmm {
namespace {

struct Entry {
    std::string arch;
    uint32_t enc, bucket;
    double costs[kTuneCosts];
};

std::mutex g_mu;
std::vector<Entry> g_entries;
bool g_env_loaded = false;

const char *const kEncNames[2] = {"int8", "fp4"};
const char *const kBucketNames[3] = {"le128", "le512", "gt512"};

int find_name(const char *const *names, int count, const std::string &s) {
    for (int i = 0; i < count; ++i)
        if (s == names[i]) return i;
    return -1;
}

bool costs_ok(const double *c) {
    for (int s = 0; s < kTuneCosts / 2; ++s)
        if (!(c[2 * s] >= 0) || !(c[2 * s + 1] > 0) || !std::isfinite(c[2 * s]) || !std::isfinite(c[2 * s + 1]))
            return false;
    return true;
}

void put_locked(const std::string &arch, uint32_t enc, uint32_t bucket, const double *costs) {
    for (Entry &e : g_entries)
        if (e.arch == arch && e.enc == enc && e.bucket == bucket) {
            std::memcpy(e.costs, costs, sizeof(e.costs));
            return;
        }
    Entry e{arch, enc, bucket, {}};
    std::memcpy(e.costs, costs, sizeof(e.costs));
    g_entries.push_back(e);
}

// --- a small JSON reader, enough for the cache file ------------------------------
struct Json {
    enum Kind { NUL, BOOL, NUM, STR, ARR, OBJ } kind = NUL;
    double num = 0;
    std::string str;
    std::vector<Json> items;                       // ARR
    std::vector<std::pair<std::string, Json>> kv;  // OBJ
    const Json *get(const char *key) const {
        for (const auto &p : kv)
            if (p.first == key) return &p.second;
        return nullptr;
    }
};

struct Parser {
    const char *s, *end;
    void ws() {
        while (s < end && std::isspace((unsigned char)*s)) ++s;
    }
    bool lit(const char *w) {
        const size_t n = std::strlen(w);
        if ((size_t)(end - s) < n || std::strncmp(s, w, n) != 0) return false;
        s += n;
        return true;
    }
    bool string(std::string &out) {
        if (s >= end || *s != '"') return false;
        ++s;
        while (s < end && *s != '"') {
            char c = *s++;
            if (c == '\\') {
                if (s >= end) return false;
                c = *s++;
                if (c == 'n') c = '\n';
                else if (c == 't') c = '\t';
                else if (c != '"' && c != '\\' && c != '/') return false;
            }
            out.push_back(c);
        }
        if (s >= end) return false;
        ++s;
        return true;
    }
    bool value(Json &v, int depth) {
        if (depth > 16) return false;
        ws();
        if (s >= end) return false;
        if (*s == '{') {
            ++s;
            v.kind = Json::OBJ;
            ws();
            if (s < end && *s == '}') return ++s, true;
            for (;;) {
                ws();
                std::string key;
                if (!string(key)) return false;
                ws();
                if (s >= end || *s != ':') return false;
                ++s;
                Json child;
                if (!value(child, depth + 1)) return false;
                v.kv.emplace_back(key, child);
                ws();
                if (s < end && *s == ',') {
                    ++s;
                    continue;
                }
                if (s < end && *s == '}') return ++s, true;
                return false;
            }
        }
        if (*s == '[') {
            ++s;
            v.kind = Json::ARR;
            ws();
            if (s < end && *s == ']') return ++s, true;
            for (;;) {
                Json child;
                if (!value(child, depth + 1)) return false;
                v.items.push_back(child);
                ws();
                if (s < end && *s == ',') {
                    ++s;
                    continue;
                }
                if (s < end && *s == ']') return ++s, true;
                return false;
            }
        }
        if (*s == '"') {
            v.kind = Json::STR;
            return string(v.str);
        }
        if (lit("true")) return v.kind = Json::BOOL, v.num = 1, true;
        if (lit("false")) return v.kind = Json::BOOL, v.num = 0, true;
        if (lit("null")) return v.kind = Json::NUL, true;
        char *stop = nullptr;
        const std::string tok(s, (size_t)std::min<ptrdiff_t>(end - s, 64));
        const double x = std::strtod(tok.c_str(), &stop);
        if (stop == tok.c_str()) return false;
        s += stop - tok.c_str();
        v.kind = Json::NUM;
        v.num = x;
        return true;
    }
};

qmm_status load_locked(const char *path, bool missing_ok) {
    FILE *f = std::fopen(path, "rb");
    if (!f) {
        if (missing_ok) return QMM_OK;
        return fail(QMM_EINVAL, std::string("tune cache ") + path + ": cannot open");
    }
    std::string text;
    char buf[4096];
    size_t got;
    while ((got = std::fread(buf, 1, sizeof(buf), f)) > 0) {
        text.append(buf, got);
        if (text.size() > (64u << 20)) break;
    }
    std::fclose(f);
    Parser ps{text.data(), text.data() + text.size()};
    Json root;
    if (!ps.value(root, 0) || root.kind != Json::OBJ)
        return fail(QMM_EINVAL, std::string("tune cache ") + path + ": not a JSON object");
    const Json *ver = root.get("version");
    if (!ver || ver->kind != Json::NUM || ver->num != 1)
        return fail(QMM_EINVAL, std::string("tune cache ") + path + ": unknown version");
    const Json *ents = root.get("entries");
    if (!ents || ents->kind != Json::ARR) return fail(QMM_EINVAL, std::string("tune cache ") + path + ": no entries");
    std::vector<Entry> parsed;
    for (const Json &e : ents->items) {
        const Json *arch = e.get("arch"), *enc = e.get("enc"), *bucket = e.get("bucket"), *costs = e.get("costs");
        if (!arch || arch->kind != Json::STR || !enc || enc->kind != Json::STR || !bucket ||
            bucket->kind != Json::STR || !costs || costs->kind != Json::ARR || costs->items.size() != kTuneCosts)
            return fail(QMM_EINVAL, std::string("tune cache ") + path + ": malformed entry");
        const int ei = find_name(kEncNames, 2, enc->str), bi = find_name(kBucketNames, 3, bucket->str);
        if (ei < 0 || bi < 0) return fail(QMM_EINVAL, std::string("tune cache ") + path + ": unknown enc or bucket");
        Entry out{arch->str, (uint32_t)ei, (uint32_t)bi, {}};
        for (int i = 0; i < kTuneCosts; ++i) {
            if (costs->items[(size_t)i].kind != Json::NUM)
                return fail(QMM_EINVAL, std::string("tune cache ") + path + ": costs must be numbers");
            out.costs[i] = costs->items[(size_t)i].num;
        }
        if (!costs_ok(out.costs)) return fail(QMM_EINVAL, std::string("tune cache ") + path + ": costs out of range");
        parsed.push_back(out);
    }
    for (const Entry &e : parsed) put_locked(e.arch, e.enc, e.bucket, e.costs);
    return QMM_OK;
}

qmm_status save_locked(const char *path) {
    const std::string tmp = std::string(path) + ".tmp";
    FILE *f = std::fopen(tmp.c_str(), "wb");
    if (!f) return fail(QMM_EINVAL, std::string("tune cache ") + path + ": cannot write");
    std::fprintf(f, "{\"version\": 1, \"entries\": [");
    for (size_t i = 0; i < g_entries.size(); ++i) {
        const Entry &e = g_entries[i];
        std::string arch;
        for (char c : e.arch)
            if (c != '"' && c != '\\' && (unsigned char)c >= 0x20) arch.push_back(c);
        std::fprintf(f, "%s\n  {\"arch\": \"%s\", \"enc\": \"%s\", \"bucket\": \"%s\", \"costs\": [", i ? "," : "",
                     arch.c_str(), kEncNames[e.enc], kBucketNames[e.bucket]);
        for (int j = 0; j < kTuneCosts; ++j) std::fprintf(f, "%s%.17g", j ? ", " : "", e.costs[j]);
        std::fprintf(f, "]}");
    }
    std::fprintf(f, "\n]}\n");
    const bool ok = std::fflush(f) == 0;
    if (std::fclose(f) != 0 || !ok) {
        std::remove(tmp.c_str());
        return fail(QMM_EINVAL, std::string("tune cache ") + path + ": write failed");
    }
    if (std::rename(tmp.c_str(), path) != 0) {
        std::remove(tmp.c_str());
        return fail(QMM_EINVAL, std::string("tune cache ") + path + ": rename failed");
    }
    return QMM_OK;
}

bool key_ok(const char *arch, uint32_t p, int64_t m, int64_t n) {
    return arch && *arch && p >= 2 && p <= 256 && m >= 0 && n >= 0;
}

}  // namespace

uint32_t tune_enc(uint32_t p) { return p <= 8 ? 1u : 0u; }

uint32_t tune_bucket(int64_t m, int64_t n) {
    const int64_t x = m > n ? m : n;
    return x <= 128 ? 0u : (x <= 512 ? 1u : 2u);
}

void tune_cache_put(const std::string &arch, uint32_t enc, uint32_t bucket, const double *costs) {
    std::lock_guard<std::mutex> lock(g_mu);
    put_locked(arch, enc, bucket, costs);
}

bool tune_cache_lookup(const std::string &arch, uint32_t enc, uint32_t bucket, double *costs) {
    std::lock_guard<std::mutex> lock(g_mu);
    const Entry *best = nullptr;
    uint32_t best_dist = 99;
    for (const Entry &e : g_entries) {
        if (e.arch != arch || e.enc != enc) continue;
        const uint32_t dist = e.bucket > bucket ? e.bucket - bucket : bucket - e.bucket;
        if (dist < best_dist) {
            best = &e;
            best_dist = dist;
        }
    }
    if (!best) return false;
    std::memcpy(costs, best->costs, sizeof(best->costs));
    return true;
}

qmm_status tune_cache_load_env_once() {
    std::lock_guard<std::mutex> lock(g_mu);
    if (g_env_loaded) return QMM_OK;
    g_env_loaded = true;
    const char *path = std::getenv("QMM_TUNE_CACHE");
    if (!path || !*path) return QMM_OK;
    return load_locked(path, true);
}

qmm_status tune_cache_save_env() {
    std::lock_guard<std::mutex> lock(g_mu);
    const char *path = std::getenv("QMM_TUNE_CACHE");
    if (!path || !*path) return QMM_OK;
    return save_locked(path);
}

}  // namespace qmm

using namespace qmm;

extern "C" qmm_status qmm_tune_cache_put(const char *arch, uint32_t p, int64_t m, int64_t n, const double *costs) {
    if (!key_ok(arch, p, m, n)) return fail(QMM_EINVAL, "tune cache key: arch non-empty, 2 <= p <= 256, m, n >= 0");
    if (!costs || !costs_ok(costs)) return fail(QMM_EINVAL, "costs: 8 values, fixed >= 0 and per_stage > 0");
    tune_cache_put(arch, tune_enc(p), tune_bucket(m, n), costs);
    return QMM_OK;
}

extern "C" qmm_status qmm_tune_cache_get(const char *arch, uint32_t p, int64_t m, int64_t n, double *costs) {
    if (!key_ok(arch, p, m, n) || !costs) return fail(QMM_EINVAL, "tune cache key or costs pointer");
    if (!tune_cache_lookup(arch, tune_enc(p), tune_bucket(m, n), costs))
        return fail(QMM_EVALUE, std::string("no tuned costs for ") + arch + " and this encoding");
    return QMM_OK;
}

extern "C" qmm_status qmm_tune_cache_load(const char *path) {
    if (!path || !*path) return fail(QMM_EINVAL, "path is empty");
    std::lock_guard<std::mutex> lock(g_mu);
    return load_locked(path, false);
}

extern "C" qmm_status qmm_tune_cache_save(const char *path) {
    if (!path || !*path) return fail(QMM_EINVAL, "path is empty");
    std::lock_guard<std::mutex> lock(g_mu);
    return save_locked(path);
}

extern "C" qmm_status qmm_tune_cache_clear(void) {
    std::lock_guard<std::mutex> lock(g_mu);
    g_entries.clear();
    return QMM_OK;
}
