// Autotuner of the breadth-first walk's launch settings (snp_tuning of snp.h)
// and its JSON cache.  A setting is measured by running the caller's whole
// walk (snp_run) with it: children per device pass, consecutive 64-child
// tiles per workgroup of the int8 form, consecutive children per wave of the
// sparse form.  A cache file maps a key of the workload and the GPU to the
// settings found, so that later handles of the same workload start from them.
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <map>
#include <string>
#include <vector>

#include "snp.h"
#include "snp_handle.hpp"

namespace {

using snp::set_error;

// FNV-1a, 64 bits.
struct Fnv {
    u64 h = 1469598103934665603ULL;
    void add(const void* p, size_t n) {
        const unsigned char* b = (const unsigned char*)p;
        for (size_t i = 0; i < n; ++i) {
            h ^= b[i];
            h *= 1099511628211ULL;
        }
    }
    template <typename T>
    void val(T v) {
        add(&v, sizeof v);
    }
    void vec(const std::vector<int32_t>& v) {
        val((u64)v.size());
        if (!v.empty()) add(v.data(), v.size() * sizeof(int32_t));
    }
};

// Key of a workload: the GPU's architecture name (letters and digits kept,
// the rest as '_'), then a hash of the system and of the options and depth
// that shape the walk.
snp_status tuning_key(const snp_system* S, int32_t max_depth, std::string* key) {
    int dev = 0;
    hipDeviceProp_t pr{};
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&pr, dev) != hipSuccess)
        return set_error(SNP_ERR_DEVICE, "autotune: no device properties");
    std::string arch;
    for (const char* c = pr.gcnArchName; *c && arch.size() < 64; ++c)
        arch.push_back(((*c >= 'a' && *c <= 'z') || (*c >= 'A' && *c <= 'Z') || (*c >= '0' && *c <= '9')) ? *c : '_');
    Fnv f;
    f.val(S->m);
    f.val(S->r);
    f.val(S->count_type);
    f.vec(S->h_rn);
    f.vec(S->h_ri);
    f.vec(S->h_rj);
    f.vec(S->h_rc);
    f.vec(S->h_rp);
    f.vec(S->h_ss);
    f.vec(S->h_sd);
    f.val(S->opt.path);
    f.val(S->opt.stop_at_cap);
    f.val(S->opt.frontier_cap);
    f.val(S->opt.child_budget);
    f.val(S->opt.expand_max_count);
    f.val(S->opt.deterministic);
    f.val(S->opt.int8_max_k);
    f.val(S->chunk_max);
    f.val(max_depth);
    char buf[32];
    snprintf(buf, sizeof buf, "%016llx", (unsigned long long)f.h);
    *key = arch + "-" + buf;
    return SNP_OK;
}

struct Entry {
    snp_tuning tu{};
    double ms = 0;
};

const char* kMagic = "\"snp_tuning_cache\": 1";

// Reads a cache file.  A missing file is an empty cache; a file that is not a
// tuning cache is an error (it is never overwritten).
snp_status read_cache(const char* path, std::map<std::string, Entry>* out, bool* exists) {
    out->clear();
    *exists = false;
    FILE* fp = fopen(path, "rb");
    if (!fp) return SNP_OK;
    std::string text;
    char buf[4096];
    size_t got;
    while ((got = fread(buf, 1, sizeof buf, fp)) > 0) text.append(buf, got);
    fclose(fp);
    *exists = true;
    if (text.find(kMagic) == std::string::npos)
        return set_error(SNP_ERR_INVALID, "%s is not a tuning cache (no %s)", path, kMagic);
    size_t pos = text.find("\"entries\"");
    if (pos == std::string::npos) return set_error(SNP_ERR_INVALID, "%s: no \"entries\"", path);
    pos = text.find('{', pos);
    if (pos == std::string::npos) return set_error(SNP_ERR_INVALID, "%s: malformed \"entries\"", path);
    ++pos;
    for (;;) {  // "key": {"chunk": N, "int8_tiles": N, "sparse_run": N, "ms": X}
        const size_t q0 = text.find_first_of("\"}", pos);
        if (q0 == std::string::npos) return set_error(SNP_ERR_INVALID, "%s: unterminated entries", path);
        if (text[q0] == '}') break;
        const size_t q1 = text.find('"', q0 + 1);
        const size_t b0 = q1 == std::string::npos ? q1 : text.find('{', q1);
        const size_t b1 = b0 == std::string::npos ? b0 : text.find('}', b0);
        if (b1 == std::string::npos) return set_error(SNP_ERR_INVALID, "%s: malformed entry", path);
        const std::string key = text.substr(q0 + 1, q1 - q0 - 1);
        const std::string obj = text.substr(b0, b1 - b0 + 1);
        long long chunk = 0, tiles = 0, run = 0;
        double ms = 0;
        const size_t a = obj.find("\"chunk\""), b = obj.find("\"int8_tiles\""), c = obj.find("\"sparse_run\""),
                     d = obj.find("\"ms\"");
        if (a == std::string::npos || b == std::string::npos || c == std::string::npos ||
            sscanf(obj.c_str() + a, "\"chunk\": %lld", &chunk) != 1 ||
            sscanf(obj.c_str() + b, "\"int8_tiles\": %lld", &tiles) != 1 ||
            sscanf(obj.c_str() + c, "\"sparse_run\": %lld", &run) != 1)
            return set_error(SNP_ERR_INVALID, "%s: malformed entry %s", path, key.c_str());
        if (d != std::string::npos) sscanf(obj.c_str() + d, "\"ms\": %lf", &ms);
        Entry e;
        e.tu.chunk = chunk;
        e.tu.int8_tiles = (int32_t)tiles;
        e.tu.sparse_run = (int32_t)run;
        e.ms = ms;
        (*out)[key] = e;
        pos = b1 + 1;
    }
    return SNP_OK;
}

snp_status write_cache(const char* path, const std::map<std::string, Entry>& entries) {
    const std::string tmp = std::string(path) + ".tmp";
    FILE* fp = fopen(tmp.c_str(), "wb");
    if (!fp) return set_error(SNP_ERR_INVALID, "cannot write %s", tmp.c_str());
    fprintf(fp, "{\n  %s,\n  \"entries\": {", kMagic);
    bool first = true;
    for (const auto& kv : entries) {
        fprintf(fp, "%s\n    \"%s\": {\"chunk\": %lld, \"int8_tiles\": %d, \"sparse_run\": %d, \"ms\": %.4f}",
                first ? "" : ",", kv.first.c_str(), (long long)kv.second.tu.chunk, kv.second.tu.int8_tiles,
                kv.second.tu.sparse_run, kv.second.ms);
        first = false;
    }
    fprintf(fp, "\n  }\n}\n");
    if (fclose(fp) != 0 || rename(tmp.c_str(), path) != 0)
        return set_error(SNP_ERR_INVALID, "cannot write %s", path);
    return SNP_OK;
}

snp_status check_tuning(const snp_system* S, const snp_tuning* tu) {
    if (tu->chunk < 0 || tu->chunk > S->chunk_max)
        return set_error(SNP_ERR_INVALID, "tuning: chunk %lld outside [0, %lld] (the handle's chunk)",
                         (long long)tu->chunk, S->chunk_max);
    if (tu->int8_tiles < 0 || tu->int8_tiles > 64) return set_error(SNP_ERR_INVALID, "tuning: int8_tiles outside [0, 64]");
    if (tu->sparse_run < 0 || tu->sparse_run > 1024)
        return set_error(SNP_ERR_INVALID, "tuning: sparse_run outside [0, 1024]");
    return SNP_OK;
}

void apply(snp_system* S, const snp_tuning& tu) {
    S->chunk_eff = tu.chunk > 0 ? tu.chunk : S->chunk_max;
    S->tune_tiles = tu.int8_tiles;
    S->tune_run = tu.sparse_run;
}

}  // namespace

extern "C" {

snp_status snp_get_tuning(const snp_system* S, snp_tuning* out) {
    if (!S || !out) return set_error(SNP_ERR_INVALID, "handle and out are required");
    out->chunk = S->chunk_eff;
    out->int8_tiles = S->tune_tiles;
    out->sparse_run = S->tune_run;
    return SNP_OK;
}

snp_status snp_set_tuning(snp_system* S, const snp_tuning* tu) {
    if (!S || !tu) return set_error(SNP_ERR_INVALID, "handle and tuning are required");
    snp_status st = check_tuning(S, tu);
    if (st) return st;
    apply(S, *tu);
    return SNP_OK;
}

snp_status snp_load_tuning(snp_system* S, const char* cache_path, int32_t max_depth, int32_t* found) {
    if (!S || !cache_path || !found) return set_error(SNP_ERR_INVALID, "handle, cache_path and found are required");
    *found = 0;
    std::string key;
    snp_status st = tuning_key(S, max_depth, &key);
    if (st) return st;
    std::map<std::string, Entry> entries;
    bool exists = false;
    if ((st = read_cache(cache_path, &entries, &exists))) return st;
    const auto it = entries.find(key);
    if (it == entries.end()) return SNP_OK;
    if ((st = check_tuning(S, &it->second.tu))) return st;
    apply(S, it->second.tu);
    *found = 1;
    return SNP_OK;
}

snp_status snp_autotune(snp_system* S, const void* c0_dev, int32_t max_depth, void* out_dev, int64_t out_capacity,
                        const char* cache_path, snp_tuning* best_out, double* best_ms_out) {
    if (!S || !c0_dev || !out_dev) return set_error(SNP_ERR_INVALID, "handle, c0 and out are required");
    std::string key;
    snp_status st = tuning_key(S, max_depth, &key);
    if (st) return st;
    std::map<std::string, Entry> entries;
    bool exists = false;
    if (cache_path && (st = read_cache(cache_path, &entries, &exists))) return st;

    constexpr int kLevels = 4096;
    std::vector<int64_t> sizes(kLevels);
    int64_t ncfg = 0;
    int32_t nlev = 0, stop = 0;
    // the fastest of a few whole walks (fewer for long ones) after one warm-up
    auto time_walks = [&](const snp_tuning& tu, double* ms) -> snp_status {
        apply(S, tu);
        double best = 1e300;
        int reps = 3;
        for (int rep = 0; rep <= reps; ++rep) {
            const auto t0 = std::chrono::steady_clock::now();
            const snp_status r = snp_run(S, c0_dev, max_depth, out_dev, out_capacity, &ncfg, sizes.data(), kLevels,
                                         &nlev, &stop, nullptr, nullptr, nullptr);
            if (r) return r;
            const double dt = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
            if (rep == 0 && dt > 100.0) reps = 1;
            if (rep > 0) best = std::min(best, dt);
        }
        *ms = best;
        return SNP_OK;
    };
    snp_tuning best{};
    best.chunk = S->chunk_max;
    double best_ms = 0;
    if ((st = time_walks(best, &best_ms))) return st;
    auto consider = [&](const snp_tuning& tu) -> snp_status {
        double ms = 0;
        const snp_status r = time_walks(tu, &ms);
        if (r) return r;
        if (ms < best_ms) {
            best_ms = ms;
            best = tu;
        }
        return SNP_OK;
    };
    // children per pass: the handle's size and smaller powers-of-two fractions
    for (long long c = S->chunk_max / 2; c >= 4096 && c >= S->chunk_max / 16; c /= 2) {
        snp_tuning tu = best;
        tu.chunk = c;
        if ((st = consider(tu))) return st;
    }
    // int8 tiles per workgroup, where the int8 form can run
    if (S->int8_ready && S->opt.path != SNP_PATH_SPARSE)
        for (int tiles : {1, 2, 4, 8, 16}) {
            snp_tuning tu = best;
            tu.int8_tiles = tiles;
            if ((st = consider(tu))) return st;
        }
    // children per wave of the sparse form, where it can run
    if (!S->lane_form && (S->opt.path != SNP_PATH_INT8 || !S->int8_ready))
        for (int run : {4, 8, 16, 32, 64}) {
            snp_tuning tu = best;
            tu.sparse_run = run;
            if ((st = consider(tu))) return st;
        }
    apply(S, best);
    if (best_out) *best_out = best;
    if (best_ms_out) *best_ms_out = best_ms;
    if (cache_path) {
        Entry e;
        e.tu = best;
        e.ms = best_ms;
        entries[key] = e;
        if ((st = write_cache(cache_path, entries))) return st;
    }
    return SNP_OK;
}

}  // extern "C"
