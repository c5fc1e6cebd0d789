// Autotune cache: the launch shapes tdct_autotune kept, in a JSON file keyed
// by GPU architecture, op set and size class, so that a later process takes
// a tuned shape without timing candidates again and the server can launch
// its batches in tuned shapes.
//
// Key: "<arch>/src=<hash>/ops=<mask>/tiles=<k>/aligned=<0|1>". <arch> is the
// device's architecture name without feature suffixes (gfx950); <hash> names
// the library's sources (the build passes it in), so shapes tuned for other
// kernel code are never taken; <mask> has bit i set
// when op i occurs; k = floor(log2(tiles)) of the batch's own tile count;
// aligned = 1 when every pixel plane's address, width and stride are
// multiples of 128 bytes (no pixel row begins or ends inside a 128-byte line,
// which decides the pixel cache policy). The file is
//
//   { "format": "tdct-autotune-1",
//     "entries": {
//       "<key>": [waves_per_group, groups_per_cu, tile_waves, xcd_remap, pixel_cache],
//       ... } }
//
// It is read when the cache is opened and rewritten whole (through a
// temporary file and a rename) after each new entry, keeping the entries
// other processes stored in it meanwhile.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

#include <map>
#include <mutex>
#include <string>

#include "tdct.h"
#include "tdct_internal.hpp"

#ifndef TDCT_SOURCE_HASH
#define TDCT_SOURCE_HASH "unversioned"
#endif

namespace tdct {
namespace {

struct TuneCache {
    std::mutex mu;
    bool env_checked = false;
    bool on = false;
    std::string path;
    std::map<std::string, tdct_tune> entries;
    tdct_tune_cache_stats stats{};
};

TuneCache& cache() {
    static TuneCache c;
    return c;
}

// Parser for the file format above (the library writes it; anything else is
// refused).
struct Scan {
    const char* p;
    const char* end;
    void ws() {
        while (p < end && (*p == ' ' || *p == '\n' || *p == '\r' || *p == '\t')) ++p;
    }
    bool eat(char c) {
        ws();
        if (p < end && *p == c) {
            ++p;
            return true;
        }
        return false;
    }
    bool str(std::string& out) {
        if (!eat('"')) return false;
        const char* q = p;
        while (p < end && *p != '"' && *p != '\\' && *p != '\n') ++p;
        if (p >= end || *p != '"') return false;
        out.assign(q, p);
        ++p;
        return true;
    }
    bool num(int32_t& out) {
        ws();
        char* e = nullptr;
        const long v = strtol(p, &e, 10);
        if (e == p || v < -(1L << 30) || v > (1L << 30)) return false;
        out = (int32_t)v;
        p = e;
        return true;
    }
};

int parse(const std::string& text, std::map<std::string, tdct_tune>& out) {
    Scan s{text.data(), text.data() + text.size()};
    std::string k;
    bool have_entries = false;
    if (!s.eat('{')) return TDCT_EINVAL;
    if (s.eat('}')) return TDCT_EINVAL;
    do {
        if (!s.str(k) || !s.eat(':')) return TDCT_EINVAL;
        if (k == "format") {
            std::string v;
            if (!s.str(v) || v != "tdct-autotune-1") return TDCT_EINVAL;
        } else if (k == "entries") {
            have_entries = true;
            if (!s.eat('{')) return TDCT_EINVAL;
            if (s.eat('}')) continue;
            do {
                std::string key;
                int32_t f[5];
                if (!s.str(key) || !s.eat(':') || !s.eat('[')) return TDCT_EINVAL;
                for (int i = 0; i < 5; ++i)
                    if ((i && !s.eat(',')) || !s.num(f[i])) return TDCT_EINVAL;
                if (!s.eat(']')) return TDCT_EINVAL;
                tdct_tune t{f[0], f[1], f[2], f[3], f[4]}, n;
                if (t.waves_per_group == 0 || t.groups_per_cu == 0 || t.tile_waves == 0 ||
                    normalise_tune(&t, &n))
                    return TDCT_EINVAL;
                out[key] = n;
            } while (s.eat(','));
            if (!s.eat('}')) return TDCT_EINVAL;
        } else {
            return TDCT_EINVAL;
        }
    } while (s.eat(','));
    if (!s.eat('}') || !have_entries) return TDCT_EINVAL;
    s.ws();
    return s.p == s.end ? TDCT_OK : TDCT_EINVAL;
}

// Reads the whole file at `path`: 1 if read, 0 if it cannot be opened, -1
// on a read error.
int read_file(const char* path, std::string* text) {
    FILE* f = fopen(path, "rb");
    if (!f) return 0;
    char buf[4096];
    size_t n;
    while ((n = fread(buf, 1, sizeof buf, f)) > 0) text->append(buf, n);
    const bool bad = ferror(f) != 0;
    fclose(f);
    return bad ? -1 : 1;
}

// Loads `path` into the cache and turns it on (a missing file is an empty
// cache). Caller holds the lock.
int load_locked(TuneCache& c, const char* path) {
    c.on = false;
    c.entries.clear();
    c.path.clear();
    if (!path || !*path) return TDCT_OK;
    std::map<std::string, tdct_tune> e;
    std::string text;
    const int got = read_file(path, &text);
    if (got < 0) return TDCT_EINVAL;
    if (got > 0) {
        if (parse(text, e)) {
            set_error_text("autotune cache: file is not in the cache's format");
            return TDCT_EINVAL;
        }
    }
    c.entries.swap(e);
    c.path = path;
    c.on = true;
    c.stats.entries = (int64_t)c.entries.size();
    TDCT_LOG(2, "autotune cache: %s, %zu entries", path, c.entries.size());
    return TDCT_OK;
}

void ensure_env_locked(TuneCache& c) {
    if (c.env_checked) return;
    c.env_checked = true;
    const char* p = getenv("TDCT_TUNE_CACHE");
    if (p && *p) (void)load_locked(c, p);
}

// Writes the whole cache through a temporary file and a rename, so a reader
// never sees half a file. Entries that another process stored in the file
// since this one read it are kept (on the same key this process's entry
// wins); a file that no longer parses is replaced. Caller holds the lock.
void write_locked(TuneCache& c) {
    std::string text;
    std::map<std::string, tdct_tune> disk;
    if (read_file(c.path.c_str(), &text) > 0 && parse(text, disk) == TDCT_OK)
        for (const auto& kv : disk) c.entries.emplace(kv.first, kv.second);
    c.stats.entries = (int64_t)c.entries.size();
    std::string out = "{\n \"format\": \"tdct-autotune-1\",\n \"entries\": {";
    bool first = true;
    for (const auto& kv : c.entries) {
        // keys hold no quote, backslash or newline (the parser refuses them),
        // so they go out as they are, whatever their length
        char nums[96];
        const tdct_tune& t = kv.second;
        snprintf(nums, sizeof nums, "[%d, %d, %d, %d, %d]", t.waves_per_group, t.groups_per_cu,
                 t.tile_waves, t.xcd_remap, t.pixel_cache);
        out += first ? "\n  \"" : ",\n  \"";
        out += kv.first;
        out += "\": ";
        out += nums;
        first = false;
    }
    out += "\n }\n}\n";
    const std::string tmp = c.path + ".tmp" + std::to_string((long)getpid());
    FILE* f = fopen(tmp.c_str(), "wb");
    bool ok = f && fwrite(out.data(), 1, out.size(), f) == out.size();
    if (f) ok = (fclose(f) == 0) && ok;
    if (ok) ok = rename(tmp.c_str(), c.path.c_str()) == 0;
    if (!ok) {
        (void)remove(tmp.c_str());
        c.stats.write_errors++;
        TDCT_LOG(1, "autotune cache: could not write %s", c.path.c_str());
    }
}

}  // namespace

int device_arch(std::string* out) {
    int dev = 0;
    hipDeviceProp_t prop;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipGetDeviceProperties(&prop, dev);
    if (e != hipSuccess) {
        set_error("device query", e);
        return TDCT_EDEVICE;
    }
    std::string a = prop.gcnArchName;
    const size_t colon = a.find(':');
    *out = colon == std::string::npos ? a : a.substr(0, colon);
    return TDCT_OK;
}

bool pixels_aligned(const ImgDesc* imgs, size_t n) {
    for (size_t i = 0; i < n; ++i) {
        const ImgDesc& d = imgs[i];
        const int64_t w = 8 * (int64_t)d.nbx;
        if (w % 128) return false;
        if (d.src && (((uintptr_t)d.src % 128) || d.src_stride % 128)) return false;
        if (d.dst && (((uintptr_t)d.dst % 128) || d.dst_stride % 128)) return false;
    }
    return true;
}

static int floor_log2(int64_t x) {
    int k = 0;
    while (x > 1) {
        x >>= 1;
        ++k;
    }
    return k;
}

std::string tune_key(const std::string& arch, int ops, int64_t tiles, bool aligned) {
    char buf[160];
    snprintf(buf, sizeof buf, "%s/src=%s/ops=%d/tiles=%d/aligned=%d", arch.c_str(), TDCT_SOURCE_HASH, ops,
             floor_log2(tiles), aligned ? 1 : 0);
    return buf;
}

bool tune_cache_get(const std::string& key, tdct_tune* out) {
    TuneCache& c = cache();
    std::lock_guard<std::mutex> lk(c.mu);
    ensure_env_locked(c);
    if (!c.on) return false;
    auto it = c.entries.find(key);
    if (it == c.entries.end()) {
        c.stats.misses++;
        return false;
    }
    c.stats.hits++;
    *out = it->second;
    return true;
}

bool tune_cache_nearest(const std::string& arch, int ops, int64_t tiles, bool aligned, tdct_tune* out) {
    TuneCache& c = cache();
    std::lock_guard<std::mutex> lk(c.mu);
    ensure_env_locked(c);
    if (!c.on || c.entries.empty()) return false;
    const int k = floor_log2(tiles);
    // the same class, else the nearest size class within a factor of 4
    // (the larger one on a tie)
    for (int d : {0, 1, -1, 2, -2}) {
        if (k + d < 0) continue;
        auto it = c.entries.find(tune_key(arch, ops, (int64_t)1 << (k + d), aligned));
        if (it != c.entries.end()) {
            c.stats.batch_hits++;
            *out = it->second;
            return true;
        }
    }
    c.stats.batch_misses++;
    return false;
}

void tune_cache_put(const std::string& key, const tdct_tune& t) {
    TuneCache& c = cache();
    std::lock_guard<std::mutex> lk(c.mu);
    ensure_env_locked(c);
    if (!c.on) return;
    c.entries[key] = t;
    c.stats.entries = (int64_t)c.entries.size();
    c.stats.stores++;
    write_locked(c);
}

}  // namespace tdct

extern "C" {

int tdct_tune_cache_open(const char* path) {
    return tdct::abi_call([&]() -> int {
        tdct::TuneCache& c = tdct::cache();
        std::lock_guard<std::mutex> lk(c.mu);
        c.env_checked = true;  // an explicit choice replaces the environment's
        c.stats = tdct_tune_cache_stats{};
        return tdct::load_locked(c, path);
    });
}

int tdct_tune_cache_info(tdct_tune_cache_stats* out) {
    return tdct::abi_call([&]() -> int {
        if (!out) return TDCT_EINVAL;
        tdct::TuneCache& c = tdct::cache();
        std::lock_guard<std::mutex> lk(c.mu);
        tdct::ensure_env_locked(c);  // may read the file $TDCT_TUNE_CACHE names
        *out = c.stats;
        out->on = c.on ? 1 : 0;
        out->entries = (int64_t)c.entries.size();
        return TDCT_OK;
    });
}

}  // extern "C"
