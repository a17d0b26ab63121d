// FFT launch-shape defaults, the autotuner's cache (with a small JSON file
// format of its own) and the cache of instantiated launch graphs.
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <sstream>

#include "fv_internal.h"

namespace fv {

bool TuneCache::find(const std::string &key, Tuning *t) {
    std::lock_guard<std::mutex> lk(mu);
    auto it = entries.find(key);
    if (it == entries.end()) return false;
    *t = it->second;
    return true;
}

// File format: one JSON object, key -> {"rows": r, "lines": l, "tpb1": a,
// "tpbm": b, "fft_ms": t}, written whole after every new entry.
void TuneCache::put(const std::string &key, const Tuning &t) {
    std::lock_guard<std::mutex> lk(mu);
    entries[key] = t;
    if (path.empty()) return;
    std::ostringstream o;
    o << "{\n";
    size_t k = 0;
    for (auto &kv : entries) {
        const Tuning &v = kv.second;
        o << "  \"" << kv.first << "\": {\"rows\": " << v.rows << ", \"lines\": " << v.lines << ", \"tpb1\": " << v.tpb1
          << ", \"tpbm\": " << v.tpbm << ", \"split\": " << v.split << ", \"fft_ms\": " << v.fft_ms << "}" << (++k < entries.size() ? "," : "")
          << "\n";
    }
    o << "}\n";
    const std::string tmp = path + ".tmp";
    {
        std::ofstream f(tmp);
        if (!f) return;  // an unwritable cache only costs a re-tune
        f << o.str();
    }
    std::rename(tmp.c_str(), path.c_str());
}

static bool read_int_field(const std::string &obj, const char *name, double *out) {
    const std::string pat = std::string("\"") + name + "\":";
    size_t p = obj.find(pat);
    if (p == std::string::npos) return false;
    *out = std::strtod(obj.c_str() + p + pat.size(), nullptr);
    return true;
}

void TuneCache::load(const std::string &file) {
    std::lock_guard<std::mutex> lk(mu);
    path = file;
    std::ifstream f(file);
    if (!f) return;
    std::stringstream ss;
    ss << f.rdbuf();
    const std::string s = ss.str();
    size_t p = 0;
    while (true) {
        const size_t k0 = s.find('"', p);
        if (k0 == std::string::npos) break;
        const size_t k1 = s.find('"', k0 + 1);
        const size_t b0 = s.find('{', k1);
        const size_t b1 = s.find('}', b0);
        if (k1 == std::string::npos || b0 == std::string::npos || b1 == std::string::npos) break;
        const std::string key = s.substr(k0 + 1, k1 - k0 - 1), obj = s.substr(b0, b1 - b0 + 1);
        Tuning t;
        double v;
        bool ok = true;
        ok = ok && read_int_field(obj, "rows", &v);
        t.rows = (int)v;
        ok = ok && read_int_field(obj, "lines", &v);
        t.lines = (int)v;
        ok = ok && read_int_field(obj, "tpb1", &v);
        t.tpb1 = (int)v;
        ok = ok && read_int_field(obj, "tpbm", &v);
        t.tpbm = (int)v;
        if (read_int_field(obj, "split", &v)) t.split = v != 0.0;
        if (read_int_field(obj, "fft_ms", &v)) t.fft_ms = v;
        if (ok && t.rows >= 1 && t.lines >= 1) entries[key] = t;
        p = b1 + 1;
    }
}

hipGraphExec_t GraphCache::find(uint64_t key) {
    for (auto it = entries.begin(); it != entries.end(); ++it)
        if (it->first == key) {
            auto e = *it;
            entries.erase(it);
            entries.push_back(e);
            return e.second;
        }
    return nullptr;
}

void GraphCache::put(uint64_t key, hipGraphExec_t g) {
    if (entries.size() >= 8) {
        (void)hipGraphExecDestroy(entries.front().second);
        entries.pop_front();
    }
    entries.push_back({key, g});
}

void GraphCache::release() {
    for (auto &e : entries) (void)hipGraphExecDestroy(e.second);
    entries.clear();
}

}  // namespace fv
