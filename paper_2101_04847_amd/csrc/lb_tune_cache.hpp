// Persisted tile choices of liblb (host code only).
//
// The timed search of lb_init (pass and tile shapes) depends only on the
// device, the storage mode, the forcing scheme, the boundary variant, the
// requested pass and tile options and the member lattice sizes.  Its result
// is kept in a small JSON file so that later processes skip the timing:
//
//   { "<key>": {"spp": 2, "tx": 128, "th": [16, 32], "th2": [8, 7], "th3": [12, 12]}, ... }
//
// with th / th2 / th3 the band heights of the single-step, the two-step and
// the three-step pass
// per size class (in the order the classes first appear among the members).
// The file is LB_TILE_CACHE if that is set ("off" or empty disables the
// cache), else $XDG_CACHE_HOME/liblb/tiles.json or ~/.cache/liblb/tiles.json.
// Writers replace the file atomically (write a temporary file, rename); a
// file that does not parse is ignored and rewritten.
#pragma once

#include <sys/stat.h>
#include <unistd.h>

#include <cctype>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <string>
#include <vector>

namespace lbtune {

struct Choice {
    int spp = 0, tx = 0;
    std::vector<int> th, th2, th3;
};

inline std::string cache_path()
{
    const char *env = std::getenv("LB_TILE_CACHE");
    if (env) {
        std::string v(env);
        if (v.empty() || v == "off") return std::string();
        return v;
    }
    std::string dir;
    if (const char *x = std::getenv("XDG_CACHE_HOME"); x && *x) dir = x;
    else if (const char *hm = std::getenv("HOME"); hm && *hm) dir = std::string(hm) + "/.cache";
    else return std::string();
    return dir + "/liblb/tiles.json";
}

// --- a reader for exactly the structure written below ---------------------
struct Reader {
    const std::string &s;
    size_t p = 0;
    bool ok = true;
    explicit Reader(const std::string &text) : s(text) {}
    void ws()
    {
        while (p < s.size() && std::isspace((unsigned char)s[p])) ++p;
    }
    bool eat(char c)
    {
        ws();
        if (p < s.size() && s[p] == c) {
            ++p;
            return true;
        }
        return false;
    }
    void need(char c)
    {
        if (!eat(c)) ok = false;
    }
    std::string str()
    {
        std::string out;
        need('"');
        while (ok && p < s.size() && s[p] != '"') {
            if (s[p] == '\\') {
                ok = false;   // keys written by this library hold no escapes
                break;
            }
            out += s[p++];
        }
        need('"');
        return out;
    }
    int num()
    {
        ws();
        size_t q = p;
        if (q < s.size() && s[q] == '-') ++q;
        while (q < s.size() && std::isdigit((unsigned char)s[q])) ++q;
        if (q == p) {
            ok = false;
            return 0;
        }
        const int v = std::atoi(s.substr(p, q - p).c_str());
        p = q;
        return v;
    }
    std::vector<int> arr()
    {
        std::vector<int> out;
        need('[');
        if (eat(']')) return out;
        do {
            out.push_back(num());
        } while (ok && eat(','));
        need(']');
        return out;
    }
};

inline bool parse(const std::string &text, std::map<std::string, Choice> &out)
{
    Reader r(text);
    r.need('{');
    if (r.eat('}')) return r.ok;
    do {
        const std::string key = r.str();
        r.need(':');
        r.need('{');
        Choice c;
        do {
            const std::string f = r.str();
            r.need(':');
            if (f == "spp") c.spp = r.num();
            else if (f == "tx") c.tx = r.num();
            else if (f == "th") c.th = r.arr();
            else if (f == "th2") c.th2 = r.arr();
            else if (f == "th3") c.th3 = r.arr();
            else r.ok = false;
        } while (r.ok && r.eat(','));
        r.need('}');
        if (!r.ok) return false;
        out[key] = c;
    } while (r.ok && r.eat(','));
    r.need('}');
    return r.ok;
}

inline std::string to_json(const std::map<std::string, Choice> &m)
{
    auto arr = [](const std::vector<int> &v) {
        std::string o = "[";
        for (size_t k = 0; k < v.size(); ++k) o += (k ? ", " : "") + std::to_string(v[k]);
        return o + "]";
    };
    std::string o = "{\n";
    size_t k = 0;
    for (const auto &kv : m) {
        o += " \"" + kv.first + "\": {\"spp\": " + std::to_string(kv.second.spp) + ", \"tx\": " +
             std::to_string(kv.second.tx) + ", \"th\": " + arr(kv.second.th) + ", \"th2\": " + arr(kv.second.th2) +
             ", \"th3\": " + arr(kv.second.th3) + "}" + (++k < m.size() ? ",\n" : "\n");
    }
    return o + "}\n";
}

inline std::mutex &mu()
{
    static std::mutex m;
    return m;
}

inline bool read_file(const std::string &path, std::string &text)
{
    FILE *fh = std::fopen(path.c_str(), "rb");
    if (!fh) return false;
    char buf[4096];
    size_t n;
    while ((n = std::fread(buf, 1, sizeof buf, fh)) > 0) text.append(buf, n);
    std::fclose(fh);
    return true;
}

// Cached choice for key (false if none or the cache is off).
inline bool lookup(const std::string &key, Choice &out)
{
    const std::string path = cache_path();
    if (path.empty()) return false;
    std::lock_guard<std::mutex> lk(mu());
    std::string text;
    std::map<std::string, Choice> m;
    if (!read_file(path, text) || !parse(text, m)) return false;
    auto it = m.find(key);
    if (it == m.end()) return false;
    out = it->second;
    return true;
}

// Record a choice (best effort: a cache that cannot be written is skipped).
inline void store(const std::string &key, const Choice &c)
{
    const std::string path = cache_path();
    if (path.empty()) return;
    std::lock_guard<std::mutex> lk(mu());
    // create the directory chain if needed
    for (size_t q = path.find('/', 1); q != std::string::npos; q = path.find('/', q + 1))
        (void)mkdir(path.substr(0, q).c_str(), 0755);
    std::string text;
    std::map<std::string, Choice> m;
    if (read_file(path, text) && !parse(text, m)) m.clear();
    m[key] = c;
    const std::string tmp = path + ".tmp" + std::to_string((long)getpid());
    FILE *fh = std::fopen(tmp.c_str(), "wb");
    if (!fh) return;
    const std::string out = to_json(m);
    const bool wrote = std::fwrite(out.data(), 1, out.size(), fh) == out.size();
    if (std::fclose(fh) != 0 || !wrote) {
        std::remove(tmp.c_str());
        return;
    }
    if (std::rename(tmp.c_str(), path.c_str()) != 0) std::remove(tmp.c_str());
}

}  // namespace lbtune
