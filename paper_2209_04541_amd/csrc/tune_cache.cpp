// Launch shapes chosen by the autotuners, kept in process memory and in a
// text file so that a later process does not search again.
//
// One line per entry: the key (no spaces), then the chosen integers.  The
// file is PGABB_TUNE_CACHE when that variable is set (empty: no file), else
// $XDG_CACHE_HOME/pgabb/tune.txt or $HOME/.cache/pgabb/tune.txt.  A file
// that cannot be read or written only costs a new search.
#include <sys/stat.h>
#include <unistd.h>

#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "common.hpp"

namespace pgabb {

namespace {

std::mutex g_mu;
std::map<std::string, std::vector<int>> g_cache;
bool g_loaded = false;

std::string cache_path() {
    if (const char *p = std::getenv("PGABB_TUNE_CACHE")) return p;
    std::string dir;
    if (const char *x = std::getenv("XDG_CACHE_HOME"); x && *x) dir = x;
    else if (const char *h = std::getenv("HOME"); h && *h) dir = std::string(h) + "/.cache";
    else return "";
    return dir + "/pgabb/tune.txt";
}

void load_locked() {
    if (g_loaded) return;
    g_loaded = true;
    const std::string path = cache_path();
    if (path.empty()) return;
    std::ifstream f(path);
    std::string line;
    while (std::getline(f, line)) {
        std::istringstream is(line);
        std::string key;
        if (!(is >> key)) continue;
        std::vector<int> v;
        int x;
        while (is >> x) v.push_back(x);
        if (!v.empty()) g_cache[key] = v;
    }
}

void mkdirs(const std::string &path) {
    for (size_t q = 1; q < path.size(); ++q)
        if (path[q] == '/') (void)mkdir(path.substr(0, q).c_str(), 0755);
}

void save_locked() {
    const std::string path = cache_path();
    if (path.empty()) return;
    mkdirs(path);
    const std::string tmp = path + ".tmp" + std::to_string(static_cast<long>(getpid()));
    {
        std::ofstream f(tmp);
        if (!f) return;
        for (const auto &kv : g_cache) {
            f << kv.first;
            for (int x : kv.second) f << ' ' << x;
            f << '\n';
        }
        if (!f) return;
    }
    (void)std::rename(tmp.c_str(), path.c_str());
}

}  // namespace

bool tune_lookup(const std::string &key, std::vector<int> &val) {
    std::lock_guard<std::mutex> lk(g_mu);
    load_locked();
    auto it = g_cache.find(key);
    if (it == g_cache.end()) return false;
    val = it->second;
    return true;
}

void tune_store(const std::string &key, const std::vector<int> &val) {
    std::lock_guard<std::mutex> lk(g_mu);
    load_locked();
    g_cache[key] = val;
    save_locked();
}

void tune_reload() {
    std::lock_guard<std::mutex> lk(g_mu);
    g_cache.clear();
    g_loaded = false;  // read the file again on next use
}

void tune_forget_all() {
    std::lock_guard<std::mutex> lk(g_mu);
    g_cache.clear();
    g_loaded = true;  // and do not read the file again
}

}  // namespace pgabb
