// The autotuner's on-disk cache: a text file of "key<TAB>value" lines, one
// per tuned shape.  Lines that do not hold a tab, and lines starting with
// '#', are kept as they are and otherwise ignored.  An update rewrites the
// file through a temporary file in the same directory and renames it over
// the old one, so a reader never sees a half-written cache.
#include <cstdio>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include <unistd.h>

#include "tune.hpp"

namespace hsp {

bool tune_cache_get(const std::string& path, const std::string& key, std::string* value) {
    std::ifstream f(path);
    if (!f) return false;
    std::string line;
    bool found = false;
    while (std::getline(f, line)) {
        if (line.empty() || line[0] == '#') continue;
        const size_t tab = line.find('\t');
        if (tab == std::string::npos) continue;
        if (line.compare(0, tab, key) == 0 && tab == key.size()) {
            *value = line.substr(tab + 1);  // the last entry of a key wins
            found = true;
        }
    }
    return found;
}

bool tune_cache_put(const std::string& path, const std::string& key, const std::string& value) {
    if (key.empty() || key.find_first_of("\t\n") != std::string::npos ||
        value.find('\n') != std::string::npos)
        return false;
    std::vector<std::string> lines;
    {
        std::ifstream f(path);
        std::string line;
        while (f && std::getline(f, line)) {
            const size_t tab = line.find('\t');
            if (tab != std::string::npos && tab == key.size() && line.compare(0, tab, key) == 0) continue;
            lines.push_back(line);
        }
    }
    lines.push_back(key + "\t" + value);
    const std::string tmp = path + ".tmp" + std::to_string((long)getpid());
    {
        std::ofstream out(tmp, std::ios::trunc);
        if (!out) return false;
        for (const std::string& l : lines) out << l << '\n';
        out.flush();
        if (!out) {
            std::remove(tmp.c_str());
            return false;
        }
    }
    if (std::rename(tmp.c_str(), path.c_str()) != 0) {
        std::remove(tmp.c_str());
        return false;
    }
    return true;
}

bool tune_parse(const std::string& value, const char* name, long* out) {
    const std::string pat = std::string(name) + "=";
    std::istringstream in(value);
    std::string tok;
    while (in >> tok) {
        if (tok.compare(0, pat.size(), pat) == 0) {
            try {
                size_t used = 0;
                *out = std::stol(tok.substr(pat.size()), &used);
                return used == tok.size() - pat.size();
            } catch (...) {
                return false;
            }
        }
    }
    return false;
}

}  // namespace hsp
