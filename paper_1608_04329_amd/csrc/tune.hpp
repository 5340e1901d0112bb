// The autotuner's cache file (host code only).
#pragma once
#include <string>

namespace hsp {

// Value stored under key in the cache file at path (false: no file or no entry).
bool tune_cache_get(const std::string& path, const std::string& key, std::string* value);
// Store key -> value, replacing an earlier entry of the key (false on an I/O
// error, or a key holding a tab or newline, or a value holding a newline).
bool tune_cache_put(const std::string& path, const std::string& key, const std::string& value);
// The integer of "name=<int>" among the space-separated fields of value.
bool tune_parse(const std::string& value, const char* name, long* out);

}  // namespace hsp
