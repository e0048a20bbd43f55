// Cache files of the Ewald table and the learned surrogate (internal).
#pragma once
#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

namespace ot {

// Every input a cached payload depends on, compared byte for byte (zero the
// whole key before filling it).
struct CacheKey {
  uint32_t kind;  // 1: Ewald table, 2: learned surrogate
  uint32_t pad;
  double d[24];
  int64_t i[16];
};

enum class CacheRead { Loaded, Regenerate, IoError };

// The path can be read (if it exists) and a file can be written next to it.
bool cache_path_usable(const char *path, std::string &why);
// Loaded: payload holds the file's payload.  Regenerate: missing, made for
// other inputs, truncated or corrupted (why says which).  IoError: the file
// exists but cannot be read.
CacheRead cache_read(const char *path, const CacheKey &key, std::vector<char> &payload, std::string &why);
// Writes header, key and payload through a temporary file renamed into place.
bool cache_write(const char *path, const CacheKey &key, const void *payload, size_t bytes, std::string &why);

}  // namespace ot
