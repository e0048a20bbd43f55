// Cache files of the Ewald table and the learned surrogate (host code).
//
// The paper's code keeps the Ewald field in a file and regenerates it when
// asked to (App. B, grv_bhEwaldAlwaysGenerate, grv_bhEwaldFName).  Here a
// file holds a fixed header, a key block that records every input the
// payload depends on, and the payload.  A file is used only when its magic,
// version, kind, key block, payload size and payload checksum (FNV-1a, 64
// bit) all match; anything else (missing, another geometry or setting,
// truncated, corrupted) makes the caller regenerate the payload and rewrite
// the file.  Files are written to a temporary name in the same directory and
// renamed into place, so a reader never sees a partial file.
#include "cache.hpp"

#include <cerrno>
#include <cstdio>
#include <cstring>

#include <sys/stat.h>
#include <unistd.h>

namespace ot {

namespace {

constexpr char MAGIC[8] = {'O', 'T', 'C', 'A', 'C', 'H', 'E', '1'};
constexpr uint32_t VERSION = 1;

struct Header {
  char magic[8];
  uint32_t version;
  uint32_t kind;
  uint64_t payload_bytes;
  uint64_t payload_hash;
  CacheKey key;
};

uint64_t fnv1a(const void *p, size_t n) {
  const unsigned char *b = static_cast<const unsigned char *>(p);
  uint64_t h = 14695981039346656037ull;
  for (size_t i = 0; i < n; ++i) {
    h ^= b[i];
    h *= 1099511628211ull;
  }
  return h;
}

std::string errno_text() { return std::string(std::strerror(errno)); }

}  // namespace

bool cache_path_usable(const char *path, std::string &why) {
  struct stat sb;
  if (stat(path, &sb) == 0) {
    if (S_ISDIR(sb.st_mode)) {
      why = std::string("cache path is a directory: ") + path;
      return false;
    }
    FILE *f = std::fopen(path, "rb");
    if (!f) {
      why = std::string("cannot read cache file ") + path + ": " + errno_text();
      return false;
    }
    std::fclose(f);
  }
  // the file is (re)written through a temporary name next to it
  const std::string tmp = std::string(path) + ".tmp";
  FILE *f = std::fopen(tmp.c_str(), "wb");
  if (!f) {
    why = std::string("cannot write next to cache file ") + path + ": " + errno_text();
    return false;
  }
  std::fclose(f);
  std::remove(tmp.c_str());
  return true;
}

CacheRead cache_read(const char *path, const CacheKey &key, std::vector<char> &payload, std::string &why) {
  FILE *f = std::fopen(path, "rb");
  if (!f) {
    if (errno == ENOENT) {
      why = "no cache file";
      return CacheRead::Regenerate;
    }
    why = std::string("cannot read cache file ") + path + ": " + errno_text();
    return CacheRead::IoError;
  }
  Header h;
  CacheRead r = CacheRead::Regenerate;
  if (std::fread(&h, sizeof(h), 1, f) != 1) {
    why = "cache file shorter than its header";
  } else if (std::memcmp(h.magic, MAGIC, sizeof(MAGIC)) != 0 || h.version != VERSION) {
    why = "not a cache file of this version";
  } else if (h.kind != key.kind || std::memcmp(&h.key, &key, sizeof(key)) != 0) {
    why = "cache file made for other inputs";
  } else if (h.payload_bytes > ((uint64_t)1 << 34)) {
    why = "cache file payload size out of range";
  } else {
    payload.resize(h.payload_bytes);
    if (h.payload_bytes && std::fread(payload.data(), 1, h.payload_bytes, f) != h.payload_bytes) {
      why = "cache file truncated";
    } else if (std::fgetc(f) != EOF) {
      why = "cache file longer than its payload";
    } else if (fnv1a(payload.data(), payload.size()) != h.payload_hash) {
      why = "cache file checksum mismatch";
    } else {
      r = CacheRead::Loaded;
    }
  }
  std::fclose(f);
  if (r != CacheRead::Loaded) payload.clear();
  return r;
}

bool cache_write(const char *path, const CacheKey &key, const void *payload, size_t bytes, std::string &why) {
  Header h;
  std::memset(&h, 0, sizeof(h));
  std::memcpy(h.magic, MAGIC, sizeof(MAGIC));
  h.version = VERSION;
  h.kind = key.kind;
  h.payload_bytes = bytes;
  h.payload_hash = fnv1a(payload, bytes);
  h.key = key;
  const std::string tmp = std::string(path) + ".tmp";
  FILE *f = std::fopen(tmp.c_str(), "wb");
  if (!f) {
    why = std::string("cannot write cache file ") + tmp + ": " + errno_text();
    return false;
  }
  bool ok = std::fwrite(&h, sizeof(h), 1, f) == 1 && (bytes == 0 || std::fwrite(payload, 1, bytes, f) == bytes);
  ok = (std::fclose(f) == 0) && ok;
  if (!ok || std::rename(tmp.c_str(), path) != 0) {
    why = std::string("cannot write cache file ") + path + ": " + errno_text();
    std::remove(tmp.c_str());
    return false;
  }
  return true;
}

}  // namespace ot
