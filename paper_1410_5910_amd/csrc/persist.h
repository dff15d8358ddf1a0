// Record I/O of a saved solver (pt_save / pt_load; internal to libpolar).
//
// A record is a 16-byte header (element count, element size, a check word)
// followed by count * elem bytes.  Device arrays are staged through host
// memory in 64 MiB pieces.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cstdio>
#include <vector>

namespace polar {

constexpr uint32_t kRecCheck = 0x52435054u;  // "TPCR"
constexpr size_t kRecChunk = (size_t)64 << 20;

inline bool rec_header(FILE* fp, uint64_t count, uint32_t elem) {
  const uint64_t h[2] = {count, ((uint64_t)kRecCheck << 32) | elem};
  return std::fwrite(h, sizeof(h), 1, fp) == 1;
}

inline bool rec_write_host(FILE* fp, const void* p, uint64_t count, uint32_t elem) {
  if (!rec_header(fp, count, elem)) return false;
  return count == 0 || std::fwrite(p, elem, count, fp) == count;
}

inline bool rec_write_device(FILE* fp, const void* d, uint64_t count, uint32_t elem) {
  if (!rec_header(fp, count, elem)) return false;
  const size_t total = (size_t)count * elem;
  std::vector<char> buf(std::min(total, kRecChunk));
  for (size_t off = 0; off < total; off += buf.size()) {
    const size_t n = std::min(buf.size(), total - off);
    if (hipMemcpy(buf.data(), (const char*)d + off, n, hipMemcpyDeviceToHost) != hipSuccess) return false;
    if (std::fwrite(buf.data(), 1, n, fp) != n) return false;
  }
  return true;
}

// the next record's header; false on a short read or a bad check word
inline bool rec_peek(FILE* fp, uint64_t& count, uint32_t& elem) {
  uint64_t h[2];
  if (std::fread(h, sizeof(h), 1, fp) != 1 || (uint32_t)(h[1] >> 32) != kRecCheck) return false;
  count = h[0];
  elem = (uint32_t)h[1];
  return true;
}

inline bool rec_read_host(FILE* fp, void* p, uint64_t count, uint32_t elem) {
  uint64_t c;
  uint32_t e;
  if (!rec_peek(fp, c, e) || c != count || e != elem) return false;
  return count == 0 || std::fread(p, elem, count, fp) == count;
}

inline bool rec_read_device(FILE* fp, void* d, uint64_t count, uint32_t elem) {
  uint64_t c;
  uint32_t e;
  if (!rec_peek(fp, c, e) || c != count || e != elem) return false;
  const size_t total = (size_t)count * elem;
  std::vector<char> buf(std::min(total, kRecChunk));
  for (size_t off = 0; off < total; off += buf.size()) {
    const size_t n = std::min(buf.size(), total - off);
    if (std::fread(buf.data(), 1, n, fp) != n) return false;
    if (hipMemcpy((char*)d + off, buf.data(), n, hipMemcpyHostToDevice) != hipSuccess) return false;
  }
  return true;
}

}  // namespace polar
