// Internal helpers shared by the library's translation units (host code).
#pragma once

#include <cstdint>
#include <string>

#include "gtsr.h"

namespace gtsr {

// Sets the calling thread's last-error message and returns `code`.
int fail(int code, const std::string& msg);
// Clears the last-error message and returns GTSR_OK.
int ok();

constexpr uint32_t kNone = 0xFFFFFFFFu;
constexpr uint32_t kMaxStripTris = 256;   // T_s limit of one meshlet
constexpr uint32_t kChunkTris = 64;       // strip triangles per flag chunk
constexpr uint32_t kChunkBytes = 16;      // u64 LR + u64 INC

inline uint32_t chunks_of(uint32_t ts) { return (ts + kChunkTris - 1) / kChunkTris; }

}  // namespace gtsr
