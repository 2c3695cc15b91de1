// closure.h -- building the partial transitive closure (Section 3.4,
// Algorithm 5) for several instances at once, shared by the batch engine and
// the serving loop.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <functional>
#include <vector>

#include "internal.h"

namespace dfamin {

struct ClosureSpec {
  uint32_t n = 0;
  const uint32_t* delta = nullptr;  // letter-major input rows (device)
  std::vector<uint32_t> letters;     // letters to close (non-identity ones)
  uint32_t L = 0;                    // levels 1..L are built
  uint32_t* storage = nullptr;       // letters.size() * L * n words (device)
};

// Scratch the builder may grow: ensure(buffer_index, bytes) returns the
// device pointer (index 0: jobs, 1: job offsets, 2: flags, 3: per-workgroup
// flags) or nullptr when memory runs out; host_flags(bytes) a pinned host
// buffer.
struct ClosureScratch {
  std::function<void*(int, size_t)> ensure;
  std::function<void*(size_t)> host_flags;
};

// Builds levels 1..L of every letter of every spec with one launch per level
// (dst[q] = src[src[q]]), then fills rows[w] with the device addresses of
// the rows each instance keeps: per letter, levels 0..l-1 where l is the
// first level that equals its predecessor or is the identity (every later
// level would be equal to it, so it cannot split any further block).
// Returns 0, or a negative DFAMIN_E_* code.
int build_closure_levels(std::vector<ClosureSpec>& specs, const ClosureScratch& scratch,
                         hipStream_t s, std::vector<std::vector<uint64_t>>& rows);

inline uint32_t floor_log2_u32(uint32_t n) {
  uint32_t L = 0;
  while (n >> 1) { n >>= 1; ++L; }
  return L;
}

}  // namespace dfamin
