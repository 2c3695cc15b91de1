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
  uint32_t L = 0;                    // levels 1..L at most
};

// Scratch the builder may grow: ensure(buffer_index, bytes) returns the
// device pointer (index 0: jobs, 1: job offsets, 2: flags, 3: per-workgroup
// flags) or nullptr when memory runs out; host_flags(bytes) a pinned host
// buffer.  level_storage(bytes) returns device memory for a batch of closure
// rows that must stay valid while the rows are used, or nullptr to stop
// building (out of memory or over the caller's cap): the levels built so far
// are kept, which is sound because any subset of closure letters preserves
// the equivalence.
// Optional: upload(dev, host, bytes) queues a host-to-device copy of the
// caller's choosing and flags_to_host(dev, bytes) a copy into the
// host_flags buffer, each returning false on failure; when unset, plain
// hipMemcpyAsync copies are queued.
struct ClosureScratch {
  std::function<void*(int, size_t)> ensure;
  std::function<void*(size_t)> host_flags;
  std::function<void*(size_t)> level_storage;
  std::function<bool(void*, const void*, size_t)> upload;
  std::function<bool(const void*, size_t)> flags_to_host;
};

// Builds closure levels (dst[q] = src[src[q]]) for every letter of every
// spec, level by level, one launch per level for all of them.  A letter
// stops at the first level that equals its predecessor or is the identity
// (every later level would equal it, so it cannot split any further block);
// its rows are levels 0..l-1.  Levels are computed in batches of 1, 2, 4, ...
// between host checks of those flags, and storage is requested per batch
// for the letters still open, so letters that stop early cost one level.
// Fills rows[w] with the device addresses of the rows instance w keeps and
// depth[w] with the closure depth reached (L unless storage ran out).
// Returns 0, or a negative DFAMIN_E_* code.
int build_closure_levels(std::vector<ClosureSpec>& specs, const ClosureScratch& scratch,
                         hipStream_t s, std::vector<std::vector<uint64_t>>& rows,
                         std::vector<uint32_t>& depth);

inline uint32_t floor_log2_u32(uint32_t n) {
  uint32_t L = 0;
  while (n >> 1) { n >>= 1; ++L; }
  return L;
}

}  // namespace dfamin
