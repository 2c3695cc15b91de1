// kernels.hip -- HIP kernels for gfx950 (CDNA4, wave64) of libdfamin.
//
// One refinement round (the loop body of the paper's Algorithm 4, Section
// 3.3) is four kernels over the active list:
//   k_signature  gather: sig(q) = (block[q], block[delta'(q,a)] for a in
//                Sigma'), a 64-bit hash of it, grouping of equal hashes in
//                LDS and one global hash-table update per local group (hash
//                grouping, the alternative to sorting that the paper
//                attributes to Tewari et al.);
//   k_resolve    every state learns its group's least member (the new block
//                id) and checks its full signature against that member's,
//                so grouping is exact and never trusts a hash alone;
//   k_compact    applies the new ids and compacts the active list with a
//                wave64 ballot/popcount scan and decoupled look-back (the
//                adjacent-difference + inclusive-scan step of Algorithm 4);
//   k_round_end  per-instance round counters.
// The closure of Algorithm 5 (Section 3.4) is k_closure_level, one launch per
// level: T_i[q] = T_{i-1}[T_{i-1}[q]] (pointer jumping).
//
// Cross-workgroup communication inside a kernel happens only through device
// atomics (hash slots, look-back status words); everything else is handed
// from one kernel to the next.  Per-workgroup partial results (flags, minima)
// are written to their own words and reduced by a second kernel, so no
// address is hammered by thousands of workgroups.
#include "internal.h"

#include <algorithm>

namespace dfamin {

namespace {

constexpr unsigned long long kFlagAgg = 1ull << 62;
constexpr unsigned long long kFlagPrefix = 2ull << 62;

__device__ __forceinline__ uint64_t hash_step(uint64_t h, uint32_t w) {
  h ^= w;
  h *= 0x9E3779B97F4A7C15ull;
  h ^= h >> 29;
  return h;
}

__device__ __forceinline__ uint64_t hash_final(uint64_t h) {
  h ^= h >> 32;
  h *= 0xD6E8FEB86659FD93ull;
  h ^= h >> 32;
  return h ? h : 1ull;  // 0 marks an empty LDS slot
}

// Dense block numbers are stored 1, 2 or 4 bytes wide: narrower arrays keep
// more of the random successor gathers in L2 / the memory-side cache.
template <int DW>
__device__ __forceinline__ uint32_t dense_at(const void* __restrict__ d, uint64_t idx) {
  if constexpr (DW == 1) return static_cast<const uint8_t*>(d)[idx];
  else if constexpr (DW == 2) return static_cast<const uint16_t*>(d)[idx];
  else return static_cast<const uint32_t*>(d)[idx];
}

__device__ __forceinline__ unsigned long long load_status(unsigned long long* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void store_status(unsigned long long* p, unsigned long long v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Decoupled look-back by the first wave of the workgroup: publishes this
// tile's aggregate, then reads 64 predecessors at a time and adds their
// aggregates back to the first inclusive prefix; publishes its own inclusive
// prefix and returns the exclusive one (valid in wave 0).  Tiles are numbered
// in the order workgroups obtained them, so every predecessor is running or
// done and the wait ends.
__device__ uint32_t lookback_wave0(unsigned long long* status, uint32_t tile, uint32_t total,
                                   Ctrl* ctrl, uint32_t seg_start = 0) {
  const uint32_t lane = threadIdx.x & 63u;
  if (tile == seg_start) {
    if (lane == 0) store_status(&status[tile], kFlagPrefix | total);
    return 0;
  }
  if (lane == 0) store_status(&status[tile], kFlagAgg | total);
  uint32_t excl = 0;
  int base = (int)tile - 1;
  uint32_t spins = 0;
  while (true) {
    const int t = base - (int)lane;
    // positions before the segment's first tile act as an inclusive prefix of 0
    const unsigned long long v = (t >= (int)seg_start) ? load_status(&status[t]) : kFlagPrefix;
    const uint32_t flag = (uint32_t)(v >> 62);
    const unsigned long long not_ready = __ballot(flag == 0);
    const unsigned long long is_prefix = __ballot(flag == 2);
    const int first_p = is_prefix ? (int)__builtin_ctzll(is_prefix) : 63;
    const unsigned long long need = (first_p >= 63) ? ~0ull : ((2ull << first_p) - 1ull);
    if (not_ready & need) {
      if (++spins > kMaxSpin) {  // a predecessor never published: give up, flag it
        if (lane == 0) atomicOr(&ctrl->fault, 1u);
        break;
      }
      __builtin_amdgcn_s_sleep(1);
      continue;
    }
    excl += wave_sum(((int)lane <= first_p) ? (uint32_t)v : 0u);
    if (is_prefix) break;
    base -= 64;
  }
  if (lane == 0) store_status(&status[tile], kFlagPrefix | (unsigned long long)(excl + total));
  return excl;
}

// Tile scan: a tile holds ITEMS x kBlock items, item e of thread t being
// element e*kBlock + t.  Each thread passes its flags as a bit mask (bit e =
// item e); one 64-lane ballot per item and wave goes to LDS, and wave 0 turns
// the ITEMS*kWaves ballot counts (in element order) into exclusive
// offsets.  Flags, ballots and offsets stay out of registers, so the scan
// kernels keep a high occupancy.  Returns the tile's flag count; tile_rank()
// gives an item's exclusive rank afterwards.
constexpr int kWaves = kBlock / 64;

template <int ITEMS>
struct TileScanLds {
  static constexpr int kWords = ITEMS * kWaves;
  static_assert(ITEMS <= 32, "flags are a 32-bit mask per thread");
  unsigned long long mask[kWords];
  uint32_t off[kWords + 1];
};

template <int ITEMS>
__device__ __forceinline__ uint32_t tile_ballot_count(uint32_t fbits, TileScanLds<ITEMS>& t) {
  constexpr int W = TileScanLds<ITEMS>::kWords;
  constexpr int PER = (W + 63) / 64;  // ballot counts per lane of wave 0
  const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
#pragma unroll
  for (int e = 0; e < ITEMS; ++e) {
    const unsigned long long m = __ballot((fbits >> e) & 1u);
    if (lane == 0) t.mask[e * kWaves + wave] = m;
  }
  __syncthreads();
  if (wave == 0) {
    uint32_t c[PER];
    uint32_t sum = 0;
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int w = (int)lane * PER + i;
      c[i] = (w < W) ? (uint32_t)__popcll(t.mask[w]) : 0u;
      sum += c[i];
    }
    uint32_t v = sum;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const uint32_t u = __shfl_up(v, off, 64);
      if ((int)lane >= off) v += u;
    }
    uint32_t excl = v - sum;
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int w = (int)lane * PER + i;
      if (w < W) t.off[w] = excl;
      excl += c[i];
    }
    if (lane == 63) t.off[W] = v;
  }
  __syncthreads();
  return t.off[W];
}

template <int ITEMS>
__device__ __forceinline__ uint32_t tile_rank(const TileScanLds<ITEMS>& t, int e) {
  const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
  const unsigned long long lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const int w = e * kWaves + (int)wave;
  return t.off[w] + (uint32_t)__popcll(t.mask[w] & lt);
}

// Workgroups are dispatched to the chip's 8 XCDs in turn (workgroup b to
// XCD b mod 8), and each XCD has its own L2.  This bijection of [0, G) gives
// each XCD one contiguous range of logical workgroup ids, so the rows that
// neighbouring tiles gather from (one instance's block ids, one closure row)
// are pulled into one L2 instead of eight.  Any order is correct; only
// locality depends on it.
constexpr uint32_t kXcds = 8;
__device__ __forceinline__ uint32_t xcd_contiguous(uint32_t b, uint32_t G) {
  const uint32_t x = b % kXcds, l = b / kXcds, q = G / kXcds, r = G % kXcds;
  return x < r ? x * (q + 1) + l : r * (q + 1) + (x - r) * q + l;
}

// Workgroup -> job by binary search over the exclusive workgroup prefix.
__device__ __forceinline__ uint32_t find_job(const uint32_t* job_wg_off, uint32_t njobs,
                                             uint32_t* s_job, uint32_t wg) {
  // Largest j with job_wg_off[j] <= wg (offsets strictly increase,
  // job_wg_off[0] = 0).  The first wave searches 64-ary: each step loads 64
  // evenly spaced offsets of [lo, hi) at once and keeps the span after the
  // last one not above wg, so 4,096 jobs take two dependent loads.
  if (threadIdx.x < 64) {
    const uint32_t lane = threadIdx.x;
    uint32_t lo = 0, hi = njobs;
    while (hi - lo > 1) {
      const uint32_t step = (hi - lo + 63) / 64;
      const uint32_t idx = lo + lane * step;
      const bool ok = idx < hi && job_wg_off[idx] <= wg;
      const unsigned long long mask = __ballot(ok);  // a prefix of lanes; lane 0 always
      const uint32_t last = 63u - (uint32_t)__builtin_clzll(mask);
      lo += last * step;
      hi = min(hi, lo + step);
    }
    if (lane == 0) *s_job = lo;
  }
  __syncthreads();
  return *s_job;
}
__device__ __forceinline__ uint32_t find_job(const uint32_t* job_wg_off, uint32_t njobs,
                                             uint32_t* s_job) {
  return find_job(job_wg_off, njobs, s_job, blockIdx.x);
}

// OR of one flag word per thread into a single word per workgroup.
__device__ __forceinline__ uint32_t block_or(uint32_t bits, uint32_t* s_or) {
  if (threadIdx.x == 0) *s_or = 0;
  __syncthreads();
  const uint32_t lane = threadIdx.x & 63u;
  bool b0 = __any(bits & 1u), b1 = __any(bits & 2u), b2 = __any(bits & 4u);
  uint32_t w = (b0 ? 1u : 0u) | (b1 ? 2u : 0u) | (b2 ? 4u : 0u);
  if (lane == 0 && w) atomicOr(s_or, w);
  __syncthreads();
  return *s_or;
}

// ---------------------------------------------------------------- row jobs
// Validation and identity detection.  Algorithmic bytes: 4 per element read.
__global__ __launch_bounds__(kBlock) void k_row_check(const RowJob* __restrict__ jobs,
                                                      const uint32_t* __restrict__ job_wg_off,
                                                      uint32_t njobs, uint32_t* __restrict__ wg_flags) {
  __shared__ uint32_t s_job, s_or;
  const uint32_t j = find_job(job_wg_off, njobs, &s_job);
  const RowJob J = jobs[j];
  const uint32_t* __restrict__ row = reinterpret_cast<const uint32_t*>(J.src);
  const uint32_t base = (blockIdx.x - job_wg_off[j]) * kLongTile;
  uint32_t bits = 0;
  auto check = [&](uint32_t v, uint32_t q) {
    if (v >= J.n) bits |= kFlagBad;
    if (v != q) bits |= kFlagNonId;
  };
  // 16-byte loads over the row from its first 16-byte boundary on: the
  // `lead` (0-3) entries before it are checked one by one by the first
  // workgroup, and each workgroup's tile is shifted by lead (the tiles still
  // cover the row, since kLongTile times the row's workgroups is at least n)
  const uint32_t lead = (uint32_t)(((16u - (J.src & 15u)) & 15u) >> 2);
  if (base == 0 && threadIdx.x < lead && threadIdx.x < J.n) check(row[threadIdx.x], threadIdx.x);
  const uint4* __restrict__ row4 = reinterpret_cast<const uint4*>(row + lead);
#pragma unroll
  for (int e = 0; e < kLongTile / (4 * kBlock); ++e) {
    const uint32_t u = base + 4u * (e * kBlock + threadIdx.x);  // offset after the lead
    const uint32_t q = lead + u;
    if (q + 3u < J.n) {
      const uint4 v = row4[u >> 2];
      check(v.x, q);
      check(v.y, q + 1u);
      check(v.z, q + 2u);
      check(v.w, q + 3u);
    } else {
      for (uint32_t t = 0; t < 4u; ++t)
        if (q + t < J.n) check(row[q + t], q + t);
    }
  }
  const uint32_t w = block_or(bits, &s_or);
  if (threadIdx.x == 0) wg_flags[blockIdx.x] = w;
}

// One closure level for every job: dst[q] = src[src[q]] (Algorithm 5).
// Algorithmic bytes: 12 per element (coalesced read, gathered read, write).
__global__ __launch_bounds__(kBlock) void k_closure_level(const RowJob* __restrict__ jobs,
                                                          const uint32_t* __restrict__ job_wg_off,
                                                          uint32_t njobs,
                                                          uint32_t* __restrict__ wg_flags) {
  __shared__ uint32_t s_job, s_or;
  const uint32_t wg = xcd_contiguous(blockIdx.x, gridDim.x);  // a row's tiles share one L2
  const uint32_t j = find_job(job_wg_off, njobs, &s_job, wg);
  const RowJob J = jobs[j];
  const uint32_t* __restrict__ src = reinterpret_cast<const uint32_t*>(J.src);
  uint32_t* __restrict__ dst = reinterpret_cast<uint32_t*>(J.dst);
  const uint32_t base = (wg - job_wg_off[j]) * kRowTile;
  constexpr int kItems = kRowTile / kBlock;
  uint32_t s1[kItems];
#pragma unroll
  for (int e = 0; e < kItems; ++e) {
    uint32_t q = base + e * kBlock + threadIdx.x;
    s1[e] = (q < J.n) ? src[q] : 0u;
  }
  uint32_t bits = 0;
#pragma unroll
  for (int e = 0; e < kItems; ++e) {
    uint32_t q = base + e * kBlock + threadIdx.x;
    if (q < J.n) {
      uint32_t s2 = src[s1[e]];
      dst[q] = s2;
      if (s2 != s1[e]) bits |= kFlagDiffers;
      if (s2 != q) bits |= kFlagNonId;
    }
  }
  if (wg_flags) {  // the same for the whole grid
    const uint32_t w = block_or(bits, &s_or);
    if (threadIdx.x == 0) wg_flags[wg] = w;
  }
}

// flags[j] = OR of the workgroup flags of job j (one workgroup per job).
__global__ __launch_bounds__(kBlock) void k_flags_reduce(const uint32_t* __restrict__ job_wg_off,
                                                         uint32_t njobs, uint32_t total_wgs,
                                                         const uint32_t* __restrict__ wg_flags,
                                                         uint32_t* __restrict__ flags) {
  __shared__ uint32_t s_or;
  const uint32_t j = blockIdx.x;
  const uint32_t b = job_wg_off[j], e = (j + 1 < njobs) ? job_wg_off[j + 1] : total_wgs;
  uint32_t bits = 0;
  for (uint32_t w = b + threadIdx.x; w < e; w += kBlock) bits |= wg_flags[w];
  const uint32_t r = block_or(bits, &s_or);
  if (threadIdx.x == 0) flags[j] = r;
}

// ---------------------------------------------------------------- init
// Per-workgroup least accepting and least non-accepting state of its chunk
// of one instance (the two initial blocks {F, Q\F} of Algorithm 4 are named
// by their least members).  Partial: (minF << 32) | minN.
__global__ __launch_bounds__(kBlock) void k_init_minmax_part(const InstDesc* __restrict__ desc,
                                                             const uint32_t* __restrict__ job_wg_off,
                                                             uint32_t ninst,
                                                             unsigned long long* __restrict__ part) {
  __shared__ uint32_t s_job, sF, sN;
  const uint32_t i = find_job(job_wg_off, ninst, &s_job);
  const InstDesc D = desc[i];
  const uint8_t* __restrict__ acc = reinterpret_cast<const uint8_t*>(D.accept);
  if (threadIdx.x == 0) { sF = 0xffffffffu; sN = 0xffffffffu; }
  __syncthreads();
  // kRowTile states = kRowTile/8 bytes per workgroup
  const uint32_t b = (blockIdx.x - job_wg_off[i]) * (kRowTile / 8) + threadIdx.x;
  const uint32_t nbytes = (D.n + 7) >> 3;
  uint32_t mf = 0xffffffffu, mn = 0xffffffffu;
  if (threadIdx.x < kRowTile / 8 && b < nbytes) {
    const uint32_t valid = D.n - b * 8;
    const uint32_t vmask = valid >= 8 ? 0xffu : ((1u << valid) - 1u);
    const uint32_t v = acc[b];
    const uint32_t f = v & vmask, nf = ~v & vmask;
    if (f) mf = b * 8 + __builtin_ctz(f);
    if (nf) mn = b * 8 + __builtin_ctz(nf);
  }
  // wave minima, then one LDS atomic per wave
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    mf = min(mf, (uint32_t)__shfl_xor(mf, off, 64));
    mn = min(mn, (uint32_t)__shfl_xor(mn, off, 64));
  }
  if ((threadIdx.x & 63u) == 0) {
    atomicMin(&sF, mf);
    atomicMin(&sN, mn);
  }
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = ((unsigned long long)sF << 32) | sN;
}

__global__ __launch_bounds__(kBlock) void k_init_minmax_reduce(const uint32_t* __restrict__ job_wg_off,
                                                               uint32_t ninst, uint32_t total_wgs,
                                                               const unsigned long long* __restrict__ part,
                                                               uint32_t* __restrict__ minF,
                                                               uint32_t* __restrict__ minN) {
  __shared__ uint32_t sF, sN;
  const uint32_t i = blockIdx.x;
  const uint32_t b = job_wg_off[i], e = (i + 1 < ninst) ? job_wg_off[i + 1] : total_wgs;
  if (threadIdx.x == 0) { sF = 0xffffffffu; sN = 0xffffffffu; }
  __syncthreads();
  uint32_t mf = 0xffffffffu, mn = 0xffffffffu;
  for (uint32_t w = b + threadIdx.x; w < e; w += kBlock) {
    const unsigned long long v = part[w];
    mf = min(mf, (uint32_t)(v >> 32));
    mn = min(mn, (uint32_t)v);
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    mf = min(mf, (uint32_t)__shfl_xor(mf, off, 64));
    mn = min(mn, (uint32_t)__shfl_xor(mn, off, 64));
  }
  if ((threadIdx.x & 63u) == 0) {
    atomicMin(&sF, mf);
    atomicMin(&sN, mn);
  }
  __syncthreads();
  if (threadIdx.x == 0) { minF[i] = sF; minN[i] = sN; }
}

// block[g] = least member of g's initial block; act = all states.
// Algorithmic bytes: 8.125 per state (bit read, block + act writes; +4 with inst_of).
__global__ __launch_bounds__(kBlock) void k_init_block(const InstDesc* __restrict__ desc,
                                                       const uint32_t* __restrict__ job_wg_off,
                                                       uint32_t ninst,
                                                       const uint32_t* __restrict__ minF,
                                                       const uint32_t* __restrict__ minN,
                                                       uint32_t* __restrict__ inst_of,
                                                       uint32_t* __restrict__ block,
                                                       uint32_t* __restrict__ act) {
  __shared__ uint32_t s_job;
  const uint32_t i = find_job(job_wg_off, ninst, &s_job);
  const InstDesc D = desc[i];
  const uint8_t* __restrict__ acc = reinterpret_cast<const uint8_t*>(D.accept);
  const uint32_t base = (blockIdx.x - job_wg_off[i]) * kRowTile;
  const uint32_t f = D.state_off + minF[i], nf = D.state_off + minN[i];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    uint32_t q = base + e * kBlock + threadIdx.x;
    if (q < D.n) {
      uint32_t g = D.state_off + q;
      bool a = (acc[q >> 3] >> (q & 7)) & 1u;
      block[g] = a ? f : nf;
      act[g] = g;
      if (inst_of) inst_of[g] = i;
    }
  }
}

// ---------------------------------------------------------------- round
// Algorithmic bytes: 8 per slot.
__global__ __launch_bounds__(kBlock) void k_clear_table(Slot* __restrict__ table, uint64_t tsize,
                                                        Ctrl* __restrict__ ctrl, uint32_t gmode,
                                                        uint32_t* __restrict__ gcount) {
  if (gmode && ctrl->stop) return;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ctrl->any_changed = 0u;
    ctrl->collision = 0u;
  }
  if (gcount && blockIdx.x == 0 && threadIdx.x < 2 * kGroupCounters) gcount[threadIdx.x] = 0u;
  const uint64_t stride = (uint64_t)gridDim.x * kBlock * 2;
  for (uint64_t s = ((uint64_t)blockIdx.x * kBlock + threadIdx.x) * 2; s < tsize; s += stride) {
    table[s] = 0ull;
    if (s + 1 < tsize) table[s + 1] = 0ull;
  }
}

// Insert a local group (least member g, a global state id, `shared` if it
// already has two members) into the global table; returns the slot.  The
// home slot is read first (a join that changes nothing then costs no
// atomic), or, with cas_first, claimed by a CAS straight away (a new group
// then costs one atomic and no read).  A slot
// belongs to one instance: its least member lies in [lo, hi), the inserting
// instance's state range, or the slot holds another instance's key and the
// probe moves on.  So exact keys (the same small numbers in every instance)
// never merge across instances.  The plain load is a shortcut only: a stale
// value just leads to a CAS that returns the current one, and slot words
// change monotonically (claimed once, index only lowered within the same
// instance, shared bit only set).
//
// `created` tells the caller that this call claimed an empty slot,
// `first_join` that it made a slot shared that was not.  The first state to
// join a slot that was not yet shared marks its claimer in `notify`
// (nullable; one byte per global state id): a claimer left unmarked is then
// known to be alone in its group without reading the slot.
__device__ __forceinline__ uint32_t table_insert(Slot* __restrict__ table, uint64_t mask, uint64_t h,
                                                 uint32_t frag, uint32_t g, bool shared, uint32_t lo,
                                                 uint32_t hi, bool cas_first, Ctrl* __restrict__ ctrl,
                                                 uint8_t* __restrict__ notify, bool& created,
                                                 bool& first_join) {
  uint64_t p = h & mask;
  created = false;
  first_join = false;
  const unsigned long long mine =
      ((unsigned long long)frag << 32) | (shared ? kSlotShared : 0u) | (unsigned long long)g;
  for (uint64_t probes = 0; probes <= mask; ++probes) {
    unsigned long long cur;
    if (cas_first) {
      cur = atomicCAS(&table[p], 0ull, mine);
      if (cur == 0ull) {
        created = true;
        return (uint32_t)p;
      }
    } else {
      cur = table[p];
    }
    while (true) {
      if (cur == 0ull) {
        const unsigned long long prev = atomicCAS(&table[p], 0ull, mine);
        if (prev == 0ull) {
          created = true;
          return (uint32_t)p;
        }
        cur = prev;
        continue;
      }
      const uint32_t cw = (uint32_t)cur;
      const uint32_t cg = cw & kSlotIndexMask;
      if ((uint32_t)(cur >> 32) != frag || cg < lo || cg >= hi) break;  // another key: next slot
      const uint32_t want_lo = min(cg, g) | kSlotShared;
      if (want_lo == cw) return (uint32_t)p;
      const unsigned long long want = (cur & 0xffffffff00000000ull) | want_lo;
      const unsigned long long prev = atomicCAS(&table[p], cur, want);
      if (prev == cur) {
        // the first joiner: the slot's least member so far is its claimer
        if (!(cw & kSlotShared)) {
          first_join = true;
          if (notify) notify[cg] = 1;
        }
        return (uint32_t)p;
      }
      cur = prev;  // re-examined from the top: empty, other key or same key
    }
    p = (p + 1) & mask;
  }
  atomicOr(&ctrl->fault, 1u);  // a table at most half full has a free slot
  return (uint32_t)(h & mask);
}

// Signature gather + grouping.  Hash mode: algorithmic bytes per active
// state 4 (act) [+4 inst_of] + 4 (own block) + 8*kp (delta' row entry and
// the gathered successor block per letter) + 4*(kp+1) (signature record) + 4
// (slot id) + 8 (one hash-slot update per local group, upper bound).  Exact
// mode: the same without the record, with dense numbers (or accept bits)
// gathered instead of block ids.
template <bool BATCH, int DW, int SI>
__global__ __launch_bounds__(kBlock) void k_signature(
    const uint32_t* __restrict__ act, uint32_t m, const uint32_t* __restrict__ inst_of,
    const InstDesc* __restrict__ desc, const uint64_t* __restrict__ rows,
    const uint32_t* __restrict__ block, const void* __restrict__ dense,
    Slot* __restrict__ table, uint32_t tbits, uint32_t* __restrict__ slot_of, uint64_t salt,
    Ctrl* __restrict__ ctrl, uint32_t gmode, uint8_t* __restrict__ notify, uint32_t* __restrict__ gcount,
    uint32_t* __restrict__ dtab) {
  if (gmode & 1u) {  // a queued round: live count and salt from the control block
    if (ctrl->stop) return;
    m = ctrl->m_cur;
    salt = ctrl->salt;
  }
  // SI states per thread; an LDS table of twice the tile's states
  constexpr uint32_t kTile = kBlock * SI, kSlots = 2 * kTile;
  __shared__ unsigned long long lkey[kSlots];
  __shared__ uint32_t lmin[kSlots], lcnt[kSlots], lslot[kSlots];
  __shared__ uint32_t s_formed, s_shared;  // slots claimed / made shared by this workgroup
  for (uint32_t s = threadIdx.x; s < kSlots; s += kBlock) {
    lkey[s] = 0ull;
    lmin[s] = 0xffffffffu;
    lcnt[s] = 0u;
  }
  if (threadIdx.x == 0) {
    s_formed = 0u;
    s_shared = 0u;
  }
  __syncthreads();
  uint64_t h[SI];
  uint32_t frag[SI], lp[SI], jj[SI], gg[SI], glo[SI], ghi[SI];
  bool valid[SI], cfirst[SI];
  // batched: neighbouring tiles (mostly one instance's states) on one XCD
  // (one instance gathers from its whole block array: no locality to keep)
  const uint32_t wg = BATCH ? xcd_contiguous(blockIdx.x, gridDim.x) : blockIdx.x;
#pragma unroll
  for (int e = 0; e < SI; ++e) {
    const uint32_t j = wg * kTile + e * kBlock + threadIdx.x;
    jj[e] = j;
    gg[e] = 0;
    glo[e] = 0;
    ghi[e] = 0;
    valid[e] = j < m;
    h[e] = 0;
    frag[e] = 0;
    lp[e] = 0;
    cfirst[e] = false;
    if (!valid[e]) continue;
    const uint32_t g = act[j];
    gg[e] = g;
    const uint32_t i = BATCH ? inst_of[g] : 0u;
    const InstDesc D = desc[i];
    const uint32_t q = g - D.state_off;
    glo[e] = D.state_off;
    ghi[e] = D.state_off + D.n;
    const uint32_t kp = D.kp;
    const uint64_t* __restrict__ R = rows + D.rows_off;
    cfirst[e] = (gmode & (D.ebits ? 4u : 2u)) != 0u;
    unsigned long long lk;  // local grouping key (exact key + 1, or the hash)
    if (D.ebits) {
      // exact key: own dense number, then one per letter, ebits each
      const uint8_t* __restrict__ acc = reinterpret_cast<const uint8_t*>(D.accept);
      uint32_t key = D.dsrc ? ((acc[q >> 3] >> (q & 7)) & 1u) : dense_at<DW>(dense, g);
      uint32_t shift = D.ebits;
      for (uint32_t r0 = 0; r0 < kp; r0 += 8) {
        const uint32_t cnt = (kp - r0) < 8u ? (kp - r0) : 8u;
        uint32_t s[8], b[8];
#pragma unroll
        for (uint32_t t = 0; t < 8; ++t)
          if (t < cnt) s[t] = reinterpret_cast<const uint32_t*>(R[r0 + t])[q];
#pragma unroll
        for (uint32_t t = 0; t < 8; ++t)
          if (t < cnt)
            b[t] = D.dsrc ? ((acc[s[t] >> 3] >> (s[t] & 7)) & 1u)
                          : dense_at<DW>(dense, (uint64_t)D.state_off + s[t]);
#pragma unroll
        for (uint32_t t = 0; t < 8; ++t)
          if (t < cnt) {
            key |= b[t] << shift;
            shift += D.ebits;
          }
      }
      // Keys are numbers within one instance: the instance joins the local
      // key and the home position, and a global slot is only joined by
      // states of the instance that claimed it (table_insert).
      frag[e] = key + 1u;  // < 2^31 + 1, never 0
      h[e] = hash_final(hash_step(hash_step(salt ^ 0x13198A2E03707344ull, key), i));
      lk = ((unsigned long long)i << 32) | frag[e];
    } else {
      uint32_t* __restrict__ rec = reinterpret_cast<uint32_t*>(D.sig) + (uint64_t)q * (kp + 1);
      const uint32_t own = block[g];
      rec[0] = own;
      uint64_t hh = hash_step(salt ^ 0x243F6A8885A308D3ull, own);
      for (uint32_t r0 = 0; r0 < kp; r0 += 8) {
        const uint32_t cnt = (kp - r0) < 8u ? (kp - r0) : 8u;
        uint32_t s[8], b[8];
#pragma unroll
        for (uint32_t t = 0; t < 8; ++t)
          if (t < cnt) s[t] = reinterpret_cast<const uint32_t*>(R[r0 + t])[q];
#pragma unroll
        for (uint32_t t = 0; t < 8; ++t)
          if (t < cnt) b[t] = block[D.state_off + s[t]];
#pragma unroll
        for (uint32_t t = 0; t < 8; ++t)
          if (t < cnt) {
            rec[1 + r0 + t] = b[t];
            hh = hash_step(hh, b[t]);
          }
      }
      hh = hash_final(hh);
      // testing: a hash with only a few bits of entropy (spread again), so
      // that different signatures share hashes and the rounds are redone
      if (const uint64_t hm = ctrl->hash_mask) hh = hash_final(hh & hm);
      h[e] = hh;
      frag[e] = (uint32_t)(hh >> 32) | 1u;
      lk = hh | (1ull << 63);  // hash keys and exact keys (< 2^32) never meet
    }
    uint32_t p = (uint32_t)h[e] & (kSlots - 1);
    while (true) {
      const unsigned long long prev = atomicCAS(&lkey[p], 0ull, lk);
      if (prev == 0ull || prev == lk) break;
      p = (p + 1) & (kSlots - 1);
    }
    lp[e] = p;
    atomicMin(&lmin[p], g);
    atomicAdd(&lcnt[p], 1u);
  }
  __syncthreads();
  const uint64_t mask = (1ull << tbits) - 1ull;
  // slot ids below 2^31: bit 31 of slot_of marks a state that claimed its
  // slot alone (no other state of its tile in its group)
  uint8_t* const nt = tbits <= 31u ? notify : nullptr;
#pragma unroll
  for (int e = 0; e < SI; ++e) {
    if (valid[e] && lmin[lp[e]] == gg[e]) {
      bool created = false, first_join = false;
      const bool alone = lcnt[lp[e]] == 1u;
      uint32_t p;
      if (dtab) {
        // direct count table: the exact key is the word's index
        p = frag[e] - 1u;
        const uint32_t old = atomicAdd(&dtab[p], lcnt[lp[e]]);
        created = old == 0u;
        first_join = old == 1u;
        lslot[lp[e]] = p | ((created && alone) ? kSlotClaimedAlone : 0u);
      } else {
        p = table_insert(table, mask, h[e], frag[e], gg[e], !alone, glo[e], ghi[e], cfirst[e], ctrl, nt,
                         created, first_join);
        lslot[lp[e]] = p | ((nt && created && alone) ? kSlotClaimedAlone : 0u);
      }
      if (gcount) {
        if (created) atomicAdd(&s_formed, 1u);
        if ((created && !alone) || first_join) atomicAdd(&s_shared, 1u);
      }
    }
  }
  __syncthreads();
  if (gcount && threadIdx.x == 0) {
    const uint32_t w = blockIdx.x % kGroupCounters;
    if (s_formed) atomicAdd(&gcount[w], s_formed);
    if (s_shared) atomicAdd(&gcount[kGroupCounters + w], s_shared);
  }
#pragma unroll
  for (int e = 0; e < SI; ++e)
    if (valid[e]) slot_of[jj[e]] = lslot[lp[e]];
}

// New block id = least member of the state's hash group; exact check of the
// full signature against that member's.  Algorithmic bytes per active state:
// 4 (act) [+4 inst_of] + 4 (slot id) + 8 (slot) + 4 (old block) + 4 (new
// id) + 1 (keep flag), plus 4 + 8*(kp+1) when the state is not the least
// member of its group (its record and the least member's).
template <bool BATCH>
__global__ __launch_bounds__(kBlock) void k_resolve(
    const uint32_t* __restrict__ act, uint32_t m, const uint32_t* __restrict__ inst_of,
    const InstDesc* __restrict__ desc,
    const Slot* __restrict__ table, const uint32_t* __restrict__ slot_of,
    const uint32_t* __restrict__ block, uint32_t* __restrict__ nb, uint8_t* __restrict__ keep,
    uint32_t* __restrict__ changed_inst, Ctrl* __restrict__ ctrl,
    unsigned long long* __restrict__ scan_status, uint32_t ntiles, uint32_t gmode,
    uint8_t* __restrict__ notify, const uint32_t* __restrict__ count_gcount) {
  if (gmode) {
    if (ctrl->stop) return;
    m = ctrl->m_cur;
  }
  const uint32_t j = blockIdx.x * kBlock + threadIdx.x;
  if (j < ntiles) store_status(&scan_status[j], 0ull);
  if (j == 0) atomicExch(&ctrl->tile_counter, 0u);
  if (count_gcount && j < 64) {
    // split iff more groups than the shared groups the labels stand for
    const uint32_t formed = wave_sum(count_gcount[j]);
    if (j == 0 && formed > ctrl->prev_shared) changed_inst[0] = 1u;
  }
  bool changed = false, coll = false;
  uint32_t i = 0xffffffffu;
  if (j < m) {
    const uint32_t g = act[j];
    i = BATCH ? inst_of[g] : 0u;
    const uint32_t so = slot_of[j];
    uint32_t w;
    if (notify && (so & kSlotClaimedAlone)) {
      // claimed its slot alone: still alone unless a joiner marked it
      if (notify[g]) {
        notify[g] = 0;
        w = (uint32_t)table[so & ~kSlotClaimedAlone];
      } else {
        w = g;  // its own group, not shared
      }
    } else {
      w = (uint32_t)table[so];
    }
    const uint32_t gc = w & kSlotIndexMask;  // least member of the group
    const uint32_t rep = gc;
    if (gc != g) {
      const InstDesc D = desc[i];
      const uint32_t words = D.kp + 1;
      if (gc < D.state_off || gc - D.state_off >= D.n) {
        coll = true;  // the group's least member belongs to another instance
      } else if (!D.ebits) {  // exact keys need no check
        const uint32_t* __restrict__ sg = reinterpret_cast<const uint32_t*>(D.sig);
        const uint32_t* __restrict__ r1 = sg + (uint64_t)(g - D.state_off) * words;
        const uint32_t* __restrict__ r2 = sg + (uint64_t)(gc - D.state_off) * words;
        for (uint32_t t = 0; t < words; ++t) coll |= (r1[t] != r2[t]);
      }
    }
    changed = !count_gcount && rep != block[g];
    nb[j] = rep;
    keep[j] = (w & kSlotShared) ? 1 : 0;
  }
  // Flags only ever go from 0 to 1 inside this kernel: plain stores of the
  // same value, made visible to the next kernel by the kernel boundary.  A
  // wave stores each instance's flag once (its states are contiguous in the
  // active list), so no word takes more than a few stores per wave.
  const uint32_t lane = threadIdx.x & 63u;
  const unsigned long long cm = __ballot(changed);
  const int first = cm ? __builtin_ctzll(cm) : 0;
  const uint32_t i0 = __shfl(i, first, 64);
  if (changed && ((int)lane == first || i != i0)) changed_inst[i] = 1u;
  if (__any(coll) && lane == 0) ctrl->collision = 1u;
}

// Apply the new ids and keep the states whose block is still shared and whose
// instance split this round.  Algorithmic bytes per active state: 4 (act)
// [+4 inst_of] + 4 (new id) + 1 (keep) + 4 (block write) + 4 per kept state
// (next active list).
template <bool BATCH, int ITEMS>
__global__ __launch_bounds__(kBlock) void k_compact(
    const uint32_t* __restrict__ act, uint32_t m, const uint32_t* __restrict__ inst_of,
    const uint32_t* __restrict__ nb, const uint8_t* __restrict__ keep,
    uint32_t* __restrict__ changed_inst, const uint32_t* __restrict__ dead,
    uint32_t* __restrict__ block, uint32_t* __restrict__ act_next, Ctrl* __restrict__ ctrl,
    unsigned long long* __restrict__ scan_status, uint32_t gmode,
    const uint32_t* __restrict__ slot_of, uint8_t* __restrict__ notify,
    const uint32_t* __restrict__ gcount, uint32_t prev_count, const uint32_t* __restrict__ dtab) {
  if (gmode) {  // every workgroup reads the same flag: all of them leave, or none
    if (ctrl->stop) return;
    m = ctrl->m_cur;
  }
  // On a hash collision the round is redone with another salt: nothing is
  // written (in a queued round the active list is carried over unchanged),
  // but every tile still takes part in the look-back so that no workgroup
  // can wait for one that left early.
  __shared__ uint32_t s_tile, s_prefix, s_coll, s_split;
  __shared__ TileScanLds<ITEMS> s_scan;
  if (threadIdx.x == 0) {
    s_tile = atomicAdd(&ctrl->tile_counter, 1u);
    s_coll = ctrl->collision;
  }
  if (slot_of && threadIdx.x < 64) {
    // slot labels: the round split iff it formed more groups than before
    const uint32_t formed = wave_sum(gcount[threadIdx.x]);
    const uint32_t shared = wave_sum(gcount[kGroupCounters + threadIdx.x]);
    // A count table tells a lone claimer from a shared one only by a random
    // read of its word.  Where groups of one state are rare, every state
    // stays instead (a group of one stays a group of one, under a label):
    // the groups kept are then all groups formed.
    const bool keep_all = dtab && (formed - shared) * 64ull <= m;
    if (threadIdx.x == 0) {
      s_split = (formed > prev_count ? 1u : 0u) | (keep_all ? 2u : 0u);
      if (blockIdx.x == 0 && formed > prev_count) {
        changed_inst[0] = 1u;
        ctrl->prev_shared = keep_all ? formed : shared;
      }
    }
  }
  __syncthreads();
  const uint32_t tile = s_tile;
  const bool coll = s_coll != 0;
  const uint32_t base = tile * (kBlock * ITEMS);
  uint32_t fb = 0;
  if (slot_of && (s_split & 3u) == 3u) {
    // every state stays, under its label: the list is left as it is (the
    // caller keeps using it) and only the labels are written
#pragma unroll 8
    for (int e = 0; e < ITEMS; ++e) {
      const uint32_t j = base + e * kBlock + threadIdx.x;
      if (j < m) {
        const uint32_t g = act[j];
        block[g] = kSlotLabel | (slot_of[j] & ~kSlotClaimedAlone);
      }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicExch(&ctrl->m_next, m);
    return;
  }
  if (slot_of) {
    // one instance, exact keys (no collision): ids change only if it split
    if (s_split & 1u) {
      const bool keep_all = (s_split & 2u) != 0;
#pragma unroll 8
      for (int e = 0; e < ITEMS; ++e) {
        const uint32_t j = base + e * kBlock + threadIdx.x;
        if (j < m) {
          const uint32_t g = act[j];
          const uint32_t so = slot_of[j];
          bool shared = keep_all || !(so & kSlotClaimedAlone);
          if (!shared) {
            if (dtab) {
              shared = dtab[so & ~kSlotClaimedAlone] >= 2u;  // a count table: its word
            } else if (notify[g]) {
              notify[g] = 0;
              shared = true;
            }
          }
          block[g] = shared ? (kSlotLabel | (so & ~kSlotClaimedAlone)) : g;
          if (shared) fb |= 1u << e;
        }
      }
    }
  } else {
#pragma unroll 8
    for (int e = 0; e < ITEMS; ++e) {
      const uint32_t j = base + e * kBlock + threadIdx.x;
      // a queued round that collided is redone from the next buffer: same list
      if (gmode && coll && j < m) act_next[j] = act[j];
      if (j < m && !coll) {
        const uint32_t g = act[j];
        block[g] = nb[j];
        const uint32_t i = BATCH ? inst_of[g] : 0u;
        if (keep[j] && changed_inst[i] && !(dead && dead[i])) fb |= 1u << e;
      }
    }
  }
  const uint32_t total = tile_ballot_count<ITEMS>(fb, s_scan);
  if (threadIdx.x < 64) {
    const uint32_t excl = lookback_wave0(scan_status, tile, total, ctrl);
    if (threadIdx.x == 0) {
      s_prefix = excl;
      if (base + kBlock * ITEMS >= m && tile < gridDim.x) atomicExch(&ctrl->m_next, excl + total);
    }
  }
  __syncthreads();
  const uint32_t pre = s_prefix;
  // kept states are re-read from act (the tile was just read: cache hits)
  for (int e = 0; e < ITEMS; ++e)
    if ((fb >> e) & 1u) act_next[pre + tile_rank<ITEMS>(s_scan, e)] = act[base + e * kBlock + threadIdx.x];
}

// Per-instance round counters; optionally also clears clear_tiles scan
// status words and the tile counter for a look-back scan queued next.
__global__ __launch_bounds__(kBlock) void k_round_end(uint32_t ninst,
                                                      uint32_t* __restrict__ changed_inst,
                                                      uint32_t* __restrict__ refine_cnt,
                                                      uint32_t* __restrict__ last,
                                                      Ctrl* __restrict__ ctrl,
                                                      unsigned long long* __restrict__ clear_status,
                                                      uint32_t clear_tiles, uint32_t gmode) {
  if (gmode && ctrl->stop) return;
  const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
  if (clear_status) {
    if (i < clear_tiles) store_status(&clear_status[i], 0ull);
    if (i == 0) atomicExch(&ctrl->tile_counter, 0u);
  }
  const uint32_t ch = (i < ninst) ? changed_inst[i] : 0u;
  if (__any(ch != 0u) && (threadIdx.x & 63u) == 0) ctrl->any_changed = 1u;
  if (i >= ninst) return;
  const uint32_t coll = ctrl->collision;
  if (last) last[i] = coll ? 0u : ch;
  if (ch) {
    if (!coll) refine_cnt[i] += 1u;
    changed_inst[i] = 0u;
  }
}

// Queued signature rounds: see launch_queue_start / launch_round_step.
__global__ void k_queue_start(Ctrl* __restrict__ ctrl, uint32_t m, uint64_t salt) {
  if (threadIdx.x != 0) return;
  ctrl->stop = 0u;
  ctrl->iterations = 0u;
  ctrl->retries = 0u;
  ctrl->m_cur = m;
  ctrl->salt = salt;
}

__global__ void k_store_u64(uint64_t* __restrict__ p, uint64_t v) {
  if (threadIdx.x == 0) *p = v;
}

// Stream-ordered copy of `units` elements (see launch_copy_bytes).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_copy_units(T* __restrict__ dst, const T* __restrict__ src,
                                                       uint64_t units) {
  const uint64_t stride = (uint64_t)gridDim.x * kBlock;
  for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < units; i += stride) dst[i] = src[i];
  __threadfence_system();
}

// Up to kMemSegs copies (src set) and byte fills (src null) in one launch:
// every workgroup strides over every segment, 16 bytes at a time where the
// segment allows it.
__global__ __launch_bounds__(kBlock) void k_mem_segs(MemSegs q) {
  const uint64_t t0 = (uint64_t)blockIdx.x * kBlock + threadIdx.x, stride = (uint64_t)gridDim.x * kBlock;
  for (uint32_t k = 0; k < q.n; ++k) {
    const MemSeg g = q.seg[k];
    uint8_t* d = static_cast<uint8_t*>(g.dst);
    const uint8_t* sp = static_cast<const uint8_t*>(g.src);
    const bool wide = ((reinterpret_cast<uintptr_t>(d) | reinterpret_cast<uintptr_t>(sp)) & 15u) == 0;
    const uint64_t body = wide ? (g.bytes & ~uint64_t(15)) : 0;
    const uint32_t f = g.fill * 0x01010101u;
    for (uint64_t u = t0; u < body / 16; u += stride)
      reinterpret_cast<uint4*>(d)[u] = sp ? reinterpret_cast<const uint4*>(sp)[u] : make_uint4(f, f, f, f);
    for (uint64_t b = body + t0; b < g.bytes; b += stride) d[b] = sp ? sp[b] : (uint8_t)g.fill;
  }
}

__global__ __launch_bounds__(kBlock) void k_queue_plan(QueueDbl q, InstDesc* __restrict__ desc,
                                                       const Ctrl* __restrict__ ctrl) {
  const uint32_t t = blockIdx.x * kBlock + threadIdx.x;
  if (t >= q.count || ctrl->stop) return;
  const uint32_t i = q.list[t];
  uint32_t lvl = 0;
  for (uint64_t x = q.mj[t] + 1; x >> 1; x >>= 1) ++lvl;  // floor(log2(j+1))
  if (lvl > q.lmax[t]) lvl = q.lmax[t];
  desc[i].rows_off = q.rbase[t] + lvl;
  q.need[t] = lvl > q.built[t] ? lvl : 0u;
  if (lvl > q.built[t]) q.built[t] = lvl;
  q.lv[t] = lvl;
}

__global__ __launch_bounds__(kBlock) void k_queue_levels(QueueDbl q, const uint64_t* __restrict__ rows,
                                                         const Ctrl* __restrict__ ctrl) {
  __shared__ uint32_t s_job;
  if (ctrl->stop) return;
  const uint32_t wg = xcd_contiguous(blockIdx.x, gridDim.x);
  const uint32_t t = find_job(q.wgoff, q.count, &s_job, wg);
  const uint32_t lvl = q.need[t];
  if (!lvl) return;
  const uint32_t* __restrict__ src = reinterpret_cast<const uint32_t*>(rows[q.rbase[t] + lvl - 1]);
  uint32_t* __restrict__ dst = reinterpret_cast<uint32_t*>(rows[q.rbase[t] + lvl]);
  const uint32_t n = q.n[t];
  const uint32_t base = (wg - q.wgoff[t]) * kRowTile;
#pragma unroll
  for (int e = 0; e < kRowTile / kBlock; ++e) {
    const uint32_t x = base + e * kBlock + threadIdx.x;
    if (x < n) dst[x] = src[src[x]];
  }
}

__global__ __launch_bounds__(kBlock) void k_queue_advance(QueueDbl q, const Ctrl* __restrict__ ctrl) {
  const uint32_t t = blockIdx.x * kBlock + threadIdx.x;
  if (t >= q.count || ctrl->stop || ctrl->collision) return;
  q.mj[t] += 1ull << q.lv[t];
  if (q.last[q.list[t]] && q.lv[t] > q.used[t]) q.used[t] = q.lv[t];  // the highest level a splitting round read
}

__global__ void k_round_step(Ctrl* __restrict__ ctrl) {
  if (threadIdx.x != 0 || ctrl->stop) return;
  if (ctrl->collision) {  // redo the round with another salt
    ctrl->salt = hash_final(ctrl->salt + 0x9E3779B97F4A7C15ull);
    if (++ctrl->retries > kMaxSaltRetries) {
      ctrl->fault = 1u;
      ctrl->stop = 1u;
    }
    return;
  }
  ctrl->iterations += 1u;
  ctrl->retries = 0u;  // the bound is on redoing one round
  ctrl->m_cur = ctrl->m_next;
  if (!ctrl->any_changed || ctrl->m_next == 0u) ctrl->stop = 1u;
}

// ------------------------------------------------ leader-based refinement
// Algorithm 2 (Section 3.2).  A state q whose block leader L = block[q]
// reaches a different block under some letter differs from L; the least
// such state of L's block becomes new_leader[L] (the paper elects by a
// concurrent write; the least candidate keeps leaders the least members of
// their blocks).  Algorithmic bytes per state: 4 (block) + 8k' (delta'
// entries of q and L) + 8k' (their successors' blocks) + 1 (flag), in the
// worst case of no early exit.
template <bool BATCH>
__global__ __launch_bounds__(kBlock) void k_naive_elect(uint32_t N, const uint32_t* __restrict__ inst_of,
                                                        const InstDesc* __restrict__ desc,
                                                        const uint64_t* __restrict__ rows,
                                                        const uint32_t* __restrict__ block,
                                                        uint32_t* __restrict__ new_leader,
                                                        uint8_t* __restrict__ differs,
                                                        const Ctrl* __restrict__ ctrl) {
  if (ctrl->stop) return;
  const uint32_t g = blockIdx.x * kBlock + threadIdx.x;
  if (g >= N) return;
  const uint32_t L = block[g];
  uint8_t d = 0;
  if (L != g) {
    const uint32_t i = BATCH ? inst_of[g] : 0u;
    const InstDesc D = desc[i];
    const uint64_t* __restrict__ R = rows + D.rows_off;
    const uint32_t q = g - D.state_off, l = L - D.state_off;
    for (uint32_t r = 0; r < D.kp && !d; ++r) {
      const uint32_t* __restrict__ row = reinterpret_cast<const uint32_t*>(R[r]);
      if (block[D.state_off + row[q]] != block[D.state_off + row[l]]) d = 1;
    }
  }
  differs[g] = d;
  if (d) atomicMin(&new_leader[L], g);
}

// Differing states join their new leader's block.  Each thread reads and
// writes only its own block entry, so the update is in place.  Resets the
// other round's election array.  Algorithmic bytes per state: 1 + 4 + 4
// (flag, block, next_leader reset) + 8 for a moving state.
template <bool BATCH>
__global__ __launch_bounds__(kBlock) void k_naive_move(uint32_t N, const uint32_t* __restrict__ inst_of,
                                                       uint32_t* __restrict__ block,
                                                       const uint32_t* __restrict__ new_leader,
                                                       uint32_t* __restrict__ next_leader,
                                                       const uint8_t* __restrict__ differs,
                                                       uint32_t* __restrict__ changed_inst,
                                                       const Ctrl* __restrict__ ctrl) {
  if (ctrl->stop) return;
  const uint32_t g = blockIdx.x * kBlock + threadIdx.x;
  bool moved = false;
  uint32_t i = 0xffffffffu;
  if (g < N) {
    next_leader[g] = 0xffffffffu;
    if (differs[g]) {
      block[g] = new_leader[block[g]];
      moved = true;
      i = BATCH ? inst_of[g] : 0u;
    }
  }
  const uint32_t lane = threadIdx.x & 63u;
  const unsigned long long cm = __ballot(moved);
  const int first = cm ? __builtin_ctzll(cm) : 0;
  const uint32_t i0 = __shfl(i, first, 64);
  if (moved && ((int)lane == first || i != i0)) changed_inst[i] = 1u;
}

__global__ void k_naive_check(Ctrl* __restrict__ ctrl) {
  if (threadIdx.x != 0 || ctrl->stop) return;
  ctrl->iterations += 1u;
  if (ctrl->any_changed) ctrl->any_changed = 0u;
  else ctrl->stop = 1u;
}

// ------------------------------------------- reachability and the quotient
// One breadth-first level from q0 (Section 2: the minimal DFA keeps the
// classes of reachable states): every frontier state follows each row; a
// successor whose visited bit this thread sets first joins the next
// frontier.  New states are staged in LDS and appended with one global
// atomicAdd per workgroup and chunk of rows.  Algorithmic bytes per
// frontier state: 4 + per row 4 (entry) + 4 (visited word) + 4 (append).
constexpr uint32_t kBfsRowChunk = 8;
__global__ __launch_bounds__(kBlock) void k_bfs_level(const uint64_t* __restrict__ rows, uint32_t nrows,
                                                      const uint32_t* __restrict__ frontier,
                                                      uint32_t fcount, uint32_t* __restrict__ visited,
                                                      uint32_t* __restrict__ next,
                                                      uint32_t* __restrict__ next_count) {
  __shared__ uint32_t s_new[kBlock * kBfsRowChunk];
  __shared__ uint32_t s_cnt, s_base;
  const uint32_t j = blockIdx.x * kBlock + threadIdx.x;
  const bool valid = j < fcount;
  const uint32_t q = valid ? frontier[j] : 0u;
  for (uint32_t r0 = 0; r0 < nrows; r0 += kBfsRowChunk) {
    if (threadIdx.x == 0) s_cnt = 0;
    __syncthreads();
    const uint32_t r1 = min(nrows, r0 + kBfsRowChunk);
    if (valid) {
      for (uint32_t r = r0; r < r1; ++r) {
        const uint32_t t = reinterpret_cast<const uint32_t*>(rows[r])[q];
        const uint32_t bit = 1u << (t & 31u);
        if (!(visited[t >> 5] & bit) && !(atomicOr(&visited[t >> 5], bit) & bit))
          s_new[atomicAdd(&s_cnt, 1u)] = t;
      }
    }
    __syncthreads();
    const uint32_t cnt = s_cnt;
    if (threadIdx.x == 0 && cnt) s_base = atomicAdd(next_count, cnt);
    __syncthreads();
    for (uint32_t x = threadIdx.x; x < cnt; x += kBlock) next[s_base + x] = s_new[x];
    __syncthreads();
  }
}

// sel[c] = c for every class c that holds a reachable state (sel starts as
// all ones), so that a scan over "sel[c] == c" numbers the kept classes.
__global__ __launch_bounds__(kBlock) void k_mark_classes(uint32_t n, const uint32_t* __restrict__ visited,
                                                         const uint32_t* __restrict__ cls,
                                                         uint32_t* __restrict__ sel) {
  const uint32_t q = blockIdx.x * kBlock + threadIdx.x;
  if (q >= n) return;
  if ((visited[q >> 5] >> (q & 31u)) & 1u) sel[cls[q]] = cls[q];
}

// rep[c] = least member of class c (block ids are least members).
__global__ __launch_bounds__(kBlock) void k_class_reps(uint32_t n, const uint32_t* __restrict__ block,
                                                       const uint32_t* __restrict__ cls,
                                                       uint32_t* __restrict__ rep) {
  const uint32_t q = blockIdx.x * kBlock + threadIdx.x;
  if (q < n && block[q] == q) rep[cls[q]] = q;
}

// The quotient: kept class c becomes state s = rid[c]; letter a leads to
// rid[class of delta(rep_c, a)] (the same class for every member of c); s
// accepts iff rep_c does.  m = rid[nb] kept classes; min_delta is
// letter-major with m entries per letter.
__global__ __launch_bounds__(kBlock) void k_quotient(uint32_t nb, uint32_t n, uint32_t k,
                                                     const uint32_t* __restrict__ delta,
                                                     const uint8_t* __restrict__ accept,
                                                     const uint32_t* __restrict__ cls,
                                                     const uint32_t* __restrict__ sel,
                                                     const uint32_t* __restrict__ rid,
                                                     const uint32_t* __restrict__ rep,
                                                     uint32_t* __restrict__ min_delta,
                                                     uint8_t* __restrict__ min_acc) {
  const uint32_t c = blockIdx.x * kBlock + threadIdx.x;
  if (c >= nb || sel[c] != c) return;
  const uint32_t m = rid[nb], s = rid[c], r = rep[c];
  for (uint32_t a = 0; a < k; ++a) min_delta[(uint64_t)a * m + s] = rid[cls[delta[(uint64_t)a * n + r]]];
  min_acc[s] = (accept[r >> 3] >> (r & 7u)) & 1u;
}

// LSB-first bitmap from one byte per state; m = *count.
__global__ __launch_bounds__(kBlock) void k_pack_bits(const uint32_t* __restrict__ count,
                                                      const uint8_t* __restrict__ bytes,
                                                      uint8_t* __restrict__ bits) {
  const uint32_t b = blockIdx.x * kBlock + threadIdx.x;
  const uint32_t m = *count;
  if ((uint64_t)b * 8 >= m) return;
  uint32_t v = 0;
  for (uint32_t t = 0; t < 8; ++t)
    if (b * 8 + t < m && bytes[b * 8 + t]) v |= 1u << t;
  bits[b] = (uint8_t)v;
}

// ---------------------------------------------------------------- finalize
__global__ __launch_bounds__(kBlock) void k_prep_scan(unsigned long long* __restrict__ scan_status,
                                                      uint32_t ntiles, Ctrl* __restrict__ ctrl) {
  const uint32_t j = blockIdx.x * kBlock + threadIdx.x;
  if (j < ntiles) store_status(&scan_status[j], 0ull);
  if (j == 0) atomicExch(&ctrl->tile_counter, 0u);
}

// rank[g] = number of block representatives (block[x] == x) with x < g;
// rank[N] = their total.  Algorithmic bytes: 8 per state.
template <int ITEMS>
__global__ __launch_bounds__(kBlock) void k_scan_reps(const uint32_t* __restrict__ block,
                                                      uint32_t N, uint32_t* __restrict__ rank,
                                                      Ctrl* __restrict__ ctrl,
                                                      unsigned long long* __restrict__ scan_status) {
  __shared__ uint32_t s_tile, s_prefix;
  __shared__ TileScanLds<ITEMS> s_scan;
  if (threadIdx.x == 0) s_tile = atomicAdd(&ctrl->tile_counter, 1u);
  __syncthreads();
  const uint32_t tile = s_tile;
  const uint32_t base = tile * (kBlock * ITEMS);
  uint32_t fb = 0;
#pragma unroll 8
  for (int e = 0; e < ITEMS; ++e) {
    const uint32_t g = base + e * kBlock + threadIdx.x;
    if (g < N && block[g] == g) fb |= 1u << e;
  }
  const uint32_t total = tile_ballot_count<ITEMS>(fb, s_scan);
  if (threadIdx.x < 64) {
    const uint32_t excl = lookback_wave0(scan_status, tile, total, ctrl);
    if (threadIdx.x == 0) {
      s_prefix = excl;
      if (base + kBlock * ITEMS >= N) rank[N] = excl + total;
    }
  }
  __syncthreads();
  const uint32_t pre = s_prefix;
  for (int e = 0; e < ITEMS; ++e) {
    const uint32_t g = base + e * kBlock + threadIdx.x;
    if (g < N) rank[g] = pre + tile_rank<ITEMS>(s_scan, e);
  }
}

// out[q] = rank[block[g]] - rank[state_off]: canonical ids by least member.
// Algorithmic bytes: 12 per state (block, gathered rank, out write; +4 inst_of).
template <bool BATCH>
__global__ __launch_bounds__(kBlock) void k_emit(uint32_t N, const uint32_t* __restrict__ inst_of,
                                                 const InstDesc* __restrict__ desc,
                                                 const uint32_t* __restrict__ block,
                                                 const uint32_t* __restrict__ rank) {
  const uint32_t g = blockIdx.x * kBlock + threadIdx.x;
  if (g >= N) return;
  const uint32_t i = BATCH ? inst_of[g] : 0u;
  const uint32_t off = desc[i].state_off;
  uint32_t* __restrict__ out = reinterpret_cast<uint32_t*>(desc[i].out);
  out[g - off] = rank[block[g]] - rank[off];
}

__global__ __launch_bounds__(kBlock) void k_results(uint32_t ninst, const InstDesc* __restrict__ desc,
                                                    const uint32_t* __restrict__ rank,
                                                    const uint32_t* __restrict__ refine_cnt,
                                                    ResultDev* __restrict__ res) {
  const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= ninst) return;
  const InstDesc D = desc[i];
  ResultDev r;
  r.num_blocks = rank[D.state_off + D.n] - rank[D.state_off];
  r.initial_block = reinterpret_cast<const uint32_t*>(D.out)[D.q0];
  r.refine_rounds = refine_cnt[i];
  r.pad = 0;
  res[i] = r;
}

// Algorithmic bytes: 8 + DW per state (block, gathered rank, dense write;
// +4 inst_of).  The caller picks DW so that every dense number fits.
template <bool BATCH, int DW>
__global__ __launch_bounds__(kBlock) void k_dense(uint32_t N, const uint32_t* __restrict__ inst_of,
                                                  const InstDesc* __restrict__ desc,
                                                  const uint32_t* __restrict__ block,
                                                  const uint32_t* __restrict__ rank,
                                                  void* __restrict__ dense) {
  const uint32_t g = blockIdx.x * kBlock + threadIdx.x;
  if (g >= N) return;
  const uint32_t i = BATCH ? inst_of[g] : 0u;
  const uint32_t v = rank[block[g]] - rank[desc[i].state_off];
  if constexpr (DW == 1) static_cast<uint8_t*>(dense)[g] = (uint8_t)v;
  else if constexpr (DW == 2) static_cast<uint16_t*>(dense)[g] = (uint16_t)v;
  else static_cast<uint32_t*>(dense)[g] = v;
}

__global__ __launch_bounds__(kBlock) void k_block_counts(uint32_t ninst, const InstDesc* __restrict__ desc,
                                                         const uint32_t* __restrict__ rank,
                                                         uint32_t* __restrict__ counts) {
  const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= ninst) return;
  counts[i] = rank[desc[i].state_off + desc[i].n] - rank[desc[i].state_off];
}

// ------------------------------------------------------- joining instances
__global__ __launch_bounds__(kBlock) void k_init_minmax_slots(const InstDesc* __restrict__ desc,
                                                              const uint32_t* __restrict__ slot,
                                                              const uint32_t* __restrict__ job_wg_off,
                                                              uint32_t njobs,
                                                              unsigned long long* __restrict__ part) {
  __shared__ uint32_t s_job, sF, sN;
  const uint32_t j = find_job(job_wg_off, njobs, &s_job);
  const InstDesc D = desc[slot[j]];
  const uint8_t* __restrict__ acc = reinterpret_cast<const uint8_t*>(D.accept);
  if (threadIdx.x == 0) { sF = 0xffffffffu; sN = 0xffffffffu; }
  __syncthreads();
  const uint32_t b = (blockIdx.x - job_wg_off[j]) * (kRowTile / 8) + threadIdx.x;
  const uint32_t nbytes = (D.n + 7) >> 3;
  uint32_t mf = 0xffffffffu, mn = 0xffffffffu;
  if (threadIdx.x < kRowTile / 8 && b < nbytes) {
    const uint32_t valid = D.n - b * 8;
    const uint32_t vmask = valid >= 8 ? 0xffu : ((1u << valid) - 1u);
    const uint32_t v = acc[b];
    const uint32_t f = v & vmask, nf = ~v & vmask;
    if (f) mf = b * 8 + __builtin_ctz(f);
    if (nf) mn = b * 8 + __builtin_ctz(nf);
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    mf = min(mf, (uint32_t)__shfl_xor(mf, off, 64));
    mn = min(mn, (uint32_t)__shfl_xor(mn, off, 64));
  }
  if ((threadIdx.x & 63u) == 0) {
    atomicMin(&sF, mf);
    atomicMin(&sN, mn);
  }
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = ((unsigned long long)sF << 32) | sN;
}

__global__ __launch_bounds__(kBlock) void k_init_minmax_slots_reduce(
    const uint32_t* __restrict__ slot, const uint32_t* __restrict__ job_wg_off, uint32_t njobs,
    uint32_t total_wgs, const unsigned long long* __restrict__ part, uint32_t* __restrict__ minF,
    uint32_t* __restrict__ minN) {
  __shared__ uint32_t sF, sN;
  const uint32_t j = blockIdx.x;
  const uint32_t b = job_wg_off[j], e = (j + 1 < njobs) ? job_wg_off[j + 1] : total_wgs;
  if (threadIdx.x == 0) { sF = 0xffffffffu; sN = 0xffffffffu; }
  __syncthreads();
  uint32_t mf = 0xffffffffu, mn = 0xffffffffu;
  for (uint32_t w = b + threadIdx.x; w < e; w += kBlock) {
    const unsigned long long v = part[w];
    mf = min(mf, (uint32_t)(v >> 32));
    mn = min(mn, (uint32_t)v);
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    mf = min(mf, (uint32_t)__shfl_xor(mf, off, 64));
    mn = min(mn, (uint32_t)__shfl_xor(mn, off, 64));
  }
  if ((threadIdx.x & 63u) == 0) {
    atomicMin(&sF, mf);
    atomicMin(&sN, mn);
  }
  __syncthreads();
  if (threadIdx.x == 0) { minF[slot[j]] = sF; minN[slot[j]] = sN; }
}

// Initial partition of joining instances; their states are appended to act.
__global__ __launch_bounds__(kBlock) void k_init_join(const InstDesc* __restrict__ desc,
                                                      const uint32_t* __restrict__ slot,
                                                      const uint32_t* __restrict__ job_wg_off,
                                                      uint32_t njobs,
                                                      const uint32_t* __restrict__ act_off,
                                                      const uint32_t* __restrict__ minF,
                                                      const uint32_t* __restrict__ minN,
                                                      uint32_t* __restrict__ inst_of,
                                                      uint32_t* __restrict__ block,
                                                      uint32_t* __restrict__ act,
                                                      uint32_t* __restrict__ zero_a,
                                                      uint32_t* __restrict__ zero_b,
                                                      uint32_t* __restrict__ zero_c) {
  __shared__ uint32_t s_job;
  const uint32_t j = find_job(job_wg_off, njobs, &s_job);
  const uint32_t i = slot[j];
  const InstDesc D = desc[i];
  if (blockIdx.x == job_wg_off[j] && threadIdx.x == 0) {  // the slot's counters start at 0
    zero_a[i] = 0u;
    zero_b[i] = 0u;
    zero_c[i] = 0u;
  }
  const uint8_t* __restrict__ acc = reinterpret_cast<const uint8_t*>(D.accept);
  const uint32_t base = (blockIdx.x - job_wg_off[j]) * kRowTile;
  const uint32_t f = D.state_off + minF[i], nf = D.state_off + minN[i];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const uint32_t q = base + e * kBlock + threadIdx.x;
    if (q < D.n) {
      const uint32_t g = D.state_off + q;
      const bool a = (acc[q >> 3] >> (q & 7)) & 1u;
      block[g] = a ? f : nf;
      inst_of[g] = i;
      act[act_off[j] + q] = g;
    }
  }
}

// --------------------------------------------------- per-instance numbering
// Segmented version of k_scan_reps over the instances slot[j]: every job
// starts its own prefix at 0.  Algorithmic bytes: 8 per state.
template <int ITEMS>
__global__ __launch_bounds__(kBlock) void k_scan_jobs(const InstDesc* __restrict__ desc,
                                                      const uint32_t* __restrict__ slot,
                                                      const uint32_t* __restrict__ job_tile_off,
                                                      uint32_t njobs,
                                                      const uint32_t* __restrict__ block,
                                                      uint32_t* __restrict__ rank,
                                                      uint32_t* __restrict__ totals,
                                                      Ctrl* __restrict__ ctrl,
                                                      unsigned long long* __restrict__ scan_status) {
  __shared__ uint32_t s_tile, s_job, s_prefix;
  __shared__ TileScanLds<ITEMS> s_scan;
  if (threadIdx.x == 0) {
    const uint32_t t = atomicAdd(&ctrl->tile_counter, 1u);
    uint32_t lo = 0, hi = njobs;
    while (hi - lo > 1) {
      const uint32_t mid = (lo + hi) >> 1;
      if (job_tile_off[mid] <= t) lo = mid; else hi = mid;
    }
    s_tile = t;
    s_job = lo;
  }
  __syncthreads();
  const uint32_t tile = s_tile, j = s_job;
  const InstDesc D = desc[slot[j]];
  const uint32_t base = (tile - job_tile_off[j]) * (kBlock * ITEMS);
  uint32_t fb = 0;
#pragma unroll 8
  for (int e = 0; e < ITEMS; ++e) {
    const uint32_t q = base + e * kBlock + threadIdx.x;
    if (q < D.n && block[D.state_off + q] == D.state_off + q) fb |= 1u << e;
  }
  const uint32_t total = tile_ballot_count<ITEMS>(fb, s_scan);
  if (threadIdx.x < 64) {
    const uint32_t excl = lookback_wave0(scan_status, tile, total, ctrl, job_tile_off[j]);
    if (threadIdx.x == 0) {
      s_prefix = excl;
      if (base + kBlock * ITEMS >= D.n) totals[j] = excl + total;
    }
  }
  __syncthreads();
  const uint32_t pre = s_prefix;
  for (int e = 0; e < ITEMS; ++e) {
    const uint32_t q = base + e * kBlock + threadIdx.x;
    if (q < D.n) rank[D.state_off + q] = pre + tile_rank<ITEMS>(s_scan, e);
  }
}

// out[q] = rank[block[g]] (ranks are already relative to the instance).
__global__ __launch_bounds__(kBlock) void k_emit_jobs(const InstDesc* __restrict__ desc,
                                                      const uint32_t* __restrict__ slot,
                                                      const uint32_t* __restrict__ job_wg_off,
                                                      uint32_t njobs,
                                                      const uint32_t* __restrict__ block,
                                                      const uint32_t* __restrict__ rank) {
  __shared__ uint32_t s_job;
  const uint32_t j = find_job(job_wg_off, njobs, &s_job);
  const InstDesc D = desc[slot[j]];
  uint32_t* __restrict__ out = reinterpret_cast<uint32_t*>(D.out);
  const uint32_t base = (blockIdx.x - job_wg_off[j]) * kRowTile;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const uint32_t q = base + e * kBlock + threadIdx.x;
    if (q < D.n) out[q] = rank[block[D.state_off + q]];
  }
}

// dense[g] = rank[block[g]] for the states of the listed instances (ranks
// from k_scan_jobs are relative to the instance), DW bytes wide.
// Algorithmic bytes: 8 + DW per state.
template <int DW>
__global__ __launch_bounds__(kBlock) void k_dense_jobs(const InstDesc* __restrict__ desc,
                                                       const uint32_t* __restrict__ slot,
                                                       const uint32_t* __restrict__ job_wg_off,
                                                       uint32_t njobs,
                                                       const uint32_t* __restrict__ block,
                                                       const uint32_t* __restrict__ rank,
                                                       void* __restrict__ dense) {
  __shared__ uint32_t s_job;
  const uint32_t j = find_job(job_wg_off, njobs, &s_job);
  const InstDesc D = desc[slot[j]];
  const uint32_t base = (blockIdx.x - job_wg_off[j]) * kRowTile;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const uint32_t q = base + e * kBlock + threadIdx.x;
    if (q < D.n) {
      const uint32_t g = D.state_off + q;
      const uint32_t v = rank[block[g]];
      if constexpr (DW == 1) static_cast<uint8_t*>(dense)[g] = (uint8_t)v;
      else if constexpr (DW == 2) static_cast<uint16_t*>(dense)[g] = (uint16_t)v;
      else static_cast<uint32_t*>(dense)[g] = v;
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_results_jobs(const InstDesc* __restrict__ desc,
                                                         const uint32_t* __restrict__ slot,
                                                         uint32_t njobs,
                                                         const uint32_t* __restrict__ totals,
                                                         const uint32_t* __restrict__ refine_cnt,
                                                         ResultDev* __restrict__ res) {
  const uint32_t j = blockIdx.x * kBlock + threadIdx.x;
  if (j >= njobs) return;
  const InstDesc D = desc[slot[j]];
  ResultDev r;
  r.num_blocks = totals[j];
  r.initial_block = reinterpret_cast<const uint32_t*>(D.out)[D.q0];
  r.refine_rounds = refine_cnt[slot[j]];
  r.pad = 0;
  res[j] = r;
}

// ------------------------------------------------- first round by labels
// From P_0 = {F, Q\F} the first round of Algorithm 4 needs no grouping: the
// signature of q is the accept bit of q and of each successor, and with at
// most kMaxLabelLetters signature letters that bit string (own bit in bit
// 0, letter t in bit t+1) is itself the exact key and a block label below
// NL (256 with up to 7 letters, stored in a byte; 512 with 8, in two bytes,
// type LT).  k_label writes the labels and the least member of every label
// (lmin, NL words per instance, all ones where absent); k_label_rank numbers
// the labels present (rank: the dense block numbers of the next round),
// counts them and flags the instances that split; k_label_apply turns labels
// into least-member ids and dense numbers.  Each workgroup covers kRowTile
// states of one instance.
// Algorithmic bytes per state: 1/8 (own bit) + kp * (4 + 1) (row entry, the
// successor's bitmap byte) + sizeof(LT) (label).
template <int NL, typename LT>
__global__ __launch_bounds__(kBlock) void k_label(const InstDesc* __restrict__ desc,
                                                  const uint32_t* __restrict__ job_wg_off, uint32_t ninst,
                                                  const uint64_t* __restrict__ rows,
                                                  uint32_t* __restrict__ lmin, LT* __restrict__ label) {
  __shared__ uint32_t s_job;
  __shared__ uint32_t s_min[NL];
  for (uint32_t l = threadIdx.x; l < (uint32_t)NL; l += kBlock) s_min[l] = 0xffffffffu;
  const uint32_t i = find_job(job_wg_off, ninst, &s_job);
  const InstDesc D = desc[i];
  const uint8_t* __restrict__ acc = reinterpret_cast<const uint8_t*>(D.accept);
  const uint64_t* __restrict__ R = rows + D.rows_off;
  const uint32_t kp = D.kp;
  const uint32_t base = (blockIdx.x - job_wg_off[i]) * kRowTile;
  uint32_t lab[4];
  // every row entry of the tile first, then the bitmap gathers
  uint32_t s[4][kMaxLabelLetters];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const uint32_t q = base + e * kBlock + threadIdx.x;
#pragma unroll
    for (uint32_t t = 0; t < kMaxLabelLetters; ++t)
      if (t < kp && q < D.n) s[e][t] = reinterpret_cast<const uint32_t*>(R[t])[q];
  }
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const uint32_t q = base + e * kBlock + threadIdx.x;
    lab[e] = 0;
    if (q >= D.n) continue;
    uint32_t L = (acc[q >> 3] >> (q & 7)) & 1u;
#pragma unroll
    for (uint32_t t = 0; t < kMaxLabelLetters; ++t)
      if (t < kp) L |= ((acc[s[e][t] >> 3] >> (s[e][t] & 7)) & 1u) << (t + 1);
    lab[e] = L;
  }
  __syncthreads();  // s_min initialised
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const uint32_t q = base + e * kBlock + threadIdx.x;
    if (q >= D.n) continue;
    label[D.state_off + q] = (LT)lab[e];
    atomicMin(&s_min[lab[e]], D.state_off + q);
  }
  __syncthreads();
  for (uint32_t l = threadIdx.x; l < (uint32_t)NL; l += kBlock) {
    const uint32_t v = s_min[l];
    if (v == 0xffffffffu) continue;
    // Workgroups of one instance run roughly in state order, so the word
    // mostly holds a smaller member already.  A plain read can only be
    // stale upwards (the word only decreases), which at worst costs an
    // atomic that changes nothing.
    uint32_t* p = &lmin[(size_t)i * NL + l];
    if (*p > v) atomicMin(p, v);
  }
}

// One workgroup of NL threads per instance, one thread per label.  Also
// clears the round flags of the control block (no table is cleared in this
// round) and, with set_m, sets m_next to m (every state stays active: no
// compaction).
template <int NL, typename LT>
__global__ __launch_bounds__(NL) void k_label_rank(const uint32_t* __restrict__ lmin, LT* __restrict__ rank,
                                                   uint32_t* __restrict__ counts,
                                                   uint32_t* __restrict__ changed_inst,
                                                   Ctrl* __restrict__ ctrl, uint32_t set_m, uint32_t m) {
  constexpr int kW = NL / 64;
  __shared__ uint32_t s_cnt[kW], s_par;
  const uint32_t i = blockIdx.x, L = threadIdx.x, lane = L & 63u, w = L >> 6;
  if (L == 0) s_par = 0;
  const bool present = lmin[(size_t)i * NL + L] != 0xffffffffu;
  const unsigned long long b = __ballot(present);
  if (lane == 0) s_cnt[w] = (uint32_t)__popcll(b);
  __syncthreads();
  if (present) atomicOr(&s_par, 1u << (L & 1u));  // blocks of P_0 present: accept bit 0 and / or 1
  uint32_t before = (uint32_t)__popcll(b & ((1ull << lane) - 1ull)), total = 0;
#pragma unroll
  for (int v = 0; v < kW; ++v) {
    if (v < (int)w) before += s_cnt[v];
    total += s_cnt[v];
  }
  rank[(size_t)i * NL + L] = (LT)before;
  __syncthreads();
  if (L == 0) {
    counts[i] = total;
    if (total > (uint32_t)__builtin_popcount(s_par)) changed_inst[i] = 1u;
    if (i == 0) {
      ctrl->any_changed = 0u;
      ctrl->collision = 0u;
      if (set_m) ctrl->m_next = m;
    }
  }
}

// label[g] -> the label's least member in block[g], the label's number in
// dense[g] (one byte: an instance whose next round groups on exact keys
// has at most 32 blocks, as (kp+1) * ceil(log2 B) <= 31 with B <= 2^(kp+1)
// gives ceil(log2 B) <= 5; for the others the byte is never read), act[g] =
// g (every state in order: list position and state id agree) and
// inst_of[g] = i where given.  With one-byte labels, dense may be label
// itself (each thread reads its state's label before it writes there).
// Algorithmic bytes per state: sizeof(LT) (label) + 1 (dense) + 4 (id) + 4
// (act) [+4 inst_of].
template <int NL, typename LT>
__global__ __launch_bounds__(kBlock) void k_label_apply(const InstDesc* __restrict__ desc,
                                                        const uint32_t* __restrict__ job_wg_off,
                                                        uint32_t ninst, const uint32_t* __restrict__ lmin,
                                                        const LT* __restrict__ rank, const LT* label,
                                                        uint8_t* dense, uint32_t* __restrict__ block,
                                                        uint32_t* __restrict__ act,
                                                        uint32_t* __restrict__ inst_of) {
  __shared__ uint32_t s_job;
  const uint32_t i = find_job(job_wg_off, ninst, &s_job);
  const InstDesc D = desc[i];
  const uint32_t* __restrict__ lm = lmin + (size_t)i * NL;
  const LT* __restrict__ rk = rank + (size_t)i * NL;
  const uint32_t base = (blockIdx.x - job_wg_off[i]) * kRowTile;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const uint32_t q = base + e * kBlock + threadIdx.x;
    if (q >= D.n) continue;
    const uint32_t g = D.state_off + q;
    const uint32_t L = label[g];
    dense[g] = (uint8_t)rk[L];
    block[g] = lm[L];
    act[g] = g;
    if (inst_of) inst_of[g] = i;
  }
}

// Every block a singleton (one instance): block q has least member q, so
// its canonical number is q.  out[q] = q; the results follow.
// Algorithmic bytes per state: 4 (out).
__global__ __launch_bounds__(kBlock) void k_identity_out(const InstDesc* __restrict__ desc,
                                                         const uint32_t* __restrict__ refine_cnt,
                                                         ResultDev* __restrict__ res) {
  const InstDesc D = desc[0];
  uint32_t* __restrict__ out = reinterpret_cast<uint32_t*>(D.out);
  const uint32_t base = blockIdx.x * kRowTile;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const uint32_t q = base + e * kBlock + threadIdx.x;
    if (q < D.n) out[q] = q;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ResultDev r;
    r.num_blocks = D.n;
    r.initial_block = D.q0;
    r.refine_rounds = refine_cnt[0];
    r.pad = 0;
    res[0] = r;
  }
}

inline uint32_t grid_for(uint64_t items, uint64_t per_wg) {
  return (uint32_t)((items + per_wg - 1) / per_wg);
}

}  // namespace

// ---------------------------------------------------------------- launchers
void launch_row_check(const RowJob* jobs, const uint32_t* job_wg_off, uint32_t njobs,
                      uint32_t total_wgs, uint32_t* wg_flags, uint32_t* flags, hipStream_t s) {
  if (!total_wgs) return;
  hipLaunchKernelGGL(k_row_check, dim3(total_wgs), dim3(kBlock), 0, s, jobs, job_wg_off, njobs, wg_flags);
  hipLaunchKernelGGL(k_flags_reduce, dim3(njobs), dim3(kBlock), 0, s, job_wg_off, njobs, total_wgs,
                     wg_flags, flags);
}

void launch_closure_level(const RowJob* jobs, const uint32_t* job_wg_off, uint32_t njobs,
                          uint32_t total_wgs, uint32_t* wg_flags, uint32_t* flags, hipStream_t s) {
  if (!total_wgs) return;
  hipLaunchKernelGGL(k_closure_level, dim3(total_wgs), dim3(kBlock), 0, s, jobs, job_wg_off, njobs,
                     flags ? wg_flags : nullptr);
  if (flags)
    hipLaunchKernelGGL(k_flags_reduce, dim3(njobs), dim3(kBlock), 0, s, job_wg_off, njobs, total_wgs,
                       wg_flags, flags);
}

void launch_init_minmax(const InstDesc* desc, const uint32_t* job_wg_off, uint32_t ninst,
                        uint32_t total_wgs, unsigned long long* wg_part, uint32_t* minF,
                        uint32_t* minN, hipStream_t s) {
  if (!ninst || !total_wgs) return;
  hipLaunchKernelGGL(k_init_minmax_part, dim3(total_wgs), dim3(kBlock), 0, s, desc, job_wg_off, ninst,
                     wg_part);
  hipLaunchKernelGGL(k_init_minmax_reduce, dim3(ninst), dim3(kBlock), 0, s, job_wg_off, ninst, total_wgs,
                     wg_part, minF, minN);
}

void launch_init_block(const InstDesc* desc, const uint32_t* job_wg_off, uint32_t ninst,
                       uint32_t total_wgs, const uint32_t* minF, const uint32_t* minN,
                       uint32_t* inst_of, uint32_t* block, uint32_t* act, hipStream_t s) {
  if (!total_wgs) return;
  hipLaunchKernelGGL(k_init_block, dim3(total_wgs), dim3(kBlock), 0, s, desc, job_wg_off, ninst, minF,
                     minN, inst_of, block, act);
}

void launch_clear_table(Slot* table, uint64_t tsize, Ctrl* ctrl, hipStream_t s, int gmode,
                        uint32_t* gcount) {
  uint32_t grid = grid_for(tsize, 2 * kBlock);
  if (grid > 65536u) grid = 65536u;
  if (grid == 0) grid = 1;
  hipLaunchKernelGGL(k_clear_table, dim3(grid), dim3(kBlock), 0, s, table, tsize, ctrl, (uint32_t)gmode, gcount);
}

void launch_queue_start(Ctrl* ctrl, uint32_t m, uint64_t salt, hipStream_t s) {
  hipLaunchKernelGGL(k_queue_start, dim3(1), dim3(64), 0, s, ctrl, m, salt);
}

void launch_queue_plan(const QueueDbl& q, InstDesc* desc, const Ctrl* ctrl, hipStream_t s) {
  if (!q.count) return;
  hipLaunchKernelGGL(k_queue_plan, dim3(grid_for(q.count, kBlock)), dim3(kBlock), 0, s, q, desc, ctrl);
}

void launch_queue_levels(const QueueDbl& q, const uint64_t* rows, const Ctrl* ctrl, hipStream_t s) {
  if (!q.count || !q.wgs) return;
  hipLaunchKernelGGL(k_queue_levels, dim3(q.wgs), dim3(kBlock), 0, s, q, rows, ctrl);
}

void launch_queue_advance(const QueueDbl& q, const Ctrl* ctrl, hipStream_t s) {
  if (!q.count) return;
  hipLaunchKernelGGL(k_queue_advance, dim3(grid_for(q.count, kBlock)), dim3(kBlock), 0, s, q, ctrl);
}

void launch_store_u64(uint64_t* p, uint64_t v, hipStream_t s) {
  hipLaunchKernelGGL(k_store_u64, dim3(1), dim3(64), 0, s, p, v);
}

void launch_round_step(Ctrl* ctrl, hipStream_t s) {
  hipLaunchKernelGGL(k_round_step, dim3(1), dim3(64), 0, s, ctrl);
}

void launch_copy_bytes(void* dst, const void* src, size_t bytes, hipStream_t s) {
  if (!bytes) return;
  const uintptr_t a = reinterpret_cast<uintptr_t>(dst) | reinterpret_cast<uintptr_t>(src) | (uintptr_t)bytes;
  const uint32_t unit = (a & 15u) == 0 ? 16u : ((a & 3u) == 0 ? 4u : 1u);
  const uint64_t units = bytes / unit;
  const uint32_t grid = (uint32_t)std::min<uint64_t>((units + kBlock - 1) / kBlock, 128);
  if (unit == 16)
    hipLaunchKernelGGL(k_copy_units<uint4>, dim3(grid), dim3(kBlock), 0, s, static_cast<uint4*>(dst),
                       static_cast<const uint4*>(src), units);
  else if (unit == 4)
    hipLaunchKernelGGL(k_copy_units<uint32_t>, dim3(grid), dim3(kBlock), 0, s, static_cast<uint32_t*>(dst),
                       static_cast<const uint32_t*>(src), units);
  else
    hipLaunchKernelGGL(k_copy_units<uint8_t>, dim3(grid), dim3(kBlock), 0, s, static_cast<uint8_t*>(dst),
                       static_cast<const uint8_t*>(src), units);
}

void launch_mem_segs(const MemSegs& q, hipStream_t s) {
  if (!q.n) return;
  uint64_t most = 0;
  for (uint32_t k = 0; k < q.n; ++k) most = std::max<uint64_t>(most, q.seg[k].bytes);
  const uint32_t grid = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>((most / 16 + kBlock - 1) / kBlock, 1024));
  hipLaunchKernelGGL(k_mem_segs, dim3(grid), dim3(kBlock), 0, s, q);
}

namespace {
template <bool BATCH, int SI>
void launch_signature_si(int dw, uint32_t m, const uint32_t* act, const uint32_t* inst_of,
                         const InstDesc* desc, const uint64_t* rows, const uint32_t* block,
                         const void* dense, Slot* table, uint32_t tbits, uint32_t* slot_of, uint64_t salt,
                         Ctrl* ctrl, hipStream_t s, uint32_t gm, uint8_t* notify, uint32_t* gcount,
                         uint32_t* dtab) {
  const dim3 grid(grid_for(m, kBlock * SI));
  if (dw == 1)
    hipLaunchKernelGGL((k_signature<BATCH, 1, SI>), grid, dim3(kBlock), 0, s, act, m, inst_of, desc, rows,
                       block, dense, table, tbits, slot_of, salt, ctrl, gm, notify, gcount, dtab);
  else if (dw == 2)
    hipLaunchKernelGGL((k_signature<BATCH, 2, SI>), grid, dim3(kBlock), 0, s, act, m, inst_of, desc, rows,
                       block, dense, table, tbits, slot_of, salt, ctrl, gm, notify, gcount, dtab);
  else
    hipLaunchKernelGGL((k_signature<BATCH, 4, SI>), grid, dim3(kBlock), 0, s, act, m, inst_of, desc, rows,
                       block, dense, table, tbits, slot_of, salt, ctrl, gm, notify, gcount, dtab);
}

template <bool BATCH>
void launch_signature_w(int dw, int variant, uint32_t m, const uint32_t* act, const uint32_t* inst_of,
                        const InstDesc* desc, const uint64_t* rows, const uint32_t* block,
                        const void* dense, Slot* table, uint32_t tbits, uint32_t* slot_of, uint64_t salt,
                        Ctrl* ctrl, hipStream_t s, uint32_t gm, uint8_t* notify, uint32_t* gcount,
                        uint32_t* dtab) {
  if (variant == 0)
    launch_signature_si<BATCH, 1>(dw, m, act, inst_of, desc, rows, block, dense, table, tbits, slot_of, salt,
                                  ctrl, s, gm, notify, gcount, dtab);
  else if (variant == 2)
    launch_signature_si<BATCH, 4>(dw, m, act, inst_of, desc, rows, block, dense, table, tbits, slot_of, salt,
                                  ctrl, s, gm, notify, gcount, dtab);
  else
    launch_signature_si<BATCH, 2>(dw, m, act, inst_of, desc, rows, block, dense, table, tbits, slot_of, salt,
                                  ctrl, s, gm, notify, gcount, dtab);
}

template <bool BATCH>
void launch_dense_w(int dw, uint32_t N, const uint32_t* inst_of, const InstDesc* desc,
                    const uint32_t* block, const uint32_t* rank, void* dense, hipStream_t s) {
  const dim3 grid(grid_for(N, kBlock));
  if (dw == 1)
    hipLaunchKernelGGL((k_dense<BATCH, 1>), grid, dim3(kBlock), 0, s, N, inst_of, desc, block, rank, dense);
  else if (dw == 2)
    hipLaunchKernelGGL((k_dense<BATCH, 2>), grid, dim3(kBlock), 0, s, N, inst_of, desc, block, rank, dense);
  else
    hipLaunchKernelGGL((k_dense<BATCH, 4>), grid, dim3(kBlock), 0, s, N, inst_of, desc, block, rank, dense);
}
}  // namespace

void launch_signature(bool batch, const uint32_t* act, uint32_t m, const uint32_t* inst_of,
                      const InstDesc* desc, const uint64_t* rows, const uint32_t* block,
                      const void* dense, int dense_width, Slot* table, uint32_t tbits,
                      uint32_t* slot_of, uint64_t salt, Ctrl* ctrl, int variant, hipStream_t s,
                      int gmode, uint8_t* notify, uint32_t* gcount, uint32_t* dtab) {
  if (!m) return;
  if (batch)
    launch_signature_w<true>(dense_width, variant, m, act, inst_of, desc, rows, block, dense, table, tbits,
                             slot_of, salt, ctrl, s, (uint32_t)gmode, notify, gcount, dtab);
  else
    launch_signature_w<false>(dense_width, variant, m, act, inst_of, desc, rows, block, dense, table, tbits,
                              slot_of, salt, ctrl, s, (uint32_t)gmode, notify, gcount, dtab);
}

void launch_dense(bool batch, uint32_t N, const uint32_t* inst_of, const InstDesc* desc,
                  const uint32_t* block, const uint32_t* rank, void* dense, int dense_width,
                  hipStream_t s) {
  if (!N) return;
  if (batch)
    launch_dense_w<true>(dense_width, N, inst_of, desc, block, rank, dense, s);
  else
    launch_dense_w<false>(dense_width, N, inst_of, desc, block, rank, dense, s);
}

void launch_block_counts(uint32_t ninst, const InstDesc* desc, const uint32_t* rank,
                         uint32_t* counts, hipStream_t s) {
  if (!ninst) return;
  hipLaunchKernelGGL(k_block_counts, dim3(grid_for(ninst, kBlock)), dim3(kBlock), 0, s, ninst, desc, rank,
                     counts);
}

void launch_resolve(bool batch, const uint32_t* act, uint32_t m, const uint32_t* inst_of,
                    const InstDesc* desc, const Slot* table,
                    const uint32_t* slot_of, const uint32_t* block, uint32_t* nb, uint8_t* keep,
                    uint32_t* changed_inst, Ctrl* ctrl, unsigned long long* scan_status,
                    uint32_t ntiles, hipStream_t s, int gmode, uint8_t* notify,
                    const uint32_t* count_gcount) {
  if (!m) return;
  const uint32_t grid = grid_for(std::max(m, ntiles), kBlock);
  if (batch)
    hipLaunchKernelGGL(k_resolve<true>, dim3(grid), dim3(kBlock), 0, s, act, m, inst_of, desc, table,
                       slot_of, block, nb, keep, changed_inst, ctrl, scan_status, ntiles, (uint32_t)gmode, notify,
                       count_gcount);
  else
    hipLaunchKernelGGL(k_resolve<false>, dim3(grid), dim3(kBlock), 0, s, act, m, inst_of, desc, table,
                       slot_of, block, nb, keep, changed_inst, ctrl, scan_status, ntiles, (uint32_t)gmode, notify,
                       count_gcount);
}

void launch_compact(bool batch, const uint32_t* act, uint32_t m, const uint32_t* inst_of,
                    const uint32_t* nb, const uint8_t* keep, uint32_t* changed_inst,
                    const uint32_t* dead, uint32_t* block, uint32_t* act_next, Ctrl* ctrl,
                    unsigned long long* scan_status, int items, hipStream_t s, int gmode,
                    const uint32_t* slot_of, uint8_t* notify, const uint32_t* gcount, uint32_t prev_count,
                    const uint32_t* dtab) {
  if (!m) return;
  const dim3 grid(scan_tiles(m, items));
  const uint32_t gm = (uint32_t)gmode;
  if (items == kScanItemsLarge) {
    if (batch)
      hipLaunchKernelGGL((k_compact<true, kScanItemsLarge>), grid, dim3(kBlock), 0, s, act, m, inst_of, nb,
                         keep, changed_inst, dead, block, act_next, ctrl, scan_status, gm,
                         slot_of, notify, gcount, prev_count, dtab);
    else
      hipLaunchKernelGGL((k_compact<false, kScanItemsLarge>), grid, dim3(kBlock), 0, s, act, m, inst_of, nb,
                         keep, changed_inst, dead, block, act_next, ctrl, scan_status, gm,
                         slot_of, notify, gcount, prev_count, dtab);
  } else {
    if (batch)
      hipLaunchKernelGGL((k_compact<true, kScanItemsSmall>), grid, dim3(kBlock), 0, s, act, m, inst_of, nb,
                         keep, changed_inst, dead, block, act_next, ctrl, scan_status, gm,
                         slot_of, notify, gcount, prev_count, dtab);
    else
      hipLaunchKernelGGL((k_compact<false, kScanItemsSmall>), grid, dim3(kBlock), 0, s, act, m, inst_of, nb,
                         keep, changed_inst, dead, block, act_next, ctrl, scan_status, gm,
                         slot_of, notify, gcount, prev_count, dtab);
  }
}

void launch_round_end(uint32_t ninst, uint32_t* changed_inst, uint32_t* refine_cnt, uint32_t* last,
                      Ctrl* ctrl, hipStream_t s, unsigned long long* clear_status, uint32_t clear_tiles,
                      int gmode) {
  const uint32_t threads = std::max(ninst, clear_status ? clear_tiles : 0u);
  if (!threads) return;
  hipLaunchKernelGGL(k_round_end, dim3(grid_for(threads, kBlock)), dim3(kBlock), 0, s, ninst,
                     changed_inst, refine_cnt, last, ctrl, clear_status, clear_tiles, (uint32_t)gmode);
}

void launch_init_join(const InstDesc* desc, const uint32_t* slot, const uint32_t* job_wg_off,
                      uint32_t njobs, uint32_t total_wgs, const uint32_t* act_off,
                      const uint32_t* minF, const uint32_t* minN, uint32_t* inst_of,
                      uint32_t* block, uint32_t* act, uint32_t* zero_a, uint32_t* zero_b, uint32_t* zero_c,
                      hipStream_t s) {
  if (!total_wgs) return;
  hipLaunchKernelGGL(k_init_join, dim3(total_wgs), dim3(kBlock), 0, s, desc, slot, job_wg_off, njobs,
                     act_off, minF, minN, inst_of, block, act, zero_a, zero_b, zero_c);
}

void launch_init_minmax_slots(const InstDesc* desc, const uint32_t* slot, const uint32_t* job_wg_off,
                              uint32_t njobs, uint32_t total_wgs, unsigned long long* wg_part,
                              uint32_t* minF, uint32_t* minN, hipStream_t s) {
  if (!njobs || !total_wgs) return;
  hipLaunchKernelGGL(k_init_minmax_slots, dim3(total_wgs), dim3(kBlock), 0, s, desc, slot, job_wg_off,
                     njobs, wg_part);
  hipLaunchKernelGGL(k_init_minmax_slots_reduce, dim3(njobs), dim3(kBlock), 0, s, slot, job_wg_off, njobs,
                     total_wgs, wg_part, minF, minN);
}

void launch_scan_jobs(const InstDesc* desc, const uint32_t* slot, const uint32_t* job_tile_off,
                      uint32_t njobs, uint32_t total_tiles, const uint32_t* block, uint32_t* rank,
                      uint32_t* totals, Ctrl* ctrl, unsigned long long* scan_status, int items,
                      hipStream_t s) {
  if (!total_tiles) return;
  if (items == kScanItemsLarge)
    hipLaunchKernelGGL(k_scan_jobs<kScanItemsLarge>, dim3(total_tiles), dim3(kBlock), 0, s, desc, slot,
                       job_tile_off, njobs, block, rank, totals, ctrl, scan_status);
  else
    hipLaunchKernelGGL(k_scan_jobs<kScanItemsSmall>, dim3(total_tiles), dim3(kBlock), 0, s, desc, slot,
                       job_tile_off, njobs, block, rank, totals, ctrl, scan_status);
}

void launch_emit_jobs(const InstDesc* desc, const uint32_t* slot, const uint32_t* job_wg_off,
                      uint32_t njobs, uint32_t total_wgs, const uint32_t* block, const uint32_t* rank,
                      hipStream_t s) {
  if (!total_wgs) return;
  hipLaunchKernelGGL(k_emit_jobs, dim3(total_wgs), dim3(kBlock), 0, s, desc, slot, job_wg_off, njobs,
                     block, rank);
}

void launch_dense_jobs(const InstDesc* desc, const uint32_t* slot, const uint32_t* job_wg_off,
                       uint32_t njobs, uint32_t total_wgs, const uint32_t* block, const uint32_t* rank,
                       void* dense, int dense_width, hipStream_t s) {
  if (!total_wgs) return;
  const dim3 grid(total_wgs);
  if (dense_width == 1)
    hipLaunchKernelGGL(k_dense_jobs<1>, grid, dim3(kBlock), 0, s, desc, slot, job_wg_off, njobs, block, rank,
                       dense);
  else if (dense_width == 2)
    hipLaunchKernelGGL(k_dense_jobs<2>, grid, dim3(kBlock), 0, s, desc, slot, job_wg_off, njobs, block, rank,
                       dense);
  else
    hipLaunchKernelGGL(k_dense_jobs<4>, grid, dim3(kBlock), 0, s, desc, slot, job_wg_off, njobs, block, rank,
                       dense);
}

namespace {
template <int NL, typename LT>
void launch_label_t(const InstDesc* desc, const uint32_t* job_wg_off, uint32_t ninst, uint32_t total_wgs,
                    const uint64_t* rows, uint32_t* lmin, void* rank, void* label, uint8_t* dense,
                    uint32_t* counts, uint32_t* changed_inst, Ctrl* ctrl, uint32_t* block, uint32_t set_m,
                    uint32_t m, uint32_t* act, uint32_t* inst_of, hipStream_t s) {
  hipLaunchKernelGGL((k_label<NL, LT>), dim3(total_wgs), dim3(kBlock), 0, s, desc, job_wg_off, ninst, rows, lmin,
                     static_cast<LT*>(label));
  hipLaunchKernelGGL((k_label_rank<NL, LT>), dim3(ninst), dim3(NL), 0, s, lmin, static_cast<LT*>(rank), counts,
                     changed_inst, ctrl, set_m, m);
  hipLaunchKernelGGL((k_label_apply<NL, LT>), dim3(total_wgs), dim3(kBlock), 0, s, desc, job_wg_off, ninst, lmin,
                     static_cast<const LT*>(rank), static_cast<const LT*>(label), dense, block, act, inst_of);
}
}  // namespace

void launch_label(const InstDesc* desc, const uint32_t* job_wg_off, uint32_t ninst, uint32_t total_wgs,
                  const uint64_t* rows, uint32_t label_bits, uint32_t* lmin, void* rank, void* label,
                  uint8_t* dense, uint32_t* counts, uint32_t* changed_inst, Ctrl* ctrl, uint32_t* block,
                  uint32_t set_m, uint32_t m, uint32_t* act, uint32_t* inst_of, hipStream_t s) {
  if (!total_wgs || !ninst) return;
  if (label_bits <= 8)
    launch_label_t<256, uint8_t>(desc, job_wg_off, ninst, total_wgs, rows, lmin, rank, label, dense, counts,
                                 changed_inst, ctrl, block, set_m, m, act, inst_of, s);
  else
    launch_label_t<512, uint16_t>(desc, job_wg_off, ninst, total_wgs, rows, lmin, rank, label, dense, counts,
                                  changed_inst, ctrl, block, set_m, m, act, inst_of, s);
}

void launch_identity_out(const InstDesc* desc, uint32_t n, const uint32_t* refine_cnt, ResultDev* res,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_identity_out, dim3(std::max<uint32_t>(1, grid_for(n, kRowTile))), dim3(kBlock), 0, s,
                     desc, refine_cnt, res);
}

void launch_results_jobs(const InstDesc* desc, const uint32_t* slot, uint32_t njobs,
                         const uint32_t* totals, const uint32_t* refine_cnt, ResultDev* res,
                         hipStream_t s) {
  if (!njobs) return;
  hipLaunchKernelGGL(k_results_jobs, dim3(grid_for(njobs, kBlock)), dim3(kBlock), 0, s, desc, slot, njobs,
                     totals, refine_cnt, res);
}

void launch_naive_round(bool batch, uint32_t N, uint32_t ninst, const uint32_t* inst_of,
                        const InstDesc* desc, const uint64_t* rows, uint32_t* block, uint32_t* new_leader,
                        uint32_t* next_leader, uint8_t* differs, uint32_t* changed_inst, uint32_t* refine_cnt,
                        Ctrl* ctrl, hipStream_t s) {
  const dim3 grid(grid_for(N, kBlock));
  if (batch) {
    hipLaunchKernelGGL(k_naive_elect<true>, grid, dim3(kBlock), 0, s, N, inst_of, desc, rows, block,
                       new_leader, differs, ctrl);
    hipLaunchKernelGGL(k_naive_move<true>, grid, dim3(kBlock), 0, s, N, inst_of, block, new_leader,
                       next_leader, differs, changed_inst, ctrl);
  } else {
    hipLaunchKernelGGL(k_naive_elect<false>, grid, dim3(kBlock), 0, s, N, inst_of, desc, rows, block,
                       new_leader, differs, ctrl);
    hipLaunchKernelGGL(k_naive_move<false>, grid, dim3(kBlock), 0, s, N, inst_of, block, new_leader,
                       next_leader, differs, changed_inst, ctrl);
  }
  launch_round_end(ninst, changed_inst, refine_cnt, nullptr, ctrl, s);
  hipLaunchKernelGGL(k_naive_check, dim3(1), dim3(64), 0, s, ctrl);
}

void launch_bfs_level(const uint64_t* rows, uint32_t nrows, const uint32_t* frontier, uint32_t fcount,
                      uint32_t* visited, uint32_t* next, uint32_t* next_count, hipStream_t s) {
  if (!fcount || !nrows) return;
  hipLaunchKernelGGL(k_bfs_level, dim3(grid_for(fcount, kBlock)), dim3(kBlock), 0, s, rows, nrows, frontier,
                     fcount, visited, next, next_count);
}

void launch_quotient(uint32_t n, uint32_t k, uint32_t nb, const uint32_t* delta, const uint8_t* accept,
                     const uint32_t* block, const uint32_t* cls, const uint32_t* visited, uint32_t* sel,
                     uint32_t* rid, uint32_t* rep, uint32_t* min_delta, uint8_t* min_acc8, uint8_t* min_acc,
                     Ctrl* ctrl, unsigned long long* scan_status, hipStream_t s) {
  hipLaunchKernelGGL(k_mark_classes, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, s, n, visited, cls, sel);
  const int items = scan_items_for(nb);
  launch_prep_scan(scan_status, scan_tiles(nb, items), ctrl, s);
  launch_scan_reps(sel, nb, rid, ctrl, scan_status, items, s);
  hipLaunchKernelGGL(k_class_reps, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, s, n, block, cls, rep);
  hipLaunchKernelGGL(k_quotient, dim3(grid_for(nb, kBlock)), dim3(kBlock), 0, s, nb, n, k, delta, accept, cls,
                     sel, rid, rep, min_delta, min_acc8);
  hipLaunchKernelGGL(k_pack_bits, dim3(grid_for((n + 7) / 8, kBlock)), dim3(kBlock), 0, s, rid + nb, min_acc8,
                     min_acc);
}

void launch_prep_scan(unsigned long long* scan_status, uint32_t ntiles, Ctrl* ctrl, hipStream_t s) {
  uint32_t grid = grid_for(ntiles ? ntiles : 1, kBlock);
  hipLaunchKernelGGL(k_prep_scan, dim3(grid), dim3(kBlock), 0, s, scan_status, ntiles, ctrl);
}

void launch_scan_reps(const uint32_t* block, uint32_t N, uint32_t* rank, Ctrl* ctrl,
                      unsigned long long* scan_status, int items, hipStream_t s) {
  if (!N) return;
  const dim3 grid(scan_tiles(N, items));
  if (items == kScanItemsLarge)
    hipLaunchKernelGGL(k_scan_reps<kScanItemsLarge>, grid, dim3(kBlock), 0, s, block, N, rank, ctrl,
                       scan_status);
  else
    hipLaunchKernelGGL(k_scan_reps<kScanItemsSmall>, grid, dim3(kBlock), 0, s, block, N, rank, ctrl,
                       scan_status);
}

void launch_emit(bool batch, uint32_t N, const uint32_t* inst_of, const InstDesc* desc,
                 const uint32_t* block, const uint32_t* rank, hipStream_t s) {
  if (!N) return;
  if (batch)
    hipLaunchKernelGGL(k_emit<true>, dim3(grid_for(N, kBlock)), dim3(kBlock), 0, s, N, inst_of, desc,
                       block, rank);
  else
    hipLaunchKernelGGL(k_emit<false>, dim3(grid_for(N, kBlock)), dim3(kBlock), 0, s, N, inst_of, desc,
                       block, rank);
}

void launch_results(uint32_t ninst, const InstDesc* desc, const uint32_t* rank,
                    const uint32_t* refine_cnt, ResultDev* res, hipStream_t s) {
  if (!ninst) return;
  hipLaunchKernelGGL(k_results, dim3(grid_for(ninst, kBlock)), dim3(kBlock), 0, s, ninst, desc, rank,
                     refine_cnt, res);
}

}  // namespace dfamin
