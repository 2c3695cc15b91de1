// fused.hip -- the whole minimization of a small instance in one workgroup.
//
// An instance of up to 16,384 states keeps its partition (block id = least
// member state, 16 bits), the closure level a doubling round reads, and the
// grouping table of a round in LDS.  One workgroup runs validation, the
// initial partition {F, Q\F}, every signature round (Section 3.3,
// Algorithm 4: group equal (own block, successor blocks) signatures, new id =
// least member, stop when the block count does not grow) and the canonical
// numbering, with barriers between the steps and no host decision between
// rounds.  The transition rows stay in global memory (they are read once per
// round and the second time from L2).
//
// Rounds follow the round engine exactly, so both give the same partition
// and the same counts:
//   * closure OFF: rounds over the non-identity letters;
//   * closure AUTO with one non-identity letter a: doubling rounds.  From
//     P_j the round gathers the level a^(2^l), 2^l <= j+1 (l capped at L),
//     which gives P_(j+2^l); each level is the square of the previous one
//     (pointer jumping, Section 3.4, Algorithm 5), computed in LDS in the
//     round that first reads it;
//   * closure AUTO with two or more non-identity letters: plain rounds; an
//     instance still splitting after auto_rounds rounds is handed back
//     (kFusedHandOff) and the caller runs it through the round engine,
//     which then builds its closure letters.
#include "../../include/dfamin.h"
#include "internal.h"

namespace dfamin {

namespace {

constexpr uint32_t kNone = 0xFFFFFFFFu;

__device__ __forceinline__ uint32_t wave_or(uint32_t v) {
  for (int o = 32; o > 0; o >>= 1) v |= __shfl_xor(v, o);
  return v;
}
__device__ __forceinline__ uint32_t wave_min(uint32_t v) {
  for (int o = 32; o > 0; o >>= 1) v = min(v, (uint32_t)__shfl_xor(v, o));
  return v;
}
__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}
// inclusive prefix sum over the wave's lanes
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
  const uint32_t lane = threadIdx.x & 63u;
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t t = __shfl_up(v, o);
    if (lane >= (uint32_t)o) v += t;
  }
  return v;
}

__device__ __forceinline__ uint32_t mix_step(uint32_t h, uint32_t c) {
  h = (h ^ c) * 0x9E3779B1u;
  return h ^ (h >> 15);
}
__device__ __forceinline__ uint32_t mix_final(uint32_t h) {
  h ^= h >> 13;
  h *= 0x85EBCA6Bu;
  return h ^ (h >> 16);
}

// The grouping table is probed a bucket of kBucket consecutive slots at a
// time (one 16-byte LDS read): a state looks for its group among the
// bucket's occupied slots and otherwise claims the bucket's first empty
// slot, moving on to the next bucket only when one is full.  A wave then
// waits for few probe steps, where single-slot linear probing at this load
// factor lets one lane of the wave run through a long cluster.
constexpr uint32_t kBucket = 4;
// states of a thread whose successors are loaded together (one or two
// signature letters)
constexpr int kChunk = 4;

// Slot word: bits 31..16 a 16-bit fragment of the signature hash, bits
// 15..1 the least state id + 1 of the group, bit 0 set once a second state
// joined it (0 = empty slot).
constexpr uint32_t kFragShift = 16;
constexpr uint32_t kIdMask = 0x7FFFu;  // (word >> 1) & kIdMask = least id + 1
constexpr uint32_t kShared = 1u;
// blk[q]: bits 13..0 the block id (least member), bit 15 set when that block
// is a single state, which can never split again: such a state skips the
// grouping of later rounds and stays its own block.
constexpr uint16_t kSingle = 0x8000u;
constexpr uint16_t kBlkMask = 0x3FFFu;

template <int MAXN, int NT>
__global__ void __launch_bounds__(NT) k_fused(const FusedJob* __restrict__ jobs, FusedRes* __restrict__ res,
                                              uint32_t njobs, FusedJob one) {
  static_assert(MAXN % NT == 0 && MAXN <= (1 << 14) && (MAXN / NT) % kChunk == 0, "fused tile: ids fit 14 bits");
  static_assert(MAXN / NT <= 32, "accept bits of a thread's states fit one word");
  static_assert(((3u * MAXN) / 2u - 64u) % kBucket == 0, "table of whole buckets");
  constexpr int ITEMS = MAXN / NT;
  constexpr uint32_t NW = NT / 64;
  // table slots: load factor at most 2/3; 64 slots fewer than 1.5 MAXN
  // leave room for the shared words in 160 KB at MAXN = 16,384
  constexpr uint32_t SMAX = (3u * MAXN) / 2u - 64u;
  __shared__ uint16_t blk[MAXN];   // block id (least member) per state
  __shared__ uint16_t lvl[MAXN];   // doubling: the closure level a^(2^built)
  __shared__ __align__(16) uint32_t slot[SMAX];  // grouping table (buckets of kBucket slots); ranks at the end
  __shared__ uint32_t sh[64];      // 0 bad, 1 non-identity letters, 2 min F, 3 min Q\F,
                                   // 4/5 leaders (alternate rounds), 6 fault, 32.. wave totals
  const uint32_t j = blockIdx.x;
  if (j >= njobs) return;
  const FusedJob J = jobs ? jobs[j] : one;  // one job may come as an argument
  const uint32_t n = J.n, k = J.k, tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6;
  const uint32_t* __restrict__ delta = reinterpret_cast<const uint32_t*>(J.delta);
  const uint8_t* __restrict__ acc = reinterpret_cast<const uint8_t*>(J.accept);
  FusedRes R{};
  if (tid == 0) {
    sh[0] = 0;
    sh[1] = 0;
    sh[2] = kNone;
    sh[3] = kNone;
    sh[4] = sh[5] = sh[6] = 0;
  }
  __syncthreads();

  // ---- validation (every entry < n) and identity letters (Section 2).
  // Thread tid owns states tid + i*NT, i < ITEMS (n <= MAXN); its loads of
  // one row go out together, so each row costs one memory latency.
  uint32_t fbits = 0;  // accept bit of owned state i in bit i
  {
    uint32_t bad = 0, nonid = 0;
    for (uint32_t a = 0; a < k; ++a) {
      const uint32_t* __restrict__ row = delta + (size_t)a * n;
      uint32_t v[ITEMS];
#pragma unroll
      for (int i = 0; i < ITEMS; ++i) {
        const uint32_t q = tid + (uint32_t)i * NT;
        v[i] = q < n ? row[q] : q;
      }
      uint32_t d = 0;
#pragma unroll
      for (int i = 0; i < ITEMS; ++i) {
        const uint32_t q = tid + (uint32_t)i * NT;
        bad |= (uint32_t)(q < n && v[i] >= n);
        d |= (uint32_t)(v[i] != q);
      }
      if (d) nonid |= 1u << a;
    }
    uint8_t ab[ITEMS];
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
      const uint32_t q = tid + (uint32_t)i * NT;
      ab[i] = q < n ? acc[q >> 3] : 0u;
    }
    uint32_t mf = kNone, mn = kNone;
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
      const uint32_t q = tid + (uint32_t)i * NT;
      if (q >= n) continue;
      if ((ab[i] >> (q & 7)) & 1u) {
        mf = min(mf, q);
        fbits |= 1u << i;
      } else {
        mn = min(mn, q);
      }
    }
    bad = wave_or(bad);
    nonid = wave_or(nonid);
    mf = wave_min(mf);
    mn = wave_min(mn);
    if (lane == 0) {
      if (bad) atomicOr(&sh[0], 1u);
      if (nonid) atomicOr(&sh[1], nonid);
      atomicMin(&sh[2], mf);
      atomicMin(&sh[3], mn);
    }
  }
  __syncthreads();
  if (sh[0]) {  // the same for every thread: the output is not touched
    if (tid == 0) {
      R.status = kFusedBad;
      res[j] = R;
    }
    return;
  }
  const uint32_t mask = sh[1];
  const uint32_t knon = __popc(mask);
  const bool autom = J.closure == DFAMIN_CLOSURE_AUTO;
  const bool dbl = autom && knon == 1;
  const uint32_t minF = sh[2], minN = sh[3];
  // the first two non-identity letters
  const uint32_t l0 = mask ? (uint32_t)__ffs(mask) - 1u : 0u;
  const uint32_t m1 = mask & (mask - 1u);
  const uint32_t l1 = m1 ? (uint32_t)__ffs(m1) - 1u : 0u;
  // ---- initial partition {F, Q\F}; ids are least members (Section 3.2)
  uint32_t count = (minF < n ? 1u : 0u) + (minN < n ? 1u : 0u);
#pragma unroll
  for (int i = 0; i < ITEMS; ++i) {
    const uint32_t q = tid + (uint32_t)i * NT;
    if (q >= n) continue;
    const bool f = (fbits >> i) & 1u;
    blk[q] = (uint16_t)(f ? minF : minN);
    // a doubling instance keeps its closure level in lvl[]; any other
    // starts with its accept bit there, the exact label of its class
    lvl[q] = dbl ? (uint16_t)delta[(size_t)l0 * n + q] : (uint16_t)f;
  }
  // > n slots, so an empty one always exists
  const uint32_t S = min(SMAX, max(64u, (n + n / 2u + kBucket - 1u) & ~(kBucket - 1u)));
  const uint32_t NB = S / kBucket;  // < 2^16: the bucket comes from the low half of the hash,
                                    // the fragment from the high half
  uint32_t rounds = 0, refine = 0, built = 0, used = 0;
  uint64_t jlen = 0;  // this partition is P_jlen (states agree on words of length <= jlen)
  // Exact-key rounds: while the signature in labels of lw bits each (block
  // numbers 0..B-1, or the accept bit in the first round) fits in
  // floor(log2 S) bits, it is itself the slot index: no hashing, no
  // comparison of signatures.  lvl[] then holds each state's label.
  const uint32_t lgS = 31u - (uint32_t)__clz(S);
  uint32_t lw = 1;
  // a direct round needs 2^bits table slots and n 16-bit keys behind them
  auto fits_direct = [&](uint32_t bits) {
    return !dbl && bits <= lgS && bits <= 14u && (4u << bits) + 2u * n <= 4u * SMAX;
  };
  bool direct_next = fits_direct((knon + 1u) * lw);
  // rank of each block's least member among the least members (states in
  // order), into slot[p] for every state p
  auto rank_leaders = [&]() {
    const uint32_t base = tid * (uint32_t)ITEMS;
    uint32_t c = 0;
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
      const uint32_t p = base + (uint32_t)i;
      if (p < n && (blk[p] & kBlkMask) == p) ++c;
    }
    const uint32_t incl = wave_incl_scan(c);
    if (lane == 63) sh[32 + wave] = incl;
    __syncthreads();
    uint32_t off = 0;
    for (uint32_t w = 0; w < wave; ++w) off += sh[32 + w];
    uint32_t r = off + incl - c;
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
      const uint32_t p = base + (uint32_t)i;
      if (p < n) {
        slot[p] = r;
        if ((blk[p] & kBlkMask) == p) ++r;
      }
    }
    __syncthreads();
  };
  int32_t status = kFusedOk;
  __syncthreads();

  // ---- rounds
  while (true) {
    if (autom && !dbl && knon >= 2 && rounds == J.auto_rounds) {
      status = kFusedHandOff;  // still splitting: its closure letters come from the round engine
      break;
    }
    if (rounds >= J.max_rounds) {
      status = kFusedRoundCap;
      break;
    }
    uint32_t l = 0;
    if (dbl) {
      l = 63u - (uint32_t)__clzll(jlen + 1ull);
      if (l > J.levels) l = J.levels;
      for (; built < l; ++built) {  // level built+1 = level built, squared
        uint16_t nxt[ITEMS];
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
          const uint32_t q = tid + (uint32_t)i * NT;
          if (q < n) nxt[i] = lvl[lvl[q]];
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
          const uint32_t q = tid + (uint32_t)i * NT;
          if (q < n) lvl[q] = nxt[i];
        }
        __syncthreads();
      }
    }
    const bool direct = direct_next;
    const uint32_t T = direct ? 1u << ((knon + 1u) * lw) : S;  // slots this round uses
    for (uint32_t s = tid; s < T; s += NT) slot[s] = 0;
    if (tid == 0) sh[4 + (rounds & 1u)] = 0;
    __syncthreads();

    // group: each state joins the slot of its signature; the slot keeps the
    // group's least state (a hash fragment match is always confirmed on the
    // full signature)
    // a direct round keeps each state's key behind the table, 16 bits each
    uint16_t* const keyat = reinterpret_cast<uint16_t*>(slot + T);
    if (direct) {
      // with one or two signature letters the successors of kChunk states
      // of the thread are loaded together, as in the hash rounds
      const bool pre = knon <= 2u;
#pragma unroll 1
      for (int c0 = 0; c0 < ITEMS; c0 += kChunk) {
      uint32_t pf[kChunk];
      if (pre) {
#pragma unroll
        for (int i = 0; i < kChunk; ++i) {
          const uint32_t q = tid + (uint32_t)(c0 + i) * NT;
          pf[i] = 0;
          if (q < n && knon > 0u) {
            pf[i] = delta[(size_t)l0 * n + q];
            if (knon > 1u) pf[i] |= delta[(size_t)l1 * n + q] << 16;
          }
        }
      }
#pragma unroll
      for (int i = 0; i < kChunk; ++i) {
        const uint32_t q = tid + (uint32_t)(c0 + i) * NT;
        if (q >= n || (blk[q] & kSingle)) continue;
        uint32_t key = lvl[q];
        if (pre) {
          if (knon > 0u) key |= (uint32_t)lvl[pf[i] & 0xFFFFu] << lw;
          if (knon > 1u) key |= (uint32_t)lvl[pf[i] >> 16] << (2u * lw);
        } else {
          uint32_t at = lw;
          for (uint32_t mm = mask; mm; mm &= mm - 1u, at += lw)
            key |= (uint32_t)lvl[delta[(size_t)(__ffs(mm) - 1) * n + q]] << at;
        }
        keyat[q] = (uint16_t)key;
        const uint32_t want = (q + 1u) << 1;
        uint32_t v = slot[key];
        if (v == 0) {
          v = atomicCAS(&slot[key], 0u, want);
          if (v == 0) continue;  // a new group
        }
        if (((v >> 1) & kIdMask) - 1u > q) atomicMin(&slot[key], want | kShared);
        else if (!(v & kShared)) atomicOr(&slot[key], kShared);
      }
      }
    } else {
    // (a plain instance keeps each state's slot in lvl[], which only
    // doubling instances use; a doubling instance finds it again below).
    // With one or two signature letters, the successors of kChunk states of
    // the thread are loaded together first, packed two to a word.
    const bool pre = !dbl && knon <= 2u;
#pragma unroll 1
    for (int c0 = 0; c0 < ITEMS; c0 += kChunk) {
    uint32_t pf[kChunk];
    if (pre) {
#pragma unroll
      for (int i = 0; i < kChunk; ++i) {
        const uint32_t q = tid + (uint32_t)(c0 + i) * NT;
        pf[i] = 0;
        if (q < n && knon > 0u) {
          pf[i] = delta[(size_t)l0 * n + q];
          if (knon > 1u) pf[i] |= delta[(size_t)l1 * n + q] << 16;
        }
      }
    }
#pragma unroll
    for (int i = 0; i < kChunk; ++i) {
      const uint32_t q = tid + (uint32_t)(c0 + i) * NT;
      if (q >= n || (blk[q] & kSingle)) continue;
      const uint32_t own = blk[q];
      uint32_t h = mix_step(0x6A09E667u, own);
      if (dbl) {
        h = mix_step(h, blk[lvl[q]] & kBlkMask);
      } else if (pre) {
        if (knon > 0u) h = mix_step(h, blk[pf[i] & 0xFFFFu] & kBlkMask);
        if (knon > 1u) h = mix_step(h, blk[pf[i] >> 16] & kBlkMask);
      } else {
        for (uint32_t mm = mask; mm; mm &= mm - 1u) {
          const uint32_t a = (uint32_t)__ffs(mm) - 1u;
          h = mix_step(h, blk[delta[(size_t)a * n + q]] & kBlkMask);
        }
      }
      h = mix_final(h);
      const uint32_t frag = h >> kFragShift;
      const uint32_t want = (frag << kFragShift) | ((q + 1u) << 1);
      // the full signature of r equals that of q
      auto same_as = [&](uint32_t r) {
        if (blk[r] != own) return false;
        if (dbl) return (blk[lvl[r]] & kBlkMask) == (blk[lvl[q]] & kBlkMask);
        if (pre) {
          bool eq = true;
          if (knon > 0u)
            eq = (blk[delta[(size_t)l0 * n + r]] & kBlkMask) == (blk[pf[i] & 0xFFFFu] & kBlkMask);
          if (knon > 1u)
            eq = eq && (blk[delta[(size_t)l1 * n + r]] & kBlkMask) == (blk[pf[i] >> 16] & kBlkMask);
          return eq;
        }
        for (uint32_t mm = mask; mm; mm &= mm - 1u) {
          const uint32_t a = (uint32_t)__ffs(mm) - 1u;
          if ((blk[delta[(size_t)a * n + r]] & kBlkMask) != (blk[delta[(size_t)a * n + q]] & kBlkMask))
            return false;
        }
        return true;
      };
      uint32_t b = (((h & 0xFFFFu) * NB) >> 16);
      uint32_t pos = 0;
      for (uint32_t steps = 0;; ++steps) {
        if (steps >= (kBucket + 1u) * NB) {  // cannot happen (S > n); bounded all the same
          sh[6] = 1;
          break;
        }
        const uint4 w0 = *reinterpret_cast<const uint4*>(&slot[b * kBucket]);
        const uint32_t w[kBucket] = {w0.x, w0.y, w0.z, w0.w};
        uint32_t cand = 0, empties = 0;
#pragma unroll
        for (int j = 0; j < (int)kBucket; ++j) {
          if (w[j] == 0) empties |= 1u << j;
          else if ((w[j] >> kFragShift) == frag) cand |= 1u << j;
        }
        int hit = -1;
        for (; cand; cand &= cand - 1u) {  // fragment matches, confirmed on the full signature
          const int j = __ffs(cand) - 1;
          // (an occupied slot changes only to a lower member of its group)
          if (same_as(((slot[b * kBucket + (uint32_t)j] >> 1) & kIdMask) - 1u)) {
            hit = j;
            break;
          }
        }
        const int empty = empties ? __ffs(empties) - 1 : -1;
        if (hit >= 0) {  // the group exists: mark it shared and keep its least member
          pos = b * kBucket + (uint32_t)hit;
          const uint32_t v = slot[pos];
          if (((v >> 1) & kIdMask) - 1u > q) atomicMin(&slot[pos], want | kShared);  // same fragment
          else if (!(v & kShared)) atomicOr(&slot[pos], kShared);
          break;
        }
        if (empty >= 0) {  // claim the bucket's first empty slot; if another state
                           // took it first, read the bucket again
          pos = b * kBucket + (uint32_t)empty;
          if (atomicCAS(&slot[pos], 0u, want) == 0u) break;
          continue;
        }
        b = (b + 1u == NB) ? 0u : b + 1u;
      }
      if (!dbl) lvl[q] = (uint16_t)pos;
    }
    }
    }
    __syncthreads();
    // new id = the group's least member (with the single-state mark);
    // count the groups
    uint32_t leaders = 0;
    if (direct) {
#pragma unroll 1
      for (int i = 0; i < ITEMS; ++i) {
        const uint32_t q = tid + (uint32_t)i * NT;
        if (q >= n) continue;
        if (blk[q] & kSingle) {
          ++leaders;
          continue;
        }
        const uint32_t v = slot[keyat[q]];
        const uint32_t nb = ((v >> 1) & kIdMask) - 1u;
        blk[q] = (uint16_t)(nb | ((v & kShared) ? 0u : kSingle));
        leaders += (uint32_t)(nb == q);
      }
    } else if (!dbl) {
#pragma unroll 1
      for (int i = 0; i < ITEMS; ++i) {
        const uint32_t q = tid + (uint32_t)i * NT;
        if (q >= n) continue;
        if (blk[q] & kSingle) {
          ++leaders;
          continue;
        }
        const uint32_t v = slot[lvl[q]];
        const uint32_t nb = ((v >> 1) & kIdMask) - 1u;
        blk[q] = (uint16_t)(nb | ((v & kShared) ? 0u : kSingle));
        leaders += (uint32_t)(nb == q);
      }
    } else {
      // the slot of each state's signature (own block, block of its level
      // successor), found again by the same probe; blocks change only
      // after every state has found its slot
      uint16_t nbs[ITEMS];
#pragma unroll
      for (int i = 0; i < ITEMS; ++i) {
        const uint32_t q = tid + (uint32_t)i * NT;
        nbs[i] = 0;
        if (q >= n || (blk[q] & kSingle)) continue;
        const uint32_t own = blk[q], succ = blk[lvl[q]] & kBlkMask;
        const uint32_t h = mix_final(mix_step(mix_step(0x6A09E667u, own), succ));
        const uint32_t frag = h >> kFragShift;
        uint32_t b = (((h & 0xFFFFu) * NB) >> 16);
        for (uint32_t probes = 0; probes < S; ++probes) {
          const uint32_t v = slot[b * kBucket + (probes % kBucket)];
          if (v && (v >> kFragShift) == frag) {
            const uint32_t r = ((v >> 1) & kIdMask) - 1u;
            if (blk[r] == own && (blk[lvl[r]] & kBlkMask) == succ) {
              nbs[i] = (uint16_t)(r | ((v & kShared) ? 0u : kSingle));
              break;
            }
          }
          if (probes % kBucket == kBucket - 1u) b = (b + 1u == NB) ? 0u : b + 1u;
        }
      }
      __syncthreads();
#pragma unroll
      for (int i = 0; i < ITEMS; ++i) {
        const uint32_t q = tid + (uint32_t)i * NT;
        if (q >= n) continue;
        if (blk[q] & kSingle) {
          ++leaders;
          continue;
        }
        blk[q] = nbs[i];
        leaders += (uint32_t)((nbs[i] & kBlkMask) == q);
      }
    }
    leaders = wave_sum(leaders);
    if (lane == 0) atomicAdd(&sh[4 + (rounds & 1u)], leaders);
    __syncthreads();
    const uint32_t cnew = sh[4 + (rounds & 1u)];
    ++rounds;
    if (sh[6]) {
      status = kFusedFault;
      break;
    }
    if (cnew == count) break;  // no block split: stable
    ++refine;
    used = max(used, l);  // the highest level a splitting round read
    count = cnew;
    jlen += dbl ? (1ull << l) : 1ull;
    if (count == n) break;  // every block a singleton: stable without another round
    // the next round's labels: block numbers, if its signature fits
    const uint32_t wn = max(1u, 32u - (uint32_t)__clz(count - 1u));
    direct_next = fits_direct((knon + 1u) * wn);
    if (direct_next) {
      rank_leaders();
      for (uint32_t q = tid; q < n; q += NT) lvl[q] = (uint16_t)slot[blk[q] & kBlkMask];
      __syncthreads();
      lw = wn;
    }
  }
  if (status != kFusedOk) {
    if (tid == 0) {
      R.status = status;
      res[j] = R;
    }
    return;
  }

  // ---- canonical numbering: out[q] = rank of q's block's least member
  rank_leaders();
  uint32_t* __restrict__ out = reinterpret_cast<uint32_t*>(J.out);
  for (uint32_t q = tid; q < n; q += NT) out[q] = slot[blk[q] & kBlkMask];
  if (tid == 0) {
    R.status = kFusedOk;
    R.num_blocks = count;
    R.initial_block = slot[blk[J.q0] & kBlkMask];
    R.refine_rounds = refine;
    R.levels_used = used;
    R.doubling = dbl ? 1u : 0u;
    res[j] = R;
  }
  (void)NW;
}

}  // namespace

void launch_fused(const FusedJob* jobs, FusedRes* res, uint32_t njobs, int cls, hipStream_t s,
                  const FusedJob* one) {
  if (!njobs) return;
  const FusedJob arg = one ? *one : FusedJob{};
  if (one) {
    jobs = nullptr;
    njobs = 1;
  }
  switch (cls) {
    case 0: hipLaunchKernelGGL((k_fused<2048, 256>), dim3(njobs), dim3(256), 0, s, jobs, res, njobs, arg); break;
    case 1: hipLaunchKernelGGL((k_fused<8192, 512>), dim3(njobs), dim3(512), 0, s, jobs, res, njobs, arg); break;
    default:
      hipLaunchKernelGGL((k_fused<16384, 1024>), dim3(njobs), dim3(1024), 0, s, jobs, res, njobs, arg);
      break;
  }
}

}  // namespace dfamin
