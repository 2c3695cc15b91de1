// closure.hip -- host side of the closure construction (Algorithm 5).
#include "closure.h"

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>

#include "../../include/dfamin.h"

namespace dfamin {

int build_closure_levels(std::vector<ClosureSpec>& specs, const ClosureScratch& scratch,
                         hipStream_t s, std::vector<std::vector<uint64_t>>& rows,
                         std::vector<uint32_t>& depth) {
  const size_t W = specs.size();
  rows.assign(W, {});
  depth.assign(W, 0);
  // per (spec, letter): the last kept row and whether the letter is still open
  std::vector<std::vector<uint64_t>> last(W);
  std::vector<std::vector<uint8_t>> open(W);
  for (size_t w = 0; w < W; ++w) {
    const ClosureSpec& sp = specs[w];
    last[w].resize(sp.letters.size());
    open[w].assign(sp.letters.size(), sp.L > 0 ? 1 : 0);
    rows[w].resize(sp.letters.size());
    for (size_t x = 0; x < sp.letters.size(); ++x)
      last[w][x] = reinterpret_cast<uint64_t>(sp.delta) + 4ull * sp.letters[x] * sp.n;
  }
  // rows[w] is built per letter first, then flattened letter by letter
  std::vector<std::vector<std::vector<uint64_t>>> kept(W);
  for (size_t w = 0; w < W; ++w) {
    kept[w].resize(specs[w].letters.size());
    for (size_t x = 0; x < specs[w].letters.size(); ++x) kept[w][x].push_back(last[w][x]);
  }
  struct Pending { uint32_t w, x, level; };
  uint32_t level = 0, batch = 1;
  const bool trace = std::getenv("DFAMIN_TRACE") != nullptr;
  auto now = [] { return std::chrono::steady_clock::now(); };
  auto us = [](auto a, auto b) { return std::chrono::duration<double, std::micro>(b - a).count(); };
  while (true) {
    const auto t0 = now();
    // levels level+1 .. level+batch for every open letter
    std::vector<RowJob> jobs;
    std::vector<uint32_t> joboff;
    std::vector<Pending> who;
    std::vector<uint32_t> lvl_begin, lvl_wgs;
    size_t words = 0;
    for (uint32_t b = 1; b <= batch; ++b)
      for (size_t w = 0; w < W; ++w)
        if (specs[w].L >= level + b)
          for (size_t x = 0; x < specs[w].letters.size(); ++x)
            if (open[w][x]) words += specs[w].n;
    if (words == 0) break;
    uint32_t* store = static_cast<uint32_t*>(scratch.level_storage(words * 4));
    if (!store) break;  // no room for more levels: keep what is built
    size_t off = 0;
    std::vector<std::vector<uint64_t>> src = last;
    uint32_t max_wgs = 0;
    for (uint32_t b = 1; b <= batch; ++b) {
      lvl_begin.push_back((uint32_t)jobs.size());
      uint32_t wgs = 0;
      for (size_t w = 0; w < W; ++w) {
        if (specs[w].L < level + b) continue;
        for (size_t x = 0; x < specs[w].letters.size(); ++x) {
          if (!open[w][x]) continue;
          RowJob J;
          J.src = src[w][x];
          J.dst = reinterpret_cast<uint64_t>(store + off);
          J.n = specs[w].n;
          J.flag_idx = (uint32_t)jobs.size();
          off += specs[w].n;
          src[w][x] = J.dst;
          joboff.push_back(wgs);
          wgs += (J.n + kRowTile - 1) / kRowTile;
          jobs.push_back(J);
          who.push_back({(uint32_t)w, (uint32_t)x, level + b});
        }
      }
      lvl_wgs.push_back(wgs);
      max_wgs = std::max(max_wgs, wgs);
    }
    lvl_begin.push_back((uint32_t)jobs.size());
    RowJob* d_jobs = static_cast<RowJob*>(scratch.ensure(0, jobs.size() * sizeof(RowJob)));
    uint32_t* d_off = static_cast<uint32_t*>(scratch.ensure(1, joboff.size() * 4));
    uint32_t* d_flags = static_cast<uint32_t*>(scratch.ensure(2, jobs.size() * 4));
    uint32_t* d_wg = static_cast<uint32_t*>(scratch.ensure(3, (size_t)max_wgs * 4));
    uint32_t* h_flags = static_cast<uint32_t*>(scratch.host_flags(jobs.size() * 4));
    if (!d_jobs || !d_off || !d_flags || !d_wg || !h_flags) return DFAMIN_E_NOMEM;
    auto up = [&](void* d, const void* h, size_t bytes) {
      return scratch.upload ? scratch.upload(d, h, bytes)
                            : hipMemcpyAsync(d, h, bytes, hipMemcpyHostToDevice, s) == hipSuccess;
    };
    if (!up(d_jobs, jobs.data(), jobs.size() * sizeof(RowJob)) || !up(d_off, joboff.data(), joboff.size() * 4))
      return DFAMIN_E_DEVICE;
    for (uint32_t b = 0; b < batch; ++b) {
      const uint32_t lb = lvl_begin[b], le = lvl_begin[b + 1];
      if (lb == le) continue;
      launch_closure_level(d_jobs + lb, d_off + lb, le - lb, lvl_wgs[b], d_wg, d_flags + lb, s);
    }
    if (hipGetLastError() != hipSuccess) return DFAMIN_E_DEVICE;
    const auto t1 = now();
    const bool copied = scratch.flags_to_host
                            ? scratch.flags_to_host(d_flags, jobs.size() * 4)
                            : hipMemcpyAsync(h_flags, d_flags, jobs.size() * 4, hipMemcpyDeviceToHost, s) == hipSuccess;
    if (!copied || stream_wait(s) != hipSuccess) return DFAMIN_E_DEVICE;
    if (trace)
      std::fprintf(stderr, "[dfamin] closure levels %u..%u: %zu jobs, %zu words, host %.0f us, device wait %.0f us\n",
                   level + 1, level + batch, jobs.size(), words, us(t0, t1), us(t1, now()));
    // keep each letter's levels in order up to its first equal/identity one
    for (size_t j = 0; j < who.size(); ++j) {
      const Pending& p = who[j];
      if (!open[p.w][p.x]) continue;
      const uint32_t f = h_flags[j];
      if (!(f & kFlagDiffers) || !(f & kFlagNonId)) {
        open[p.w][p.x] = 0;
        continue;
      }
      kept[p.w][p.x].push_back(jobs[j].dst);
      last[p.w][p.x] = jobs[j].dst;
    }
    level += batch;
    batch *= 2;
  }
  for (size_t w = 0; w < W; ++w) {
    rows[w].clear();
    for (auto& kx : kept[w]) rows[w].insert(rows[w].end(), kx.begin(), kx.end());
    // depth: L, unless letters were still open when building stopped
    bool any_open = false;
    for (size_t x = 0; x < specs[w].letters.size(); ++x) any_open |= open[w][x] && level < specs[w].L;
    depth[w] = any_open ? std::min(level, specs[w].L) : specs[w].L;
  }
  return DFAMIN_OK;
}

}  // namespace dfamin
