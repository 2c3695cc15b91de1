// closure.hip -- host side of the closure construction (Algorithm 5).
#include "closure.h"

#include <algorithm>

#include "../../include/dfamin.h"

namespace dfamin {

int build_closure_levels(std::vector<ClosureSpec>& specs, const ClosureScratch& scratch,
                         hipStream_t s, std::vector<std::vector<uint64_t>>& rows) {
  rows.assign(specs.size(), {});
  uint32_t Lmax = 0;
  for (auto& sp : specs) Lmax = std::max(Lmax, sp.L);
  auto row_ptr = [&](size_t w, size_t x, uint32_t l) -> uint64_t {
    const ClosureSpec& sp = specs[w];
    if (l == 0) return reinterpret_cast<uint64_t>(sp.delta) + 4ull * sp.letters[x] * sp.n;
    return reinterpret_cast<uint64_t>(sp.storage) + 4ull * ((uint64_t)x * sp.L + (l - 1)) * sp.n;
  };
  // jobs grouped by level; each level's workgroups are numbered from 0
  std::vector<RowJob> jobs;
  std::vector<uint32_t> joboff;
  std::vector<uint32_t> lvl_begin(Lmax + 2, 0), lvl_wgs(Lmax + 2, 0);
  std::vector<std::vector<std::vector<int64_t>>> job_of(specs.size());
  for (size_t w = 0; w < specs.size(); ++w)
    job_of[w].assign(specs[w].letters.size(), std::vector<int64_t>(specs[w].L + 1, -1));
  uint32_t max_wgs = 0;
  for (uint32_t l = 1; l <= Lmax; ++l) {
    lvl_begin[l] = (uint32_t)jobs.size();
    uint32_t wgs = 0;
    for (size_t w = 0; w < specs.size(); ++w) {
      if (specs[w].L < l) continue;
      for (size_t x = 0; x < specs[w].letters.size(); ++x) {
        RowJob J;
        J.src = row_ptr(w, x, l - 1);
        J.dst = row_ptr(w, x, l);
        J.n = specs[w].n;
        J.flag_idx = (uint32_t)jobs.size();
        job_of[w][x][l] = (int64_t)jobs.size();
        joboff.push_back(wgs);
        wgs += (J.n + kRowTile - 1) / kRowTile;
        jobs.push_back(J);
      }
    }
    lvl_wgs[l] = wgs;
    max_wgs = std::max(max_wgs, wgs);
  }
  lvl_begin[Lmax + 1] = (uint32_t)jobs.size();
  const uint32_t* flags = nullptr;
  if (!jobs.empty()) {
    RowJob* d_jobs = static_cast<RowJob*>(scratch.ensure(0, jobs.size() * sizeof(RowJob)));
    uint32_t* d_off = static_cast<uint32_t*>(scratch.ensure(1, joboff.size() * 4));
    uint32_t* d_flags = static_cast<uint32_t*>(scratch.ensure(2, jobs.size() * 4));
    uint32_t* d_wg = static_cast<uint32_t*>(scratch.ensure(3, (size_t)max_wgs * 4));
    uint32_t* h_flags = static_cast<uint32_t*>(scratch.host_flags(jobs.size() * 4));
    if (!d_jobs || !d_off || !d_flags || !d_wg || !h_flags) return DFAMIN_E_NOMEM;
    if (hipMemcpyAsync(d_jobs, jobs.data(), jobs.size() * sizeof(RowJob), hipMemcpyHostToDevice, s) !=
            hipSuccess ||
        hipMemcpyAsync(d_off, joboff.data(), joboff.size() * 4, hipMemcpyHostToDevice, s) != hipSuccess)
      return DFAMIN_E_DEVICE;
    for (uint32_t l = 1; l <= Lmax; ++l) {
      const uint32_t b = lvl_begin[l], e = lvl_begin[l + 1];
      if (b == e) continue;
      launch_closure_level(d_jobs + b, d_off + b, e - b, lvl_wgs[l], d_wg, d_flags + b, s);
    }
    if (hipGetLastError() != hipSuccess) return DFAMIN_E_DEVICE;
    if (hipMemcpyAsync(h_flags, d_flags, jobs.size() * 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
        stream_wait(s) != hipSuccess)
      return DFAMIN_E_DEVICE;
    flags = h_flags;
  }
  for (size_t w = 0; w < specs.size(); ++w) {
    for (size_t x = 0; x < specs[w].letters.size(); ++x) {
      rows[w].push_back(row_ptr(w, x, 0));
      for (uint32_t l = 1; l <= specs[w].L; ++l) {
        const int64_t j = job_of[w][x][l];
        if (j < 0) break;
        const uint32_t f = flags[j];
        if (!(f & kFlagDiffers) || !(f & kFlagNonId)) break;
        rows[w].push_back(row_ptr(w, x, l));
      }
    }
  }
  return DFAMIN_OK;
}

}  // namespace dfamin
