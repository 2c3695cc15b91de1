// serving.h -- continuous-batching request loop of one context.
#pragma once

#include <stdint.h>

#include "../../include/dfamin.h"

namespace dfamin {

class Context;

class Serving {
 public:
  explicit Serving(Context* ctx);
  ~Serving();
  int submit(const dfamin_dfa& dfa, const dfamin_opts& opts, uint64_t* ticket);
  int wait(uint64_t ticket, int64_t timeout_us, uint32_t* out, dfamin_result* result);
  int cancel(uint64_t ticket);

 private:
  struct Impl;
  Impl* impl_;
};

}  // namespace dfamin
