// serving.hip -- continuous-batching request loop (placeholder: not yet wired).
#include "serving.h"

#include "engine.h"

namespace dfamin {

struct Serving::Impl {};

Serving::Serving(Context*) : impl_(new Impl) {}
Serving::~Serving() { delete impl_; }
int Serving::submit(const dfamin_dfa&, const dfamin_opts&, uint64_t*) { return DFAMIN_E_INTERNAL; }
int Serving::wait(uint64_t, int64_t, uint32_t*, dfamin_result*) { return DFAMIN_E_INTERNAL; }
int Serving::cancel(uint64_t) { return DFAMIN_E_INTERNAL; }

}  // namespace dfamin
