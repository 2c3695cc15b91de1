// capi.hip -- the extern "C" boundary of libdfamin (declared in dfamin.h).
//
// Argument checks happen here on the host; everything the method computes
// happens in the kernels driven by Engine.  No exception crosses the ABI.
#include <hip/hip_runtime.h>

#include <cstring>
#include <algorithm>
#include <thread>
#include <atomic>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/dfamin.h"
#include "engine.h"
#include "serving.h"

struct dfamin_ctx {
  dfamin::Context c;
};

// Device memory of dfamin_minimize_device_noalloc: one array per device,
// held from the module's load until the process ends.  In host code its name
// is a host-side stand-in, never a device address: kernels receive the
// address that hipGetSymbolAddress returned for the current device.
static __device__ __align__(256) unsigned char scratch[DFAMIN_NOALLOC_SCRATCH_BYTES];

namespace {

using dfamin::Context;

constexpr int kMaxDevices = 64;
// page-locked bytes of each host buffer of a fixed-region engine (control
// block and result readbacks, job lists, the two upload arenas)
constexpr size_t kFixedHostBytes = 256u << 10;
// the array's last bytes are left out of the region, as a margin behind the
// last carved buffer
constexpr size_t kScratchTail = 64u << 10;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on `device`, which must be current; looked up
// once per device.
int scratch_address(int device, void** out) {
  if (device < 0 || device >= kMaxDevices) return DFAMIN_E_INVAL;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      return DFAMIN_E_DEVICE;
    }
    g_scratch_ptr[device] = p;
  }
  *out = g_scratch_ptr[device];
  return DFAMIN_OK;
}

// Device bytes a single-instance call of dfamin_minimize_device_noalloc may
// carve, per state: block, act, act2, slot_of and nb (4 B each), keep (1),
// rank (4), dense numbers (4), a hash table of up to 2^ceil(log2 2n) 8-byte
// slots (at most 32 B), and signature records of k + 1 words counted four
// times over (the plain letters' records, then those of closure levels,
// which take at most a third of what is left); plus 1 MiB of job lists,
// descriptors and scan status.
uint64_t noalloc_bytes(uint32_t n, uint32_t k) {
  return (uint64_t)n * (66ull + 16ull * ((uint64_t)k + 1)) + (1ull << 20);
}
using dfamin::InstInput;
using dfamin::InstOutcome;

int check_dfa_shape(const dfamin_dfa* d) {
  if (!d || !d->delta || !d->accept) return DFAMIN_E_INVAL;
  if (d->n == 0 || d->k == 0 || d->q0 >= d->n || d->n >= dfamin::kMaxStates) return DFAMIN_E_INVAL;
  if ((uint64_t)d->n * d->k > (1ull << 40)) return DFAMIN_E_INVAL;
  return DFAMIN_OK;
}

int check_opts(const dfamin_opts* o) {
  const bool closure_ok = !o || o->closure == DFAMIN_CLOSURE_AUTO || o->closure == DFAMIN_CLOSURE_OFF ||
                          o->closure == DFAMIN_CLOSURE_ON;
  if (o && (!closure_ok || o->method > DFAMIN_METHOD_LEADER ||
            (o->flags & ~(DFAMIN_FLAG_NO_GRAPH | DFAMIN_FLAG_QUEUE))))
    return DFAMIN_E_INVAL;
  return DFAMIN_OK;
}

dfamin_opts opts_or_default(const dfamin_opts* o) {
  dfamin_opts d{};
  if (o) d = *o;
  return d;
}

void to_result(const InstOutcome& o, dfamin_result* r) {
  if (!r) return;
  r->num_blocks = o.num_blocks;
  r->initial_block = o.initial_block;
  r->refine_rounds = o.refine_rounds;
  r->rounds_executed = o.rounds_executed;
  r->closure_levels = o.closure_levels;
  r->closure_letters = o.closure_letters;
  r->status = o.status;
  r->reserved = 0;
}

int set_device(Context& c) {
  if (c.device_lost) return DFAMIN_E_DEVICE;
  return hipSetDevice(c.device) == hipSuccess ? DFAMIN_OK : DFAMIN_E_DEVICE;
}

int ensure(Context& c, dfamin::DevBuf& b, size_t bytes) {
  if (bytes == 0) bytes = 256;
  if (b.cap >= bytes) return DFAMIN_OK;
  if (b.p) {
    (void)hipFree(b.p);
    c.used -= b.cap;
    b.p = nullptr;
    b.cap = 0;
  }
  size_t want = (bytes + bytes / 8 + 4095) & ~size_t(4095);
  if (c.used + want > c.budget) {
    want = (bytes + 4095) & ~size_t(4095);
    if (c.used + want > c.budget) return DFAMIN_E_NOMEM;
  }
  if (hipMalloc(&b.p, want) != hipSuccess) {
    b.p = nullptr;
    (void)hipGetLastError();
    return DFAMIN_E_NOMEM;
  }
  b.cap = want;
  c.used += want;
  return DFAMIN_OK;
}

int ensure_host(dfamin::HostBuf& b, size_t bytes) {
  if (bytes == 0) bytes = 64;
  if (b.cap >= bytes) return DFAMIN_OK;
  if (b.p) (void)hipHostFree(b.p);
  b.p = nullptr;
  b.cap = 0;
  size_t want = bytes + bytes / 8 + 64;
  if (hipHostMalloc(&b.p, want, hipHostMallocDefault) != hipSuccess) {
    b.p = nullptr;
    return DFAMIN_E_NOMEM;
  }
  b.cap = want;
  return DFAMIN_OK;
}

inline size_t accept_bytes(uint32_t n) { return ((size_t)n + 7) / 8; }
inline size_t align16(size_t x) { return (x + 15) & ~size_t(15); }

// One contiguous host copy of a staged transfer.
struct Piece {
  char* dst;
  const char* src;
  size_t bytes;
  size_t dev_off;  // where the piece goes in device memory (uploads)
};
constexpr size_t kPieceBytes = 4u << 20;

// Runs pieces on up to 8 host threads (fewer for small transfers); each
// piece, once copied, is handed to after(piece) on the same thread.  Threads
// started here make `device` current first (-1: none).  Returns false if any
// after() failed.
template <typename After>
bool run_pieces(const std::vector<Piece>& pieces, size_t total_bytes, int device, After after) {
  const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
  const unsigned nt = (unsigned)std::min<size_t>({8u, hw, (total_bytes + kPieceBytes - 1) / kPieceBytes});
  std::atomic<size_t> next{0};
  std::atomic<bool> ok{true};
  auto work = [&] {
    for (size_t j = next++; j < pieces.size(); j = next++) {
      std::memcpy(pieces[j].dst, pieces[j].src, pieces[j].bytes);
      if (!after(pieces[j])) ok = false;
    }
  };
  if (nt <= 1) {
    work();
  } else {
    std::vector<std::thread> ts;
    for (unsigned t = 1; t < nt; ++t)
      ts.emplace_back([&] {
        if (device >= 0 && hipSetDevice(device) != hipSuccess) {
          ok = false;
          return;
        }
        work();
      });
    work();
    for (auto& t : ts) t.join();
  }
  return ok;
}

// Splits [src, src + bytes) into pieces of at most kPieceBytes.
void add_pieces(std::vector<Piece>& out, char* dst, const char* src, size_t bytes, size_t dev_off) {
  for (size_t o = 0; o < bytes; o += kPieceBytes) {
    const size_t b = std::min(kPieceBytes, bytes - o);
    out.push_back({dst + o, src + o, b, dev_off + o});
  }
}

// Host-input batch: pack every instance into pinned staging, one H2D copy,
// run, one D2H copy, scatter into the caller's buffers.
int run_host_batch(Context& c, uint32_t count, const dfamin_dfa* dfas, const dfamin_opts& o,
                   uint32_t* const* outs, dfamin_result* results) {
  std::vector<size_t> d_off(count), a_off(count), o_off(count);
  size_t in_bytes = 0, out_bytes = 0;
  for (uint32_t i = 0; i < count; ++i) {
    d_off[i] = in_bytes;
    in_bytes = align16(in_bytes + 4ull * dfas[i].n * dfas[i].k);
    a_off[i] = in_bytes;
    in_bytes = align16(in_bytes + accept_bytes(dfas[i].n));
    o_off[i] = out_bytes;
    out_bytes = align16(out_bytes + 4ull * dfas[i].n);
  }
  int rc;
  if ((rc = ensure_host(c.h_in, in_bytes)) != DFAMIN_OK) return rc;
  if ((rc = ensure_host(c.h_out, out_bytes)) != DFAMIN_OK) return rc;
  if ((rc = ensure(c, c.in_delta, in_bytes)) != DFAMIN_OK) return rc;
  if ((rc = ensure(c, c.in_out, out_bytes)) != DFAMIN_OK) return rc;
  // Staging: pieces of the caller's buffers are copied into page-locked
  // memory by several threads, and each piece is uploaded as soon as it is
  // there, so the host copies overlap the transfers (all are queued before
  // any kernel of the call).
  char* hin = c.h_in.as<char>();
  char* din = c.in_delta.as<char>();
  std::vector<Piece> pieces;
  for (uint32_t i = 0; i < count; ++i) {
    add_pieces(pieces, hin + d_off[i], reinterpret_cast<const char*>(dfas[i].delta), 4ull * dfas[i].n * dfas[i].k,
               d_off[i]);
    add_pieces(pieces, hin + a_off[i], reinterpret_cast<const char*>(dfas[i].accept), accept_bytes(dfas[i].n),
               a_off[i]);
  }
  if (!run_pieces(pieces, in_bytes, c.device, [&](const Piece& p) {
        return hipMemcpyAsync(din + p.dev_off, p.dst, p.bytes, hipMemcpyHostToDevice, c.stream) == hipSuccess;
      }))
    return DFAMIN_E_DEVICE;
  std::vector<InstInput> in(count);
  char* dbase = c.in_delta.as<char>();
  char* obase = c.in_out.as<char>();
  for (uint32_t i = 0; i < count; ++i) {
    in[i].n = dfas[i].n;
    in[i].k = dfas[i].k;
    in[i].q0 = dfas[i].q0;
    in[i].closure = o.closure;
    in[i].delta = reinterpret_cast<const uint32_t*>(dbase + d_off[i]);
    in[i].accept = reinterpret_cast<const uint8_t*>(dbase + a_off[i]);
    in[i].out = reinterpret_cast<uint32_t*>(obase + o_off[i]);
  }
  std::vector<InstOutcome> res;
  rc = c.engine.run(in, o, c.stream, res);
  if (rc == DFAMIN_E_BAD_DFA) {
    for (uint32_t i = 0; i < count; ++i) to_result(res[i], results ? &results[i] : nullptr);
    return rc;
  }
  if (rc != DFAMIN_OK) return rc;
  if (hipMemcpyAsync(c.h_out.p, obase, out_bytes, hipMemcpyDeviceToHost, c.stream) != hipSuccess)
    return DFAMIN_E_DEVICE;
  if (hipStreamSynchronize(c.stream) != hipSuccess) return DFAMIN_E_DEVICE;
  const char* hout = c.h_out.as<char>();
  std::vector<Piece> back;
  for (uint32_t i = 0; i < count; ++i) {
    add_pieces(back, reinterpret_cast<char*>(outs[i]), hout + o_off[i], 4ull * dfas[i].n, 0);
    to_result(res[i], results ? &results[i] : nullptr);
  }
  (void)run_pieces(back, out_bytes, -1, [](const Piece&) { return true; });
  return DFAMIN_OK;
}

}  // namespace

extern "C" {

int dfamin_create(int hip_device, uint64_t hbm_budget_bytes, dfamin_ctx** out) {
  if (!out) return DFAMIN_E_INVAL;
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) {
    (void)hipGetLastError();
    return DFAMIN_E_DEVICE;
  }
  if (hip_device < 0 || hip_device >= count) return DFAMIN_E_INVAL;
  if (hipSetDevice(hip_device) != hipSuccess) return DFAMIN_E_DEVICE;
  size_t free_b = 0, total_b = 0;
  if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) return DFAMIN_E_DEVICE;
  dfamin_ctx* ctx = new (std::nothrow) dfamin_ctx;
  if (!ctx) return DFAMIN_E_NOMEM;
  ctx->c.device = hip_device;
  ctx->c.budget = hbm_budget_bytes ? hbm_budget_bytes : (uint64_t)(0.9 * (double)free_b);
  if (hipStreamCreateWithFlags(&ctx->c.stream, hipStreamNonBlocking) != hipSuccess) {
    delete ctx;
    return DFAMIN_E_DEVICE;
  }
  // set-up of dfamin_minimize_device_noalloc, so that the call itself needs
  // no allocation: this device's scratch address, the fixed engine's
  // page-locked host buffers and events, and the tile autotuner's events
  void* sp = nullptr;
  int rc = scratch_address(hip_device, &sp);
  if (rc == DFAMIN_OK) rc = ctx->c.fixed_engine.set_fixed_region(sp, DFAMIN_NOALLOC_SCRATCH_BYTES - kScratchTail,
                                                                kFixedHostBytes);
  if (rc == DFAMIN_OK && !ctx->c.tuner.have_events) {
    for (hipEvent_t& e : ctx->c.tuner.ev)
      if (hipEventCreate(&e) != hipSuccess) rc = DFAMIN_E_DEVICE;
    ctx->c.tuner.have_events = true;
  }
  if (rc != DFAMIN_OK) {
    dfamin_destroy(ctx);
    return rc;
  }
  *out = ctx;
  return DFAMIN_OK;
}

void dfamin_destroy(dfamin_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->c.device);
  if (ctx->c.serving) {
    delete ctx->c.serving;
    ctx->c.serving = nullptr;
  }
  dfamin::DevBuf* bufs[] = {&ctx->c.in_delta, &ctx->c.in_accept, &ctx->c.in_out};
  for (auto* b : bufs)
    if (b->p) (void)hipFree(b->p);
  if (ctx->c.h_in.p) (void)hipHostFree(ctx->c.h_in.p);
  if (ctx->c.h_out.p) (void)hipHostFree(ctx->c.h_out.p);
  if (ctx->c.stream) (void)hipStreamSynchronize(ctx->c.stream);
  if (ctx->c.tuner.have_events) {
    (void)hipDeviceSynchronize();
    for (hipEvent_t e : ctx->c.tuner.ev) (void)hipEventDestroy(e);
  }
  hipStream_t s = ctx->c.stream;
  delete ctx;
  if (s) (void)hipStreamDestroy(s);
}

int dfamin_minimize(dfamin_ctx* ctx, const dfamin_dfa* host_dfa, const dfamin_opts* opts,
                    uint32_t* out, dfamin_result* result) {
  if (!ctx || !out) return DFAMIN_E_INVAL;
  int rc = check_dfa_shape(host_dfa);
  if (rc == DFAMIN_OK) rc = check_opts(opts);
  if (rc != DFAMIN_OK) return rc;
  if ((rc = set_device(ctx->c)) != DFAMIN_OK) return rc;
  uint32_t* outs[1] = {out};
  dfamin_result tmp{};
  rc = run_host_batch(ctx->c, 1, host_dfa, opts_or_default(opts), outs, &tmp);
  if (result && (rc == DFAMIN_OK || rc == DFAMIN_E_BAD_DFA)) *result = tmp;
  return rc;
}

int dfamin_minimal_dfa(dfamin_ctx* ctx, const dfamin_dfa* host_dfa, const dfamin_opts* opts,
                       uint32_t* min_delta, uint8_t* min_accept, uint32_t* out, dfamin_minimal* info) {
  if (!ctx || !min_delta || !min_accept) return DFAMIN_E_INVAL;
  int rc = check_dfa_shape(host_dfa);
  if (rc == DFAMIN_OK) rc = check_opts(opts);
  if (rc != DFAMIN_OK) return rc;
  if ((rc = set_device(ctx->c)) != DFAMIN_OK) return rc;
  std::vector<uint32_t> tmp;
  if (!out) {
    tmp.resize(host_dfa->n);
    out = tmp.data();
  }
  uint32_t* outs[1] = {out};
  dfamin_result r{};
  const dfamin_opts o = opts_or_default(opts);
  // the reachability search and the quotient read the round engine's
  // buffers (block ids, closure rows): this instance goes through it
  ctx->c.engine.no_fused = true;
  rc = run_host_batch(ctx->c, 1, host_dfa, o, outs, &r);
  ctx->c.engine.no_fused = false;
  if (rc != DFAMIN_OK) return rc;
  dfamin::MinimalInfo mi;
  const uint32_t* d_delta = nullptr;
  const uint8_t* d_acc = nullptr;
  rc = ctx->c.engine.minimal_dfa(o, ctx->c.stream, r.num_blocks, r.initial_block, mi, &d_delta, &d_acc);
  if (rc != DFAMIN_OK) return rc;
  // back through page-locked staging on the context's stream, then to the
  // caller's buffers by several threads
  const size_t dbytes = 4ull * host_dfa->k * mi.n, abytes = ((size_t)mi.n + 7) / 8;
  if ((rc = ensure_host(ctx->c.h_out, align16(dbytes) + abytes)) != DFAMIN_OK) return rc;
  char* hb = ctx->c.h_out.as<char>();
  if (hipMemcpyAsync(hb, d_delta, dbytes, hipMemcpyDeviceToHost, ctx->c.stream) != hipSuccess ||
      hipMemcpyAsync(hb + align16(dbytes), d_acc, abytes, hipMemcpyDeviceToHost, ctx->c.stream) != hipSuccess ||
      hipStreamSynchronize(ctx->c.stream) != hipSuccess)
    return DFAMIN_E_DEVICE;
  std::vector<Piece> back;
  add_pieces(back, reinterpret_cast<char*>(min_delta), hb, dbytes, 0);
  add_pieces(back, reinterpret_cast<char*>(min_accept), hb + align16(dbytes), abytes, 0);
  (void)run_pieces(back, dbytes + abytes, -1, [](const Piece&) { return true; });
  if (info) {
    *info = dfamin_minimal{};
    info->n = mi.n;
    info->q0 = mi.q0;
    info->num_blocks = r.num_blocks;
    info->reachable = mi.reachable;
    info->bfs_levels = mi.bfs_levels;
    info->refine_rounds = r.refine_rounds;
  }
  return DFAMIN_OK;
}

int dfamin_minimize_device(dfamin_ctx* ctx, const dfamin_dfa* dev_dfa, const dfamin_opts* opts,
                           uint32_t* dev_out, dfamin_result* result, void* hip_stream) {
  if (!ctx || !dev_out) return DFAMIN_E_INVAL;
  int rc = check_dfa_shape(dev_dfa);
  if (rc == DFAMIN_OK) rc = check_opts(opts);
  if (rc != DFAMIN_OK) return rc;
  if ((rc = set_device(ctx->c)) != DFAMIN_OK) return rc;
  const dfamin_opts o = opts_or_default(opts);
  std::vector<InstInput> in(1);
  in[0].n = dev_dfa->n;
  in[0].k = dev_dfa->k;
  in[0].q0 = dev_dfa->q0;
  in[0].closure = o.closure;
  in[0].delta = dev_dfa->delta;
  in[0].accept = dev_dfa->accept;
  in[0].out = dev_out;
  std::vector<InstOutcome> res;
  rc = ctx->c.engine.run(in, o, static_cast<hipStream_t>(hip_stream), res);
  if (rc == DFAMIN_OK || rc == DFAMIN_E_BAD_DFA) to_result(res[0], result);
  return rc;
}

int dfamin_minimize_device_noalloc(dfamin_ctx* ctx, const dfamin_dfa* dev_dfa, const dfamin_opts* opts,
                                   uint32_t* dev_out, dfamin_result* result, void* hip_stream) {
  if (!ctx || !dev_out) return DFAMIN_E_INVAL;
  int rc = check_dfa_shape(dev_dfa);
  if (rc == DFAMIN_OK) rc = check_opts(opts);
  // leader rounds and queued rounds instantiate HIP graphs
  if (rc == DFAMIN_OK && opts && (opts->method != DFAMIN_METHOD_SIGNATURE || (opts->flags & DFAMIN_FLAG_QUEUE)))
    rc = DFAMIN_E_INVAL;
  if (rc != DFAMIN_OK) return rc;
  if (noalloc_bytes(dev_dfa->n, dev_dfa->k) > DFAMIN_NOALLOC_SCRATCH_BYTES) return DFAMIN_E_NOMEM;
  if (!ctx->c.fixed_engine.fixed()) return DFAMIN_E_INTERNAL;
  if ((rc = set_device(ctx->c)) != DFAMIN_OK) return rc;
  const dfamin_opts o = opts_or_default(opts);
  std::vector<InstInput> in(1);
  in[0].n = dev_dfa->n;
  in[0].k = dev_dfa->k;
  in[0].q0 = dev_dfa->q0;
  in[0].closure = o.closure;
  in[0].delta = dev_dfa->delta;
  in[0].accept = dev_dfa->accept;
  in[0].out = dev_out;
  std::vector<InstOutcome> res;
  // kernel timing would create events: off for this call
  const bool prof_was = ctx->c.prof.swap_enabled(false);
  rc = ctx->c.fixed_engine.run(in, o, static_cast<hipStream_t>(hip_stream), res);
  ctx->c.prof.swap_enabled(prof_was);
  if (rc == DFAMIN_OK || rc == DFAMIN_E_BAD_DFA) to_result(res[0], result);
  return rc;
}

int dfamin_minimize_batch(dfamin_ctx* ctx, uint32_t count, const dfamin_dfa* dfas,
                          const dfamin_opts* opts, uint32_t* const* outs, dfamin_result* results) {
  if (!ctx || (count && (!dfas || !outs))) return DFAMIN_E_INVAL;
  int rc = check_opts(opts);
  if (rc != DFAMIN_OK) return rc;
  for (uint32_t i = 0; i < count; ++i) {
    if ((rc = check_dfa_shape(&dfas[i])) != DFAMIN_OK) return rc;
    if (!outs[i]) return DFAMIN_E_INVAL;
  }
  if (count == 0) return DFAMIN_OK;
  if ((rc = set_device(ctx->c)) != DFAMIN_OK) return rc;
  return run_host_batch(ctx->c, count, dfas, opts_or_default(opts), outs, results);
}

int dfamin_minimize_batch_device(dfamin_ctx* ctx, uint32_t count, const dfamin_dfa* dev_dfas,
                                 const dfamin_opts* opts, uint32_t* const* dev_outs,
                                 dfamin_result* results, void* hip_stream) {
  if (!ctx || (count && (!dev_dfas || !dev_outs))) return DFAMIN_E_INVAL;
  int rc = check_opts(opts);
  if (rc != DFAMIN_OK) return rc;
  for (uint32_t i = 0; i < count; ++i) {
    if ((rc = check_dfa_shape(&dev_dfas[i])) != DFAMIN_OK) return rc;
    if (!dev_outs[i]) return DFAMIN_E_INVAL;
  }
  if (count == 0) return DFAMIN_OK;
  if ((rc = set_device(ctx->c)) != DFAMIN_OK) return rc;
  const dfamin_opts o = opts_or_default(opts);
  std::vector<InstInput> in(count);
  for (uint32_t i = 0; i < count; ++i) {
    in[i].n = dev_dfas[i].n;
    in[i].k = dev_dfas[i].k;
    in[i].q0 = dev_dfas[i].q0;
    in[i].closure = o.closure;
    in[i].delta = dev_dfas[i].delta;
    in[i].accept = dev_dfas[i].accept;
    in[i].out = dev_outs[i];
  }
  std::vector<InstOutcome> res;
  rc = ctx->c.engine.run(in, o, static_cast<hipStream_t>(hip_stream), res);
  if ((rc == DFAMIN_OK || rc == DFAMIN_E_BAD_DFA) && results)
    for (uint32_t i = 0; i < count; ++i) to_result(res[i], &results[i]);
  return rc;
}

int dfamin_submit(dfamin_ctx* ctx, const dfamin_dfa* host_dfa, const dfamin_opts* opts,
                  uint64_t* ticket) {
  if (!ctx || !ticket) return DFAMIN_E_INVAL;
  int rc = check_dfa_shape(host_dfa);
  if (rc == DFAMIN_OK) rc = check_opts(opts);
  if (rc == DFAMIN_OK && opts && opts->method != DFAMIN_METHOD_SIGNATURE) rc = DFAMIN_E_INVAL;
  if (rc != DFAMIN_OK) return rc;
  if (!ctx->c.serving) {
    ctx->c.serving = new (std::nothrow) dfamin::Serving(&ctx->c);
    if (!ctx->c.serving) return DFAMIN_E_NOMEM;
  }
  return ctx->c.serving->submit(*host_dfa, opts_or_default(opts), ticket);
}

int dfamin_wait(dfamin_ctx* ctx, uint64_t ticket, int64_t timeout_us, uint32_t* out,
                dfamin_result* result) {
  if (!ctx || !out) return DFAMIN_E_INVAL;
  if (!ctx->c.serving) return DFAMIN_E_INVAL;
  return ctx->c.serving->wait(ticket, timeout_us, out, result);
}

int dfamin_cancel(dfamin_ctx* ctx, uint64_t ticket) {
  if (!ctx || !ctx->c.serving) return DFAMIN_E_INVAL;
  return ctx->c.serving->cancel(ticket);
}

const char* dfamin_status_str(int status) {
  switch (status) {
    case DFAMIN_OK: return "ok";
    case DFAMIN_E_INVAL: return "invalid argument";
    case DFAMIN_E_BAD_DFA: return "transition target out of range";
    case DFAMIN_E_NOMEM: return "out of device memory budget";
    case DFAMIN_E_DEVICE: return "HIP device error";
    case DFAMIN_E_TIMEOUT: return "timed out";
    case DFAMIN_E_CANCELLED: return "cancelled";
    case DFAMIN_E_BUSY: return "queue full";
    case DFAMIN_E_INTERNAL: return "internal limit exceeded";
    default: return "unknown status";
  }
}

int dfamin_set_profiling(dfamin_ctx* ctx, int on) {
  if (!ctx) return DFAMIN_E_INVAL;
  ctx->c.prof.set_enabled(on != 0);
  return DFAMIN_OK;
}

int dfamin_set_tuning(dfamin_ctx* ctx, int variant) {
  if (!ctx || variant < -1 || variant >= dfamin::kSigVariants) return DFAMIN_E_INVAL;
  ctx->c.tuner.forced = variant;
  ctx->c.tuner.best.clear();
  return DFAMIN_OK;
}

int dfamin_get_kernel_stats(dfamin_ctx* ctx, dfamin_kernel_stat* stats, int cap) {
  if (!ctx || (cap > 0 && !stats)) return DFAMIN_E_INVAL;
  return ctx->c.prof.copy_stats(stats, cap);
}

}  // extern "C"
