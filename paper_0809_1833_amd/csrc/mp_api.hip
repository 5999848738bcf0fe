// Host side of libmp.so: argument checking, context ownership, the iteration
// driver, and the C ABI declared in include/mp.h.
#include <math.h>
#include <cmath>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <climits>
#include <string>
#include <vector>

#include "mp_internal.h"

namespace {

thread_local std::string g_create_error;

constexpr int64_t kMaxN = 16384;          // the residual is staged whole in LDS
constexpr int64_t kMaxSignN = 16384;      // two 16-byte chunks of a column per lane
constexpr int64_t kMaxRaggedN = 8192;     // per-instance residual in LDS, 32 KB
constexpr int kMaxRaggedSplit = 4096;     // instances cut into parts, at most
constexpr int kRaggedDefaultSplit = 3;    // parts of an instance, at most, unless configured
constexpr int64_t kLdAlign = 64;          // padded column length (floats): 256 B aligned
constexpr int kMaxChunk = 64;             // iterations enqueued per host check
constexpr double kNormTol = 1e-4;

mp_status fail(mp_ctx* ctx, mp_status s, const std::string& msg) {
  if (ctx) ctx->err = msg;
  else g_create_error = msg;
  return s;
}

#define HIP_TRY(ctx, expr)                                                            \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess)                                                             \
      return fail((ctx), MP_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

int64_t round_up(int64_t v, int64_t a) { return (v + a - 1) / a * a; }

void free_batched(mp_ctx* c) {
  (void)hipFree(c->b_r32);
  (void)hipFree(c->b_rq);
  (void)hipFree(c->b_slots);
  (void)hipFree(c->b_act);
  (void)hipFree(c->b_state);
  (void)hipFree(c->b_partials);
  (void)hipFree(c->b_keep);
  (void)hipFree(c->b_tcap);
  if (c->h_slots) (void)hipHostFree(c->h_slots);
  if (c->h_bstate) (void)hipHostFree(c->h_bstate);
  c->b_r32 = nullptr;
  c->b_rq = nullptr;
  c->b_slots = nullptr;
  c->b_act = nullptr;
  c->b_state = nullptr;
  c->b_partials = nullptr;
  c->b_keep = nullptr;
  c->b_tcap = nullptr;
  c->h_slots = nullptr;
  c->h_bstate = nullptr;
  c->bcap = 0;
}

void free_ragged(mp_ctx* c) {
  (void)hipFree(c->r_psi32);
  (void)hipFree(c->r_psib);
  (void)hipFree(c->r_inst);
  (void)hipFree(c->r_items);
  (void)hipFree(c->r_slots);
  if (c->h_rq) (void)hipHostFree(c->h_rq);
  (void)hipFree(c->r_caps);
  (void)hipFree(c->r_res);
  (void)hipFree(c->r_queue);
  if (c->h_rres) (void)hipHostFree(c->h_rres);
  if (c->r_graph) (void)hipGraphExecDestroy(c->r_graph);
  if (c->r_cap_stream) (void)hipStreamDestroy(c->r_cap_stream);
}

void free_omp(mp_ctx* c) {
  mp::OmpBufs& b = c->omp;
  (void)hipFree(b.q);
  (void)hipFree(b.rmat);
  (void)hipFree(b.z);
  (void)hipFree(b.sel);
  (void)hipFree(b.in_s);
  (void)hipFree(b.w);
  (void)hipFree(b.h1);
  (void)hipFree(b.h2);
  (void)hipFree(b.hp);
  (void)hipFree(b.part);
  (void)hipFree(b.os);
  b = mp::OmpBufs{};
}

void free_ctx(mp_ctx* c) {
  if (!c) return;
  free_batched(c);
  free_ragged(c);
  free_omp(c);
  (void)hipFree(c->psibt);
  (void)hipFree(c->psi32);
  (void)hipFree(c->psi64);
  (void)hipFree(c->r64_work);
  (void)hipFree(c->psiq);
  (void)hipFree(c->psis);
  (void)hipFree(c->sign_c64);
  (void)hipFree(c->sign_r64);
  (void)hipFree(c->sign_rrp);
  (void)hipFree(c->sign_slots);
  (void)hipFree(c->small_slots);
  (void)hipFree(c->scales);
  (void)hipFree(c->r_work);
  (void)hipFree(c->st);
  (void)hipFree(c->partials);
  (void)hipFree(c->bal);
  if (c->async_pending && c->async_ev) (void)hipEventSynchronize(c->async_ev);
  if (c->async_ev) (void)hipEventDestroy(c->async_ev);
  if (c->h_st) (void)hipHostFree(c->h_st);
  for (hipEvent_t e : c->done_ev)
    if (e) (void)hipEventDestroy(e);
  for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
  delete c;
}

// The current device, if it is a gfx950 this library was built for.
mp_status open_device(int& dev, hipDeviceProp_t& prop) {
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count < 1)
    return fail(nullptr, MP_EDEVICE, "no HIP device");
  HIP_TRY(nullptr, hipGetDevice(&dev));
  HIP_TRY(nullptr, hipGetDeviceProperties(&prop, dev));
  if (strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(nullptr, MP_EUNSUPPORTED, std::string("device is ") + prop.gcnArchName +
                                              ", this library is built for gfx950");
  return MP_OK;
}

// Eq. 4 on the FP64 squared column norms: finite always, 1 within kNormTol
// unless MP_SKIP_NORM_CHECK.  Returns MP_OK or the status with `msg` set.
mp_status check_norms(const std::vector<double>& norm2, uint32_t flags, std::string& msg) {
  for (size_t j = 0; j < norm2.size(); ++j) {
    if (!isfinite(norm2[j])) {
      char buf[96];
      snprintf(buf, sizeof buf, "column %lld holds NaN or Inf", static_cast<long long>(j));
      msg = buf;
      return MP_ENONFINITE;
    }
    if (!(flags & MP_SKIP_NORM_CHECK) && fabs(sqrt(norm2[j]) - 1.0) > kNormTol) {
      char buf[128];
      snprintf(buf, sizeof buf, "column %lld has norm %.9g (must be 1 within 1e-4)",
               static_cast<long long>(j), sqrt(norm2[j]));
      msg = buf;
      return MP_ENOTNORM;
    }
  }
  return MP_OK;
}

// The trace's residual rows: ldr must cover the longest residual it receives.
template <class T>
mp_status check_trace(mp_ctx* c, const T* trace, int64_t rows) {
  if (!trace) return MP_OK;
  if (trace->cap < 0) return fail(c, MP_EINVAL, "trace cap must be >= 0");
  if (trace->r && trace->ldr < rows)
    return fail(c, MP_EINVAL, "trace ldr must be >= the residual length");
  return MP_OK;
}

// A context with a stream-ordered decode not yet collected takes no other
// decode (its device state and the host mirror belong to that decode).
mp_status check_not_pending(mp_ctx* c) {
  if (c->async_pending)
    return fail(c, MP_EINVAL, "a stream-ordered decode is pending: collect it with mp_solve_result");
  return MP_OK;
}

mp_status check_opts(mp_ctx* c, const mp_opts* opts,
                     uint32_t allowed = MP_SOLVE_STEP_LAUNCHES) {
  if (mp_status ps = check_not_pending(c); ps != MP_OK) return ps;
  if (!(opts->eps >= 0.0) || !isfinite(opts->eps))
    return fail(c, MP_EINVAL, "eps must be finite and >= 0");
  if (opts->max_iters < 0) return fail(c, MP_EINVAL, "max_iters must be >= 0");
  if (opts->flags & ~allowed) return fail(c, MP_EINVAL, "unknown opts.flags");
  if (opts->rescore_k < 0 || opts->rescore_k > 8)
    return fail(c, MP_EINVAL, "rescore_k must be in 0..8");
  return MP_OK;
}

// The pinned host mirror of the device state (entry 0) and the two slots
// run_iterations copies each chunk's state into (entries 1, 2), with the
// events that mark those copies: made once per context, so that a decode
// allocates nothing.
bool make_host_state(mp_ctx* c) {
  if (hipHostMalloc(&c->h_st, 3 * sizeof(mp::DevState), hipHostMallocDefault) != hipSuccess) {
    c->h_st = nullptr;
    return false;
  }
  for (hipEvent_t& e : c->done_ev)
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
      e = nullptr;
      return false;
    }
  if (hipEventCreateWithFlags(&c->async_ev, hipEventDisableTiming) != hipSuccess) {
    c->async_ev = nullptr;
    return false;
  }
  return true;
}

// Length of the next chunk of launches.  Doubling from 4 up to kMaxChunk
// while the run is young; once two chunk-end states are known, the
// remaining steps are estimated from the decay of ||r||^2 between them
// (ln rr falls about linearly once MP settles) and the chunk is cut to what
// that estimate still needs beyond the launches already in flight, plus a
// margin: launches issued past the stop return at once but still cost a
// dispatch each, which dominates short decodes.  Returns 0 when the
// launches in flight should cover the estimate (the caller then waits).
int next_chunk(int doubling, long long issued, const mp::DevState* a, const mp::DevState* b) {
  const double thr = b ? b->thr : 0.0;
  if (!a || !b || b->done || b->t <= a->t || !(b->rr > thr) || !(a->rr > b->rr) ||
      !(thr > 0.0))
    return doubling;
  const double rate = (std::log(a->rr) - std::log(b->rr)) / static_cast<double>(b->t - a->t);
  const double rem = std::log(b->rr / thr) / rate;  // steps still needed after b
  const long long ahead = issued - (b->t + 1);         // launches in flight past b
  const double want = std::ceil(rem * 1.25) + 2.0 - static_cast<double>(ahead);
  if (want <= 0.0) return 0;
  return static_cast<int>(std::min<double>(want, doubling));
}

// The single-signal iteration driver: after init (state already copied to
// c->h_st), enqueue chunks of iterations with `enqueue(e0, e1)` (record e0,
// when not null, before the iteration's launch and e1 after it); the kernels
// stop doing work once the device state says the run is over.  Two chunks
// stay in flight: after enqueuing chunk k the host waits for the state copy
// that follows chunk k-1.
//
// Timing, with profiling on.  `windowed` (one kernel launch per iteration):
// each chunk is cut from its start into windows of prof_every consecutive
// launches (at most a chunk), timed by one event before the window's first
// launch and one after its last, so the launches inside run as untimed ones
// do and the average per launch includes the gaps between them.  Otherwise
// (OMP: several kernels per iteration, `enqueue` brackets the selection
// launch) every prof_every-th iteration is timed on its own.  Only launches
// that performed an iteration are counted: a window, all its launches.
template <typename Enqueue>
mp_status run_iterations(mp_ctx* c, long long T, hipStream_t s, bool windowed, Enqueue enqueue,
                         bool known_running = false, const mp::DevState* dst = nullptr) {
  if (!dst) dst = c->st;
  c->prof_ms = 0.0;
  c->prof_launches = 0;
  long long issued = 0;
  int chunk = 4;
  hipEvent_t* done_ev = c->done_ev;
  mp::DevState* h_slot = c->h_st + 1;
  // the last two chunk-end states read back (for the chunk-length estimate)
  mp::DevState hist[2];
  int nhist = 0;
  long long slot_base[2] = {0, 0};
  int slot_len[2] = {0, 0};
  mp_status status = MP_OK;
  // Launch j of a decode ran its correlation pass unless the run had stopped
  // by then.  A run that stops after t steps stops in launch t+1 in the
  // one-bit form; in the others in launch t (converged or out of steps: step
  // t applied, no pass) or t+1 (no usable winner).  Only launches that ran a
  // pass are timed.
  auto account = [&](int k) {
    if (!c->profiling) return;
    const mp::DevState& sl = h_slot[k];
    const bool late = c->storage == MP_SIGN1 ||
                      (sl.reason != MP_STOP_CONVERGED && sl.reason != MP_STOP_MAX_ITERS);
    const long long stop_launch = sl.done ? sl.t + (late ? 1 : 0) : LLONG_MAX;
    const int w = windowed ? std::min(c->prof_every, kMaxChunk) : 1;
    for (int j = 0; j + w <= slot_len[k]; j += w) {
      if (slot_base[k] + j + w > stop_launch) break;
      if (!windowed && (slot_base[k] + j) % c->prof_every != 0) continue;
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, c->ev[(k * kMaxChunk + j) * 2],
                              c->ev[(k * kMaxChunk + j) * 2 + 1]) == hipSuccess) {
        c->prof_ms += ms;
        c->prof_launches += w;
      }
    }
  };
  bool finished = !known_running && c->h_st->done != 0;
  int next = 0;      // slot the next chunk goes to
  int inflight = 0;  // chunks enqueued but not yet waited for
  while (!finished && status == MP_OK) {
    while (inflight < 2 && issued < T && status == MP_OK) {
      const int k = next;
      int want = next_chunk(chunk, issued, nhist == 2 ? &hist[0] : nullptr,
                            nhist >= 1 ? &hist[nhist - 1] : nullptr);
      if (want == 0) {
        if (inflight > 0) break;  // wait for what is in flight
        want = 2;
      }
      const int len = static_cast<int>(std::min<long long>(want, T - issued));
      const int w = windowed ? std::min(c->prof_every, kMaxChunk) : 1;
      for (int j = 0; j < len; ++j) {
        hipEvent_t e0 = nullptr, e1 = nullptr;
        const int j0 = j - j % w;  // first launch of j's window
        if (c->profiling && j0 + w <= len &&
            (windowed || (issued + j) % c->prof_every == 0)) {
          if (j == j0) e0 = c->ev[(k * kMaxChunk + j0) * 2];
          if (j == j0 + w - 1) e1 = c->ev[(k * kMaxChunk + j0) * 2 + 1];
        }
        hipError_t e = enqueue(e0, e1);
        if (e != hipSuccess) {
          status = fail(c, MP_EDEVICE, std::string("launch: ") + hipGetErrorString(e));
          break;
        }
      }
      if (status != MP_OK) break;
      slot_base[k] = issued;
      slot_len[k] = len;
      issued += len;
      hipError_t e = hipMemcpyAsync(&h_slot[k], dst, sizeof(mp::DevState),
                                    hipMemcpyDeviceToHost, s);
      if (e == hipSuccess) e = hipEventRecord(done_ev[k], s);
      if (e != hipSuccess) {
        status = fail(c, MP_EDEVICE, std::string("state copy: ") + hipGetErrorString(e));
        break;
      }
      ++inflight;
      next ^= 1;
      chunk = std::min(chunk * 2, kMaxChunk);
    }
    if (status != MP_OK || inflight == 0) break;
    const int old = inflight == 2 ? next : (next ^ 1);  // the older chunk in flight
    hipError_t e = hipEventSynchronize(done_ev[old]);
    if (e != hipSuccess) {
      status = fail(c, MP_EDEVICE, std::string("sync: ") + hipGetErrorString(e));
      break;
    }
    --inflight;
    account(old);
    if (h_slot[old].done) finished = true;
    if (nhist == 2) hist[0] = hist[1];
    hist[nhist == 2 ? 1 : nhist] = h_slot[old];
    if (nhist < 2) ++nhist;
  }
  // drain the chunk still in flight (its launches return at once)
  if (hipStreamSynchronize(s) != hipSuccess && status == MP_OK)
    status = fail(c, MP_EDEVICE, "stream synchronize failed");
  return status;
}

// Device buffers of one carried single-signal decode (FP32, BF16, FP8): the
// context's own (mp_solve) or carved from the library's static scratch
// (mp_solve_noalloc).
struct CarriedBufs {
  mp::DevState* st;  // the decode's state
  float* r_work;     // 2 x ld floats: r_k in half k mod 2 (padding rows written 0)
  uint64_t* keys;    // 2 x grid x kLpTopK key slots
  mp::BalState* bal; // column shares and pass timings (any contents: a balance hint only)
};

mp_status finish_result(mp_ctx* c, mp_result* res);

// The carried decode: launch k takes step k (k >= 1) and runs pass k+1, so T
// steps take T+1 launches; r ends in the half the state names.  The kernels
// read the stop threshold from the device state, so the host starts
// launching without waiting for the init kernel (launches after a stop, zero
// input included, return at once).  At the end one small kernel copies r out
// of the half the state names, and the state comes back with one wait.
// Allocates nothing: every buffer is in `b`, the context (pinned state slots
// and events made at its creation) or the caller's arguments.
//
// Stream-ordered (MP_SOLVE_ASYNC): the same launches, all T+1 of them
// enqueued at once (the host does not read the state), then the state copy
// into the host mirror and the context's event; mp_solve_result waits for it.
mp_status enqueue_result(mp_ctx* c, const mp::DevState* st, hipStream_t s, int persistent) {
  HIP_TRY(c, hipMemcpyAsync(c->h_st, st, sizeof(mp::DevState), hipMemcpyDeviceToHost, s));
  HIP_TRY(c, hipEventRecord(c->async_ev, s));
  c->async_pending = true;
  c->async_persistent = persistent;
  return MP_OK;
}

mp_status solve_carried(mp_ctx* c, const float* y, float* x, float* r, const mp_opts* opts,
                        mp_result* res, const mp_trace& tr, hipStream_t s, const CarriedBufs& b,
                        bool allow_one_launch) {
  const bool async = (opts->flags & MP_SOLVE_ASYNC) != 0;
  HIP_TRY(c, mp::launch_init(y, c->n, c->ld, x, c->m, b.r_work, b.st, opts->eps,
                             static_cast<long long>(opts->max_iters), s));
  if (allow_one_launch && c->storage == MP_F32 && c->small.grid > 0 &&
      !(opts->flags & MP_SOLVE_STEP_LAUNCHES)) {
    // the whole decode in one launch, every share of the dictionary in LDS:
    // a new tag epoch for every decode (never 0 mod the epoch range: the
    // zeroed words match no step); when it wraps, clear the words so that
    // none left from a decode that many decodes ago can match
    c->small_epoch = c->small_epoch % (mp::small_epoch_mod() - 1) + 1;
    if (c->small_epoch == 1)
      HIP_TRY(c, hipMemsetAsync(c->small_slots, 0,
                                sizeof(unsigned long long) * mp::small_slot_words(), s));
    const bool timed = c->profiling && !async;
    if (timed) HIP_TRY(c, hipEventRecord(c->ev[0], s));
    HIP_TRY(c, mp::launch_f32_small(c->psi32, c->ld, c->n, c->m, b.r_work, c->small,
                                    c->small_slots, c->small_epoch, opts->max_iters, x, b.st, tr,
                                    s));
    if (timed) HIP_TRY(c, hipEventRecord(c->ev[1], s));
    if (r) HIP_TRY(c, mp::launch_copy_selected(b.r_work, c->ld, c->n, b.st, r, s));
    if (async) return enqueue_result(c, b.st, s, 1);
    HIP_TRY(c, hipMemcpyAsync(c->h_st, b.st, sizeof(mp::DevState), hipMemcpyDeviceToHost, s));
    HIP_TRY(c, hipStreamSynchronize(s));
    if (c->profiling) {
      // the launch time per step taken (t steps, t passes)
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, c->ev[0], c->ev[1]) == hipSuccess) {
        c->prof_ms = ms;
        c->prof_launches = c->h_st->t > 0 ? c->h_st->t : 1;
      }
    }
    const mp_status fs = finish_result(c, res);
    if (fs == MP_OK && res) res->persistent = 1;
    return fs;
  }
  long long k = 0;
  const long long T = opts->max_iters;
  auto step = [&](hipEvent_t e0, hipEvent_t e1) {
    hipError_t e;
    if (e0 && (e = hipEventRecord(e0, s)) != hipSuccess) return e;
    if (c->storage == MP_F32)
      e = mp::launch_mp_step_f32(c->psi32, c->ld, c->n, c->m, b.r_work, c->geom, b.keys, b.bal,
                                 k, T, x, b.st, tr, s);
    else
      e = mp::launch_mp_step_lp(c->storage, c->psiq, c->scales, c->psi32, c->ld, c->n, c->m,
                                b.r_work, c->geom, c->rescore_k, b.keys, k, T, x, b.st, tr, s);
    ++k;
    if (e != hipSuccess) return e;
    if (e1 && (e = hipEventRecord(e1, s)) != hipSuccess) return e;
    return hipSuccess;
  };
  if (async) {
    const long long launches = T > 0 ? T + 1 : 0;
    for (long long j = 0; j < launches; ++j) {
      const hipError_t e = step(nullptr, nullptr);
      if (e != hipSuccess) return fail(c, MP_EDEVICE, std::string("launch: ") + hipGetErrorString(e));
    }
    if (r) HIP_TRY(c, mp::launch_copy_selected(b.r_work, c->ld, c->n, b.st, r, s));
    return enqueue_result(c, b.st, s, 0);
  }
  const mp_status st = run_iterations(c, T > 0 ? T + 1 : 0, s, true, step,
                                      /*known_running=*/true, b.st);
  if (st != MP_OK) return st;
  if (r) HIP_TRY(c, mp::launch_copy_selected(b.r_work, c->ld, c->n, b.st, r, s));
  HIP_TRY(c, hipMemcpyAsync(c->h_st, b.st, sizeof(mp::DevState), hipMemcpyDeviceToHost, s));
  HIP_TRY(c, hipStreamSynchronize(s));
  const mp_status fs = finish_result(c, res);
  if (fs == MP_OK && res) res->persistent = 0;
  return fs;
}

// Final state of a single-signal decode into `res`, with the internal stop
// reasons mapped to errors.
mp_status finish_result(mp_ctx* c, mp_result* res) {
  const mp::DevState& d = *c->h_st;
  if (d.fail)
    return fail(c, MP_EDEVICE, "a wait of the persistent one-bit decode gave up");
  if (d.reason == mp::kStopNonFinite) return fail(c, MP_ENONFINITE, "y holds NaN or Inf");
  if (d.reason == mp::kStopInternal)
    return fail(c, MP_EDEVICE,
                "internal error: a selected index fell outside the dictionary");
  if (res) {
    res->iters = d.t;
    res->yy = d.yy;
    res->rr = d.rr;
    res->stop_reason = d.reason;
    res->persistent = 0;
  }
  return MP_OK;
}

}  // namespace

extern "C" {

const char* mp_status_str(mp_status s) {
  switch (s) {
    case MP_OK: return "MP_OK";
    case MP_EINVAL: return "MP_EINVAL";
    case MP_ENOTNORM: return "MP_ENOTNORM";
    case MP_ENONFINITE: return "MP_ENONFINITE";
    case MP_ENOMEM: return "MP_ENOMEM";
    case MP_EDEVICE: return "MP_EDEVICE";
    case MP_EUNSUPPORTED: return "MP_EUNSUPPORTED";
  }
  return "MP_UNKNOWN";
}

const char* mp_last_error(const mp_ctx* ctx) {
  return ctx ? ctx->err.c_str() : g_create_error.c_str();
}

mp_status mp_create(mp_ctx** out, const float* psi, int64_t n, int64_t m, int64_t ld,
                    mp_dtype storage, uint32_t flags, void* stream) {
  g_create_error.clear();
  if (!out) return fail(nullptr, MP_EINVAL, "out is NULL");
  *out = nullptr;
  if (!psi) return fail(nullptr, MP_EINVAL, "psi is NULL");
  if (n < 1 || m < 1) return fail(nullptr, MP_EINVAL, "n and m must be >= 1");
  if (ld < n) return fail(nullptr, MP_EINVAL, "ld must be >= n");
  if (n > kMaxN) return fail(nullptr, MP_EINVAL, "n exceeds 16384");
  if (m >= (int64_t{1} << 31)) return fail(nullptr, MP_EINVAL, "m must be < 2^31");
  if (flags & ~MP_SKIP_NORM_CHECK) return fail(nullptr, MP_EINVAL, "unknown flags");
  if (storage == MP_F64)
    return fail(nullptr, MP_EINVAL, "an FP64 dictionary is taken by mp_create_f64");
  if (storage == MP_SIGN1)
    return fail(nullptr, MP_EINVAL, "a sign-bit dictionary is taken by mp_create_signs");
  if (storage != MP_F32 && storage != MP_BF16 && storage != MP_FP8_E4M3)
    return fail(nullptr, MP_EINVAL, "unknown storage type");
  int dev = 0;
  hipDeviceProp_t prop;
  if (mp_status ds = open_device(dev, prop); ds != MP_OK) return ds;
  hipStream_t s = static_cast<hipStream_t>(stream);

  mp_ctx* c = new mp_ctx();
  c->device = dev;
  c->num_cus = prop.multiProcessorCount;
  c->n = n;
  c->m = m;
  c->ld = round_up(n, kLdAlign);
  c->storage = storage;
  c->geom = mp::corr_f32_geometry(m, c->num_cus);

  auto bail = [&](mp_status st, const std::string& msg) {
    free_ctx(c);
    return fail(nullptr, st, msg);
  };
  const size_t psi_bytes = static_cast<size_t>(c->ld) * static_cast<size_t>(m) * sizeof(float);
  if (hipMalloc(&c->psi32, psi_bytes) != hipSuccess) return bail(MP_ENOMEM, "dictionary copy");
  // r and the published keys in two halves (the reduced-precision decode
  // alternates between them by launch parity)
  if (hipMalloc(&c->r_work, 2 * c->ld * sizeof(float)) != hipSuccess)
    return bail(MP_ENOMEM, "r");
  if (hipMalloc(&c->st, sizeof(mp::DevState)) != hipSuccess) return bail(MP_ENOMEM, "state");
  if (c->geom.grid * mp::kLpTopK > 2 * 1024)
    return bail(MP_EUNSUPPORTED, "more correlation workgroups than the key slots hold");
  const size_t nkeys = 2 * static_cast<size_t>(c->geom.grid) * mp::kLpTopK;
  if (hipMalloc(&c->partials, sizeof(uint64_t) * nkeys) != hipSuccess)
    return bail(MP_ENOMEM, "partials");
  if (hipMalloc(&c->bal, sizeof(mp::BalState)) != hipSuccess) return bail(MP_ENOMEM, "shares");
  if (!make_host_state(c)) return bail(MP_ENOMEM, "pinned state");
  // the one-launch decode of small FP32 dictionaries (every share in LDS)
  if (storage == MP_F32) {
    c->small = mp::small_geometry(c->ld, m, c->num_cus);
    if (c->small.grid > 0) {
      const size_t bytes = sizeof(unsigned long long) * mp::small_slot_words();
      if (hipMalloc(&c->small_slots, bytes) != hipSuccess) return bail(MP_ENOMEM, "step records");
      if (hipMemsetAsync(c->small_slots, 0, bytes, s) != hipSuccess)
        return bail(MP_EDEVICE, "step records");
    }
  }
  // set-up of mp_solve_noalloc's scratch on this device (the entry point
  // looks it up itself if this fails)
  {
    void* scratch_ptr = nullptr;
    (void)mp::noalloc_scratch(dev, &scratch_ptr);
  }

  hipError_t e = hipMemsetAsync(c->psi32, 0, psi_bytes, s);
  if (e == hipSuccess)
    e = hipMemcpy2DAsync(c->psi32, c->ld * sizeof(float), psi, ld * sizeof(float),
                         n * sizeof(float), m, hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess) e = hipMemsetAsync(c->r_work, 0, 2 * c->ld * sizeof(float), s);
  if (e == hipSuccess) e = hipMemsetAsync(c->partials, 0, sizeof(uint64_t) * nkeys, s);
  if (e == hipSuccess) e = hipMemsetAsync(c->bal, 0, sizeof(mp::BalState), s);
  if (e != hipSuccess) return bail(MP_EDEVICE, std::string("copy: ") + hipGetErrorString(e));

  // Column norms in FP64 (eq. 4): finiteness always, unit norm unless skipped.
  double* d_norm2 = nullptr;
  if (hipMalloc(&d_norm2, sizeof(double) * m) != hipSuccess) return bail(MP_ENOMEM, "norms");
  std::vector<double> norm2(static_cast<size_t>(m));
  e = mp::launch_norms(c->psi32, c->ld, n, m, d_norm2, nullptr, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(norm2.data(), d_norm2, sizeof(double) * m, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(d_norm2);
  if (e != hipSuccess) return bail(MP_EDEVICE, std::string("norms: ") + hipGetErrorString(e));
  {
    std::string msg;
    const mp_status ns = check_norms(norm2, flags, msg);
    if (ns != MP_OK) return bail(ns, msg);
  }
  // Reduced-precision copy the correlation pass streams (same padded layout).
  if (storage == MP_BF16 || storage == MP_FP8_E4M3) {
    const size_t esize = storage == MP_BF16 ? 2 : 1;
    const size_t qbytes = static_cast<size_t>(c->ld) * static_cast<size_t>(m) * esize;
    if (hipMalloc(&c->psiq, qbytes) != hipSuccess) return bail(MP_ENOMEM, "reduced copy");
    if (storage == MP_BF16) {
      e = mp::launch_quant_bf16(c->psi32, c->ld, m, static_cast<uint16_t*>(c->psiq), s);
    } else {
      if (hipMalloc(&c->scales, sizeof(float) * m) != hipSuccess)
        return bail(MP_ENOMEM, "scales");
      e = mp::launch_quant_fp8(c->psi32, c->ld, m, static_cast<uint8_t*>(c->psiq), c->scales, s);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return bail(MP_EDEVICE, std::string("quantise: ") + hipGetErrorString(e));
  }
  *out = c;
  return MP_OK;
}

void mp_destroy(mp_ctx* ctx) { free_ctx(ctx); }

mp_status mp_set_profiling(mp_ctx* ctx, int every) {
  if (!ctx) return MP_EINVAL;
  if (every < 0) return fail(ctx, MP_EINVAL, "every must be >= 0");
  if (every > 0 && ctx->ev.empty()) {
    ctx->ev.resize(2 * 2 * kMaxChunk, nullptr);
    for (hipEvent_t& e : ctx->ev) HIP_TRY(ctx, hipEventCreate(&e));
  }
  ctx->profiling = every > 0;
  ctx->prof_every = every > 0 ? every : 1;
  return MP_OK;
}

mp_status mp_kernel_time(const mp_ctx* ctx, double* avg_ms, int64_t* launches) {
  if (!ctx || !avg_ms || !launches) return MP_EINVAL;
  *launches = ctx->prof_launches;
  *avg_ms = ctx->prof_launches ? ctx->prof_ms / static_cast<double>(ctx->prof_launches) : 0.0;
  return MP_OK;
}

mp_status mp_get_storage(const mp_ctx* ctx, void* codes, float* scales, void* stream) {
  if (!ctx || !codes) return MP_EINVAL;
  mp_ctx* c = const_cast<mp_ctx*>(ctx);
  if (c->ragged) return fail(c, MP_EINVAL, "not available for a ragged context");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (c->storage == MP_F64) {
    HIP_TRY(c, hipMemcpy2DAsync(codes, c->n * sizeof(double), c->psi64, c->ld * sizeof(double),
                                c->n * sizeof(double), c->m, hipMemcpyDeviceToDevice, s));
  } else if (c->storage == MP_SIGN1) {
    const size_t w = static_cast<size_t>((c->n + 31) / 32) * sizeof(uint32_t);
    HIP_TRY(c, hipMemcpy2DAsync(codes, w, c->psis, c->sign_ws * sizeof(uint32_t), w, c->m,
                                hipMemcpyDeviceToDevice, s));
  } else if (c->storage == MP_F32) {
    HIP_TRY(c, hipMemcpy2DAsync(codes, c->n * sizeof(float), c->psi32, c->ld * sizeof(float),
                                c->n * sizeof(float), c->m, hipMemcpyDeviceToDevice, s));
  } else {
    const size_t esize = c->storage == MP_BF16 ? 2 : 1;
    HIP_TRY(c, hipMemcpy2DAsync(codes, c->n * esize, c->psiq, c->ld * esize, c->n * esize, c->m,
                                hipMemcpyDeviceToDevice, s));
    if (c->storage == MP_FP8_E4M3 && scales)
      HIP_TRY(c, hipMemcpyAsync(scales, c->scales, sizeof(float) * c->m, hipMemcpyDeviceToDevice,
                                s));
  }
  HIP_TRY(c, hipStreamSynchronize(s));
  return MP_OK;
}

mp_status mp_solve(mp_ctx* ctx, const float* y, float* x, float* r, const mp_opts* opts,
                   mp_result* res, const mp_trace* trace, void* stream) {
  if (!ctx) return MP_EINVAL;
  ctx->err.clear();
  if (ctx->ragged) return fail(ctx, MP_EINVAL, "a ragged context is decoded with mp_solve_ragged");
  if (ctx->storage == MP_F64)
    return fail(ctx, MP_EINVAL, "an MP_F64 context is decoded with mp_solve_f64");
  if (!y || !x || !opts) return fail(ctx, MP_EINVAL, "y, x and opts must not be NULL");
  if (mp_status os = check_opts(ctx, opts, MP_SOLVE_STEP_LAUNCHES | MP_SOLVE_ASYNC); os != MP_OK)
    return os;
  if (opts->flags & MP_SOLVE_ASYNC) {
    if (ctx->storage == MP_SIGN1)
      return fail(ctx, MP_EINVAL, "stream-ordered decodes need MP_F32, MP_BF16 or MP_FP8_E4M3");
    if (res) return fail(ctx, MP_EINVAL, "a stream-ordered decode takes res = NULL");
  }
  mp_trace tr{};
  if (mp_status ts = check_trace(ctx, trace, ctx->n); ts != MP_OK) return ts;
  if (trace) tr = *trace;
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  hipStream_t s = static_cast<hipStream_t>(stream);
  mp_ctx* c = ctx;
  c->rescore_k = opts->rescore_k == 0 ? mp::kLpTopK : opts->rescore_k;
  c->prof_ms = 0.0;
  c->prof_launches = 0;
  bool persistent = false;  // the one-bit decode ran as one persistent launch

  if (c->storage != MP_SIGN1)
    return solve_carried(c, y, x, r, opts, res, tr, s,
                         CarriedBufs{c->st, c->r_work, c->partials, c->bal}, true);

  HIP_TRY(c, mp::launch_init(y, c->n, c->ld, x, c->m, c->r_work, c->st, opts->eps,
                             static_cast<long long>(opts->max_iters), s));
  {
    // the host needs the threshold and whether the run is over before it
    // chooses between the persistent and the stepping decode
    HIP_TRY(c, hipMemcpyAsync(c->h_st, c->st, sizeof(mp::DevState), hipMemcpyDeviceToHost, s));
    HIP_TRY(c, hipStreamSynchronize(s));
    // c(0) = Psi^T y and r = y in FP64; launch k runs the stop test for the
    // k-1 steps taken and takes step k, so T steps take T+2 launches
    if (!c->h_st->done)
      HIP_TRY(c, mp::launch_sign_c0(c->psis, c->sign_ws, c->n, c->m, y, c->ld, c->sign_c64,
                                    c->sign_r64, s));
    const long long T = opts->max_iters;
    const double thr = c->h_st->thr;
    // the whole decode as one persistent launch when it fits, unless the
    // caller asks for one launch per step; a launch the device refuses
    // falls back to stepping
    if (c->sign_persist && !(opts->flags & MP_SOLVE_STEP_LAUNCHES) && !c->h_st->done) {
      if (c->profiling) HIP_TRY(c, hipEventRecord(c->ev[0], s));
      // a new tag epoch for every decode (never 0 mod kSignEpochMod: the
      // zeroed words match no step); when it wraps, clear the words so that
      // none left from a decode that many decodes ago can match
      c->sign_epoch = c->sign_epoch % (mp::kSignEpochMod - 1) + 1;
      if (c->sign_epoch == 1)
        HIP_TRY(c, hipMemsetAsync(c->sign_slots, 0,
                                  sizeof(unsigned long long) * mp::kSignSlotWords * 2 *
                                      static_cast<size_t>(c->geom.grid),
                                  s));
      const hipError_t e = mp::launch_sign_persist(
          c->psis, c->sign_ws, c->n, c->m, c->ld, c->sign_c64, c->sign_r64, c->r_work, c->geom,
          c->sign_slots, c->sign_epoch, T, thr, x, c->st, tr, s);
      if (e == hipSuccess) {
        persistent = true;
        if (c->profiling) HIP_TRY(c, hipEventRecord(c->ev[1], s));
      } else {
        (void)hipGetLastError();
      }
    }
    long long k = 0;
    const mp_status st = persistent ? MP_OK :
        run_iterations(c, T > 0 ? T + 2 : 0, s, true, [&](hipEvent_t e0, hipEvent_t e1) {
      hipError_t e;
      if (e0 && (e = hipEventRecord(e0, s)) != hipSuccess) return e;
      e = mp::launch_mp_step_sign(c->psis, c->sign_ws, c->n, c->m, c->ld, c->sign_c64,
                                  c->sign_r64, c->r_work, c->sign_rrp, c->geom, c->partials, k, T,
                                  thr, x, c->st, tr, s);
      ++k;
      if (e != hipSuccess) return e;
      if (e1 && (e = hipEventRecord(e1, s)) != hipSuccess) return e;
      return hipSuccess;
    });
    if (st != MP_OK) return st;
  }

  HIP_TRY(c, hipMemcpyAsync(c->h_st, c->st, sizeof(mp::DevState), hipMemcpyDeviceToHost, s));
  HIP_TRY(c, hipStreamSynchronize(s));
  if (persistent && c->profiling) {
    // the persistent launch runs t + 2 steps (step j of it does what launch
    // j of the stepping form does): the launch time over the steps
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, c->ev[0], c->ev[1]) == hipSuccess) {
      c->prof_ms = ms;
      c->prof_launches = c->h_st->t + 2;
    }
  }
  if (r) {
    // the one-bit form keeps its FP32 r in the first n floats of r_work
    HIP_TRY(c, hipMemcpyAsync(r, c->r_work, c->n * sizeof(float), hipMemcpyDeviceToDevice, s));
  }
  HIP_TRY(c, hipStreamSynchronize(s));
  const mp_status fs = finish_result(c, res);
  if (fs == MP_OK && res) res->persistent = persistent ? 1 : 0;
  return fs;
}

mp_status mp_solve_noalloc(mp_ctx* ctx, const float* y, float* x, float* r, const mp_opts* opts,
                           mp_result* res, const mp_trace* trace, void* stream) {
  if (!ctx) return MP_EINVAL;
  ctx->err.clear();
  mp_ctx* c = ctx;
  if (c->ragged || !(c->storage == MP_F32 || c->storage == MP_BF16 ||
                     c->storage == MP_FP8_E4M3))
    return fail(c, MP_EINVAL,
                "mp_solve_noalloc decodes MP_F32, MP_BF16 and MP_FP8_E4M3 contexts of mp_create");
  if (!y || !x || !opts) return fail(c, MP_EINVAL, "y, x and opts must not be NULL");
  if (mp_status os = check_opts(c, opts, MP_SOLVE_STEP_LAUNCHES | MP_SOLVE_ASYNC); os != MP_OK)
    return os;
  if ((opts->flags & MP_SOLVE_ASYNC) && res)
    return fail(c, MP_EINVAL, "a stream-ordered decode takes res = NULL");
  if (mp_status ts = check_trace(c, trace, c->n); ts != MP_OK) return ts;
  if (c->ld > mp::kNoAllocMaxLd)
    return fail(c, MP_EINVAL, "N exceeds the static scratch (at most 16384 rows)");
  if (2 * static_cast<int64_t>(c->geom.grid) * mp::kLpTopK > mp::kNoAllocMaxKeys)
    return fail(c, MP_EINVAL, "more correlation workgroups than the static scratch holds");
  mp_trace tr{};
  if (trace) tr = *trace;
  HIP_TRY(c, hipSetDevice(c->device));
  void* base = nullptr;
  HIP_TRY(c, mp::noalloc_scratch(c->device, &base));
  unsigned char* b = static_cast<unsigned char*>(base);
  c->rescore_k = opts->rescore_k == 0 ? mp::kLpTopK : opts->rescore_k;
  c->prof_ms = 0.0;
  c->prof_launches = 0;
  return solve_carried(c, y, x, r, opts, res, tr, static_cast<hipStream_t>(stream),
                       CarriedBufs{reinterpret_cast<mp::DevState*>(b),
                                   reinterpret_cast<float*>(b + mp::kNoAllocR),
                                   reinterpret_cast<uint64_t*>(b + mp::kNoAllocKeys),
                                   reinterpret_cast<mp::BalState*>(b + mp::kNoAllocBal)},
                       false);
}

mp_status mp_solve_result(mp_ctx* ctx, mp_result* res) {
  if (!ctx) return MP_EINVAL;
  mp_ctx* c = ctx;
  if (!c->async_pending) return fail(c, MP_EINVAL, "no stream-ordered decode is pending");
  c->err.clear();
  HIP_TRY(c, hipSetDevice(c->device));
  c->async_pending = false;
  HIP_TRY(c, hipEventSynchronize(c->async_ev));
  const mp_status fs = finish_result(c, res);
  if (fs == MP_OK && res) res->persistent = c->async_persistent;
  return fs;
}

static mp_status ensure_omp(mp_ctx* c, int64_t tq) {
  mp::OmpBufs& b = c->omp;
  if (b.tq >= tq) return MP_OK;
  free_omp(c);
  const size_t ld = static_cast<size_t>(c->ld), t = static_cast<size_t>(tq);
  bool ok = hipMalloc(&b.q, sizeof(float) * t * ld) == hipSuccess &&
            hipMalloc(&b.rmat, sizeof(float) * t * t) == hipSuccess &&
            hipMalloc(&b.z, sizeof(double) * t) == hipSuccess &&
            hipMalloc(&b.sel, sizeof(int) * t) == hipSuccess &&
            hipMalloc(&b.in_s, static_cast<size_t>(c->m)) == hipSuccess &&
            hipMalloc(&b.w, sizeof(float) * ld) == hipSuccess &&
            hipMalloc(&b.h1, sizeof(float) * t) == hipSuccess &&
            hipMalloc(&b.h2, sizeof(float) * t) == hipSuccess &&
            hipMalloc(&b.hp, sizeof(float) * t * mp::kOmpProjSlices) == hipSuccess &&
            hipMalloc(&b.part, sizeof(double) * (ld / 64)) == hipSuccess &&
            hipMalloc(&b.os, sizeof(mp::OmpState)) == hipSuccess;
  if (!ok) {
    free_omp(c);
    return fail(c, MP_ENOMEM, "OMP work buffers");
  }
  b.tq = tq;
  return MP_OK;
}

mp_status mp_solve_omp(mp_ctx* ctx, const float* y, float* x, float* r, const mp_opts* opts,
                       mp_result* res, const mp_trace* trace, void* stream) {
  if (!ctx) return MP_EINVAL;
  ctx->err.clear();
  if (ctx->ragged || ctx->storage != MP_F32)
    return fail(ctx, MP_EINVAL, "mp_solve_omp needs an MP_F32 context from mp_create");
  if (!y || !x || !opts) return fail(ctx, MP_EINVAL, "y, x and opts must not be NULL");
  if (mp_status os = check_opts(ctx, opts, MP_SOLVE_STEP_LAUNCHES | MP_SOLVE_ASYNC); os != MP_OK)
    return os;
  if (opts->flags & MP_SOLVE_ASYNC) {
    if (ctx->storage == MP_SIGN1)
      return fail(ctx, MP_EINVAL, "stream-ordered decodes need MP_F32, MP_BF16 or MP_FP8_E4M3");
    if (res) return fail(ctx, MP_EINVAL, "a stream-ordered decode takes res = NULL");
  }
  mp_trace tr{};
  if (mp_status ts = check_trace(ctx, trace, ctx->n); ts != MP_OK) return ts;
  if (trace) tr = *trace;
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  hipStream_t s = static_cast<hipStream_t>(stream);
  mp_ctx* c = ctx;
  // at most min(T, N) atoms: beyond N the selected atoms span the whole space
  const long long T = std::min<long long>(opts->max_iters, c->n);
  if (mp_status bs = ensure_omp(c, std::max<long long>(T, 1)); bs != MP_OK) return bs;
  mp::OmpBufs& b = c->omp;
  HIP_TRY(c, hipMemsetAsync(b.in_s, 0, static_cast<size_t>(c->m), s));
  HIP_TRY(c, mp::launch_init(y, c->n, c->ld, x, c->m, c->r_work, c->st, opts->eps, T, s));
  HIP_TRY(c, hipMemcpyAsync(c->h_st, c->st, sizeof(mp::DevState), hipMemcpyDeviceToHost, s));
  HIP_TRY(c, hipStreamSynchronize(s));
  long long it = 0;  // iterations enqueued so far: a bound on the atoms selected
  const mp_status st = run_iterations(c, T, s, false, [&](hipEvent_t e0, hipEvent_t e1) {
    const hipError_t e = mp::launch_omp_iteration(c->psi32, c->ld, c->n, c->m, c->r_work, c->geom,
                                                  c->partials, c->st, b, it, tr, s, e0, e1);
    ++it;
    return e;
  });
  if (st != MP_OK) return st;
  HIP_TRY(c, mp::launch_omp_solve(b, c->st, x, s));
  HIP_TRY(c, hipMemcpyAsync(c->h_st, c->st, sizeof(mp::DevState), hipMemcpyDeviceToHost, s));
  if (r)
    HIP_TRY(c, hipMemcpyAsync(r, c->r_work, c->n * sizeof(float), hipMemcpyDeviceToDevice, s));
  HIP_TRY(c, hipStreamSynchronize(s));
  return finish_result(c, res);
}

mp_status mp_create_f64(mp_ctx** out, const double* psi, int64_t n, int64_t m, int64_t ld,
                        uint32_t flags, void* stream) {
  g_create_error.clear();
  if (!out) return fail(nullptr, MP_EINVAL, "out is NULL");
  *out = nullptr;
  if (!psi) return fail(nullptr, MP_EINVAL, "psi is NULL");
  if (n < 1 || m < 1) return fail(nullptr, MP_EINVAL, "n and m must be >= 1");
  if (ld < n) return fail(nullptr, MP_EINVAL, "ld must be >= n");
  if (n > kMaxN) return fail(nullptr, MP_EINVAL, "n exceeds 16384");
  if (m >= (int64_t{1} << 31)) return fail(nullptr, MP_EINVAL, "m must be < 2^31");
  if (flags & ~MP_SKIP_NORM_CHECK) return fail(nullptr, MP_EINVAL, "unknown flags");
  int dev = 0;
  hipDeviceProp_t prop;
  if (mp_status ds = open_device(dev, prop); ds != MP_OK) return ds;
  hipStream_t s = static_cast<hipStream_t>(stream);

  mp_ctx* c = new mp_ctx();
  c->device = dev;
  c->num_cus = prop.multiProcessorCount;
  c->n = n;
  c->m = m;
  c->ld = round_up(n, kLdAlign);
  c->storage = MP_F64;
  c->geom = mp::corr_f32_geometry(m, c->num_cus);  // same workgroup layout as FP32

  auto bail = [&](mp_status st, const std::string& msg) {
    free_ctx(c);
    return fail(nullptr, st, msg);
  };
  const size_t psi_bytes = static_cast<size_t>(c->ld) * static_cast<size_t>(m) * sizeof(double);
  if (hipMalloc(&c->psi64, psi_bytes) != hipSuccess) return bail(MP_ENOMEM, "dictionary copy");
  // r in two halves that alternate by launch parity
  if (hipMalloc(&c->r64_work, 2 * c->ld * sizeof(double)) != hipSuccess)
    return bail(MP_ENOMEM, "r");
  if (hipMalloc(&c->st, sizeof(mp::DevState)) != hipSuccess) return bail(MP_ENOMEM, "state");
  if (c->geom.grid * 2 > 2 * 1024)
    return bail(MP_EUNSUPPORTED, "more correlation workgroups than the key slots hold");
  // two words per workgroup, in two halves that alternate by launch parity
  const size_t nkeys = static_cast<size_t>(c->geom.grid) * 4;
  if (hipMalloc(&c->partials, sizeof(uint64_t) * nkeys) != hipSuccess)
    return bail(MP_ENOMEM, "partials");
  if (hipMalloc(&c->bal, sizeof(mp::BalState)) != hipSuccess) return bail(MP_ENOMEM, "shares");
  if (!make_host_state(c)) return bail(MP_ENOMEM, "pinned state");

  hipError_t e = hipMemsetAsync(c->psi64, 0, psi_bytes, s);
  if (e == hipSuccess)
    e = hipMemcpy2DAsync(c->psi64, c->ld * sizeof(double), psi, ld * sizeof(double),
                         n * sizeof(double), m, hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess) e = hipMemsetAsync(c->r64_work, 0, 2 * c->ld * sizeof(double), s);
  if (e == hipSuccess) e = hipMemsetAsync(c->bal, 0, sizeof(mp::BalState), s);
  if (e == hipSuccess) e = hipMemsetAsync(c->partials, 0, sizeof(uint64_t) * nkeys, s);
  if (e != hipSuccess) return bail(MP_EDEVICE, std::string("copy: ") + hipGetErrorString(e));

  double* d_norm2 = nullptr;
  if (hipMalloc(&d_norm2, sizeof(double) * m) != hipSuccess) return bail(MP_ENOMEM, "norms");
  std::vector<double> norm2(static_cast<size_t>(m));
  e = mp::launch_norms_f64(c->psi64, c->ld, n, m, d_norm2, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(norm2.data(), d_norm2, sizeof(double) * m, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(d_norm2);
  if (e != hipSuccess) return bail(MP_EDEVICE, std::string("norms: ") + hipGetErrorString(e));
  {
    std::string msg;
    const mp_status ns = check_norms(norm2, flags, msg);
    if (ns != MP_OK) return bail(ns, msg);
  }
  *out = c;
  return MP_OK;
}

mp_status mp_create_signs(mp_ctx** out, const uint32_t* signs, int64_t n, int64_t m, int64_t ldw,
                          uint32_t flags, void* stream) {
  g_create_error.clear();
  if (!out) return fail(nullptr, MP_EINVAL, "out is NULL");
  *out = nullptr;
  if (!signs) return fail(nullptr, MP_EINVAL, "signs is NULL");
  if (n < 1 || m < 1) return fail(nullptr, MP_EINVAL, "n and m must be >= 1");
  if (n > kMaxSignN) return fail(nullptr, MP_EINVAL, "n exceeds 16384");
  if (ldw < (n + 31) / 32) return fail(nullptr, MP_EINVAL, "ldw must be >= ceil(n / 32)");
  if (m >= (int64_t{1} << 31)) return fail(nullptr, MP_EINVAL, "m must be < 2^31");
  if (flags & ~MP_SKIP_NORM_CHECK) return fail(nullptr, MP_EINVAL, "unknown flags");
  int dev = 0;
  hipDeviceProp_t prop;
  if (mp_status ds = open_device(dev, prop); ds != MP_OK) return ds;
  hipStream_t s = static_cast<hipStream_t>(stream);

  mp_ctx* c = new mp_ctx();
  c->device = dev;
  c->num_cus = prop.multiProcessorCount;
  c->n = n;
  c->m = m;
  c->ld = round_up(n, kLdAlign);
  c->storage = MP_SIGN1;
  c->sign_ws = round_up((n + 31) / 32, 4);
  c->geom = mp::sign_geometry(n, m, c->num_cus);

  auto bail = [&](mp_status st, const std::string& msg) {
    free_ctx(c);
    return fail(nullptr, st, msg);
  };
  const size_t words = static_cast<size_t>(m) * static_cast<size_t>(c->sign_ws);
  if (hipMalloc(&c->psis, words * sizeof(uint32_t)) != hipSuccess)
    return bail(MP_ENOMEM, "sign-bit copy");
  if (hipMalloc(&c->sign_c64, sizeof(double) * m) != hipSuccess)
    return bail(MP_ENOMEM, "correlations");
  if (hipMalloc(&c->sign_r64, sizeof(double) * c->ld) != hipSuccess) return bail(MP_ENOMEM, "r");
  if (hipMalloc(&c->r_work, c->ld * sizeof(float)) != hipSuccess) return bail(MP_ENOMEM, "r");
  if (hipMalloc(&c->st, sizeof(mp::DevState)) != hipSuccess) return bail(MP_ENOMEM, "state");
  if (c->geom.grid > 1024)
    return bail(MP_EUNSUPPORTED, "more correlation workgroups than the key slots hold");
  // pair keys, one per workgroup, in two halves alternating by launch parity
  const size_t nkeys = 4 * static_cast<size_t>(c->geom.grid);
  if (hipMalloc(&c->partials, sizeof(uint64_t) * nkeys) != hipSuccess)
    return bail(MP_ENOMEM, "partials");
  if (hipMalloc(&c->sign_rrp, sizeof(double) * 2 * c->geom.grid) != hipSuccess)
    return bail(MP_ENOMEM, "partial norms");
  // the persistent decode (bits in LDS): one workgroup per CU, all resident
  c->sign_persist = mp::sign_persist_fits(n, m, c->ld, c->sign_ws, c->geom, c->num_cus) &&
                    mp::sign_persist_resident(n, c->sign_ws, c->geom, c->num_cus);
  const size_t slot_bytes =
      sizeof(unsigned long long) * mp::kSignSlotWords * 2 * static_cast<size_t>(c->geom.grid);
  if (hipMalloc(&c->sign_slots, slot_bytes) != hipSuccess)
    return bail(MP_ENOMEM, "step records");
  if (!make_host_state(c)) return bail(MP_ENOMEM, "pinned state");
  hipError_t e = mp::launch_copy_signs(signs, ldw, n, m, c->sign_ws, c->psis, s);
  if (e == hipSuccess) e = hipMemsetAsync(c->r_work, 0, c->ld * sizeof(float), s);
  if (e == hipSuccess) e = hipMemsetAsync(c->partials, 0, sizeof(uint64_t) * nkeys, s);
  if (e == hipSuccess)
    e = hipMemsetAsync(c->sign_slots, 0, slot_bytes, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return bail(MP_EDEVICE, std::string("copy: ") + hipGetErrorString(e));
  *out = c;
  return MP_OK;
}

mp_status mp_solve_f64(mp_ctx* ctx, const double* y, double* x, double* r, const mp_opts* opts,
                       mp_result* res, const mp_trace_f64* trace, void* stream) {
  if (!ctx) return MP_EINVAL;
  ctx->err.clear();
  if (ctx->ragged || ctx->storage != MP_F64)
    return fail(ctx, MP_EINVAL, "mp_solve_f64 needs a context from mp_create_f64");
  if (!y || !x || !opts) return fail(ctx, MP_EINVAL, "y, x and opts must not be NULL");
  if (mp_status os = check_opts(ctx, opts); os != MP_OK) return os;
  mp_trace_f64 tr{};
  if (mp_status ts = check_trace(ctx, trace, ctx->n); ts != MP_OK) return ts;
  if (trace) tr = *trace;
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  hipStream_t s = static_cast<hipStream_t>(stream);
  mp_ctx* c = ctx;

  HIP_TRY(c, mp::launch_init_f64(y, c->n, c->ld, x, c->m, c->r64_work, c->st, opts->eps,
                                 static_cast<long long>(opts->max_iters), s));
  HIP_TRY(c, hipMemcpyAsync(c->h_st, c->st, sizeof(mp::DevState), hipMemcpyDeviceToHost, s));
  HIP_TRY(c, hipStreamSynchronize(s));
  // launch k takes step k (k >= 1) and runs pass k+1: T steps take T+1
  // launches; r ends in the half the state names
  long long k = 0;
  const long long T = opts->max_iters;
  const double thr = c->h_st->thr;
  const mp_status st = run_iterations(c, T > 0 ? T + 1 : 0, s, true, [&](hipEvent_t e0, hipEvent_t e1) {
    hipError_t e;
    if (e0 && (e = hipEventRecord(e0, s)) != hipSuccess) return e;
    e = mp::launch_mp_step_f64(c->psi64, c->ld, c->n, c->m, c->r64_work, c->geom, c->partials,
                               c->bal, k, T, thr, x, c->st, tr, s);
    ++k;
    if (e != hipSuccess) return e;
    if (e1 && (e = hipEventRecord(e1, s)) != hipSuccess) return e;
    return hipSuccess;
  });
  if (st != MP_OK) return st;

  HIP_TRY(c, hipMemcpyAsync(c->h_st, c->st, sizeof(mp::DevState), hipMemcpyDeviceToHost, s));
  HIP_TRY(c, hipStreamSynchronize(s));
  if (r)
    HIP_TRY(c, hipMemcpyAsync(r, c->r64_work + (c->h_st->r_sel ? c->ld : 0),
                              c->n * sizeof(double), hipMemcpyDeviceToDevice, s));
  HIP_TRY(c, hipStreamSynchronize(s));
  return finish_result(c, res);
}


// Make sure the context has a BF16 copy for the batched product and buffers
// for `B` signals.
static mp_status ensure_batched(mp_ctx* c, int64_t B, hipStream_t s) {
  if (!c->psibt) {
    const size_t bytes =
        static_cast<size_t>(c->ld) * static_cast<size_t>(round_up(c->m, 16)) * 2;
    if (hipMalloc(&c->psibt, bytes) != hipSuccess) return fail(c, MP_ENOMEM, "BF16 tiles");
    HIP_TRY(c, mp::launch_tile_bf16(c->psi32, c->ld, c->m, c->psibt, s));
  }
  if (B <= c->bcap) return MP_OK;
  free_batched(c);
  const int64_t cap = B;
  const int mtiles = mp::bcorr_mtiles(c->m, mp::kBTileMinAtoms);  // the most lists of a tiling
  const size_t ldb = static_cast<size_t>(c->ld);
  c->ldq = c->ld + 32;
  bool ok = hipMalloc(&c->b_r32, sizeof(float) * ldb * cap) == hipSuccess &&
            hipMalloc(&c->b_rq, sizeof(uint16_t) * static_cast<size_t>(c->ldq) * cap) ==
                hipSuccess &&
            hipMalloc(&c->b_slots, sizeof(mp::BSlot) * cap) == hipSuccess &&
            hipMalloc(&c->b_act, sizeof(int) * 2 * cap) == hipSuccess &&
            hipMalloc(&c->b_state, sizeof(mp::BState)) == hipSuccess &&
            hipMalloc(&c->b_partials, sizeof(uint64_t) * cap * mtiles * 8) == hipSuccess &&
            hipMalloc(&c->b_keep, sizeof(int) * 4 * cap) == hipSuccess &&
            hipMalloc(&c->b_tcap, sizeof(long long) * cap) == hipSuccess &&
            hipHostMalloc(&c->h_slots, sizeof(mp::BSlot) * cap, hipHostMallocDefault) ==
                hipSuccess &&
            hipHostMalloc(&c->h_bstate, 2 * sizeof(mp::BState), hipHostMallocDefault) ==
                hipSuccess;
  if (!ok) {
    free_batched(c);
    return fail(c, MP_ENOMEM, "batched work buffers");
  }
  HIP_TRY(c, hipMemsetAsync(c->b_keep, 0, sizeof(int) * 4 * cap, s));
  HIP_TRY(c, hipMemsetAsync(c->b_state, 0, sizeof(mp::BState), s));
  c->bcap = cap;
  return MP_OK;
}

mp_status mp_solve_batched(mp_ctx* ctx, const float* Y, int64_t ldy, int64_t B, float* X,
                           int64_t ldx, float* R, int64_t ldr, const mp_opts* opts,
                           const int64_t* max_iters_b, mp_result* res, const mp_trace* trace,
                           void* stream) {
  if (!ctx) return MP_EINVAL;
  ctx->err.clear();
  mp_ctx* c = ctx;
  if (c->ragged) return fail(c, MP_EINVAL, "a ragged context is decoded with mp_solve_ragged");
  if (c->storage == MP_F64 || c->storage == MP_SIGN1)
    return fail(c, MP_EINVAL, "batched decoding needs an FP32, BF16 or FP8 context");
  if (mp_status ps = check_not_pending(c); ps != MP_OK) return ps;
  if (B < 0) return fail(c, MP_EINVAL, "B must be >= 0");
  if (B == 0) return MP_OK;
  if (B >= (int64_t{1} << 31) / 2) return fail(c, MP_EINVAL, "B too large");
  if (!Y || !X || !opts) return fail(c, MP_EINVAL, "Y, X and opts must not be NULL");
  if (ldy < c->n || ldx < c->m || (R && ldr < c->n))
    return fail(c, MP_EINVAL, "leading dimensions must be >= the column lengths");
  if (!(opts->eps >= 0.0) || !isfinite(opts->eps))
    return fail(c, MP_EINVAL, "eps must be finite and >= 0");
  if (opts->max_iters < 0) return fail(c, MP_EINVAL, "max_iters must be >= 0");
  if (opts->flags != 0) return fail(c, MP_EINVAL, "opts.flags must be 0");
  if (opts->rescore_k < 0 || opts->rescore_k > 8)
    return fail(c, MP_EINVAL, "rescore_k must be in 0..8");
  long long tmax = opts->max_iters;
  if (max_iters_b) {
    tmax = 0;
    for (int64_t b = 0; b < B; ++b) {
      if (max_iters_b[b] < 0) return fail(c, MP_EINVAL, "max_iters_b entries must be >= 0");
      tmax = std::max<long long>(tmax, max_iters_b[b]);
    }
  }
  mp_trace tr{};
  if (mp_status ts = check_trace(c, trace, c->n); ts != MP_OK) return ts;
  if (trace) tr = *trace;
  HIP_TRY(c, hipSetDevice(c->device));
  hipStream_t s = static_cast<hipStream_t>(stream);
  mp_status st = ensure_batched(c, B, s);
  if (st != MP_OK) return st;
  const int rk = opts->rescore_k == 0 ? mp::kLpTopK : opts->rescore_k;
  c->prof_ms = 0.0;
  c->prof_launches = 0;
  if (max_iters_b)
    HIP_TRY(c, hipMemcpyAsync(c->b_tcap, max_iters_b, sizeof(long long) * B,
                              hipMemcpyHostToDevice, s));
  HIP_TRY(c, mp::launch_binit(Y, ldy, c->n, c->ld, X, ldx, c->m, c->b_r32, c->b_rq, c->ldq,
                              c->b_slots,
                              max_iters_b ? c->b_tcap : nullptr, opts->max_iters, opts->eps,
                              static_cast<int>(B), c->b_act, c->b_keep, c->bcap, c->b_state, s));

  // Rounds in chunks, two chunks in flight; the kernels stop doing work once
  // the active list is empty.  No signal runs more than tmax rounds.
  hipEvent_t done_ev[2] = {nullptr, nullptr};
  HIP_TRY(c, hipEventCreateWithFlags(&done_ev[0], hipEventDisableTiming));
  HIP_TRY(c, hipEventCreateWithFlags(&done_ev[1], hipEventDisableTiming));
  long long issued = 0;
  int chunk = 4, next = 0, inflight = 0;
  long long slot_base[2] = {0, 0};
  int slot_len[2] = {0, 0};
  bool finished = false;
  mp_status status = MP_OK;
  // upper bound on the active count used to size each round's grids: all
  // B at first, then the count read back after each completed chunk
  int nact_hint = static_cast<int>(B);
  auto account = [&](int k, int n_after) {
    if (!c->profiling) return;
    (void)n_after;
    for (int j = 0; j < slot_len[k]; ++j) {
      if ((slot_base[k] + j) % c->prof_every != 0) continue;
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, c->ev[(k * kMaxChunk + j) * 2],
                              c->ev[(k * kMaxChunk + j) * 2 + 1]) == hipSuccess) {
        c->prof_ms += ms;
        c->prof_launches += 1;
      }
    }
  };
  while (!finished && status == MP_OK) {
    while (inflight < 2 && issued < tmax && status == MP_OK) {
      const int k = next;
      const int len = static_cast<int>(std::min<long long>(chunk, tmax - issued));
      for (int j = 0; j < len; ++j) {
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (c->profiling && (issued + j) % c->prof_every == 0) {
          e0 = c->ev[(k * kMaxChunk + j) * 2];
          e1 = c->ev[(k * kMaxChunk + j) * 2 + 1];
        }
        hipError_t e = mp::launch_bround(c->psibt, c->psi32, c->ld, c->n, c->m, c->b_r32,
                                         c->b_rq, c->ldq, X, ldx, c->b_slots, c->b_act,
                                         c->b_keep, c->bcap, c->b_state, c->b_partials,
                                         issued + j, nact_hint, c->b_cfg, c->num_cus, rk, tr, s,
                                         e0, e1);
        if (e != hipSuccess) {
          status = fail(c, MP_EDEVICE, std::string("launch: ") + hipGetErrorString(e));
          break;
        }
      }
      if (status != MP_OK) break;
      slot_base[k] = issued;
      slot_len[k] = len;
      issued += len;
      hipError_t e = hipMemcpyAsync(&c->h_bstate[k], c->b_state, sizeof(mp::BState),
                                    hipMemcpyDeviceToHost, s);
      if (e == hipSuccess) e = hipEventRecord(done_ev[k], s);
      if (e != hipSuccess) {
        status = fail(c, MP_EDEVICE, std::string("state copy: ") + hipGetErrorString(e));
        break;
      }
      ++inflight;
      next ^= 1;
      chunk = std::min(chunk * 2, kMaxChunk);
    }
    if (status != MP_OK || inflight == 0) break;
    const int old = inflight == 2 ? next : (next ^ 1);
    hipError_t e = hipEventSynchronize(done_ev[old]);
    if (e != hipSuccess) {
      status = fail(c, MP_EDEVICE, std::string("sync: ") + hipGetErrorString(e));
      break;
    }
    --inflight;
    // the length of the list the chunk's last round r left for round r+1
    // (the signals still running after round r-1): an upper bound for every
    // later round, zero once all have stopped
    const mp::BState& hb = c->h_bstate[old];
    const long long r_last = slot_base[old] + slot_len[old] - 1;
    const int n_after = hb.n_active[(r_last + 1) & 1];
    account(old, n_after);
    // rounds already in flight were sized with the older hint, which is also
    // an upper bound; the count never increases
    nact_hint = std::min(nact_hint, n_after);
    if (n_after == 0) finished = true;
  }
  if (hipStreamSynchronize(s) != hipSuccess && status == MP_OK)
    status = fail(c, MP_EDEVICE, "stream synchronize failed");
  (void)hipEventDestroy(done_ev[0]);
  (void)hipEventDestroy(done_ev[1]);
  if (status != MP_OK) return status;

  if (R)
    HIP_TRY(c, hipMemcpy2DAsync(R, ldr * sizeof(float), c->b_r32, c->ld * sizeof(float),
                                c->n * sizeof(float), B, hipMemcpyDeviceToDevice, s));
  HIP_TRY(c, hipMemcpyAsync(c->h_slots, c->b_slots, sizeof(mp::BSlot) * B, hipMemcpyDeviceToHost,
                            s));
  HIP_TRY(c, hipStreamSynchronize(s));
  bool nonfinite = false, internal = false;
  for (int64_t b = 0; b < B; ++b) {
    const mp::BSlot& d = c->h_slots[b];
    nonfinite |= d.reason == mp::kStopNonFinite;
    internal |= d.reason == mp::kStopInternal;
    if (res) {
      res[b].iters = d.t;
      res[b].yy = d.yy;
      res[b].rr = d.rr;
      res[b].stop_reason = d.reason;
      res[b].persistent = 0;
    }
  }
  if (internal)
    return fail(c, MP_EDEVICE, "internal error: a selected index fell outside the dictionary");
  if (nonfinite) return fail(c, MP_ENONFINITE, "a column of Y holds NaN or Inf");
  return MP_OK;
}


// ---------------------------------------------------------------------------
// Many independent instances

mp_status mp_create_ragged(mp_ctx** out, const mp_instance* inst, int64_t count, mp_dtype storage,
                           uint32_t flags, void* stream) {
  g_create_error.clear();
  if (!out) return fail(nullptr, MP_EINVAL, "out is NULL");
  *out = nullptr;
  if (!inst) return fail(nullptr, MP_EINVAL, "inst is NULL");
  if (count < 1 || count >= (int64_t{1} << 30)) return fail(nullptr, MP_EINVAL, "bad count");
  if (flags & ~MP_SKIP_NORM_CHECK) return fail(nullptr, MP_EINVAL, "unknown flags");
  if (storage != MP_F32 && storage != MP_BF16) {
    if (storage == MP_FP8_E4M3)
      return fail(nullptr, MP_EUNSUPPORTED, "ragged instances support MP_F32 and MP_BF16");
    return fail(nullptr, MP_EINVAL, "unknown storage type");
  }
  for (int64_t i = 0; i < count; ++i) {
    const mp_instance& d = inst[i];
    char buf[96];
    snprintf(buf, sizeof buf, "instance %lld: ", static_cast<long long>(i));
    if (!d.psi) return fail(nullptr, MP_EINVAL, std::string(buf) + "psi is NULL");
    if (d.n < 1 || d.m < 1) return fail(nullptr, MP_EINVAL, std::string(buf) + "n, m must be >= 1");
    if (d.ld < d.n) return fail(nullptr, MP_EINVAL, std::string(buf) + "ld must be >= n");
    if (d.n > kMaxRaggedN) return fail(nullptr, MP_EINVAL, std::string(buf) + "n exceeds 8192");
    if (d.m >= (int64_t{1} << 31)) return fail(nullptr, MP_EINVAL, std::string(buf) + "m too large");
  }
  int dev = 0, ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1)
    return fail(nullptr, MP_EDEVICE, "no HIP device");
  HIP_TRY(nullptr, hipGetDevice(&dev));
  hipDeviceProp_t prop;
  HIP_TRY(nullptr, hipGetDeviceProperties(&prop, dev));
  if (strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(nullptr, MP_EUNSUPPORTED, std::string("device is ") + prop.gcnArchName +
                                              ", this library is built for gfx950");
  hipStream_t s = static_cast<hipStream_t>(stream);
  mp_ctx* c = new mp_ctx();
  c->device = dev;
  c->num_cus = prop.multiProcessorCount;
  c->storage = storage;
  c->ragged = true;
  c->r_count = count;
  // the untuned shape: the tuner's choice on the 512-instance mix of
  // N in {128, ..., 1024} (one 1024-thread workgroup per CU, the largest
  // instances in three parts)
  c->r_cfg = storage == MP_BF16 ? mp::RConfig{1024, 2, 2, kRaggedDefaultSplit}
                                : mp::RConfig{1024, 1, 2, kRaggedDefaultSplit};
  auto bail = [&](mp_status st, const std::string& msg) {
    free_ctx(c);
    return fail(nullptr, st, msg);
  };
  // packed layout of the copies, descriptors, and the work order
  std::vector<mp::RInst> desc(static_cast<size_t>(count));
  std::vector<int64_t> psi_off(static_cast<size_t>(count));
  int64_t elems = 0, yo = 0, xo = 0, msum = 0;
  c->r_n.resize(count);
  c->r_m.resize(count);
  for (int64_t i = 0; i < count; ++i) {
    const int64_t ld = round_up(inst[i].n, kLdAlign);
    psi_off[i] = elems;
    desc[i].n = inst[i].n;
    desc[i].m = inst[i].m;
    desc[i].ld = ld;
    desc[i].y_off = yo;
    desc[i].x_off = xo;
    elems += ld * inst[i].m;
    yo += inst[i].n;
    xo += inst[i].m;
    msum += inst[i].m;
    c->r_max_ld = std::max(c->r_max_ld, ld);
    c->r_n[i] = inst[i].n;
    c->r_m[i] = inst[i].m;
  }
  c->r_sum_n = yo;
  c->r_sum_m = xo;
  if (hipMalloc(&c->r_psi32, sizeof(float) * elems) != hipSuccess)
    return bail(MP_ENOMEM, "dictionary copies");
  if (storage == MP_BF16 && hipMalloc(&c->r_psib, sizeof(uint16_t) * elems) != hipSuccess)
    return bail(MP_ENOMEM, "BF16 copies");
  const int64_t max_split = std::min<int64_t>(count, kMaxRaggedSplit);
  if (hipMalloc(&c->r_inst, sizeof(mp::RInst) * count) != hipSuccess ||
      hipMalloc(&c->r_items, sizeof(mp::RItem) * count * mp::kRaggedMaxParts) != hipSuccess ||
      hipMalloc(&c->r_slots, sizeof(unsigned long long) * max_split * 2 * mp::kRaggedMaxParts *
                                 mp::kRaggedRecWords) != hipSuccess ||
      hipHostMalloc(&c->h_rq, sizeof(mp::RQueue), hipHostMallocDefault) != hipSuccess ||
      hipMalloc(&c->r_caps, sizeof(long long) * count) != hipSuccess ||
      hipMalloc(&c->r_res, sizeof(mp::RResult) * count) != hipSuccess ||
      hipMalloc(&c->r_queue, sizeof(mp::RQueue)) != hipSuccess ||
      hipHostMalloc(&c->h_rres, sizeof(mp::RResult) * count, hipHostMallocDefault) != hipSuccess)
    return bail(MP_ENOMEM, "ragged buffers");
  if (hipStreamCreateWithFlags(&c->r_cap_stream, hipStreamNonBlocking) != hipSuccess)
    return bail(MP_EDEVICE, "capture stream");
  hipError_t e = hipMemsetAsync(c->r_psi32, 0, sizeof(float) * elems, s);
  for (int64_t i = 0; i < count && e == hipSuccess; ++i)
    e = hipMemcpy2DAsync(c->r_psi32 + psi_off[i], desc[i].ld * sizeof(float), inst[i].psi,
                         inst[i].ld * sizeof(float), inst[i].n * sizeof(float), inst[i].m,
                         hipMemcpyDeviceToDevice, s);
  if (e != hipSuccess) return bail(MP_EDEVICE, std::string("copy: ") + hipGetErrorString(e));
  // column norms of every instance (eq. 4)
  double* d_norm2 = nullptr;
  if (hipMalloc(&d_norm2, sizeof(double) * msum) != hipSuccess) return bail(MP_ENOMEM, "norms");
  std::vector<double> norm2(static_cast<size_t>(msum));
  int64_t mo = 0;
  for (int64_t i = 0; i < count && e == hipSuccess; ++i) {
    e = mp::launch_norms(c->r_psi32 + psi_off[i], desc[i].ld, desc[i].n, desc[i].m,
                         d_norm2 + mo, nullptr, s);
    mo += desc[i].m;
  }
  if (e == hipSuccess)
    e = hipMemcpyAsync(norm2.data(), d_norm2, sizeof(double) * msum, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(d_norm2);
  if (e != hipSuccess) return bail(MP_EDEVICE, std::string("norms: ") + hipGetErrorString(e));
  mo = 0;
  for (int64_t i = 0; i < count; ++i) {
    for (int64_t j = 0; j < desc[i].m; ++j) {
      const double v = norm2[mo + j];
      char buf[128];
      if (!isfinite(v)) {
        snprintf(buf, sizeof buf, "instance %lld column %lld holds NaN or Inf",
                 static_cast<long long>(i), static_cast<long long>(j));
        return bail(MP_ENONFINITE, buf);
      }
      if (!(flags & MP_SKIP_NORM_CHECK) && fabs(sqrt(v) - 1.0) > kNormTol) {
        snprintf(buf, sizeof buf, "instance %lld column %lld has norm %.9g",
                 static_cast<long long>(i), static_cast<long long>(j), sqrt(v));
        return bail(MP_ENOTNORM, buf);
      }
    }
    mo += desc[i].m;
  }
  if (storage == MP_BF16) {
    // padding rows are zero and quantise to zero: one pass over everything
    e = mp::launch_quant_bf16(c->r_psi32, elems, 1, c->r_psib, s);
    if (e != hipSuccess) return bail(MP_EDEVICE, "quantise");
  }
  for (int64_t i = 0; i < count; ++i) {
    desc[i].psi32 = c->r_psi32 + psi_off[i];
    desc[i].psib = storage == MP_BF16 ? c->r_psib + psi_off[i] : nullptr;
  }
  // most work first (iterations grow with n, a pass costs n * m); the work
  // list itself is built per launch shape (ragged_items)
  c->r_est.resize(count);
  for (int64_t i = 0; i < count; ++i)
    c->r_est[i] = static_cast<double>(desc[i].n) * desc[i].n * desc[i].m;
  c->r_order.resize(count);
  for (int64_t i = 0; i < count; ++i) c->r_order[i] = static_cast<int>(i);
  std::stable_sort(c->r_order.begin(), c->r_order.end(),
                   [&](int a1, int b1) { return c->r_est[a1] > c->r_est[b1]; });
  e = hipMemcpyAsync(c->r_inst, desc.data(), sizeof(mp::RInst) * count, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return bail(MP_EDEVICE, std::string("upload: ") + hipGetErrorString(e));
  *out = c;
  return MP_OK;
}

mp_status mp_batched_set_config(mp_ctx* ctx, const mp_batched_config* cfg) {
  if (!ctx || !cfg) return MP_EINVAL;
  if (ctx->ragged || ctx->storage == MP_F64 || ctx->storage == MP_SIGN1)
    return fail(ctx, MP_EINVAL, "batched decoding needs an FP32, BF16 or FP8 context");
  if (cfg->atoms128_above < 0 || cfg->atoms64_above < 0 || cfg->atoms32_above < 0)
    return fail(ctx, MP_EINVAL, "the active counts must be >= 0");
  ctx->b_cfg = mp::BConfig{cfg->atoms128_above, cfg->atoms64_above, cfg->atoms32_above};
  return MP_OK;
}

mp_status mp_batched_get_config(const mp_ctx* ctx, mp_batched_config* cfg) {
  if (!ctx || !cfg || ctx->ragged) return MP_EINVAL;
  cfg->atoms128_above = ctx->b_cfg.atoms128_above;
  cfg->atoms64_above = ctx->b_cfg.atoms64_above;
  cfg->atoms32_above = ctx->b_cfg.atoms32_above;
  return MP_OK;
}

mp_status mp_ragged_set_config(mp_ctx* ctx, const mp_ragged_config* cfg) {
  if (!ctx || !cfg) return MP_EINVAL;
  if (!ctx->ragged) return fail(ctx, MP_EINVAL, "not a ragged context");
  mp::RConfig cf{cfg->threads, cfg->cols_per_wave, cfg->wgs_per_cu,
                 cfg->split == 0 ? kRaggedDefaultSplit : cfg->split};
  if (!mp::ragged_config_valid(cf, ctx->storage == MP_BF16))
    return fail(ctx, MP_EINVAL, "threads must be 256/512/1024, cols_per_wave 1/2/4, "
                                "wgs_per_cu 1..8, split 0..8");
  ctx->r_cfg = cf;
  return MP_OK;
}

mp_status mp_ragged_get_config(const mp_ctx* ctx, mp_ragged_config* cfg) {
  if (!ctx || !cfg || !ctx->ragged) return MP_EINVAL;
  cfg->threads = ctx->r_cfg.threads;
  cfg->cols_per_wave = ctx->r_cfg.cols_per_wave;
  cfg->wgs_per_cu = ctx->r_cfg.wgs_per_cu;
  cfg->split = ctx->r_cfg.split;
  return MP_OK;
}

// The work list for the current launch shape: instances most work first; an
// instance whose work exceeds the average per workgroup of the grid is cut
// into parts (at most cfg.split, each a share of its columns; at most
// kMaxRaggedSplit instances are cut), consecutive in the list.
static mp_status ragged_items(mp_ctx* c, int grid, hipStream_t s) {
  if (c->r_nitems > 0 && memcmp(&c->r_items_cfg, &c->r_cfg, sizeof(mp::RConfig)) == 0)
    return MP_OK;
  double total = 0.0;
  for (double w : c->r_est) total += w;
  const double target = total / std::max(grid, 1);
  std::vector<mp::RItem> items;
  items.reserve(c->r_count * 2);
  int nslots = 0;
  for (int id : c->r_order) {
    int parts = 1;
    if (c->r_cfg.split > 1 && nslots < kMaxRaggedSplit && target > 0.0) {
      const double want = std::ceil(c->r_est[id] / target);
      parts = static_cast<int>(std::min<double>(want, c->r_cfg.split));
      parts = std::max(1, std::min<int>(parts, static_cast<int>(c->r_m[id])));
    }
    const int slot = parts > 1 ? nslots++ : -1;
    for (int p = 0; p < parts; ++p) items.push_back(mp::RItem{id, p, parts, slot});
  }
  HIP_TRY(c, hipMemcpyAsync(c->r_items, items.data(), sizeof(mp::RItem) * items.size(),
                            hipMemcpyHostToDevice, s));
  HIP_TRY(c, hipStreamSynchronize(s));
  c->r_nitems = static_cast<int>(items.size());
  c->r_nslots = nslots;
  c->r_items_cfg = c->r_cfg;
  return MP_OK;
}

mp_status mp_solve_ragged(mp_ctx* ctx, const float* Y, float* X, float* R, const mp_opts* opts,
                          const int64_t* max_iters, mp_result* res, const mp_trace* trace,
                          void* stream) {
  if (!ctx) return MP_EINVAL;
  ctx->err.clear();
  mp_ctx* c = ctx;
  if (!c->ragged) return fail(c, MP_EINVAL, "not a ragged context (use mp_create_ragged)");
  if (!Y || !X || !opts) return fail(c, MP_EINVAL, "Y, X and opts must not be NULL");
  if (!(opts->eps >= 0.0) || !isfinite(opts->eps))
    return fail(c, MP_EINVAL, "eps must be finite and >= 0");
  if (opts->max_iters < 0) return fail(c, MP_EINVAL, "max_iters must be >= 0");
  if (opts->flags != 0) return fail(c, MP_EINVAL, "opts.flags must be 0");
  if (opts->rescore_k < 0 || opts->rescore_k > 8)
    return fail(c, MP_EINVAL, "rescore_k must be in 0..8");
  if (max_iters)
    for (int64_t i = 0; i < c->r_count; ++i)
      if (max_iters[i] < 0) return fail(c, MP_EINVAL, "max_iters entries must be >= 0");
  mp_trace tr{};
  const int64_t max_n = *std::max_element(c->r_n.begin(), c->r_n.end());
  if (mp_status ts = check_trace(c, trace, max_n); ts != MP_OK) return ts;
  if (trace) tr = *trace;
  HIP_TRY(c, hipSetDevice(c->device));
  hipStream_t s = static_cast<hipStream_t>(stream);
  const bool lp = c->storage == MP_BF16;
  const int rk = opts->rescore_k == 0 ? mp::kLpTopK : opts->rescore_k;
  const long long* caps = max_iters ? c->r_caps : nullptr;
  if (max_iters)
    HIP_TRY(c, hipMemcpyAsync(c->r_caps, max_iters, sizeof(long long) * c->r_count,
                              hipMemcpyHostToDevice, s));
  int grid = c->num_cus * c->r_cfg.wgs_per_cu;
  if (mp_status is = ragged_items(c, grid, s); is != MP_OK) return is;
  if (grid > c->r_nitems) grid = c->r_nitems;
  const size_t lds = static_cast<size_t>(c->r_max_ld) * sizeof(float);
  // polls per wait between the parts of an instance before the solve fails;
  // MP_RAGGED_SPIN_LIMIT (a non-negative integer; 0 gives up at the first
  // wait) overrides it, so that tests can drive the failure path
  long long spin_limit = 1ll << 22;
  if (const char* env = getenv("MP_RAGGED_SPIN_LIMIT")) {
    char* end = nullptr;
    const long long v = strtoll(env, &end, 10);
    if (end != env && v >= 0) spin_limit = v;
  }

  // (re)capture the solve as a graph when its arguments change
  struct Key {
    const void *y, *x, *r, *caps, *ti, *tc, *trr, *tres;
    double eps;
    long long cap_all, tcap, tldr, spin;
    int rk, threads, cc, grid, split, nitems, nslots, pad;
  } key{Y, X, R, caps, tr.idx, tr.coef, tr.rr, tr.r, opts->eps, opts->max_iters, tr.cap, tr.ldr,
        spin_limit, rk, c->r_cfg.threads, c->r_cfg.cols_per_wave, grid, c->r_cfg.split,
        c->r_nitems, c->r_nslots, 0};
  const unsigned char* kb = reinterpret_cast<const unsigned char*>(&key);
  std::vector<unsigned char> kv(kb, kb + sizeof key);
  if (!c->r_graph || kv != c->r_graph_key) {
    if (c->r_graph) {
      (void)hipGraphExecDestroy(c->r_graph);
      c->r_graph = nullptr;
    }
    HIP_TRY(c, hipStreamBeginCapture(c->r_cap_stream, hipStreamCaptureModeThreadLocal));
    hipError_t le = mp::launch_ragged(c->r_cfg, lp, grid, lds, c->r_inst, c->r_items,
                                      c->r_nitems, Y, X, R, caps, opts->max_iters, opts->eps,
                                      rk, c->r_res, c->r_queue, c->r_slots, c->r_nslots,
                                      spin_limit, tr, c->r_cap_stream);
    hipGraph_t g = nullptr;
    hipError_t ee = hipStreamEndCapture(c->r_cap_stream, &g);
    if (le != hipSuccess || ee != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return fail(c, MP_EDEVICE, std::string("capture: ") +
                                     hipGetErrorString(le != hipSuccess ? le : ee));
    }
    hipError_t ie = hipGraphInstantiate(&c->r_graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ie != hipSuccess) {
      c->r_graph = nullptr;
      return fail(c, MP_EDEVICE, std::string("instantiate: ") + hipGetErrorString(ie));
    }
    c->r_graph_key = kv;
  }
  c->prof_ms = 0.0;
  c->prof_launches = 0;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (c->profiling) {
    e0 = c->ev[0];
    e1 = c->ev[1];
    HIP_TRY(c, hipEventRecord(e0, s));
  }
  HIP_TRY(c, hipGraphLaunch(c->r_graph, s));
  if (e1) HIP_TRY(c, hipEventRecord(e1, s));
  HIP_TRY(c, hipMemcpyAsync(c->h_rres, c->r_res, sizeof(mp::RResult) * c->r_count,
                            hipMemcpyDeviceToHost, s));
  HIP_TRY(c, hipMemcpyAsync(c->h_rq, c->r_queue, sizeof(mp::RQueue), hipMemcpyDeviceToHost, s));
  HIP_TRY(c, hipStreamSynchronize(s));
  if (e1) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, e0, e1) == hipSuccess) {
      c->prof_ms = ms;
      c->prof_launches = 1;
    }
  }
  bool nonfinite = false, internal = false;
  for (int64_t i = 0; i < c->r_count; ++i) {
    const mp::RResult& d = c->h_rres[i];
    nonfinite |= d.reason == mp::kStopNonFinite;
    internal |= d.reason == mp::kStopInternal;
    if (res) {
      res[i].iters = d.t;
      res[i].yy = d.yy;
      res[i].rr = d.rr;
      res[i].stop_reason = d.reason;
      res[i].persistent = 0;
    }
  }
  if (c->h_rq->fail)
    return fail(c, MP_EDEVICE, "a wait between the parts of an instance gave up");
  if (internal)
    return fail(c, MP_EDEVICE, "internal error: a selected index fell outside the dictionary");
  if (nonfinite) return fail(c, MP_ENONFINITE, "an instance's y holds NaN or Inf");
  return MP_OK;
}

}  // extern "C"
