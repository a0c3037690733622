// Per-kernel device timing of the online calls (instrumentation, off by
// default).  While a model's timer is enabled, each launch site brackets its
// kernel with a pair of HIP events on the launch stream and records the
// algorithmic flops and bytes of that launch; reading the timer synchronizes
// on the recorded events and sums per kernel kind.
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

namespace lrbms {

enum KernelKind {
  KK_MOMENTS = 0,
  KK_LSQ,
  KK_AFFINE_SUM,
  KK_ASM_DIAG,
  KK_ASM_REDUCE,
  KK_ASM_IFACE,
  KK_FRONT_ASM,
  KK_FRONT_FACTOR0,
  KK_FRONT_STEP,
  KK_FRONT_BACKWARD,
  KK_FRONT_UPDATE,
  KK_FRONT_BW_GEMV,
  KK_RECONSTRUCT,
  KK_FLUX,
  KK_TRANSPORT,
  KK_LIMITER,
  KK_RESIDUAL,
  KK_FRONT_FORWARD,
  KK_FRONT_FW_GEMV,
  KK_FRONT_SCHUR,
  KK_COUNT
};

const char* kernel_kind_name(int kind);

struct KernelTimer {
  struct Rec {
    int kind;
    hipEvent_t a, b;
    double flops, bytes;
  };
  bool on = false;
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
  long long n[KK_COUNT] = {};
  double ms[KK_COUNT] = {}, flops[KK_COUNT] = {}, bytes[KK_COUNT] = {};
  // launches recorded with flops < 0: their figures are the model's fixed
  // per-launch figures of that kernel kind, added when the timer is read
  long long unit_n[KK_COUNT] = {};
  hipEvent_t open = nullptr;
  int open_kind = -1;
  bool failed = false;

  hipEvent_t take();
  void reset();    // drop pending records and zero the sums
  bool drain();    // wait for pending records and add them to the sums
  ~KernelTimer();
};

// Timer of the online call running on this thread (nullptr: not timing).
extern thread_local KernelTimer* t_timer;

struct TimerScope {
  explicit TimerScope(KernelTimer* t) { t_timer = (t && t->on) ? t : nullptr; }
  ~TimerScope() { t_timer = nullptr; }
};

void ktimer_begin(int kind, hipStream_t st);
// flops/bytes < 0: the fixed per-launch figures of the kind (see unit_n).
void ktimer_end(double flops, double bytes, hipStream_t st);

}  // namespace lrbms
