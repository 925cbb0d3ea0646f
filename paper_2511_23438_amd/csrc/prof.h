// Opt-in timing of one launch class with HIP events on the launching stream,
// together with the algorithmic work (bytes or flops) of the timed launches.
#pragma once
#include <hip/hip_runtime.h>

#include <vector>

namespace mpsim {

enum ProfKind { PROF_OFF = 0, PROF_TRD_HEMV = 1, PROF_GRAM = 2, PROF_GEMM = 3, PROF_THETA = 4 };

struct Prof {
  int kind = PROF_OFF;
  std::vector<hipEvent_t> ev;  // start/stop pairs
  size_t used = 0;
  double ms = 0.0, work = 0.0;
  double min_work = 0.0;  // launches with less algorithmic work are not timed
  long launches = 0;

  bool on(int k, double w) const { return kind != PROF_OFF && k == kind && w >= min_work; }
  void begin(int k, double w, hipStream_t s) {
    if (!on(k, w)) return;
    if (2 * (used + 1) > ev.size()) {
      if (ev.size() < 8192) {
        size_t old = ev.size();
        ev.resize(old == 0 ? 512 : 2 * old);
        for (size_t i = old; i < ev.size(); ++i) (void)hipEventCreate(&ev[i]);
      } else {
        flush();
      }
    }
    (void)hipEventRecord(ev[2 * used], s);
  }
  void end(int k, double w, hipStream_t s) {
    if (!on(k, w)) return;
    (void)hipEventRecord(ev[2 * used + 1], s);
    ++used;
    ++launches;
    work += w;
  }
  void flush() {
    if (used == 0) return;
    (void)hipEventSynchronize(ev[2 * used - 1]);
    for (size_t i = 0; i < used; ++i) {
      float t = 0.f;
      if (hipEventElapsedTime(&t, ev[2 * i], ev[2 * i + 1]) == hipSuccess) ms += t;
    }
    used = 0;
  }
  void reset(int k) {
    flush();
    kind = k;
    ms = 0.0;
    work = 0.0;
    launches = 0;
  }
  ~Prof() {
    for (auto e : ev) (void)hipEventDestroy(e);
  }
};

}  // namespace mpsim
