// Host-side extent checks of device operands (see common.h).
#include <atomic>
#include <cstdio>
#include <map>
#include <mutex>
#include <string>

#include "common.h"

namespace mpsim {

namespace {
std::mutex g_mu;
std::map<uintptr_t, size_t> g_bufs;  // base address -> bytes
std::atomic<bool> g_on{false};

std::string hex(uintptr_t v) {
  char b[32];
  snprintf(b, sizeof b, "0x%llx", (unsigned long long)v);
  return b;
}
}  // namespace

void bounds_register(const void* p, size_t bytes) {
  if (!p) return;
  std::lock_guard<std::mutex> lk(g_mu);
  g_bufs[(uintptr_t)p] = bytes;
}

bool bounds_register_new(const void* p, size_t bytes) {
  if (!p) return false;
  std::lock_guard<std::mutex> lk(g_mu);
  return g_bufs.emplace((uintptr_t)p, bytes).second;
}

void bounds_unregister(const void* p) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_bufs.erase((uintptr_t)p);
}

bool bounds_checking() { return g_on.load(std::memory_order_relaxed); }

void bounds_set_checking(bool on) { g_on.store(on); }

void bounds_require(const void* p, long lo, long hi, size_t elem, const char* what) {
  if (!bounds_checking() || !p || hi < lo) return;
  const uintptr_t a = (uintptr_t)p;
  uintptr_t base = 0;
  size_t size = 0;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_bufs.upper_bound(a);
    if (it != g_bufs.begin()) {
      --it;
      base = it->first;
      size = it->second;
    }
  }
  if (size == 0 || a >= base + size)
    throw BoundsError{std::string(what) + ": base " + hex(a) + " lies in no buffer of the library"};
  const long long off = (long long)(a - base);
  const long long first = off + (long long)lo * (long long)elem;
  const long long last = off + ((long long)hi + 1) * (long long)elem;
  if (first < 0 || last > (long long)size)
    throw BoundsError{std::string(what) + ": bytes [" + std::to_string(first) + ", " +
                      std::to_string(last) + ") of a buffer of " + std::to_string(size) + " bytes"};
}

}  // namespace mpsim
