// Launch sampler of the kernel-family timer (host code only, no HIP).
//
// While a kernel family is timed, one launch of it in `every` (on average)
// carries start/stop events.  A launch is sampled when SplitMix64's finaliser
// of its sequence number among the family's launches is divisible by
// `every`, so that the sample does not lock onto a period of the launch
// sequence.  Several host threads (the pairs of a batched registration)
// launch concurrently: the decision for a launch is kept per thread, between
// the call that accounts the launch's work and the calls that hand out its
// events on the same thread, so that another thread's launch in between
// cannot change it.
#pragma once

#include <atomic>
#include <cstdint>
#include <mutex>

namespace lddmm {

inline uint64_t splitmix64_finalise(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

struct LaunchSampler {
  std::mutex mu;                 // guards seen and the sums of the owner
  std::atomic<int> family{0};    // timed family (0: none)
  std::atomic<int> every{1};
  int64_t seen = 0;              // launches of the family accounted so far

  // The decision of this thread's last accounted launch.
  static bool& decision() {
    static thread_local bool take = false;
    return take;
  }

  // Accounts one launch of `fam`: returns (and keeps for this thread)
  // whether it is sampled.  Takes `mu`; `on_sampled` runs under it.
  template <class F>
  bool account(int fam, F&& on_sampled) {
    bool& take = decision();
    take = false;
    const int f = family.load(std::memory_order_acquire);
    if (f == 0 || fam != f) return false;
    std::lock_guard<std::mutex> lk(mu);
    const uint64_t e = (uint64_t)every.load(std::memory_order_relaxed);
    take = splitmix64_finalise((uint64_t)seen++) % e == 0;
    if (take) on_sampled();
    return take;
  }

  // Whether this thread's last accounted launch of `fam` is sampled.
  bool sampled(int fam) const {
    const int f = family.load(std::memory_order_acquire);
    return f != 0 && fam == f && decision();
  }
};

}  // namespace lddmm
