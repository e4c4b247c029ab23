// Host-only check of the kernel-family timer's launch sampler under
// concurrent host threads (the pairs of a batched registration): every
// thread accounts its launches and then asks for their events, as the
// library's timed launches do.  Each launch carries a distinct amount of
// work; the work summed for sampled launches must equal the work of the
// launches that were handed events, launch by launch, and the number of
// sampled launches must equal the number of sequence numbers the hash
// selects, whatever the interleaving.
#include <cstdio>
#include <thread>
#include <vector>

#include "sampler.h"

using lddmm::LaunchSampler;

int main(int argc, char** argv) {
  const int threads = 8, per_thread = 20000, every = 4, family = 5;
  LaunchSampler smp;
  smp.family.store(family);
  smp.every.store(every);
  double accounted = 0.0;            // under smp.mu, as the library's sums
  std::vector<double> granted(threads, 0.0);
  std::vector<long long> grants(threads, 0);
  std::vector<std::thread> pool;
  for (int t = 0; t < threads; ++t) {
    pool.emplace_back([&, t] {
      for (int i = 0; i < per_thread; ++i) {
        const double work = 1.0 + t * per_thread + i;  // distinct per launch
        const int fam = (i % 7 == 3) ? family + 1 : family;  // other families interleave
        smp.account(fam, [&] { accounted += work; });
        if (i % 13 == 0) std::this_thread::yield();
        if (smp.sampled(fam)) {
          granted[t] += work;
          grants[t] += 1;
        }
      }
    });
  }
  for (auto& th : pool) th.join();
  long long expect = 0, total = 0;
  double sum = 0.0;
  for (int t = 0; t < threads; ++t) {
    total += grants[t];
    sum += granted[t];
  }
  long long family_launches = 0;
  for (int i = 0; i < per_thread; ++i) family_launches += (i % 7 == 3) ? 0 : 1;
  family_launches *= threads;
  for (long long k = 0; k < family_launches; ++k)
    if (lddmm::splitmix64_finalise((unsigned long long)k) % every == 0) ++expect;
  std::printf("launches %lld sampled %lld expected %lld work %.1f granted %.1f\n", family_launches, total, expect,
              accounted, sum);
  const bool ok = total == expect && sum == accounted && smp.seen == family_launches;
  return ok ? 0 : 1;
}
