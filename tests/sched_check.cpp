// CPU checks of the request server's admission policy (no GPU, no HIP).
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "../paper_2304_06543_amd/csrc/sched.hpp"

static int failures = 0;
#define CHECK(c)                                                   \
  do {                                                             \
    if (!(c)) { std::printf("FAIL line %d: %s\n", __LINE__, #c); ++failures; } \
  } while (0)

int main() {
  using lbdd::AdmissionQueue;
  uint64_t id = 0;
  {  // arrival order when everything fits
    AdmissionQueue q;
    for (uint64_t i = 1; i <= 4; ++i) q.push(i, 10);
    for (uint64_t i = 1; i <= 4; ++i) { CHECK(q.next(100, 0, true, &id)); CHECK(id == i); }
    CHECK(!q.next(100, 0, true, &id));
  }
  {  // no free slot: nothing admitted
    AdmissionQueue q;
    q.push(1, 10);
    CHECK(!q.next(100, 0, false, &id));
    CHECK(q.size() == 1);
  }
  {  // small requests pass a big one that does not fit, at most max_bypass times
    AdmissionQueue q(2);
    q.push(1, 1000);
    for (uint64_t i = 2; i <= 6; ++i) q.push(i, 10);
    CHECK(q.next(100, 1, true, &id) && id == 2);
    CHECK(q.next(100, 1, true, &id) && id == 3);
    CHECK(!q.next(100, 1, true, &id));                // bypass cap reached: 1 blocks
    CHECK(q.next(1000, 1, true, &id) && id == 1);     // memory freed: the old one goes
    CHECK(q.next(100, 1, true, &id) && id == 4);      // and the counter restarts
  }
  {  // a request bigger than the budget runs alone once nothing is in flight
    AdmissionQueue q(0);
    q.push(1, 1u << 30);
    CHECK(!q.next(100, 2, true, &id));
    CHECK(q.next(100, 0, true, &id) && id == 1);
  }
  {  // cancellation
    AdmissionQueue q;
    q.push(1, 5); q.push(2, 5);
    CHECK(q.erase(1));
    CHECK(!q.erase(7));
    CHECK(q.next(10, 0, true, &id) && id == 2);
  }
  {  // expiry: every matching request leaves, the others keep their order
    AdmissionQueue q(1);
    for (uint64_t i = 1; i <= 6; ++i) q.push(i, i == 1 ? 1000 : 10);
    CHECK(q.next(100, 1, true, &id) && id == 2);      // one bypass of request 1
    CHECK(!q.next(100, 1, true, &id));                // cap reached
    std::vector<uint64_t> gone;
    CHECK(q.erase_if([](uint64_t x) { return x == 1 || x == 4; }, [&](uint64_t x) { gone.push_back(x); }) == 2);
    CHECK(gone.size() == 2 && gone[0] == 1 && gone[1] == 4);
    CHECK(q.next(100, 1, true, &id) && id == 3);      // the head left: the counter restarted
    CHECK(q.next(100, 1, true, &id) && id == 5);
    CHECK(q.next(100, 1, true, &id) && id == 6);
    CHECK(q.empty());
    CHECK(q.erase_if([](uint64_t) { return true; }, [](uint64_t) {}) == 0);
  }
  {  // footprint grows with both sizes and covers the cost matrix three times
    CHECK(lbdd::instance_footprint(100, 100000) > (size_t)3 * 4 * 100 * 100000);
    CHECK(lbdd::instance_footprint(200, 1000) > lbdd::instance_footprint(100, 1000));
  }
  {  // simulated stream: memory never exceeds the budget while >1 job runs
    AdmissionQueue q(4);
    std::vector<size_t> sizes;
    srand(7);
    for (int i = 0; i < 200; ++i) { size_t s = 1 + rand() % 90; sizes.push_back(s); q.push(i + 1, s); }
    size_t budget = 100, used = 0;
    std::vector<std::pair<uint64_t, size_t>> run;
    int steps = 0, admitted = 0;
    while ((!q.empty() || !run.empty()) && steps < 100000) {
      ++steps;
      while (q.next(budget - used, (int)run.size(), true, &id)) {
        used += sizes[id - 1];
        run.push_back({id, sizes[id - 1]});
        ++admitted;
        CHECK(used <= budget || run.size() == 1);
      }
      if (!run.empty()) { used -= run.front().second; run.erase(run.begin()); }
    }
    CHECK(admitted == 200);
  }
  std::printf("%s (%d failures)\n", failures ? "FAILED" : "ok", failures);
  return failures ? 1 : 0;
}
