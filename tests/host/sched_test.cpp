// Host-only checks of the request server's admission pass and of the per-round
// precision schedule (paper_2604_17001_amd/csrc/admission.h). Built and run by
// tests/test_host_sanitized.py with the address and undefined-behaviour sanitizers.
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "admission.h"

using namespace icnnm;

static int failures = 0;
#define CHECK(c)                                                 \
  do {                                                           \
    if (!(c)) {                                                  \
      std::fprintf(stderr, "FAIL %s:%d %s\n", __FILE__, __LINE__, #c); \
      ++failures;                                                \
    }                                                            \
  } while (0)

struct Q {
  std::vector<int> bypassed;
  std::vector<AdmitView> views;
  void add(const std::string& key, size_t bytes, size_t group_bytes) {
    bypassed.reserve(64);
    bypassed.push_back(0);
    views.push_back(AdmitView{key, bytes, group_bytes, nullptr});
  }
  std::vector<AdmitView>& get() {
    for (size_t i = 0; i < views.size(); ++i) views[i].bypassed = &bypassed[i];
    return views;
  }
  void erase(const std::vector<size_t>& idx) {  // ascending positions
    for (size_t j = idx.size(); j-- > 0;) {
      views.erase(views.begin() + (long)idx[j]);
      bypassed.erase(bypassed.begin() + (long)idx[j]);
    }
  }
};

static AdmitLimits lim(size_t used, size_t limit, int slots = 512, int max_bypass = 32, int scan = 16) {
  return AdmitLimits{used, limit, slots, max_bypass, scan};
}

int main() {
  // cumulative reservation: a budget for two of six equal requests admits two
  {
    Q q;
    for (int i = 0; i < 6; ++i) q.add("g", 100, 0);
    AdmitResult r = admission_pass(q.get(), {{"g", 512}}, lim(0, 250));
    CHECK(r.admitted.size() == 2 && r.admitted[0] == 0 && r.admitted[1] == 1);
    CHECK(!r.head_blocked);
    q.erase(r.admitted);
    // nothing freed: the new head is blocked and nothing passes it (all equal)
    r = admission_pass(q.get(), {{"g", 510}}, lim(200, 250));
    CHECK(r.admitted.empty() && r.head_blocked);
    // two members retire: two more fit
    r = admission_pass(q.get(), {{"g", 512}}, lim(0, 250));
    CHECK(r.admitted.size() == 2);
  }
  // a new group's bytes are reserved with its first request only
  {
    Q q;
    q.add("a", 10, 100);
    q.add("a", 10, 100);
    q.add("b", 10, 100);
    AdmitResult r = admission_pass(q.get(), {}, lim(0, 125));
    CHECK(r.admitted.size() == 2 && r.admitted[1] == 1);  // 110 + 10; "b" would need 110 more
    r = admission_pass(q.get(), {{"a", 512}}, lim(0, 130));
    CHECK(r.admitted.size() == 3);  // "a" exists: 10 + 10 + 110
  }
  // slots: a group with one free slot takes one member per pass
  {
    Q q;
    q.add("g", 1, 0);
    q.add("g", 1, 0);
    AdmitResult r = admission_pass(q.get(), {{"g", 1}}, lim(0, 1000));
    CHECK(r.admitted.size() == 1 && r.admitted[0] == 0);
    CHECK(!r.head_blocked);
    // a new group starts with group_slots free slots
    Q q2;
    for (int i = 0; i < 5; ++i) q2.add("n", 1, 0);
    r = admission_pass(q2.get(), {}, lim(0, 1000, 3));
    CHECK(r.admitted.size() == 3);
  }
  // bounded bypass: small requests pass a blocked large head at most max_bypass
  // times in all, then the queue waits for the head
  {
    Q q;
    q.add("g", 1000, 0);  // does not fit until the budget frees
    for (int i = 0; i < 20; ++i) q.add("g", 1, 0);
    AdmitResult r = admission_pass(q.get(), {{"g", 512}}, lim(0, 500, 512, 5, 16));
    CHECK(r.head_blocked);
    CHECK(r.admitted.size() == 5);
    CHECK(q.bypassed[0] == 5);
    q.erase(r.admitted);
    r = admission_pass(q.get(), {{"g", 512}}, lim(0, 500, 512, 5, 16));
    CHECK(r.admitted.empty() && r.head_blocked);  // strict arrival order from now on
    // the budget frees: the head goes first, then the others in order
    r = admission_pass(q.get(), {{"g", 512}}, lim(0, 2000, 512, 5, 16));
    CHECK(!r.admitted.empty() && r.admitted[0] == 0 && !r.head_blocked);
  }
  // the scan past a blocked head is bounded
  {
    Q q;
    q.add("g", 1000, 0);
    for (int i = 0; i < 10; ++i) q.add("g", 600, 0);  // do not fit either
    q.add("g", 1, 0);                                  // would fit, but lies past the scan
    AdmitResult r = admission_pass(q.get(), {{"g", 512}}, lim(0, 500, 512, 32, 4));
    CHECK(r.admitted.empty() && r.head_blocked);
    r = admission_pass(q.get(), {{"g", 512}}, lim(0, 500, 512, 32, 16));
    CHECK(r.admitted.size() == 1 && r.admitted[0] == 11);
  }
  // a request larger than the whole budget never fits (no overflow in the test)
  {
    Q q;
    q.add("g", (size_t)-1 - 5, 0);
    AdmitResult r = admission_pass(q.get(), {{"g", 512}}, lim(100, 1000));
    CHECK(r.admitted.empty() && r.head_blocked);
  }
  // empty queue
  {
    Q q;
    AdmitResult r = admission_pass(q.get(), {}, lim(0, 10));
    CHECK(r.admitted.empty() && !r.head_blocked);
  }
  // precision schedule: FP32 at round 0 (initialisation), iteration 1, every
  // refresh_every-th after it and from the last iteration on; FP32 members always
  {
    const int prec = 1, iters = 25, every = 10;
    std::vector<int> fp32;
    for (int r = 0; r <= iters + 2; ++r)
      if (round_kind(r, prec, iters, every) == 0) fp32.push_back(r);
    const std::vector<int> want = {0, 1, 11, 21, 25, 26, 27};
    CHECK(fp32 == want);
    for (int r = 0; r < 30; ++r) CHECK(round_kind(r, 0, iters, every) == 0);
    for (int r = 0; r < 30; ++r) CHECK(round_kind(r, 2, iters, 1) == 0);
  }
  if (failures) {
    std::fprintf(stderr, "%d check(s) failed\n", failures);
    return 1;
  }
  std::printf("sched ok\n");
  return 0;
}
