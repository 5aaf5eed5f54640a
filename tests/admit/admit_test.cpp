// Unit test of the serving loop's admission arithmetic (xd_admit.h), built
// with g++ on a machine without a GPU by tests/test_admission.py.  Prints
// "ok <checks>" or the first failed check.
#include <cstdio>
#include <vector>

#include "xd_admit.h"

using namespace xd;

static int checks = 0;
#define CHECK(c)                                                              \
  do {                                                                        \
    ++checks;                                                                 \
    if (!(c)) {                                                               \
      std::printf("check failed: %s (line %d)\n", #c, __LINE__);              \
      return 1;                                                               \
    }                                                                         \
  } while (0)

static AdmitItem item(uint64_t a, uint64_t b, uint32_t n, int cls, int32_t match = 1) {
  AdmitItem it;
  it.a_words = a;
  it.b_words = b;
  it.n_pairs = n;
  it.scores = {match, -1, -1};
  it.cls = cls;
  return it;
}

int main() {
  std::vector<size_t> take;
  // slot memory: the context's budget is half the share; arenas get the rest
  SlotPlan p;
  CHECK(plan_slot(1000000, 100, 0, &p) && p.ctx_budget == 500000);
  CHECK(p.pair_bytes == 100 * (sizeof(xd_pair) + sizeof(xd_result)));
  CHECK(plan_slot(1000000, 100, 400000, &p));
  CHECK(p.cap_words == (1000000 - 400000 - p.pair_bytes) / 8);
  CHECK(400000 + p.pair_bytes + 8 * p.cap_words <= 1000000);   // all inside the share
  CHECK(!plan_slot(1000000, 100, 500001, &p));                 // context over its budget
  CHECK(!plan_slot(10000, 1000, 0, &p));                        // no room for the arenas
  // cost classes: X tier and the octave of the longest pair
  xd_pair prs[3] = {};
  prs[0].a_len = 1000; prs[0].b_len = 1000; prs[0].x = 10;
  prs[1].a_len = 3000; prs[1].b_len = 2000; prs[1].x = 10;
  prs[2].a_len = 10; prs[2].b_len = 10; prs[2].x = 100;
  CHECK(cost_class(prs, 2) == 12);            // longest 5,000 bases: octave 12
  CHECK(cost_class(prs, 1) == 10);            // 2,000 bases: octave 10
  CHECK(cost_class(prs + 2, 1) == 64 + 4);    // X = 100: the wide tier class
  CHECK(cost_class(prs, 3) == 64 + 12);
  // admission: oldest first, same scores, same class, while it fits
  std::vector<AdmitItem> q = {item(10, 10, 5, 1), item(10, 10, 5, 2), item(10, 10, 5, 1),
                              item(50, 1, 5, 1), item(10, 10, 5, 1, 2), item(10, 10, 5, 1)};
  admit(q.data(), q.size(), 30, 100, true, 64, &take);
  CHECK((take == std::vector<size_t>{0, 2, 5}));          // class 2, too big, other scores skipped
  admit(q.data(), q.size(), 30, 100, false, 64, &take);
  CHECK((take == std::vector<size_t>{0, 1, 2}));          // any class: arena full after three
  admit(q.data(), q.size(), 1000, 12, false, 64, &take);
  CHECK((take == std::vector<size_t>{0, 1}));             // pair capacity 12: two of 5
  admit(q.data(), q.size(), 1000, 100, true, 3, &take);
  CHECK((take == std::vector<size_t>{0, 2}));             // scan window of three
  admit(q.data(), 0, 1000, 100, true, 64, &take);
  CHECK(take.empty());
  std::vector<AdmitItem> big = {item(40, 1, 1, 0)};
  admit(big.data(), 1, 30, 100, true, 64, &take);
  CHECK(take.empty());                                     // a head that cannot fit is not taken
  std::vector<AdmitItem> exact = {item(1, 1, 4, 0), item(1, 1, 4, 0), item(1, 1, 4, 0)};
  admit(exact.data(), 3, 100, 8, true, 64, &take);
  CHECK((take == std::vector<size_t>{0, 1}));             // stops once the batch is full
  std::printf("ok %d\n", checks);
  return 0;
}
