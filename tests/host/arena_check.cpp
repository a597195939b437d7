// Checks of the serving arena's first-fit node ranges and memory budget
// (arena.h), built with the host compiler under AddressSanitizer and
// UndefinedBehaviorSanitizer.  Random sequences of takes and gives are replayed
// against a brute-force model (one flag per node): every take must return the
// lowest offset of a free run long enough (first fit), fail exactly when no such
// run exists, and the free list must stay sorted, merged and equal to the
// model's free runs.  Exit status 0 when every check passes.
#include <cstdio>
#include <random>
#include <vector>

#include "arena.h"

static int failures = 0;
#define CHECK(c, ...)                                        \
  do {                                                       \
    if (!(c)) {                                              \
      if (failures < 20) {                                   \
        std::printf("FAIL %s:%d: ", __FILE__, __LINE__);     \
        std::printf(__VA_ARGS__);                            \
        std::printf("\n");                                   \
      }                                                      \
      ++failures;                                            \
    }                                                        \
  } while (0)

static int64_t first_fit(const std::vector<char>& used, int64_t n) {
  int64_t run = 0;
  for (int64_t i = 0; i < (int64_t)used.size(); ++i) {
    run = used[i] ? 0 : run + 1;
    if (run == n) return i - n + 1;
  }
  return -1;
}

static void compare_runs(const yq::NodeArena& a, const std::vector<char>& used) {
  std::vector<std::pair<int64_t, int64_t>> runs;
  for (int64_t i = 0; i < (int64_t)used.size();) {
    if (used[i]) {
      ++i;
      continue;
    }
    int64_t j = i;
    while (j < (int64_t)used.size() && !used[j]) ++j;
    runs.push_back({i, j - i});
    i = j;
  }
  CHECK(runs == a.ranges(), "free list differs from the model (%zu vs %zu runs)", a.ranges().size(),
        runs.size());
}

int main() {
  std::mt19937_64 rng(7);
  for (int trial = 0; trial < 40; ++trial) {
    const int64_t cap = 64 + (int64_t)(rng() % 4000);
    yq::NodeArena a(cap);
    std::vector<char> used(cap, 0);
    std::vector<std::pair<int64_t, int64_t>> held;
    for (int op = 0; op < 2000; ++op) {
      if (held.empty() || rng() % 3 != 0) {
        const int64_t n = 1 + (int64_t)(rng() % (cap / 4 + 1));
        int64_t off = -7;
        const bool ok = a.take(n, off);
        const int64_t want = first_fit(used, n);
        CHECK(ok == (want >= 0), "take(%lld) returned %d, model %lld", (long long)n, ok,
              (long long)want);
        if (ok) {
          CHECK(off == want, "first fit: %lld vs %lld", (long long)off, (long long)want);
          for (int64_t i = off; i < off + n; ++i) used[i] = 1;
          held.push_back({off, n});
        } else {
          CHECK(off == -7, "failed take changed the offset");
        }
      } else {
        const size_t k = rng() % held.size();
        a.give(held[k].first, held[k].second);
        for (int64_t i = held[k].first; i < held[k].first + held[k].second; ++i) used[i] = 0;
        held.erase(held.begin() + (std::ptrdiff_t)k);
      }
      compare_runs(a, used);
    }
    for (auto& h : held) a.give(h.first, h.second);
    CHECK(a.free_total() == cap && a.ranges().size() == 1, "arena not whole after every give");
  }
  // degenerate requests
  yq::NodeArena z(0);
  int64_t off = 3;
  CHECK(!z.take(1, off) && off == 3, "take from an empty arena");
  yq::NodeArena b(10);
  CHECK(!b.take(0, off) && !b.take(-1, off) && !b.take(11, off), "take of 0, -1 or too many");
  CHECK(b.take(10, off) && off == 0 && b.ranges().empty(), "take of the whole arena");
  b.give(0, 10);
  CHECK(b.free_total() == 10, "give back the whole arena");
  // budget
  yq::MemBudget m{100.0, 0.0};
  CHECK(m.fits(100.0) && !m.fits(100.5), "budget limit");
  m.take(60.0);
  CHECK(m.fits(40.0) && !m.fits(41.0), "budget after a take");
  m.give(60.0);
  m.give(1.0);
  CHECK(m.used == 0.0, "budget never below zero");
  std::printf("%s (%d failures)\n", failures ? "FAILED" : "ok", failures);
  return failures ? 1 : 0;
}
