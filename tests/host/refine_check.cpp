// Runs the library's host refinement (refine.h) on particles read from stdin and
// prints the panel descriptors, for comparison with the oracle's refinement.
// Input: n P levels ratio win, then n lines "cx cy theta A B".
// Output: one line per particle: its panel count, then k lev idx of every panel.
// Built with the host compiler under AddressSanitizer and UndefinedBehaviorSanitizer.
#include <cstdio>
#include <vector>

#include "refine.h"

int main() {
  int n, P, levels, win;
  double ratio;
  if (std::scanf("%d %d %d %lf %d", &n, &P, &levels, &ratio, &win) != 5) return 2;
  std::vector<double> pc(5 * (size_t)n);
  for (int i = 0; i < n; ++i)
    for (int c = 0; c < 5; ++c)
      if (std::scanf("%lf", &pc[5 * (size_t)i + c]) != 1) return 2;
  // 16-point Gauss-Legendre rule (Newton on P16 from Chebyshev guesses)
  const int q = 16;
  const double pi = 3.14159265358979323846264338327950288;
  double xg[q], wg[q];
  for (int m = 0; m < q; ++m) {
    double x = -std::cos(pi * (m + 0.75) / (q + 0.5)), dp = 0.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = x;
      for (int l = 2; l <= q; ++l) {
        const double p2 = ((2 * l - 1) * x * p1 - (l - 1) * p0) / l;
        p0 = p1;
        p1 = p2;
      }
      dp = q * (x * p1 - p0) / (x * x - 1.0);
      const double dx = p1 / dp;
      x -= dx;
      if (std::fabs(dx) < 1e-16) break;
    }
    xg[m] = x;
    wg[m] = 2.0 / ((1.0 - x * x) * dp * dp);
  }
  // every particle is a candidate neighbour of every other
  std::vector<int> nbp(n + 1), nbi;
  for (int i = 0; i < n; ++i) {
    for (int j = 0; j < n; ++j) nbi.push_back(j);
    nbp[i + 1] = (int)nbi.size();
  }
  const auto pans = yq::refine_panels(pc.data(), n, P, levels, ratio, win, xg, wg, q, nbp, nbi);
  for (int i = 0; i < n; ++i) {
    std::printf("%zu", pans[i].size());
    for (const auto& d : pans[i]) std::printf(" %d %d %d", d.k, d.lev, d.idx);
    std::printf("\n");
  }
  return 0;
}
