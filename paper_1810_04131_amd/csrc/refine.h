// Adaptive panel refinement near contact (host code only; builds with a plain C++
// compiler).
//
// Section 5 states QBX's preconditions after Theorem qbx-accuracy (expansion disks
// free of other geometry, the panels next to a target adequately resolved) and the
// paper refines at most 3-5 levels per time step.  A panel is the parameter
// interval 2 pi / P (k + [idx, idx + 1] 2^-lev) of base panel k of its ellipse.
// Refinement passes split (at the parameter midpoint) every panel whose arclength
// exceeds ratio times its distance to the nearest node of another particle, at
// most `levels` times; then every particle's panels are balanced so that the
// `win` panels on either side of any panel (those its QBX expansion takes) are at
// most one level coarser than it, by splitting the coarser ones.  Distances and
// arclengths are FP64, nodes the 16-point Gauss-Legendre nodes of each panel.
#pragma once

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <vector>

namespace yq {

struct PanelDesc {
  int k, lev, idx;
};

// Nodes (x, y) and the arclength (sum of the weights, in node order) of one panel
// of the ellipse pc = (cx, cy, theta, A, B); xg, wg the q-point rule on [-1, 1].
inline void refine_panel_nodes(const double* pc, int P, const PanelDesc& d, const double* xg,
                               const double* wg, int q, double* x, double* y, double& h) {
  const double pi = 3.14159265358979323846264338327950288;
  const double sa = std::sin(pc[2]), ca = std::cos(pc[2]);
  const double dt = std::ldexp(pi / P, -d.lev);
  h = 0.0;
  for (int m = 0; m < q; ++m) {
    const double t = 2.0 * pi / P * (d.k + std::ldexp(d.idx + 0.5 * (xg[m] + 1.0), -d.lev));
    const double st = std::sin(t), ct = std::cos(t);
    const double ex = pc[3] * ct, ey = pc[4] * st;
    const double ddx = -pc[3] * st, ddy = pc[4] * ct;
    x[m] = pc[0] + ca * ex - sa * ey;
    y[m] = pc[1] + sa * ex + ca * ey;
    const double gx = ca * ddx - sa * ddy, gy = sa * ddx + ca * ddy;
    h += dt * wg[m] * std::sqrt(gx * gx + gy * gy);
  }
}

// Panels of n ellipses pc[5 n] after refinement, per particle in increasing t.
// nbp, nbi: for every particle the particles that can come within the refinement
// distance of it (CSR, may include the particle itself, which is skipped); a
// particle outside its list never decides a split.
inline std::vector<std::vector<PanelDesc>> refine_panels(const double* pc, int n, int P,
                                                         int levels, double ratio, int win,
                                                         const double* xg, const double* wg,
                                                         int q, const std::vector<int>& nbp,
                                                         const std::vector<int>& nbi) {
  std::vector<std::vector<PanelDesc>> pans(n);
  for (int i = 0; i < n; ++i)
    for (int k = 0; k < P; ++k) pans[i].push_back(PanelDesc{k, 0, 0});
  if (levels <= 0 || n < 2) return pans;
  std::vector<std::vector<double>> nx(n), ny(n), hh(n);
  for (int pass = 0; pass < levels; ++pass) {
    for (int i = 0; i < n; ++i) {
      const size_t m = pans[i].size();
      nx[i].resize(m * q);
      ny[i].resize(m * q);
      hh[i].resize(m);
      for (size_t a = 0; a < m; ++a)
        refine_panel_nodes(pc + 5 * (size_t)i, P, pans[i][a], xg, wg, q, &nx[i][a * q],
                           &ny[i][a * q], hh[i][a]);
    }
    bool any = false;
    std::vector<std::vector<PanelDesc>> next(n);
    for (int i = 0; i < n; ++i) {
      for (size_t a = 0; a < pans[i].size(); ++a) {
        const PanelDesc d = pans[i][a];
        double d2 = INFINITY;
        if (d.lev < levels)
          for (int e = nbp[i]; e < nbp[i + 1]; ++e) {
            const int j = nbi[e];
            if (j == i) continue;
            for (int m = 0; m < q; ++m) {
              const double px = nx[i][a * q + m], py = ny[i][a * q + m];
              for (size_t b = 0; b < nx[j].size(); ++b) {
                const double dx = px - nx[j][b], dy = py - ny[j][b];
                d2 = std::min(d2, dx * dx + dy * dy);
              }
            }
          }
        if (d.lev < levels && hh[i][a] > ratio * std::sqrt(d2)) {
          next[i].push_back(PanelDesc{d.k, d.lev + 1, 2 * d.idx});
          next[i].push_back(PanelDesc{d.k, d.lev + 1, 2 * d.idx + 1});
          any = true;
        } else {
          next[i].push_back(d);
        }
      }
    }
    pans.swap(next);
    if (!any) break;
  }
  // balance: the panels within win of a panel are at most one level coarser
  const int w = std::max(win, 1);
  for (int i = 0; i < n; ++i) {
    for (;;) {
      const std::vector<PanelDesc>& ring = pans[i];
      const int m = (int)ring.size();
      std::vector<char> bad(m, 0);
      bool anybad = false;
      for (int a = 0; a < m; ++a) {
        int mx = ring[a].lev;
        for (int o = -w; o <= w; ++o) mx = std::max(mx, ring[((a + o) % m + m) % m].lev);
        if (ring[a].lev + 1 < mx) bad[a] = anybad = 1;
      }
      if (!anybad) break;
      std::vector<PanelDesc> out;
      for (int a = 0; a < m; ++a) {
        const PanelDesc d = ring[a];
        if (bad[a]) {
          out.push_back(PanelDesc{d.k, d.lev + 1, 2 * d.idx});
          out.push_back(PanelDesc{d.k, d.lev + 1, 2 * d.idx + 1});
        } else {
          out.push_back(d);
        }
      }
      pans[i].swap(out);
    }
  }
  return pans;
}

}  // namespace yq
