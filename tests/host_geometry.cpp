// Host build of the contour geometry (arc-length density, admissibility checks) and of the
// log-singular moment tables of the near-field rule, for CPU tests.
#include <cstdio>
#include <string>
#include <vector>

#include "../paper_2203_13283_amd/csrc/internal.h"
using namespace cfie;

// out: c0, L, minimum curvature, convex (0/1), number of retained speed modes.  Returns 0 on
// success, else 1 with the error text in err.
extern "C" int geo_build(int n_nodes, int n_modes, const double *zhat, double *out, char *err,
                         int nerr) {
    cfie_contour c{};
    c.n_nodes = n_nodes;
    c.n_modes = n_modes;
    c.zhat = zhat;
    HostGeometry g;
    const std::string e = build_geometry(c, g);
    std::snprintf(err, (size_t)nerr, "%s", e.c_str());
    if (!e.empty()) return 1;
    out[0] = g.c0;
    out[1] = g.L;
    out[2] = g.min_curvature;
    out[3] = g.convex ? 1.0 : 0.0;
    out[4] = (double)g.cm.size();
    return 0;
}

// the 3 x 5 x q x q table of log_moments
extern "C" void geo_log_moments(int q, double *out) {
    std::vector<double> m;
    log_moments(q, m);
    for (size_t i = 0; i < m.size(); ++i) out[i] = m[i];
}
