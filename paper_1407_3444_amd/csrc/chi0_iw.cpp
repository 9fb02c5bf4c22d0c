// chi0_iw.cpp -- the irreducible wedge of a Gamma-centred simple-cubic mesh under the cubic
// point group O_h, decomposed into tetrahedra (Sec. II, Fig. 1(a)); host code only.
//
// The wedge 0 <= z <= y <= x <= 1/2 is one 48th of the zone.  In mesh units (m = n/2) it is the
// union of the cubes with corner (i, j, l), m > i >= j >= l >= 0, each cube cut into the six
// tetrahedra of the orders in which the three axes are stepped from the corner to the opposite
// one; in a cube on the plane x = y (i == j) only the tetrahedra stepping x before y lie in the
// wedge, on y = z (j == l) only those stepping y before z.  That leaves exactly m^3 tetrahedra
// of volume 1/(6 n^3) each, and the 48 images of the set tile the zone.
#include "../../include/chi0.h"

#include <cstdint>

namespace {

// Index of wedge point (i, j, l), i >= j >= l >= 0, in the order i, then j, then l ascending.
int64_t wedge_point(int64_t i, int64_t j, int64_t l) { return i * (i + 1) * (i + 2) / 6 + j * (j + 1) / 2 + l; }

constexpr int kAxisOrders[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};

}  // namespace

extern "C" chi0_status chi0_iw_cubic(int32_t n, int64_t *n_kp, int64_t *n_tet, double *volume, double *kfrac,
                                     int32_t *tets, int32_t *ops)
{
    if (!n_kp || !n_tet || !volume) return CHI0_E_INVALID_ARG;
    if (n < 2 || n > 1024 || n % 2 != 0) return CHI0_E_SHAPE;
    const int64_t m = n / 2;
    *n_kp = (m + 1) * (m + 2) * (m + 3) / 6;
    *n_tet = m * m * m;
    *volume = 1.0 / (6.0 * (double)n * (double)n * (double)n);
    if (kfrac) {
        for (int64_t i = 0; i <= m; ++i)
            for (int64_t j = 0; j <= i; ++j)
                for (int64_t l = 0; l <= j; ++l) {
                    double *p = kfrac + 3 * wedge_point(i, j, l);
                    p[0] = (double)i / n;
                    p[1] = (double)j / n;
                    p[2] = (double)l / n;
                }
    }
    if (tets) {
        int64_t t = 0;
        for (int64_t i = 0; i < m; ++i)
            for (int64_t j = 0; j <= i; ++j)
                for (int64_t l = 0; l <= j; ++l)
                    for (const auto &ord : kAxisOrders) {
                        int pos[3];
                        for (int r = 0; r < 3; ++r) pos[ord[r]] = r;
                        if (i == j && pos[0] > pos[1]) continue;   // steps y before x on x = y
                        if (j == l && pos[1] > pos[2]) continue;   // steps z before y on y = z
                        int64_t c[3] = {i, j, l};
                        int32_t *out = tets + 4 * t;
                        out[0] = (int32_t)wedge_point(c[0], c[1], c[2]);
                        for (int r = 0; r < 3; ++r) {
                            ++c[ord[r]];
                            out[r + 1] = (int32_t)wedge_point(c[0], c[1], c[2]);
                        }
                        ++t;
                    }
    }
    if (ops) {
        // signed permutation matrices g[r][perm[r]] = sign[r]; the identity comes first
        int32_t *g = ops;
        for (const auto &perm : kAxisOrders)
            for (int s = 0; s < 8; ++s) {
                for (int e = 0; e < 9; ++e) g[e] = 0;
                for (int r = 0; r < 3; ++r) g[3 * r + perm[r]] = (s >> r) & 1 ? -1 : 1;
                g += 9;
            }
    }
    return CHI0_OK;
}
