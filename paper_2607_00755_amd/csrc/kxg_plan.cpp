// Host-only planning of libkxg: Gauss-Legendre rule and GEMM work units.
#include "kxg_plan.h"

#include <algorithm>
#include <cmath>
#include <utility>

#include "kxg_geom.h"

namespace kxg {

// Gauss-Legendre rule by Golub-Welsch: the nodes are the eigenvalues of the
// symmetric tridiagonal Jacobi matrix of the Legendre polynomials
// (zero diagonal, off-diagonal k / sqrt(4k^2 - 1)), the weights 2 v_0^2 with
// v_0 the first component of each normalised eigenvector.  Implicit QL with
// Wilkinson-type shifts, tracking only the first row of the eigenvectors.
void gauss_legendre(int n, double *x, double *w)
{
    std::vector<double> d(n, 0.0), e(n, 0.0), z(n, 0.0);
    for (int k = 1; k < n; ++k) e[k - 1] = k / std::sqrt(4.0 * k * k - 1.0);
    z[0] = 1.0;
    for (int l = 0; l < n; ++l) {
        for (int iter = 0; iter < 200; ++iter) {
            int m = l;
            for (; m < n - 1; ++m) {
                const double dd = std::fabs(d[m]) + std::fabs(d[m + 1]);
                if (std::fabs(e[m]) <= 2.220446049250313e-16 * dd || e[m] == 0.0) break;
            }
            if (m == l) break;
            double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
            double r = std::hypot(g, 1.0);
            g = d[m] - d[l] + e[l] / (g + (g >= 0 ? r : -r));
            double s = 1.0, c = 1.0, p = 0.0;
            int i = m - 1;
            for (; i >= l; --i) {
                double f = s * e[i];
                const double b = c * e[i];
                r = std::hypot(f, g);
                e[i + 1] = r;
                if (r == 0.0) {
                    d[i + 1] -= p;
                    e[m] = 0.0;
                    break;
                }
                s = f / r;
                c = g / r;
                g = d[i + 1] - p;
                r = (d[i] - g) * s + 2.0 * c * b;
                p = s * r;
                d[i + 1] = g + p;
                g = c * r - b;
                f = z[i + 1];
                z[i + 1] = s * z[i] + c * f;
                z[i] = c * z[i] - s * f;
            }
            if (r == 0.0 && i >= l) continue;
            d[l] -= p;
            e[l] = g;
            e[m] = 0.0;
        }
    }
    std::vector<int> idx(n);
    for (int i = 0; i < n; ++i) idx[i] = i;
    std::sort(idx.begin(), idx.end(), [&](int a, int b) { return d[a] < d[b]; });
    for (int i = 0; i < n; ++i) {
        // symmetrise: the rule is exactly symmetric about 0
        const int j = idx[i], jm = idx[n - 1 - i];
        x[i] = 0.5 * (d[j] - d[jm]);
        w[i] = 0.5 * (2.0 * z[j] * z[j] + 2.0 * z[jm] * z[jm]);
    }
}


// GEMMs over non-zero blocks only.  The kinematic cuts leave whole
// 32 x 16 x 16 blocks of the packed operand at zero (about a quarter at
// n = 256, most of them at large i); they are dropped from the operands and
// from the K loops, which is exact.  The FP32 operand keeps the blocks of
// each i-block; the 16-bit operand, whose workgroups cover KXG_LDS_IBW
// i-blocks at once, keeps the union over such a group.  The kept blocks of
// each group are cut into work units of about equal length (in super-steps
// of a few dk steps), so that one launch at the handle's largest batch has
// at most the targeted number of workgroups; the partial of unit j of a
// group goes to K slot j.  The units depend on the handle only, so the
// reduction order of a row does not depend on the batch.
Units make_units(const std::vector<int> &cnt, const std::vector<int> &first, int pps,
                        int nbt, int wg_target)
{
    Units U;
    const int ng = (int)cnt.size();
    long total = 0;
    for (int c : cnt) total += (long)c * pps;
    U.nslot.assign(ng, 0);
    if (total == 0) return U;
    // units in all: one launch of at most wg_target workgroups (a second
    // round of workgroups would double the time of its CUs), and at least
    // 4 super-steps a wave
    int target = std::max(1, wg_target / nbt);
    target = (int)std::max<long>(1, std::min<long>(target, total / (4 * kWaves)));
    // shared out in proportion to each group's blocks (largest remainders),
    // at least one per non-empty group
    std::vector<int> nu(ng, 0);
    int given = 0;
    std::vector<std::pair<double, int>> rem;
    for (int q = 0; q < ng; ++q) {
        if (cnt[q] == 0) continue;
        const double share = (double)target * cnt[q] * pps / (double)total;
        nu[q] = std::max(1, (int)share);
        given += nu[q];
        rem.push_back({share - (int)share, q});
    }
    std::sort(rem.begin(), rem.end(), [](const std::pair<double, int> &x, const std::pair<double, int> &y) {
        return x.first > y.first || (x.first == y.first && x.second < y.second);
    });
    for (size_t j = 0; j < rem.size() && given < target; ++j, ++given) ++nu[rem[j].second];
    for (int q = 0; q < ng; ++q) {
        const long len = (long)cnt[q] * pps, base = (long)first[q] * pps;
        if (len == 0) continue;
        const int m = (int)std::min<long>(nu[q], len);
        for (int j = 0; j < m; ++j) {
            U.units.push_back(q);
            U.units.push_back(j);
            U.units.push_back((int)(base + len * j / m));
            U.units.push_back((int)(base + len * (j + 1) / m));
        }
        U.nslot[q] = m;
        U.maxslots = std::max(U.maxslots, m);
    }
    return U;
}

}  // namespace kxg
