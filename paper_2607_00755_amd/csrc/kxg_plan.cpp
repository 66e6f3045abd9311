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
// units in all for one launch of at most wg_target workgroups (a second
// round of workgroups would double the time of its CUs), and at least 4
// super-steps a wave
static int unit_target(long total, int nbt, int wg_target)
{
    const int target = std::max(1, wg_target / nbt);
    return (int)std::max<long>(1, std::min<long>(target, total / (4 * kWaves)));
}

Units make_units(const std::vector<int> &cnt, const std::vector<int> &first, int pps,
                        int nbt, int wg_target)
{
    Units U;
    const int ng = (int)cnt.size();
    long total = 0;
    for (int c : cnt) total += (long)c * pps;
    U.nslot.assign(ng, 0);
    if (total == 0) return U;
    const int target = unit_target(total, nbt, wg_target);
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

Units make_units_cost(const std::vector<int> &cnt, const std::vector<int> &first,
                      const std::vector<double> &w, int pps, int nbt, int wg_target)
{
    Units U;
    const int ng = (int)cnt.size();
    long total = 0;
    double wmax = 0.0;
    int nonempty = 0;
    for (int q = 0; q < ng; ++q) {
        total += (long)cnt[q] * pps;
        nonempty += cnt[q] > 0;
        for (int b = first[q]; b < first[q] + cnt[q]; ++b) wmax = std::max(wmax, w[b]);
    }
    U.nslot.assign(ng, 0);
    if (total == 0) return U;
    const int target = std::max(unit_target(total, nbt, wg_target), nonempty);
    // greedy cut of every group at unit cost T: a unit from super-step s runs
    // floor(T / w) super-steps (at least one), w that of its first block
    auto cut = [&](double T, bool emit) {
        int units = 0;
        for (int q = 0; q < ng; ++q) {
            long s = (long)first[q] * pps;
            const long e = (long)(first[q] + cnt[q]) * pps;
            while (s < e) {
                const long len = std::max<long>(1, (long)(T / w[s / pps]));
                const long s1 = std::min(e, s + len);
                if (emit) {
                    U.units.push_back(q);
                    U.units.push_back(U.nslot[q]++);
                    U.units.push_back((int)s);
                    U.units.push_back((int)s1);
                }
                s = s1;
                ++units;
            }
        }
        return units;
    };
    // the least T (to a part in 1e6) whose cut has at most target units; a
    // whole group as one unit costs at most wmax * total
    double lo = 0.0, hi = wmax * (double)total;
    for (int it = 0; it < 60 && hi - lo > 1e-6 * hi; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (cut(mid, false) <= target)
            hi = mid;
        else
            lo = mid;
    }
    cut(hi, true);
    for (int c : U.nslot) U.maxslots = std::max(U.maxslots, c);
    return U;
}

}  // namespace kxg
