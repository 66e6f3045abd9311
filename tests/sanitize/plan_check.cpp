// Property checks of libkxg's host-only planning code (GEMM work units,
// Gauss-Legendre rule), built with AddressSanitizer and
// UndefinedBehaviorSanitizer by tests/test_sanitizers_cpu.py.  Prints "ok"
// and exits 0 when every check holds.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <random>
#include <vector>

#include "../../paper_2607_00755_amd/csrc/kxg_plan.h"

static int fails = 0;
#define CHECK(c)                                                             \
    do {                                                                     \
        if (!(c)) {                                                          \
            if (fails < 20) std::printf("check failed: %s (line %d)\n", #c, __LINE__); \
            ++fails;                                                         \
        }                                                                    \
    } while (0)

static void check_units(std::mt19937 &rng)
{
    std::uniform_int_distribution<int> ngd(1, 40), cntd(0, 200), zero(0, 4);
    const int pps_choices[] = {1, 2, 4, 8};
    const int wg_choices[] = {64, 256, 512, 1024};
    const int ng = ngd(rng);
    std::vector<int> cnt(ng), first(ng);
    int acc = 0;
    for (int q = 0; q < ng; ++q) {
        cnt[q] = zero(rng) == 0 ? 0 : cntd(rng);
        first[q] = acc;
        acc += cnt[q];
    }
    const int pps = pps_choices[rng() % 4];
    const int nbt = 1 + (int)(rng() % 64);
    const int wg = wg_choices[rng() % 4];
    const kxg::Units U = kxg::make_units(cnt, first, pps, nbt, wg);
    CHECK(U.units.size() % 4 == 0);
    CHECK((int)U.nslot.size() == ng);
    const int nu = (int)U.units.size() / 4;
    int maxs = 0, nonempty = 0;
    long cover = 0;
    for (int q = 0; q < ng; ++q) {
        if (cnt[q] > 0) ++nonempty;
        // the units of group q, in slot order, tile its super-steps exactly
        long pos = (long)first[q] * pps, minlen = 1L << 40, maxlen = 0;
        int m = 0;
        for (int u = 0; u < nu; ++u) {
            const int *x = &U.units[4 * u];
            if (x[0] != q) continue;
            CHECK(x[1] == m);
            CHECK(x[2] == pos);
            CHECK(x[3] > x[2]);
            const long len = x[3] - x[2];
            minlen = std::min(minlen, len);
            maxlen = std::max(maxlen, len);
            pos = x[3];
            ++m;
        }
        CHECK(pos == (long)(first[q] + cnt[q]) * pps);
        CHECK(U.nslot[q] == m);
        CHECK((cnt[q] == 0) == (m == 0));
        if (m > 0) CHECK(maxlen - minlen <= 1);       // balanced within a group
        cover += (long)cnt[q] * pps;
        maxs = std::max(maxs, m);
    }
    CHECK(U.maxslots == maxs);
    long total = 0;
    for (int u = 0; u < nu; ++u) total += U.units[4 * u + 3] - U.units[4 * u + 2];
    CHECK(total == cover);
    // no more units than the launch target allows, beyond one per group
    if (cover > 0) CHECK(nu <= std::max(nonempty, std::max(1, wg / nbt)) + nonempty);
}

// Cost-balanced units: per-block costs non-increasing within each group;
// units tile each group in order with K slots 0, 1, ..., a unit's cost is
// its length times the cost of its first block, the number of units stays
// within the target (or one per non-empty group), and the costliest unit is
// within the bound the least feasible cut implies.
static void check_units_cost(std::mt19937 &rng)
{
    std::uniform_int_distribution<int> ngd(1, 12), cntd(0, 150), wd(0, 4);
    const int pps_choices[] = {2, 4, 8};
    const int ng = ngd(rng);
    std::vector<int> cnt(ng), first(ng);
    std::vector<double> w;
    int acc = 0, nonempty = 0;
    for (int q = 0; q < ng; ++q) {
        cnt[q] = cntd(rng);
        first[q] = acc;
        acc += cnt[q];
        nonempty += cnt[q] > 0;
        std::vector<double> g(cnt[q]);
        for (double &x : g) x = 3.0 + wd(rng);
        std::sort(g.begin(), g.end(), [](double a, double b) { return a > b; });
        w.insert(w.end(), g.begin(), g.end());
    }
    const int pps = pps_choices[rng() % 3];
    const int nbt = 1 + (int)(rng() % 32);
    const int wg = 512;
    const kxg::Units U = kxg::make_units_cost(cnt, first, w, pps, nbt, wg);
    CHECK(U.units.size() % 4 == 0);
    CHECK((int)U.nslot.size() == ng);
    const int nu = (int)U.units.size() / 4;
    long total = 0;
    double tcost = 0.0, wmax = 0.0, wmin = 1e300, umax = 0.0;
    for (int q = 0; q < ng; ++q) {
        total += (long)cnt[q] * pps;
        for (int b = first[q]; b < first[q] + cnt[q]; ++b) {
            tcost += w[b] * pps;
            wmax = std::max(wmax, w[b]);
            wmin = std::min(wmin, w[b]);
        }
        long pos = (long)first[q] * pps;
        int m = 0;
        for (int u = 0; u < nu; ++u) {
            const int *x = &U.units[4 * u];
            if (x[0] != q) continue;
            CHECK(x[1] == m);
            CHECK(x[2] == pos);
            CHECK(x[3] > x[2]);
            umax = std::max(umax, (x[3] - x[2]) * w[x[2] / pps]);
            pos = x[3];
            ++m;
        }
        CHECK(pos == (long)(first[q] + cnt[q]) * pps);
        CHECK(U.nslot[q] == m);
    }
    if (total == 0) {
        CHECK(nu == 0);
        return;
    }
    const int target = std::max(nonempty, (int)std::max<long>(1, std::min<long>(std::max(1, wg / nbt), total / 16)));
    CHECK(nu <= target);
    // (a unit is charged its first block's cost for every super-step, at most
    // wmax / wmin times what its super-steps cost on their own)
    if (target > ng) CHECK(umax <= wmax / wmin * tcost / (target - ng) + wmax + 1e-6 * tcost);
}

static void check_gauss_legendre()
{
    for (int n = 1; n <= 64; ++n) {
        std::vector<double> x(n), w(n);
        kxg::gauss_legendre(n, x.data(), w.data());
        double ws = 0.0;
        for (int i = 0; i < n; ++i) {
            CHECK(x[i] > -1.0 && x[i] < 1.0 && w[i] > 0.0);
            if (i > 0) CHECK(x[i] > x[i - 1]);
            CHECK(x[i] == -x[n - 1 - i] && w[i] == w[n - 1 - i]);
            ws += w[i];
        }
        CHECK(std::fabs(ws - 2.0) < 1e-13);
        // exact for polynomials of degree <= 2n - 1
        for (int k = 0; k <= 2 * n - 1 && k <= 40; ++k) {
            double s = 0.0;
            for (int i = 0; i < n; ++i) s += w[i] * std::pow(x[i], k);
            const double ref = (k % 2) ? 0.0 : 2.0 / (k + 1);
            CHECK(std::fabs(s - ref) < 1e-13);
        }
    }
}

int main()
{
    std::mt19937 rng(20261202u);
    for (int t = 0; t < 3000; ++t) check_units(rng);
    for (int t = 0; t < 3000; ++t) check_units_cost(rng);
    check_gauss_legendre();
    if (fails) {
        std::printf("%d checks failed\n", fails);
        return 1;
    }
    std::printf("ok\n");
    return 0;
}
