// Host-only planning of libkxg (no HIP): the Gauss-Legendre rule of the
// angular quadrature and the partition of the packed GEMM operand into work
// units.  Kept apart from the HIP translation units so that the host checks
// (and a sanitizer build of them) can run without a GPU.
#pragma once

#include <vector>

namespace kxg {

// Gauss-Legendre nodes (ascending) and weights on [-1, 1], n >= 1.
void gauss_legendre(int n, double *x, double *w);

// Work units of a packed GEMM: group q has cnt[q] kept blocks starting at
// block first[q], each of pps super-steps; the units of a group cover its
// super-steps [first*pps, (first+cnt)*pps) in order without gaps or overlap,
// unit j of a group writing K slot j.  At most about wg_target / nbt units
// in all (nbt batch tiles share each unit), at least one per non-empty group
// and at least 4 super-steps per wave of a unit where the work allows.
struct Units {
    std::vector<int> units, nslot;   // [u][4] = (group, slot, first, end); [group]
    int maxslots = 0;
};
Units make_units(const std::vector<int> &cnt, const std::vector<int> &first, int pps, int nbt,
                 int wg_target);

// The same where a unit's super-steps cost w[b] each, b the unit's first
// block (w[] per kept block, non-increasing within each group): every unit
// costs at most T, for the least T that keeps the number of units within
// the same target (or one per non-empty group).  A group's units are cut
// greedily in order; its last one may be short.
Units make_units_cost(const std::vector<int> &cnt, const std::vector<int> &first,
                      const std::vector<double> &w, int pps, int nbt, int wg_target);

}  // namespace kxg
