// Host-side planning of the all-pairs refinement (no device code): the order
// of the Rayleigh quotients and the blocks of coupled pairs.
#pragma once

#include <algorithm>
#include <numeric>
#include <utility>
#include <vector>

namespace zk {

// Ascending order of n double-double values (hi[0..n), lo at hi[n..2n)),
// stable for equal values.
inline void ap_sorted_order(const double *th, int n, std::vector<int> &order)
{
    order.resize(n);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        return th[a] < th[b] || (th[a] == th[b] && th[n + a] < th[n + b]);
    });
}

// Blocks of coupled pairs as runs [start, end) of sorted positions.
// reach[p] is the smallest sorted position coupled to position p and below it
// (p itself when there is none).  A block boundary sits before position p
// exactly when no coupled pair (a, b), a < p <= b, straddles it, i.e. when
// every position q >= p has reach[q] >= p.
inline void ap_runs(const int *reach, int n, std::vector<std::pair<int, int>> &runs)
{
    runs.clear();
    int end = n, runmin = n;
    for (int p = n - 1; p >= 0; p--) {
        runmin = std::min(runmin, reach[p]);
        if (runmin >= p) {
            runs.push_back(std::make_pair(p, end));
            end = p;
        }
    }
    std::reverse(runs.begin(), runs.end());
}

}  // namespace zk
