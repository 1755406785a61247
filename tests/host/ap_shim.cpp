// Host build of the all-pairs planning helpers, exported with C linkage.
#include "../../paper_2402_11868_amd/csrc/ap_host.h"

extern "C" {
// starts[k], ends[k] of the runs; returns their number
int t_ap_runs(const int *reach, int n, int *starts, int *ends)
{
    std::vector<std::pair<int, int>> runs;
    zk::ap_runs(reach, n, runs);
    for (size_t k = 0; k < runs.size(); k++) {
        starts[k] = runs[k].first;
        ends[k] = runs[k].second;
    }
    return (int)runs.size();
}

void t_ap_sorted_order(const double *th, int n, int *order)
{
    std::vector<int> o;
    zk::ap_sorted_order(th, n, o);
    for (int k = 0; k < n; k++) order[k] = o[k];
}
}
