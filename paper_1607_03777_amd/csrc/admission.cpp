// Host-only discrete-event simulation of the admission policy (admission.h).
#include "admission.h"

#include <algorithm>
#include <deque>
#include <numeric>
#include <queue>
#include <utility>

#include "../../include/sdg.h"

namespace sdg {

int simulate_admission(int n, const double* arrival_ms, const double* service_ms, const size_t* bytes,
                       int slots, size_t budget, int bypass, double* start_ms) {
  std::vector<int> order(n);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return arrival_ms[a] < arrival_ms[b]; });
  Admission adm(budget, slots, bypass);
  using Run = std::pair<double, int>;  // (end time, request)
  std::priority_queue<Run, std::vector<Run>, std::greater<Run>> running;
  std::deque<int> waiting;
  size_t next = 0;
  int started = 0;
  double t = n > 0 ? arrival_ms[order[0]] : 0.0;
  while (started < n) {
    while (next < order.size() && arrival_ms[order[next]] <= t) waiting.push_back(order[next++]);
    while (true) {
      std::vector<size_t> need(waiting.size());
      for (size_t i = 0; i < waiting.size(); ++i) need[i] = bytes[waiting[i]];
      const int pick = adm.pick(need);
      if (pick < 0) break;
      const int r = waiting[pick];
      waiting.erase(waiting.begin() + pick);
      start_ms[r] = t;
      adm.start(bytes[r]);
      running.push({t + service_ms[r], r});
      ++started;
    }
    if (started == n) break;
    const double t_arr = next < order.size() ? arrival_ms[order[next]] : 1e300;
    if (!running.empty() && running.top().first <= t_arr) {
      const Run e = running.top();
      running.pop();
      adm.end(bytes[e.second]);
      t = std::max(t, e.first);
    } else if (next < order.size()) {
      t = std::max(t, t_arr);
    } else {
      return SDG_ERR_INVALID;  // cannot happen when every request fits the budget
    }
  }
  return SDG_OK;
}

}  // namespace sdg
