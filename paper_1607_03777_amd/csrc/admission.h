// Admission policy of the request server: a request starts when a slot is
// free and its device memory fits into what the budget has left.  The oldest
// waiting request (the head) goes first; a later request may overtake a head
// that does not fit, at most `bypass` times per head, so no request waits
// forever.  The same class drives the live server and the host-only
// simulation used to test the policy and to plan capacity.
#pragma once

#include <cstddef>
#include <vector>

namespace sdg {

class Admission {
 public:
  Admission() = default;
  Admission(size_t budget, int slots, int bypass) : budget_(budget), slots_(slots), bypass_(bypass) {}

  // index into `need` (bytes of the waiting requests, oldest first) of the
  // request to start now, or -1
  int pick(const std::vector<size_t>& need) {
    if (busy_ >= slots_ || need.empty()) return -1;
    if (fits(need[0])) {
      head_skips_ = 0;
      return 0;
    }
    if (head_skips_ >= bypass_) return -1;
    for (size_t i = 1; i < need.size(); ++i)
      if (fits(need[i])) {
        ++head_skips_;
        return (int)i;
      }
    return -1;
  }
  bool fits(size_t bytes) const { return in_use_ + bytes <= budget_; }
  void start(size_t bytes) {
    in_use_ += bytes;
    ++busy_;
  }
  void end(size_t bytes) {
    in_use_ -= bytes < in_use_ ? bytes : in_use_;
    --busy_;
  }
  size_t in_use() const { return in_use_; }
  int busy() const { return busy_; }

 private:
  size_t budget_ = 0;
  int slots_ = 1;
  int bypass_ = 0;
  size_t in_use_ = 0;
  int busy_ = 0;
  int head_skips_ = 0;
};

// Discrete-event run of the policy: request i arrives at arrival_ms[i],
// occupies a slot and bytes[i] for service_ms[i]; start_ms[i] receives its
// start time.  Every bytes[i] must be <= budget.
int simulate_admission(int n, const double* arrival_ms, const double* service_ms, const size_t* bytes,
                       int slots, size_t budget, int bypass, double* start_ms);

}  // namespace sdg
