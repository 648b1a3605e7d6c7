// Internal state behind the opaque qtn_plan handle.
#pragma once

#include <string>
#include <vector>

#include "planner.h"

namespace qtn {
struct DeviceState;  // defined by the HIP runtime
void device_state_free(DeviceState *d);
void set_error(const std::string &msg);
}  // namespace qtn

struct qtn_plan_s {
  qtn::Network net;
  std::vector<int> cut;    // ascending; slice bit b fixes cut[b]
  std::vector<int> order;  // elimination order of the free variables
  qtn::Schedule sched;
  qtn::PlanOpts popts;
  int precision = 0;
  int mf_width = 0;        // min-fill width of G - C
  uint64_t work = 0;       // sum 2^(|N+(v)|+1)
  double search_seconds = 0.0;
  int f64_below_rank = 0;  // intermediates of smaller rank are stored as complex128
  qtn::DeviceState *dev = nullptr;
};
