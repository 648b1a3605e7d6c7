// Internal state behind the opaque qtn_plan handle.
#pragma once

#include <string>
#include <vector>

#include "planner.h"

namespace qtn {
struct DeviceState;  // defined by the HIP runtime
struct NoAllocState; // tables of qtn_contract_noalloc, defined by the HIP runtime
constexpr uint32_t kLdsBudget = 56 * 1024;   // LDS bytes for program tensors
constexpr uint64_t kMaxWorkgroups = 1024;    // persistent workgroups of a program launch

// Execution mode for `slices_per_wave` slices: one workgroup per instance
// (MODE_SLICE) when there are enough instances to fill the chip and their
// scratch fits, else grid-wide streaming steps (MODE_WIDE).
int choose_mode(const struct qtn_plan_s *P, uint64_t S);
uint64_t wg_slots_for(const struct qtn_plan_s *P, int mode, uint64_t S);
void device_state_free(DeviceState *d);
void noalloc_state_free(NoAllocState *n);
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
  // per execution mode: the rescaling kernels run, i.e. the mixed form keeps
  // at least one intermediate in the 64-bit form outside LDS (values kept in
  // range for its 8-bit exponent); with every stored tensor complex128 (LDS
  // holds complex128 anyway) the FP64 kernels compute the same thing
  bool scaled[2] = {false, false};
  int exec_mode = -1;      // -1 chosen per binding, else qtn::ExecMode
  qtn::ExecPlan exec[2];   // MODE_WIDE, MODE_SLICE
  qtn::DeviceState *dev = nullptr;
  qtn::NoAllocState *na = nullptr;
  // a fault forced from the host for tests of re-issue: the next fault_count
  // range calls of qtn_contract_ranges that start at fault_lo fail
  uint64_t fault_lo = 0;
  int32_t fault_count = 0;
};
