// Internal interface between the cost-model features / exact costs (host)
// and the device MLP with the model-guided cut search.
#pragma once

#include <cstdint>
#include <vector>

#include "../../include/qtn.h"

namespace qtn {

struct CostContext;  // network, line graph and uncut elimination statistics

CostContext *cost_context_new(const qtn_graph *graph, uint32_t p);  // NULL if invalid
void cost_context_free(CostContext *c);
int cost_context_vars(const CostContext *c);
const std::vector<std::vector<int>> &cost_context_adj(const CostContext *c);
void cost_features(const CostContext *c, const uint32_t *cut, uint32_t k, float *f);
void cost_exact(const CostContext *c, const uint32_t *cut, uint32_t k, int32_t &width,
                double &log2cost);

}  // namespace qtn
