// Stage plan of a set of signals executed together: one launch per stage and
// kernel variant, each covering every signal of the set through its own
// exclusive prefix of workgroups per signal. Shared by batches and the server.
#pragma once

#include <stdint.h>

#include <vector>

#include "common.hpp"
#include "host.hpp"

namespace sfft {

enum StepKind : uint32_t {
    kStepFold = 0, kStepFft = 1, kStepVote = 2, kStepFin = 3, kStepRes = 4, kStepFftLarge = 5, kStepComb = 6,
    kStepSub = 7, kStepReselect = 8, kStepEst = 9, kStepDecode = 10, kStepResSum = 11, kStepFused = 12
};

struct Step {
    StepKind kind;
    uint32_t param;       // fold variant / log2B / (staged | lmax << 8 | round << 16) / round /
                          // 0 / (log2B | pass << 8) / log2Bc / 0 / log2B / (lmax | round << 8) / round /
                          // 0 / L (fused)
    uint32_t units;       // workgroups of the launch
    uint32_t lds;         // dynamic LDS bytes
    size_t prefix_off;    // offset (in entries) of this launch's prefix of n+1 entries
};

// Fill `steps` and `prefix` (appended) for the signals `sig` (in launch order).
// Launches with no work are left out.
void plan_steps(const std::vector<const Resolved*>& sig, std::vector<Step>* steps, std::vector<uint32_t>* prefix);

// Upper bound of the prefix entries plan_steps appends for n signals.
size_t max_prefix_entries(size_t n);

// Launch the steps over the device arrays (descs[n], ios[n], prefix). part 0:
// bucketization launches only, 1: every later stage, -1: all.
hipError_t issue_steps(const std::vector<Step>& steps, const SigDesc* d_descs, const IoDesc* d_ios,
                       const uint32_t* d_prefix, uint32_t n, uint32_t xcd_order, int part, hipStream_t s);

}  // namespace sfft
