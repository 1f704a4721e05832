// hbm_imm.h -- the IMM query state machine (imm.hip), shared by hbm_imm, hbm_imm_batch
// and the serving loop.
#pragma once

#include <chrono>
#include <string>
#include <vector>

#include "hbm_internal.h"

// the opaque handle of the C ABI
struct hbm_ctx {
    hbm::Ctx c;
};

namespace hbm {

// IMM parameters (Tang, Shi, Xiao 2015), evaluated in double in a fixed order.
struct ImmParams {
    double l_adj = 0, eps_prime = 0, lnC = 0, lambda_prime = 0, lambda_star = 0;
};
ImmParams imm_params(int32_t n, int32_t k, double eps, double l);

struct ImmJob {
    enum Phase { EST_SAMPLE, EST_SELECT, FIN_SAMPLE, FIN_SELECT, DONE, FAILED };
    Ctx *c = nullptr;
    int32_t k = 0;
    double eps = 0, l = 1;
    uint64_t seed = 0;
    ImmParams P;
    Phase phase = FAILED;
    int32_t round = 0;   // estimation round i
    double x = 0;        // n / 2^i of the current round
    int64_t target = 0;  // sets the current round needs
    double lb = 1.0;
    hbm_imm_stats st{};
    std::vector<int32_t> seeds;
    std::vector<uint64_t> gains;
    hbm_status status = HBM_OK;
    std::string error;
    std::chrono::steady_clock::time_point t0;
};

// Validate the query, reset the job's store and set the first target (FAILED on a bad query).
void imm_start(ImmJob &J);
bool imm_sampling(const ImmJob &J);
// One step for every listed job (none DONE or FAILED): a sampling block for each job short of
// its target (cap[i] >= 0 bounds its sets in this step; cap[i] == 0 skips it; empty: no bound),
// then one batched selection for every job whose target is met.  Device errors throw.
void imm_step(Ctx &root, const std::vector<ImmJob *> &jobs, const std::vector<int64_t> &cap);
// The two halves of a step, for drivers that run them on different streams: sampling blocks
// (jobs that meet their target move to their selection phase), and the batched selection of
// every job in a selection phase (which then moves on: next round, final round or DONE).
void imm_sample_step(Ctx &root, const std::vector<ImmJob *> &jobs, const std::vector<int64_t> &cap);
void imm_select_step(Ctx &root, const std::vector<ImmJob *> &jobs);
bool imm_selecting(const ImmJob &J);
// imm_start every job, then step until each is DONE or FAILED.
void imm_run(Ctx &root, const std::vector<ImmJob *> &jobs);

}  // namespace hbm
