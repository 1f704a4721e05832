// imm.hip -- the IMM driver as a resumable state machine.
//
// One query (k, eps, l, seed) on one context walks: estimation rounds i = 1, 2, ...
// (sample to theta_i, select k, test the lower bound), then the final round (sample
// to max(theta, sets so far), select k).  The schedule is the paper's Eq. 1 read as
// Tang, Shi and Xiao's lambda' together with their lower bound and final theta.
// Every step advances all given queries at once: one sampling block for each query
// that is short of its target, then one batched greedy selection for each query that
// reached it.  A single hbm_imm, a batch of instances and the serving loop all run
// this same code, so a query's result does not depend on what ran beside it.
#include <chrono>
#include <cmath>

#include "hbm_imm.h"

namespace hbm {

ImmParams imm_params(int32_t n, int32_t k, double eps, double l) {
    ImmParams p;
    const double dn = (double)n;
    p.l_adj = l * (1.0 + log(2.0) / log(dn));
    p.eps_prime = sqrt(2.0) * eps;
    double lc = 0.0;
    for (int32_t i = 1; i <= k; i++) lc += log((double)(n - k + i)) - log((double)i);
    p.lnC = lc;
    const double ep = p.eps_prime, la = p.l_adj;
    p.lambda_prime = (2.0 + 2.0 * ep / 3.0) * (lc + la * log(dn) + log(log2(dn))) * dn / (ep * ep);
    const double e1 = 1.0 - 1.0 / exp(1.0);
    const double alpha = sqrt(la * log(dn) + log(2.0));
    const double beta = sqrt(e1 * (lc + la * log(dn) + log(2.0)));
    p.lambda_star = 2.0 * dn * (e1 * alpha + beta) * (e1 * alpha + beta) / (eps * eps);
    return p;
}

static void fail(ImmJob &J, hbm_status st, const std::string &msg) {
    J.phase = ImmJob::FAILED;
    J.status = st;
    J.error = msg;
}

// The final round: theta = ceil(lambda* / LB) over at least the sets already drawn.
static void go_final(ImmJob &J, double lb) {
    J.lb = lb;
    const double thf = ceil(J.P.lambda_star / lb);
    if (!(thf < 2147483648.0)) {
        fail(J, HBM_EBUDGET, "final theta exceeds 2^31 sets");
        return;
    }
    J.st.lb = lb;
    J.st.theta_final = (int64_t)thf;
    J.target = std::max<int64_t>((int64_t)thf, J.c->s.nsets);
    J.phase = ImmJob::FIN_SAMPLE;
}

static bool round_ok(const ImmJob &J, int32_t i) { return (double)i <= log2((double)J.c->g.n) - 1.0; }

static void go_round(ImmJob &J, int32_t i) {
    const double dn = (double)J.c->g.n;
    J.round = i;
    J.x = dn / pow(2.0, (double)i);
    J.target = (int64_t)ceil(J.P.lambda_prime / J.x);
    J.phase = ImmJob::EST_SAMPLE;
}

void imm_start(ImmJob &J) {
    J.t0 = std::chrono::steady_clock::now();
    J.st = hbm_imm_stats{};
    J.status = HBM_OK;
    J.error.clear();
    J.seeds.clear();
    J.gains.clear();
    Ctx &c = *J.c;
    const int32_t k = J.k;
    const double eps = J.eps, l = J.l;
    if (!c.g.loaded) return fail(J, HBM_ESTATE, "no graph loaded");
    const int32_t n = c.g.n;
    if (n < 2) return fail(J, HBM_EINVAL, "IMM needs n >= 2");
    if (k < 1 || k > n) return fail(J, HBM_EINVAL, "k must be in [1, n]");
    if (!(eps > 0.0 && std::isfinite(eps))) return fail(J, HBM_EINVAL, "eps must be positive");
    if (!(l > 0.0 && std::isfinite(l))) return fail(J, HBM_EINVAL, "l must be positive");
    c.t_sample = c.t_select = c.t_encode = 0;
    store_reset(c);
    J.P = imm_params(n, k, eps, l);
    J.st.lambda_prime = J.P.lambda_prime;
    J.st.lambda_star = J.P.lambda_star;
    if (round_ok(J, 1)) go_round(J, 1);
    else go_final(J, 1.0);
}

static void finish(ImmJob &J, uint64_t cov) {
    Ctx &c = *J.c;
    J.st.nsets_final = c.s.nsets;
    J.st.coverage = cov;
    J.st.influence = (double)c.g.n * (double)cov / (double)c.s.nsets;
    J.st.t_sample_ms = c.t_sample;
    J.st.t_encode_ms = c.t_encode;
    J.st.t_select_ms = c.t_select;
    J.st.t_total_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - J.t0).count();
    store_stats(c, &J.st.store);
    J.phase = ImmJob::DONE;
}

// After a selection over the job's current target.
static void selected(ImmJob &J, std::vector<int32_t> &&s, std::vector<uint64_t> &&g, uint64_t cov) {
    J.seeds = std::move(s);
    J.gains = std::move(g);
    if (J.phase == ImmJob::FIN_SELECT) return finish(J, cov);
    const double dn = (double)J.c->g.n;
    const int64_t th = J.target;
    if (J.st.rounds < 64) {
        J.st.theta_round[J.st.rounds] = th;
        J.st.cov_round[J.st.rounds] = cov;
    }
    J.st.rounds++;
    if (dn * (double)cov / (double)th >= (1.0 + J.P.eps_prime) * J.x)
        return go_final(J, dn * (double)cov / ((double)th * (1.0 + J.P.eps_prime)));
    if (round_ok(J, J.round + 1)) go_round(J, J.round + 1);
    else go_final(J, 1.0);
}

bool imm_sampling(const ImmJob &J) { return J.phase == ImmJob::EST_SAMPLE || J.phase == ImmJob::FIN_SAMPLE; }

// Jobs whose sampling target is met move on to their selection.
static void promote(const std::vector<ImmJob *> &jobs) {
    for (ImmJob *J : jobs)
        if (imm_sampling(*J) && J->c->s.nsets >= J->target)
            J->phase = J->phase == ImmJob::EST_SAMPLE ? ImmJob::EST_SELECT : ImmJob::FIN_SELECT;
}

bool imm_selecting(const ImmJob &J) { return J.phase == ImmJob::EST_SELECT || J.phase == ImmJob::FIN_SELECT; }

void imm_sample_step(Ctx &root, const std::vector<ImmJob *> &jobs, const std::vector<int64_t> &cap) {
    promote(jobs);
    std::vector<Ctx *> sc;
    std::vector<int64_t> th, cp;
    std::vector<uint64_t> sd;
    std::vector<ImmJob *> sj;
    for (size_t i = 0; i < jobs.size(); i++) {
        ImmJob *J = jobs[i];
        if (!imm_sampling(*J)) continue;
        const Store &S = J->c->s;
        const bool warming = S.enc != HBM_ENC_NONE && !S.model_ready;
        if (!cap.empty() && cap[i] == 0 && !warming) continue;  // warm-up blocks store nothing
        sj.push_back(J);
        sc.push_back(J->c);
        th.push_back(J->target);
        sd.push_back(J->seed);
        cp.push_back(cap.empty() ? -1 : cap[i]);
    }
    if (!sc.empty()) {
        std::vector<hbm_status> st;
        extend_step(root, sc, th, sd, cp, st);
        for (size_t q = 0; q < sj.size(); q++)
            if (st[q] != HBM_OK)
                fail(*sj[q], st[q], "store budget exceeded at " + std::to_string(sj[q]->c->s.nsets) + " sets");
    }
    promote(jobs);
}

void imm_select_step(Ctx &root, const std::vector<ImmJob *> &jobs) {
    std::vector<Ctx *> lc;
    std::vector<int32_t> lk;
    std::vector<ImmJob *> lj;
    for (ImmJob *J : jobs)
        if (imm_selecting(*J)) {
            lj.push_back(J);
            lc.push_back(J->c);
            lk.push_back(J->k);
        }
    if (lc.empty()) return;
    std::vector<std::vector<int32_t>> s;
    std::vector<std::vector<uint64_t>> g;
    std::vector<uint64_t> cov;
    select_batch(root, lc, lk, s, g, cov);
    for (size_t q = 0; q < lj.size(); q++) selected(*lj[q], std::move(s[q]), std::move(g[q]), cov[q]);
}

void imm_step(Ctx &root, const std::vector<ImmJob *> &jobs, const std::vector<int64_t> &cap) {
    imm_sample_step(root, jobs, cap);
    imm_select_step(root, jobs);
}

void imm_run(Ctx &root, const std::vector<ImmJob *> &jobs) {
    for (ImmJob *J : jobs) imm_start(*J);
    for (;;) {
        std::vector<ImmJob *> live;
        for (ImmJob *J : jobs)
            if (J->phase != ImmJob::DONE && J->phase != ImmJob::FAILED) live.push_back(J);
        if (live.empty()) return;
        imm_step(root, live, {});
    }
}

}  // namespace hbm
