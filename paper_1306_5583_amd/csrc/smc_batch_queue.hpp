// smc_batch_queue.hpp -- the work queue of the persistent batched step:
// item kinds, the dependency counters, and the host-side builder that lists
// one step's items so that every item comes after all the items it waits
// for (the condition that lets workgroups taking tickets in order always
// make progress).
#pragma once

#include <stdint.h>

#include <algorithm>
#include <vector>

namespace smc {

// Kinds of work item (see smc_persist.hip for what each does).
enum : int32_t {
    IT_PF_MOVE = 0,
    IT_GMM_REWEIGHT = 1,
    IT_FINAL = 2,
    IT_RESAMPLE = 3,
    IT_GMM_STEP = 4,
    IT_MONITOR = 5  // mixture sampler: path-sampling integrand after all its M items
};

struct QItem {
    int32_t kind;
    int32_t prob;
    int32_t tile;   // 1024-particle tile (A, R), 64-particle tile (M); 0 for F
    int32_t count;  // M: consecutive 64-particle tiles of the item; monitor: the
                    // problem's 64-particle tiles; 1 otherwise
};

// Per-problem completion counters (uint32 each, DEP_STRIDE per problem):
// DEP_A counts finished A tiles, DEP_F finished normalisations, DEP_R
// finished resampling tiles of mixture samplers, DEP_M the 64-particle tiles
// of their finished Metropolis items (an item adds its tile count, so the
// targets do not depend on the item size a schedule chooses).  At step t the
// targets are t * tiles (A, R), t (F) and t * 64-particle tiles (the
// monitor).
enum : int { DEP_A = 0, DEP_F = 1, DEP_R = 2, DEP_M = 3, DEP_STRIDE = 4 };
// Launch-wide words: the ticket counter and the abort flag.
enum : int { SYNC_TICKET = 0, SYNC_ABORT = 1, SYNC_WORDS = 64 };

// Mixture samplers of the persistent step have at most this many components.
constexpr int BATCH_MAX_K = 8;

// Orders of the queue the autotuner chooses between.
enum : int32_t {
    // mixture samplers' A, F, R items, then their Metropolis tiles with the
    // most expensive problems first and their monitors, then the tracking
    // filters' items (which fill the workgroups freed at the tail of the
    // Metropolis phase)
    ORDER_COST_FIRST = 0,
    // phase by phase in problem order: every A item, every F, every R, then
    // the Metropolis tiles and the monitors
    ORDER_PHASES = 1
};

struct QProblem {
    bool gmm;
    int64_t tiles;     // 1024-particle tiles
    int64_t tiles64;   // 64-particle tiles
    double cost;       // relative cost of one 64-particle Metropolis tile
};

// One step's items.  `per_item` 64-particle tiles make one Metropolis item.
inline std::vector<QItem> build_queue(const std::vector<QProblem> &pr, int32_t order,
                                      int per_item)
{
    std::vector<QItem> q;
    const int np = (int)pr.size();
    std::vector<int> gm, pf;
    for (int p = 0; p < np; ++p)
        (pr[p].gmm ? gm : pf).push_back(p);
    auto phase_a = [&](const std::vector<int> &ps) {
        for (int p : ps)
            for (int64_t b = 0; b < pr[p].tiles; ++b)
                q.push_back(QItem{pr[p].gmm ? IT_GMM_REWEIGHT : IT_PF_MOVE, p, (int32_t)b, 1});
    };
    auto phase_f = [&](const std::vector<int> &ps) {
        for (int p : ps)
            q.push_back(QItem{IT_FINAL, p, 0, 1});
    };
    auto phase_r = [&](const std::vector<int> &ps) {
        for (int p : ps)
            for (int64_t b = 0; b < pr[p].tiles; ++b)
                q.push_back(QItem{IT_RESAMPLE, p, (int32_t)b, 1});
    };
    auto phase_m = [&](const std::vector<int> &ps) {
        for (int p : ps)
            for (int64_t b = 0; b < pr[p].tiles64; b += per_item)
                q.push_back(QItem{IT_GMM_STEP, p, (int32_t)b,
                                  (int32_t)std::min<int64_t>(per_item, pr[p].tiles64 - b)});
    };
    auto phase_mon = [&](const std::vector<int> &ps) {
        for (int p : ps)
            q.push_back(QItem{IT_MONITOR, p, 0, (int32_t)pr[p].tiles64});
    };
    if (order == ORDER_PHASES) {
        std::vector<int> all(np);
        for (int p = 0; p < np; ++p)
            all[p] = p;
        phase_a(all);
        phase_f(all);
        phase_r(all);
        phase_m(gm);
        phase_mon(gm);
    } else {
        std::vector<int> byc = gm;
        std::stable_sort(byc.begin(), byc.end(),
                         [&](int a, int b) { return pr[a].cost > pr[b].cost; });
        phase_a(byc);
        phase_f(byc);
        phase_r(byc);
        phase_m(byc);
        phase_mon(byc);
        phase_a(pf);
        phase_f(pf);
        phase_r(pf);
    }
    return q;
}

}  // namespace smc
