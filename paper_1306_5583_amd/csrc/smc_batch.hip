// smc_batch.hip -- the batched form of the sweep: many independent filters
// and samplers advanced together, one launch per phase over all of their
// tiles, the step index on the device so that one captured HIP graph serves
// every step, and an autotuner for the waves per mixture tile.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <new>
#include <string>
#include <vector>

#include "smc_internal.hpp"
#include "smc_batch_queue.hpp"

namespace smc {

// Problems of one mixture size and move kind, initialised by one launch.
struct KGroup {
    int K = 0;
    bool mala = false;
    int2 *map64 = nullptr;
    int64_t tiles64 = 0;
    int W = 1;
    int64_t sum_n = 0;
    int64_t max_nd = 0;
};

}  // namespace smc

using namespace smc;

struct smc_batch {
    std::vector<smc_batch_problem> probs;
    std::vector<Prob> P;
    std::vector<QProblem> qp;
    hipStream_t stream = nullptr;
    char *table = nullptr;
    Prob *dprobs = nullptr;
    int2 *map_pf = nullptr, *map_gmm = nullptr, *map_all = nullptr;
    int64_t pf_tiles = 0, gmm_tiles = 0, all_tiles = 0;
    std::vector<KGroup> groups;
    int32_t *step = nullptr;        // step index of the initialisation kernels
    QItem *queue = nullptr;         // one step's work items
    int64_t queue_cap = 0;
    uint32_t nitems = 0;
    uint32_t *deps = nullptr;       // per-problem completion counters
    uint32_t *sync = nullptr;       // ticket counter, abort flag
    int cus = 0;                    // compute units of the device
    int max_wgs_per_cu = 0;         // co-resident step workgroups per CU
    int32_t order = ORDER_COST_FIRST, per_item = 1, wgs_per_cu = 0;
    uint32_t nwg = 0;               // workgroups of the step launch
    bool initialised = false;
    int host_step = 0;
    int max_steps = 0;
    int64_t max_count = 1;          // largest per-step counter target unit (tiles per problem)
    int counter_steps = 0;          // steps the 32-bit ticket and counters can index
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::string last_error;
};

namespace {

struct Plan {
    size_t probs = 0, map_pf = 0, map_gmm = 0, map_all = 0, step = 0, queue = 0, deps = 0,
           sync = 0, total = 0;
    std::vector<size_t> map64;
    std::vector<std::pair<int, bool>> keys;  // (K, mala) of each mixture group
    std::vector<int64_t> tiles64;
    int64_t pf_tiles = 0, gmm_tiles = 0, queue_cap = 0;
};

size_t al(size_t v) { return (v + 255) & ~size_t(255); }

Plan plan(const smc_batch_problem *probs, int32_t np)
{
    Plan pl;
    std::map<std::pair<int, bool>, int64_t> t64;
    for (int32_t i = 0; i < np; ++i) {
        const smc_config &c = probs[i].cfg;
        const int64_t nt = ceil_div(c.n, TILE);
        if (c.model == SMC_MODEL_CV_TRACK) {
            pl.pf_tiles += nt;
            pl.queue_cap += 2 * nt + 1;
        } else {
            pl.gmm_tiles += nt;
            t64[{c.K, c.move_kind == SMC_MOVE_MALA}] += ceil_div(c.n, WAVE);
            pl.queue_cap += 2 * nt + 2 + ceil_div(c.n, WAVE);
        }
    }
    size_t off = 0;
    pl.probs = off;
    off = al(off + sizeof(Prob) * (size_t)np);
    pl.map_pf = off;
    off = al(off + sizeof(int2) * (size_t)pl.pf_tiles);
    pl.map_gmm = off;
    off = al(off + sizeof(int2) * (size_t)pl.gmm_tiles);
    pl.map_all = off;
    off = al(off + sizeof(int2) * (size_t)(pl.pf_tiles + pl.gmm_tiles));
    for (auto &kv : t64) {
        pl.keys.push_back(kv.first);
        pl.tiles64.push_back(kv.second);
        pl.map64.push_back(off);
        off = al(off + sizeof(int2) * (size_t)kv.second);
    }
    pl.step = off;
    off = al(off + 256);
    pl.queue = off;
    off = al(off + sizeof(QItem) * (size_t)pl.queue_cap);
    pl.deps = off;
    off = al(off + sizeof(uint32_t) * DEP_STRIDE * (size_t)np);
    pl.sync = off;
    off = al(off + sizeof(uint32_t) * SYNC_WORDS);
    pl.total = off;
    return pl;
}

// What the queue needs to know of each problem: its tiles and the relative
// cost of one Metropolis tile (data points x components, MALA's gradient
// and the sweeps).
std::vector<QProblem> queue_problems(const smc_batch_problem *probs, int32_t np)
{
    std::vector<QProblem> q;
    for (int32_t i = 0; i < np; ++i) {
        const smc_config &c = probs[i].cfg;
        QProblem r;
        r.gmm = c.model == SMC_MODEL_GMM_TEMPERED;
        r.tiles = ceil_div(c.n, TILE);
        r.tiles64 = r.gmm ? ceil_div(c.n, WAVE) : 0;
        r.cost = r.gmm ? (double)c.n_data * c.K * (c.move_kind == SMC_MOVE_MALA ? 1.4 : 1.0) *
                             (c.sweeps > 0 ? c.sweeps : 1)
                       : 0.0;
        q.push_back(r);
    }
    return q;
}

smc_status bfail(smc_batch *b, smc_status s, const std::string &m)
{
    b->last_error = m;
    return s;
}

smc_status bhip(smc_batch *b, hipError_t e, const char *where)
{
    if (e == hipSuccess)
        return SMC_OK;
    b->last_error = std::string(where) + ": " + hipGetErrorString(e);
    return SMC_ERR_DEVICE;
}

// Validation shared by the table size, the queue inspection and creation.
smc_status check_problem(const smc_batch_problem &q, std::string &err)
{
    smc_status s = validate_config(&q.cfg, err);
    if (s != SMC_OK)
        return s;
    if (q.cfg.scheme != SMC_RS_SYSTEMATIC && q.cfg.scheme != SMC_RS_STRATIFIED)
        return SMC_ERR_UNSUPPORTED;
    if (q.cfg.model == SMC_MODEL_GMM_TEMPERED && q.cfg.K > BATCH_MAX_K)
        return SMC_ERR_UNSUPPORTED;
    return SMC_OK;
}

// Builds and uploads the step's queue for a schedule choice (not while a
// step is captured: it copies from the host).
hipError_t set_schedule(smc_batch *b, int32_t order, int32_t per_item, int32_t wgs_per_cu)
{
    const std::vector<QItem> q = build_queue(b->qp, order, per_item);
    if ((int64_t)q.size() > b->queue_cap)
        return hipErrorInvalidValue;
    // steps already enqueued read the old queue
    hipError_t e = hipStreamSynchronize(b->stream);
    if (e == hipSuccess)
        e = hipMemcpy(b->queue, q.data(), sizeof(QItem) * q.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess)
        return e;
    const uint32_t old_per_step = b->nitems + b->nwg;
    b->order = order;
    b->per_item = per_item;
    b->wgs_per_cu = std::max(1, std::min(wgs_per_cu, b->max_wgs_per_cu));
    b->nitems = (uint32_t)q.size();
    // no more workgroups than the step has items (a small batch's launch
    // then costs what its few tiles need)
    b->nwg = std::max(1u, std::min((uint32_t)(b->wgs_per_cu * b->cus), b->nitems));
    // The ticket and the completion counters are 32-bit and only grow: step t
    // takes tickets up to t * (items + workgroups) and waits for counter
    // targets up to t * (tiles of the largest problem), so the step index is
    // capped where either would wrap.
    {
        const uint64_t per = (uint64_t)b->nitems + b->nwg;
        const uint64_t lim = std::min<uint64_t>(0xFFFFFFFFull / per,
                                                0xFFFFFFFFull / (uint64_t)b->max_count);
        b->counter_steps = (int)std::min<uint64_t>(lim, (uint64_t)INT_MAX);
    }
    // steps already taken keep their index under the new ticket count
    if (b->initialised && old_per_step != b->nitems + b->nwg)
        e = launch_batch_ticket_rebase(b->sync, old_per_step, b->nitems + b->nwg, b->stream);
    if (e != hipSuccess)
        return e;
    if (b->exec) {  // a captured step used the old schedule
        (void)hipGraphExecDestroy(b->exec);
        b->exec = nullptr;
    }
    if (b->graph) {
        (void)hipGraphDestroy(b->graph);
        b->graph = nullptr;
    }
    return hipSuccess;
}

// One step: a single launch of the persistent step kernel.
hipError_t enqueue_step(smc_batch *b)
{
    return launch_batch_step(b->dprobs, b->queue, b->nitems, b->nwg, b->sync, b->deps,
                             b->stream);
}

std::string cache_key(const smc_batch *b)
{
    int dev = 0;
    hipDeviceProp_t prop;
    (void)hipGetDevice(&dev);
    (void)hipGetDeviceProperties(&prop, dev);
    // shape bucket: per problem type and mixture size, the problem count and
    // the rounded-up log2 of the particles and of the data points
    std::map<std::string, int> buckets;
    for (const smc_batch_problem &q : b->probs) {
        const smc_config &c = q.cfg;
        char k[96];
        if (c.model == SMC_MODEL_CV_TRACK)
            snprintf(k, sizeof(k), "pf%d", (int)ceil(log2((double)c.n)));
        else
            snprintf(k, sizeof(k), "g%d%c%d.%d", c.K, c.move_kind == SMC_MOVE_MALA ? 'm' : 'r',
                     (int)ceil(log2((double)c.n)), (int)ceil(log2((double)c.n_data)));
        buckets[k] += 1;
    }
    std::string key = prop.gcnArchName;
    for (auto &kv : buckets)
        key += " " + kv.first + "x" + std::to_string(kv.second);
    std::replace(key.begin(), key.end(), ':', '_');
    return key;
}

}  // namespace

extern "C" {

smc_status smc_batch_table_size(const smc_batch_problem *probs, int32_t nprob, size_t *bytes)
{
    if (!probs || nprob < 1 || !bytes)
        return SMC_ERR_INVALID_ARG;
    std::string err;
    for (int32_t i = 0; i < nprob; ++i) {
        const smc_status s = check_problem(probs[i], err);
        if (s != SMC_OK)
            return s;
    }
    *bytes = plan(probs, nprob).total;
    return SMC_OK;
}

smc_status smc_batch_plan_queue(const smc_batch_problem *probs, int32_t nprob, int32_t order,
                                int32_t per_item, int32_t *items, int64_t capacity,
                                int64_t *count)
{
    if (!probs || nprob < 1 || !count || (order != ORDER_COST_FIRST && order != ORDER_PHASES) ||
        per_item < 1 || per_item > 2 || capacity < 0 || (capacity > 0 && !items))
        return SMC_ERR_INVALID_ARG;
    std::string err;
    for (int32_t i = 0; i < nprob; ++i) {
        const smc_status s = check_problem(probs[i], err);
        if (s != SMC_OK)
            return s;
    }
    const std::vector<QItem> q = build_queue(queue_problems(probs, nprob), order, per_item);
    *count = (int64_t)q.size();
    if (capacity < (int64_t)q.size())
        return capacity == 0 ? SMC_OK : SMC_ERR_INVALID_ARG;
    for (size_t k = 0; k < q.size(); ++k) {
        items[4 * k] = q[k].kind;
        items[4 * k + 1] = q[k].prob;
        items[4 * k + 2] = q[k].tile;
        items[4 * k + 3] = q[k].count;
    }
    return SMC_OK;
}

smc_status smc_batch_create(const smc_batch_problem *probs, int32_t nprob, void *table,
                            size_t table_bytes, void *hip_stream, smc_batch **out)
{
    if (!out)
        return SMC_ERR_INVALID_ARG;
    *out = nullptr;
    if (!probs || nprob < 1 || !table || (reinterpret_cast<uintptr_t>(table) % 256) != 0)
        return SMC_ERR_INVALID_ARG;
    std::string err;
    for (int32_t i = 0; i < nprob; ++i) {
        const smc_batch_problem &q = probs[i];
        smc_status s = check_problem(q, err);
        if (s != SMC_OK)
            return s;
        s = validate_buffers(q.cfg, &q.buf, err);
        if (s != SMC_OK)
            return s;
        if (q.cfg.model == SMC_MODEL_GMM_TEMPERED && (!q.schedule || q.schedule_len < 2))
            return SMC_ERR_INVALID_ARG;
    }
    const Plan pl = plan(probs, nprob);
    if (table_bytes < pl.total)
        return SMC_ERR_INVALID_ARG;
    smc_status s = device_ok(err);
    if (s != SMC_OK)
        return s;
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
        return SMC_ERR_DEVICE;
    const int per_cu = batch_step_blocks_per_cu();
    if (per_cu < 1)
        return SMC_ERR_DEVICE;
    smc_batch *b = new (std::nothrow) smc_batch();
    if (!b)
        return SMC_ERR_DEVICE;
    b->probs.assign(probs, probs + nprob);
    b->qp = queue_problems(probs, nprob);
    b->stream = static_cast<hipStream_t>(hip_stream);
    b->table = static_cast<char *>(table);
    b->dprobs = reinterpret_cast<Prob *>(b->table + pl.probs);
    b->map_pf = reinterpret_cast<int2 *>(b->table + pl.map_pf);
    b->map_gmm = reinterpret_cast<int2 *>(b->table + pl.map_gmm);
    b->map_all = reinterpret_cast<int2 *>(b->table + pl.map_all);
    b->step = reinterpret_cast<int32_t *>(b->table + pl.step);
    b->queue = reinterpret_cast<QItem *>(b->table + pl.queue);
    b->queue_cap = pl.queue_cap;
    b->deps = reinterpret_cast<uint32_t *>(b->table + pl.deps);
    b->sync = reinterpret_cast<uint32_t *>(b->table + pl.sync);
    b->pf_tiles = pl.pf_tiles;
    b->gmm_tiles = pl.gmm_tiles;
    b->all_tiles = pl.pf_tiles + pl.gmm_tiles;
    b->cus = prop.multiProcessorCount;
    b->max_wgs_per_cu = per_cu;
    // descriptors and maps, staged on the host
    std::vector<int2> mpf, mgmm, mall;
    std::map<std::pair<int, bool>, std::vector<int2>> m64;
    std::map<std::pair<int, bool>, KGroup> grp;
    b->max_steps = 1 << 30;
    for (int32_t i = 0; i < nprob; ++i) {
        const smc_batch_problem &q = probs[i];
        const Workspace ws = plan_workspace(q.cfg);
        Prob P = prob_from(q.cfg, q.buf, ws, q.buf.state, q.buf.state_alt);
        P.sched = q.schedule;
        b->P.push_back(P);
        const int64_t nt = ceil_div(q.cfg.n, TILE);
        // counter targets per step: tiles (move, reweight, resampling), and
        // for a mixture sampler its 64-particle tiles (Metropolis items)
        b->max_count = std::max(b->max_count, q.cfg.model == SMC_MODEL_CV_TRACK
                                                  ? nt
                                                  : ceil_div(q.cfg.n, WAVE));
        for (int64_t t = 0; t < nt; ++t) {
            (q.cfg.model == SMC_MODEL_CV_TRACK ? mpf : mgmm).push_back(make_int2(i, (int)t));
            mall.push_back(make_int2(i, (int)t));
        }
        if (q.buf.history)
            b->max_steps = std::min<int>(b->max_steps, (int)q.buf.history_len - 1);
        if (q.cfg.model == SMC_MODEL_CV_TRACK) {
            b->max_steps = std::min<int>(b->max_steps, q.cfg.n_obs - 1);
        } else {
            b->max_steps = std::min<int>(b->max_steps, q.schedule_len - 1);
            const std::pair<int, bool> key{q.cfg.K, q.cfg.move_kind == SMC_MOVE_MALA};
            const int64_t t64 = ceil_div(q.cfg.n, WAVE);
            auto &v = m64[key];
            for (int64_t t = 0; t < t64; ++t)
                v.push_back(make_int2(i, (int)t));
            KGroup &g = grp[key];
            g.K = key.first;
            g.mala = key.second;
            g.sum_n += q.cfg.n;
            g.max_nd = std::max<int64_t>(g.max_nd, q.cfg.n_data);
        }
    }
    hipError_t e = hipMemcpy(b->dprobs, b->P.data(), sizeof(Prob) * b->P.size(),
                             hipMemcpyHostToDevice);
    if (e == hipSuccess && !mpf.empty())
        e = hipMemcpy(b->map_pf, mpf.data(), sizeof(int2) * mpf.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess && !mgmm.empty())
        e = hipMemcpy(b->map_gmm, mgmm.data(), sizeof(int2) * mgmm.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(b->map_all, mall.data(), sizeof(int2) * mall.size(), hipMemcpyHostToDevice);
    for (size_t k = 0; k < pl.keys.size() && e == hipSuccess; ++k) {
        KGroup g = grp[pl.keys[k]];
        g.map64 = reinterpret_cast<int2 *>(b->table + pl.map64[k]);
        g.tiles64 = pl.tiles64[k];
        g.W = gmm_waves(g.sum_n, g.max_nd);
        const auto &v = m64[pl.keys[k]];
        e = hipMemcpy(g.map64, v.data(), sizeof(int2) * v.size(), hipMemcpyHostToDevice);
        b->groups.push_back(g);
    }
    if (e == hipSuccess)
        e = set_schedule(b, ORDER_COST_FIRST, 1, per_cu);
    if (e != hipSuccess) {
        delete b;
        return SMC_ERR_DEVICE;
    }
    *out = b;
    return SMC_OK;
}

smc_status smc_batch_destroy(smc_batch *b)
{
    if (!b)
        return SMC_OK;
    if (b->exec)
        (void)hipGraphExecDestroy(b->exec);
    if (b->graph)
        (void)hipGraphDestroy(b->graph);
    delete b;
    return SMC_OK;
}

smc_status smc_batch_waves(const smc_batch *b, int32_t K, int32_t *waves)
{
    if (!b || !waves)
        return SMC_ERR_INVALID_ARG;
    for (const KGroup &g : b->groups)
        if (g.K == K) {
            *waves = g.W;
            return SMC_OK;
        }
    return SMC_ERR_INVALID_ARG;
}

smc_status smc_batch_init(smc_batch *b)
{
    if (!b)
        return SMC_ERR_INVALID_ARG;
    hipStream_t s = b->stream;
    const int32_t np = (int32_t)b->P.size();
    hipError_t e = launch_set_step(b->step, 0, 0, s);
    if (e == hipSuccess)
        e = launch_reset_scalars_batch(b->dprobs, np, s);
    if (e == hipSuccess)
        e = launch_pf_init_batch(b->dprobs, b->map_pf, b->pf_tiles, s);
    for (const KGroup &g : b->groups)
        if (e == hipSuccess)
            e = launch_gmm_init_batch(b->dprobs, g.map64, g.tiles64, g.K, g.W, g.mala, s);
    if (e == hipSuccess)
        e = launch_const_partials_batch(b->dprobs, b->map_gmm, b->gmm_tiles, s);
    if (e == hipSuccess)
        e = launch_finalize_batch(b->dprobs, np, b->step, s);
    if (e == hipSuccess)
        e = launch_resample_batch(b->dprobs, b->map_all, b->all_tiles, b->step, s);
    // the mixture samplers' step-0 path-sampling point (alpha_0, U_0)
    if (e == hipSuccess && b->gmm_tiles > 0)
        e = launch_batch_monitor0(b->dprobs, np, s);
    // the step kernel's tickets and completion counters start from zero
    if (e == hipSuccess)
        e = launch_batch_sync_reset(b->sync, b->deps, np, s);
    if (e == hipSuccess) {
        b->initialised = true;
        b->host_step = 0;
    }
    return bhip(b, e, "smc_batch_init");
}

smc_status smc_batch_step(smc_batch *b)
{
    if (!b)
        return SMC_ERR_INVALID_ARG;
    if (!b->initialised)
        return bfail(b, SMC_ERR_BAD_STATE, "smc_batch_step before smc_batch_init");
    if (b->host_step >= b->max_steps)
        return bfail(b, SMC_ERR_BAD_STATE, "no observations / schedule rows / history rows left");
    if (b->host_step >= b->counter_steps)
        return bfail(b, SMC_ERR_UNSUPPORTED,
                     "step index beyond the 32-bit step counters for this batch and schedule");
    const hipError_t e = enqueue_step(b);
    if (e == hipSuccess)
        b->host_step++;
    return bhip(b, e, "smc_batch_step");
}

smc_status smc_batch_capture(smc_batch *b)
{
    if (!b)
        return SMC_ERR_INVALID_ARG;
    if (b->exec) {
        (void)hipGraphExecDestroy(b->exec);
        b->exec = nullptr;
    }
    if (b->graph) {
        (void)hipGraphDestroy(b->graph);
        b->graph = nullptr;
    }
    hipError_t e = hipStreamBeginCapture(b->stream, hipStreamCaptureModeRelaxed);
    if (e != hipSuccess)
        return bhip(b, e, "smc_batch_capture (begin)");
    const hipError_t e1 = enqueue_step(b);
    e = hipStreamEndCapture(b->stream, &b->graph);
    if (e1 != hipSuccess)
        return bhip(b, e1, "smc_batch_capture (enqueue)");
    if (e != hipSuccess)
        return bhip(b, e, "smc_batch_capture (end)");
    e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
    return bhip(b, e, "smc_batch_capture (instantiate)");
}

smc_status smc_batch_replay(smc_batch *b)
{
    if (!b)
        return SMC_ERR_INVALID_ARG;
    if (!b->exec)
        return bfail(b, SMC_ERR_BAD_STATE, "smc_batch_replay before smc_batch_capture");
    if (!b->initialised)
        return bfail(b, SMC_ERR_BAD_STATE, "smc_batch_replay before smc_batch_init");
    if (b->host_step >= b->max_steps)
        return bfail(b, SMC_ERR_BAD_STATE, "no observations / schedule rows / history rows left");
    if (b->host_step >= b->counter_steps)
        return bfail(b, SMC_ERR_UNSUPPORTED,
                     "step index beyond the 32-bit step counters for this batch and schedule");
    const hipError_t e = hipGraphLaunch(b->exec, b->stream);
    if (e == hipSuccess)
        b->host_step++;
    return bhip(b, e, "smc_batch_replay");
}

smc_status smc_batch_check(smc_batch *b, int32_t *first_bad)
{
    if (!b)
        return SMC_ERR_INVALID_ARG;
    if (first_bad)
        *first_bad = -1;
    hipError_t e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess)
        return bhip(b, e, "smc_batch_check");
    for (size_t i = 0; i < b->P.size(); ++i) {
        int32_t word = 0;
        e = hipMemcpy(&word, b->P[i].counters + CNT_ERR, sizeof(int32_t), hipMemcpyDeviceToHost);
        if (e != hipSuccess)
            return bhip(b, e, "smc_batch_check");
        if (word != 0) {
            if (first_bad)
                *first_bad = (int32_t)i;
            b->last_error = "problem " + std::to_string(i) + ": device error word " +
                            std::to_string(word);
            return SMC_ERR_NUMERIC;
        }
    }
    return SMC_OK;
}

const char *smc_batch_last_error(const smc_batch *b)
{
    return b ? b->last_error.c_str() : "null batch";
}

smc_status smc_batch_schedule(const smc_batch *b, int32_t *out)
{
    if (!b || !out)
        return SMC_ERR_INVALID_ARG;
    out[0] = b->order;
    out[1] = b->per_item;
    out[2] = b->wgs_per_cu;
    out[3] = (int32_t)b->nwg;
    out[4] = (int32_t)b->nitems;
    return SMC_OK;
}

smc_status smc_batch_set_schedule(smc_batch *b, int32_t order, int32_t per_item,
                                  int32_t wgs_per_cu)
{
    if (!b || (order != ORDER_COST_FIRST && order != ORDER_PHASES) || per_item < 1 ||
        per_item > 2 || wgs_per_cu < 1)
        return SMC_ERR_INVALID_ARG;
    return bhip(b, set_schedule(b, order, per_item, wgs_per_cu), "smc_batch_set_schedule");
}

// Autotuner of the persistent step: times whole steps (from a fresh
// initialisation) for every candidate schedule -- queue order, 64-particle
// tiles per Metropolis item, step workgroups per compute unit -- and keeps
// the fastest; results are cached per device and batch shape bucket.
smc_status smc_batch_autotune(smc_batch *b, int32_t repeats, const char *cache_path)
{
    if (!b || repeats < 1)
        return SMC_ERR_INVALID_ARG;
    const std::string key = cache_key(b);
    if (cache_path) {
        if (FILE *f = fopen(cache_path, "r")) {
            char line[4096];
            int o = -1, q = -1, w = -1;
            while (fgets(line, sizeof(line), f)) {
                char *tail = strstr(line, " | order=");
                if (!tail)
                    continue;
                *tail = 0;
                int oo, qq, ww;
                if (key == line && sscanf(tail + 3, "order=%d per_item=%d wgs_per_cu=%d", &oo,
                                          &qq, &ww) == 3) {
                    o = oo;
                    q = qq;
                    w = ww;
                }
            }
            fclose(f);
            if ((o == ORDER_COST_FIRST || o == ORDER_PHASES) && (q == 1 || q == 2) && w >= 1) {
                const hipError_t e = set_schedule(b, o, q, w);
                b->initialised = false;
                return bhip(b, e, "smc_batch_autotune (cached schedule)");
            }
        }
    }
    const int steps = std::min(repeats + 1, b->max_steps);
    if (steps < 2)
        return bfail(b, SMC_ERR_BAD_STATE, "smc_batch_autotune needs two steps of schedule");
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return bfail(b, SMC_ERR_DEVICE, "hipEventCreate");
    float best = 1e30f;
    int bo = b->order, bq = b->per_item, bw = b->wgs_per_cu;
    hipError_t err = hipSuccess;
    for (int o : {ORDER_COST_FIRST, ORDER_PHASES})
        for (int q = 1; q <= 2; ++q)
            for (int w = 1; w <= b->max_wgs_per_cu && err == hipSuccess; ++w) {
                err = set_schedule(b, o, q, w);
                if (err != hipSuccess)
                    break;
                smc_status st = smc_batch_init(b);
                if (st != SMC_OK) {
                    err = hipErrorUnknown;
                    break;
                }
                // the first step warms up; the rest are timed one by one
                // (within what the step counters can index)
                const int nsteps = std::min(steps, b->counter_steps);
                std::vector<float> ms;
                for (int k = 0; k < nsteps && err == hipSuccess; ++k) {
                    err = hipEventRecord(e0, b->stream);
                    if (err == hipSuccess)
                        err = enqueue_step(b);
                    if (err == hipSuccess)
                        err = hipEventRecord(e1, b->stream);
                    if (err == hipSuccess)
                        err = hipEventSynchronize(e1);
                    float t = 0.f;
                    if (err == hipSuccess)
                        err = hipEventElapsedTime(&t, e0, e1);
                    if (k > 0)
                        ms.push_back(t);
                }
                if (err != hipSuccess)
                    break;
                if (ms.empty())  // no timed step fits this schedule's counters
                    continue;
                std::sort(ms.begin(), ms.end());
                const float med = ms[ms.size() / 2];
                if (med < best) {
                    best = med;
                    bo = o;
                    bq = q;
                    bw = w;
                }
            }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    b->initialised = false;
    if (err == hipSuccess)
        err = set_schedule(b, bo, bq, bw);
    if (err != hipSuccess)
        return bhip(b, err, "smc_batch_autotune");
    if (cache_path) {
        if (FILE *f = fopen(cache_path, "a")) {
            fprintf(f, "%s | order=%d per_item=%d wgs_per_cu=%d step_ms=%.4f\n", key.c_str(), bo,
                    bq, bw, best);
            fclose(f);
        }
    }
    return SMC_OK;
}

}  // extern "C"
