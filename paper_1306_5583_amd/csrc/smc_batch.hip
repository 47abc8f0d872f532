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

namespace smc {

struct KGroup {
    int K = 0;
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
    hipStream_t stream = nullptr;
    char *table = nullptr;
    Prob *dprobs = nullptr;
    int2 *map_pf = nullptr, *map_gmm = nullptr, *map_all = nullptr;
    int64_t pf_tiles = 0, gmm_tiles = 0, all_tiles = 0;
    std::vector<KGroup> groups;
    int32_t *step = nullptr;
    bool mala = false;
    int sweeps = 1;
    bool initialised = false;
    int host_step = 0;
    int max_steps = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::string last_error;
};

namespace {

struct Plan {
    size_t probs = 0, map_pf = 0, map_gmm = 0, map_all = 0, step = 0, total = 0;
    std::vector<size_t> map64;
    std::vector<int> ks;
    std::vector<int64_t> tiles64;
    int64_t pf_tiles = 0, gmm_tiles = 0;
};

size_t al(size_t v) { return (v + 255) & ~size_t(255); }

Plan plan(const smc_batch_problem *probs, int32_t np)
{
    Plan pl;
    std::map<int, int64_t> t64;
    for (int32_t i = 0; i < np; ++i) {
        const smc_config &c = probs[i].cfg;
        const int64_t nt = ceil_div(c.n, TILE);
        if (c.model == SMC_MODEL_CV_TRACK)
            pl.pf_tiles += nt;
        else {
            pl.gmm_tiles += nt;
            t64[c.K] += ceil_div(c.n, WAVE);
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
        pl.ks.push_back(kv.first);
        pl.tiles64.push_back(kv.second);
        pl.map64.push_back(off);
        off = al(off + sizeof(int2) * (size_t)kv.second);
    }
    pl.step = off;
    off = al(off + 256);
    pl.total = off;
    return pl;
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

hipError_t enqueue_step(smc_batch *b)
{
    hipStream_t s = b->stream;
    hipError_t e = launch_set_step(b->step, 1, 1, s);
    if (e == hipSuccess)
        e = launch_pf_move_batch(b->dprobs, b->map_pf, b->pf_tiles, b->step, s);
    if (e == hipSuccess)
        e = launch_gmm_reweight_batch(b->dprobs, b->map_gmm, b->gmm_tiles, b->step, s);
    if (e == hipSuccess)
        e = launch_finalize_batch(b->dprobs, (int32_t)b->P.size(), b->step, s);
    if (e == hipSuccess)
        e = launch_resample_batch(b->dprobs, b->map_all, b->all_tiles, b->step, s);
    for (int sw = 0; sw < b->sweeps && e == hipSuccess; ++sw)
        for (int blk = 0; blk < 3 && e == hipSuccess; ++blk)
            for (const KGroup &g : b->groups) {
                if (blk == 2 && g.K == 1)
                    continue;
                const int first = (sw == 0 && blk == 0) ? 1 : 0;
                e = launch_gmm_block_batch(b->dprobs, g.map64, g.tiles64, g.K, b->step, g.W, blk,
                                           sw, first, b->mala, s);
                if (e != hipSuccess)
                    break;
            }
    return e;
}

std::string cache_key(const KGroup &g)
{
    int dev = 0;
    hipDeviceProp_t prop;
    (void)hipGetDevice(&dev);
    (void)hipGetDeviceProperties(&prop, dev);
    char buf[256];
    snprintf(buf, sizeof(buf), "%s K=%d log2n=%d log2nd=%d", prop.gcnArchName, g.K,
             (int)ceil(log2((double)std::max<int64_t>(g.sum_n, 1))),
             (int)ceil(log2((double)std::max<int64_t>(g.max_nd, 1))));
    std::string k(buf);
    std::replace(k.begin(), k.end(), ':', '_');
    return k;
}

}  // namespace

extern "C" {

smc_status smc_batch_table_size(const smc_batch_problem *probs, int32_t nprob, size_t *bytes)
{
    if (!probs || nprob < 1 || !bytes)
        return SMC_ERR_INVALID_ARG;
    std::string err;
    for (int32_t i = 0; i < nprob; ++i) {
        const smc_status s = validate_config(&probs[i].cfg, err);
        if (s != SMC_OK)
            return s;
    }
    *bytes = plan(probs, nprob).total;
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
    int gmm_kind = -1, gmm_sweeps = -1;
    for (int32_t i = 0; i < nprob; ++i) {
        const smc_batch_problem &q = probs[i];
        smc_status s = validate_config(&q.cfg, err);
        if (s != SMC_OK)
            return s;
        s = validate_buffers(q.cfg, &q.buf, err);
        if (s != SMC_OK)
            return s;
        if (q.cfg.scheme != SMC_RS_SYSTEMATIC)
            return SMC_ERR_UNSUPPORTED;
        if (q.cfg.model == SMC_MODEL_CV_TRACK && q.cfg.precision != SMC_F64)
            return SMC_ERR_UNSUPPORTED;
        if (q.cfg.model == SMC_MODEL_GMM_TEMPERED) {
            if (!q.schedule || q.schedule_len < 2)
                return SMC_ERR_INVALID_ARG;
            const int sw = q.cfg.sweeps > 0 ? q.cfg.sweeps : 1;
            if (gmm_kind >= 0 && (gmm_kind != q.cfg.move_kind || gmm_sweeps != sw))
                return SMC_ERR_UNSUPPORTED;
            gmm_kind = q.cfg.move_kind;
            gmm_sweeps = sw;
        }
    }
    const Plan pl = plan(probs, nprob);
    if (table_bytes < pl.total)
        return SMC_ERR_INVALID_ARG;
    smc_status s = device_ok(err);
    if (s != SMC_OK)
        return s;
    smc_batch *b = new (std::nothrow) smc_batch();
    if (!b)
        return SMC_ERR_DEVICE;
    b->probs.assign(probs, probs + nprob);
    b->stream = static_cast<hipStream_t>(hip_stream);
    b->table = static_cast<char *>(table);
    b->dprobs = reinterpret_cast<Prob *>(b->table + pl.probs);
    b->map_pf = reinterpret_cast<int2 *>(b->table + pl.map_pf);
    b->map_gmm = reinterpret_cast<int2 *>(b->table + pl.map_gmm);
    b->map_all = reinterpret_cast<int2 *>(b->table + pl.map_all);
    b->step = reinterpret_cast<int32_t *>(b->table + pl.step);
    b->pf_tiles = pl.pf_tiles;
    b->gmm_tiles = pl.gmm_tiles;
    b->all_tiles = pl.pf_tiles + pl.gmm_tiles;
    b->mala = gmm_kind == SMC_MOVE_MALA;
    b->sweeps = gmm_sweeps > 0 ? gmm_sweeps : 1;
    // descriptors and maps, staged on the host
    std::vector<int2> mpf, mgmm, mall;
    std::map<int, std::vector<int2>> m64;
    std::map<int, KGroup> grp;
    b->max_steps = 1 << 30;
    for (int32_t i = 0; i < nprob; ++i) {
        const smc_batch_problem &q = probs[i];
        const Workspace ws = plan_workspace(q.cfg);
        Prob P = prob_from(q.cfg, q.buf, ws, q.buf.state, q.buf.state_alt);
        P.sched = q.schedule;
        b->P.push_back(P);
        const int64_t nt = ceil_div(q.cfg.n, TILE);
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
            const int64_t t64 = ceil_div(q.cfg.n, WAVE);
            auto &v = m64[q.cfg.K];
            for (int64_t t = 0; t < t64; ++t)
                v.push_back(make_int2(i, (int)t));
            KGroup &g = grp[q.cfg.K];
            g.K = q.cfg.K;
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
    for (size_t k = 0; k < pl.ks.size() && e == hipSuccess; ++k) {
        KGroup g = grp[pl.ks[k]];
        g.map64 = reinterpret_cast<int2 *>(b->table + pl.map64[k]);
        g.tiles64 = pl.tiles64[k];
        g.W = gmm_waves(g.sum_n, g.max_nd);
        const auto &v = m64[pl.ks[k]];
        e = hipMemcpy(g.map64, v.data(), sizeof(int2) * v.size(), hipMemcpyHostToDevice);
        b->groups.push_back(g);
    }
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
            e = launch_gmm_init_batch(b->dprobs, g.map64, g.tiles64, g.K, g.W, b->mala, s);
    if (e == hipSuccess)
        e = launch_const_partials_batch(b->dprobs, b->map_gmm, b->gmm_tiles, s);
    if (e == hipSuccess)
        e = launch_finalize_batch(b->dprobs, np, b->step, s);
    if (e == hipSuccess)
        e = launch_resample_batch(b->dprobs, b->map_all, b->all_tiles, b->step, s);
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

smc_status smc_batch_autotune(smc_batch *b, int32_t repeats, const char *cache_path)
{
    if (!b || repeats < 1)
        return SMC_ERR_INVALID_ARG;
    std::map<std::string, int> cache;
    if (cache_path) {
        if (FILE *f = fopen(cache_path, "r")) {
            char line[512];
            while (fgets(line, sizeof(line), f)) {
                char *eq = strrchr(line, '=');
                char *sp = strstr(line, " W=");
                if (!eq || !sp)
                    continue;
                *sp = 0;
                cache[line] = atoi(eq + 1);
            }
            fclose(f);
        }
    }
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return bfail(b, SMC_ERR_DEVICE, "hipEventCreate");
    std::vector<std::string> fresh;
    hipError_t err = hipSuccess;
    for (KGroup &g : b->groups) {
        const std::string key = cache_key(g);
        auto it = cache.find(key);
        if (it != cache.end() && (it->second == 1 || it->second == 2 || it->second == 4 ||
                                  it->second == 8)) {
            g.W = it->second;
            continue;
        }
        float best = 1e30f;
        int bestW = g.W;
        for (int W = 1; W <= 8 && err == hipSuccess; W *= 2) {
            std::vector<float> ms;
            for (int r = 0; r <= repeats && err == hipSuccess; ++r) {
                err = hipEventRecord(e0, b->stream);
                if (err == hipSuccess)
                    err = launch_gmm_init_batch(b->dprobs, g.map64, g.tiles64, g.K, W, b->mala,
                                                b->stream);
                if (err == hipSuccess)
                    err = hipEventRecord(e1, b->stream);
                if (err == hipSuccess)
                    err = hipEventSynchronize(e1);
                float t = 0.f;
                if (err == hipSuccess)
                    err = hipEventElapsedTime(&t, e0, e1);
                if (r > 0)  // the first launch warms up
                    ms.push_back(t);
            }
            if (err != hipSuccess)
                break;
            std::sort(ms.begin(), ms.end());
            const float med = ms[ms.size() / 2];
            if (med < best) {
                best = med;
                bestW = W;
            }
        }
        g.W = bestW;
        fresh.push_back(key + " W=" + std::to_string(bestW));
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    b->initialised = false;
    if (b->exec) {  // the captured graph used the old tile shapes
        (void)hipGraphExecDestroy(b->exec);
        b->exec = nullptr;
    }
    if (err != hipSuccess)
        return bhip(b, err, "smc_batch_autotune");
    if (cache_path && !fresh.empty()) {
        if (FILE *f = fopen(cache_path, "a")) {
            for (const std::string &l : fresh)
                fprintf(f, "%s\n", l.c_str());
            fclose(f);
        }
    }
    return SMC_OK;
}

}  // extern "C"
