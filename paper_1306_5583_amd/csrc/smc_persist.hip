// smc_persist.hip -- the batched step as ONE persistent launch: every
// workgroup takes work items (problem, phase, tile) from a queue in ticket
// order until the step's items are exhausted.  The queue lists the items of
// a step in an order in which every item comes after all the items it
// depends on, so a workgroup waiting for a dependency waits only for items
// already taken by running workgroups: the step makes progress whatever the
// number of co-resident workgroups, and the grid is sized from occupancy
// only to keep the chip full.
//
// Per problem and step (the phases of Algorithm "pf" / Algorithm "gmm"):
//   A  tracking filter: fused move + weight of one 1024-particle tile;
//      mixture sampler: tempering reweight of one 1024-particle tile;
//   F  normalisation (after all its A tiles), plus the tracking filter's
//      monitor of the previous step;
//   R  resampling of one 1024-particle tile (after its F);
//   M  mixture sampler: every Metropolis block and sweep of one or two
//      64-particle tiles (after all its R tiles);
//   U  mixture sampler: the path-sampling integrand and trapezoid (after all
//      its M items).
// Per-problem completion counters only ever grow (a step's targets are
// multiples of the step index), so nothing is reset between steps; the step
// index itself comes from the ticket: a step consumes exactly
// items + workgroups tickets (each workgroup exits on the first ticket past
// the items), so ticket / (items + workgroups) + 1 is the step.
//
// A producer's stores are released (agent scope) before it advances the
// counter, a consumer acquires after seeing the target.  Every wait is
// bounded: past WAIT_TICKS of the constant clock the workgroup raises the
// abort flag and the problem's SMC_DEVERR_TIMEOUT bit, and every later item
// of the launch is skipped, so all workgroups still exit normally.
#include "smc_gmm_impl.hpp"
#include "smc_tiles.hpp"
#include "smc_batch_queue.hpp"

namespace smc {

constexpr uint64_t WAIT_TICKS = 200000000ull;  // 2 s of the 100 MHz constant clock
constexpr int GMM_STASH_MAX = gmm_stash_doubles<BATCH_MAX_K, true>();

__device__ __forceinline__ uint32_t load_relaxed(const uint32_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Publishing an item's results: every wave drains its own stores before
// the workgroup barrier, then thread 0 writes the L2 back (agent-scope
// release), waits for the write-back to complete and only then advances the
// counter.  The waits are explicit: when the releasing wave has no store of
// its own in flight, the compiler emits the write-back and the atomic
// back to back, and a workgroup on another XCD could then see the counter
// before the data reached memory (it read a previous step's tile partials).
__device__ __forceinline__ void drain_memory() { __builtin_amdgcn_s_waitcnt(0); }

__device__ __forceinline__ void release_add(uint32_t *ctr, uint32_t units)
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    drain_memory();
    __hip_atomic_fetch_add(ctr, units, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Thread 0 only: waits until *ctr >= target, then acquires (the cache
// invalidation completes before the workgroup barrier that follows, so the
// other waves' loads cannot overtake it).  False on an abort raised
// elsewhere or on a time-out (which raises it).
__device__ bool wait_at_least(const uint32_t *ctr, uint32_t target, uint32_t *abort_flag,
                              int32_t *err_word)
{
    if (load_relaxed(ctr) < target) {
        const uint64_t t0 = wall_clock64();
        for (;;) {
            __builtin_amdgcn_s_sleep(2);
            if (load_relaxed(ctr) >= target)
                break;
            if (load_relaxed(abort_flag) != 0)
                return false;
            if (wall_clock64() - t0 > WAIT_TICKS) {
                atomicOr(err_word, SMC_DEVERR_TIMEOUT);
                __hip_atomic_fetch_or(abort_flag, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                return false;
            }
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    drain_memory();
    return true;
}

template <int K, bool MALA>
__device__ __attribute__((noinline)) void gmm_item(const Prob &P, int64_t tile0, int count, int32_t t,
                                         double *red, double *stash)
{
    const double *sch = P.sched + 4 * (int64_t)t;
    const double a = fmin(fmax(sch[0], 0.0), 1.0);
    double *cur = (double *)P.state[t & 1];
    const double *prev = (const double *)P.state[(t - 1) & 1];
    const int nb = K == 1 ? 2 : 3;
    for (int q = 0; q < count; ++q) {
        for (int sw = 0; sw < P.sweeps; ++sw)
            for (int b = 0; b < nb; ++b) {
                const bool first = sw == 0 && b == 0;
                __syncthreads();  // LDS and the rows the previous block wrote
                gmm_block_tile<K, MALA>(P, first ? prev : cur, cur, first ? 1 : 0, NWAVES,
                                        tile0 + q, (uint32_t)t, b, sw, a, sch[1 + b], t, red,
                                        stash);
            }
    }
}

__device__ __forceinline__ void gmm_item_dispatch(const Prob &P, int64_t tile0, int count,
                                                  int32_t t, double *red, double *stash)
{
    const bool mala = P.move_kind == SMC_MOVE_MALA;
#define SMC_GMM_ITEM(k)                                                                           \
    case k:                                                                                       \
        if (mala)                                                                                 \
            gmm_item<k, true>(P, tile0, count, t, red, stash);                                    \
        else                                                                                      \
            gmm_item<k, false>(P, tile0, count, t, red, stash);                                   \
        break;
    switch (P.K) {
        SMC_GMM_ITEM(1)
        SMC_GMM_ITEM(2)
        SMC_GMM_ITEM(3)
        SMC_GMM_ITEM(4)
        SMC_GMM_ITEM(5)
        SMC_GMM_ITEM(6)
        SMC_GMM_ITEM(7)
        SMC_GMM_ITEM(8)
    default:
        break;
    }
#undef SMC_GMM_ITEM
}

// Path-sampling integrand of a mixture sampler at step t (Eq. path_import:
// U_t = sum_i W_i l_i over the population after the Metropolis moves) and
// one trapezoid of Eq. path_est, as the single-problem sampler's monitor
// takes them: per 64-particle tile the sums of w_i and w_i l_i (w_i = 1
// after a resample, else exp(lw_i - M)) in the tile's wave, written
// column-major to the problem's monitor partials, then combined over the
// tiles in a fixed order by the workgroup.
__device__ __forceinline__ void gmm_path_monitor(const Prob &P, int32_t t)
{
    const int64_t n = P.n, t64 = ceil_div(n, WAVE);
    const int D = 3 * P.K - 1;
    const double *__restrict__ ll = (const double *)P.state[t & 1] + (int64_t)D * n;
    const bool reset = P.scalars[SMC_S_RESAMPLED] != 0.0;
    const double M = P.scalars[SMC_S_M];
    for (int64_t b = wave_id(); b < t64; b += NWAVES) {
        const int64_t i = b * WAVE + lane_id();
        double w = 0.0, wl = 0.0;
        if (i < n) {
            w = reset ? 1.0 : exp_nonpos_d(P.lw[i] - M);
            if (w != 0.0)
                wl = w * ll[i];
        }
        w = wave_sum(w);
        wl = wave_sum(wl);
        if (lane_id() == 0) {
            P.mon[b] = w;
            P.mon[t64 + b] = wl;
        }
    }
    __syncthreads();
    __shared__ double red[MON_STRIDE * NWAVES];
    __shared__ double col[MON_STRIDE];
    MonDest md;
    md.step = t;
    md.rows = 1;
    md.hist_col = SMC_H_PATH;
    md.hist_ncols = 1;
    md.out = nullptr;
    md.scalars = P.scalars;
    md.alpha = fmin(fmax(P.sched[4 * (int64_t)t], 0.0), 1.0);
    mon_combine<TPB>(P.mon, t64, md, P.hist, P.hist_len, red, col);
}

__global__ __launch_bounds__(TPB, 2) void batch_step_kernel(const Prob *__restrict__ probs,
                                                         const QItem *__restrict__ queue,
                                                         uint32_t nitems, uint32_t per_step,
                                                         uint32_t *__restrict__ sync,
                                                         uint32_t *__restrict__ deps)
{
    __shared__ uint32_t sh_ticket;
    __shared__ int sh_go;
    // one LDS arena for the two largest users, which never run at the same
    // time: a Metropolis item (wave-combine buffer + stash) and a stratified
    // resampling tile (cumulative weights + slot uniforms)
    constexpr int ARENA = GMM_RED_DOUBLES + GMM_STASH_MAX > TILE + RS_UCAP
                              ? GMM_RED_DOUBLES + GMM_STASH_MAX
                              : TILE + RS_UCAP;
    __shared__ double arena[ARENA];
    double *gred = arena, *gstash = arena + GMM_RED_DOUBLES;
    const int tid = threadIdx.x;
    // thread 0's record of the last dependency it saw satisfied in this
    // launch (the step does not change within a launch)
    int ok_prob = -1, ok_kind = -1;
    for (;;) {
        if (tid == 0)
            sh_ticket = atomicAdd(&sync[SYNC_TICKET], 1u);
        __syncthreads();
        const uint32_t tk = sh_ticket;
        const uint32_t k = tk % per_step;
        const int32_t t = (int32_t)(tk / per_step) + 1;
        if (k >= nitems)
            break;
        const QItem it = queue[k];
        const Prob &P = probs[it.prob];
        uint32_t *dc = deps + DEP_STRIDE * (int64_t)it.prob;
        if (tid == 0) {
            bool go = load_relaxed(&sync[SYNC_ABORT]) == 0;
            const uint32_t ntl = (uint32_t)P.ntiles;
            int dkind = -1;
            uint32_t target = 0;
            if (it.kind == IT_FINAL) {
                dkind = DEP_A;
                target = (uint32_t)t * ntl;
            } else if (it.kind == IT_RESAMPLE) {
                dkind = DEP_F;
                target = (uint32_t)t;
            } else if (it.kind == IT_GMM_STEP) {
                dkind = DEP_R;
                target = (uint32_t)t * ntl;
            } else if (it.kind == IT_MONITOR) {
                dkind = DEP_M;
                target = (uint32_t)t * (uint32_t)it.count;
            }
            if (go && dkind >= 0 && !(ok_prob == it.prob && ok_kind == dkind)) {
                go = wait_at_least(dc + dkind, target, &sync[SYNC_ABORT],
                                   &P.counters[CNT_ERR]);
                if (go) {
                    ok_prob = it.prob;
                    ok_kind = dkind;
                }
            }
            sh_go = go;
        }
        __syncthreads();
        if (!sh_go)
            continue;  // aborted: the remaining tickets are drained without work
        int release = -1;
        uint32_t units = 1;  // what the item adds to its counter
        switch (it.kind) {
        case IT_PF_MOVE: {
            const int32_t obs = t < P.n_data ? t : (int32_t)P.n_data - 1;
            const double *y = P.data + 2 * (int64_t)obs;
            if (P.elem_bytes == 4)
                pf_move_tile<float, true, true>(P, (const float *)P.state[(t - 1) & 1],
                                                (float *)P.state[t & 1], it.tile, (uint32_t)t, y,
                                                true, true);
            else
                pf_move_tile<double, true, true>(P, (const double *)P.state[(t - 1) & 1],
                                                 (double *)P.state[t & 1], it.tile, (uint32_t)t,
                                                 y, true, true);
            release = DEP_A;
            break;
        }
        case IT_GMM_REWEIGHT: {
            const double a = fmin(fmax(P.sched[4 * (int64_t)t], 0.0), 1.0);
            const double ap = fmin(fmax(P.sched[4 * (int64_t)(t - 1)], 0.0), 1.0);
            const double dalpha = a == 0.0 ? 0.0 : a - ap;
            const int D = 3 * P.K - 1;
            const double *llrow = (const double *)P.state[(t - 1) & 1] + (int64_t)D * P.n;
            gmm_reweight_tile(P, llrow, it.tile, 1, dalpha);
            release = DEP_A;
            break;
        }
        case IT_FINAL: {
            normalise_block<TPB>(P, t);
            if (P.kind == SMC_MODEL_CV_TRACK && t >= 1) {
                __syncthreads();
                MonDest md;
                md.out = nullptr;
                md.scalars = nullptr;
                md.alpha = 0.0;
                md.rows = FIN_MON_ROWS;
                md.hist_col = SMC_H_MON;
                md.hist_ncols = FIN_MON_ROWS;
                md.step = t - 1;
                monitor_block<TPB>(P, md);
            }
            release = DEP_F;
            break;
        }
        case IT_RESAMPLE:
            if (P.scheme == SMC_RS_STRATIFIED)
                resample_tile<SMC_RS_STRATIFIED>(P, it.tile, (uint32_t)t, 0, nullptr, arena,
                                                 arena + TILE);
            else
                resample_sys_tile(P, it.tile, (uint32_t)t, 0);
            release = P.kind == SMC_MODEL_GMM_TEMPERED ? DEP_R : -1;
            break;
        case IT_GMM_STEP:
            gmm_item_dispatch(P, it.tile, it.count, t, gred, gstash);
            release = DEP_M;
            units = (uint32_t)it.count;
            break;
        case IT_MONITOR:
            gmm_path_monitor(P, t);
            break;
        default:
            break;
        }
        drain_memory();   // this wave's stores of the item have reached L2
        __syncthreads();
        if (release >= 0 && tid == 0)
            release_add(dc + release, units);
    }
}

// The mixture samplers' step-0 monitor (the prior draws, alpha_0): one
// workgroup per problem, filters skipped.
__global__ __launch_bounds__(TPB) void batch_monitor0_kernel(const Prob *__restrict__ probs)
{
    const Prob &P = probs[blockIdx.x];
    if (P.kind == SMC_MODEL_GMM_TEMPERED)
        gmm_path_monitor(P, 0);
}

__global__ void batch_sync_reset_kernel(uint32_t *sync, uint32_t *deps, int64_t ndeps)
{
    for (int64_t k = threadIdx.x; k < ndeps; k += blockDim.x)
        deps[k] = 0u;
    if (threadIdx.x < SYNC_WORDS)
        sync[threadIdx.x] = 0u;
}

// A new schedule changes the tickets a step consumes (items + workgroups);
// the steps already taken keep their count, so the next ticket is rebased
// to steps * new_per_step (no step in flight).
__global__ void batch_ticket_rebase_kernel(uint32_t *sync, uint32_t old_per_step,
                                           uint32_t new_per_step)
{
    if (threadIdx.x == 0)
        sync[SYNC_TICKET] = sync[SYNC_TICKET] / old_per_step * new_per_step;
}

hipError_t launch_batch_ticket_rebase(uint32_t *sync, uint32_t old_per_step,
                                      uint32_t new_per_step, hipStream_t s)
{
    hipLaunchKernelGGL(batch_ticket_rebase_kernel, dim3(1), dim3(WAVE), 0, s, sync, old_per_step,
                       new_per_step);
    return hipGetLastError();
}

int batch_step_blocks_per_cu()
{
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, batch_step_kernel, TPB, 0) !=
        hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return nb;
}

hipError_t launch_batch_step(const Prob *probs, const QItem *queue, uint32_t nitems,
                             uint32_t nwg, uint32_t *sync, uint32_t *deps, hipStream_t s)
{
    hipLaunchKernelGGL(batch_step_kernel, dim3(nwg), dim3(TPB), 0, s, probs, queue, nitems,
                       nitems + nwg, sync, deps);
    return hipGetLastError();
}

hipError_t launch_batch_monitor0(const Prob *probs, int32_t nprob, hipStream_t s)
{
    hipLaunchKernelGGL(batch_monitor0_kernel, dim3((unsigned)nprob), dim3(TPB), 0, s, probs);
    return hipGetLastError();
}

hipError_t launch_batch_sync_reset(uint32_t *sync, uint32_t *deps, int64_t nprob, hipStream_t s)
{
    hipLaunchKernelGGL(batch_sync_reset_kernel, dim3(1), dim3(256), 0, s, sync, deps,
                       (int64_t)DEP_STRIDE * nprob);
    return hipGetLastError();
}

}  // namespace smc
