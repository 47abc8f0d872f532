"""Batched driver: many independent filters and samplers of uneven sizes
advanced together through the smc_batch_* entry points (each step one
launch of a persistent kernel that works through a dependency-ordered queue
of (problem, phase, tile) items; one step capturable as a HIP graph).  Host
logic only; every numeric step is a HIP kernel behind include/smc.h.

Each problem is the single-problem algorithm of its kind (Section 5.1's
filter, Section 5.2's tempered sampler) with its own seed and problem id in
the Philox counter, so the batch computes exactly what the problems would
compute one by one.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional, Sequence

import numpy as np
import torch

from . import _lib as L
from .sampler import BlockAdapter, ProblemBuffers, mala_scales, rw_scales


@dataclasses.dataclass
class PfSpec:
    """A bootstrap filter of the almost-constant-velocity model over
    observations y[S+1][2] (S steps after the initial weighting)."""
    n: int
    y: np.ndarray
    seed: int = 1
    problem_id: int = 0
    threshold: float = 0.5
    obs_nu: float = 10.0
    fp32_state: bool = False
    scheme: str = "systematic"


@dataclasses.dataclass
class GmmSpec:
    """A tempered mixture sampler over data y with exponents alphas[S+1]
    (alphas[0] = 0) and per-step block scales [S+1][3] (None: the default
    random-walk or MALA scales of each alpha)."""
    n: int
    y: np.ndarray
    K: int
    alphas: np.ndarray
    scales: Optional[np.ndarray] = None
    move: str = "mala"
    sweeps: int = 1
    seed: int = 1
    problem_id: int = 0
    threshold: float = 0.5
    prior: tuple = (0.0, 10.0, 1.0, 1.0, 1.0)
    scheme: str = "systematic"


def gmm_schedule(alphas, scales, move):
    """Rows [alpha_t, s_mu, s_eta, s_z] of the device schedule."""
    alphas = np.asarray(alphas, dtype=np.float64)
    if scales is None:
        f = rw_scales if move == "rw" else mala_scales
        scales = np.array([f(min(max(a, 0.0), 1.0)) for a in alphas])
    scales = np.asarray(scales, dtype=np.float64).reshape(alphas.size, 3)
    return np.ascontiguousarray(np.column_stack([alphas, scales]))


class BatchRunner:
    def __init__(self, specs: Sequence, device="cuda", stream=None):
        self.device = torch.device(device)
        self.specs = list(specs)
        # a stream of its own (default priority): the legacy null stream
        # cannot be captured into a graph
        self.stream = stream if stream is not None else torch.cuda.Stream(self.device)
        self.bufs: List[ProblemBuffers] = []
        self.schedules: List[Optional[torch.Tensor]] = []
        self._base_scales = {}   # mixture sampler index -> its schedule's block scales
        probs = []
        for sp in self.specs:
            bp = L.smc_batch_problem()
            if isinstance(sp, PfSpec):
                y = torch.as_tensor(np.ascontiguousarray(sp.y, dtype=np.float64))
                T = int(y.shape[0])
                cfg = L.make_config(L.SMC_MODEL_CV_TRACK, sp.n, seed=sp.seed,
                                    problem_id=sp.problem_id, threshold=sp.threshold,
                                    obs_nu=sp.obs_nu, n_obs=T, scheme=sp.scheme,
                                    precision=L.SMC_F32_STATE if sp.fp32_state else L.SMC_F64)
                buf = ProblemBuffers(cfg, y, T, self.device)
                self.schedules.append(None)
                bp.schedule = None
                bp.schedule_len = 0
            elif isinstance(sp, GmmSpec):
                y = torch.as_tensor(np.ascontiguousarray(sp.y, dtype=np.float64))
                sched_h = gmm_schedule(sp.alphas, sp.scales, sp.move)
                self._base_scales[len(self.schedules)] = sched_h[:, 1:4].copy()
                sched = torch.as_tensor(sched_h, device=self.device)
                S = int(sched.shape[0]) - 1
                cfg = L.make_config(L.SMC_MODEL_GMM_TEMPERED, sp.n, seed=sp.seed,
                                    problem_id=sp.problem_id, threshold=sp.threshold, K=sp.K,
                                    scheme=sp.scheme,
                                    n_data=int(y.numel()), prior=sp.prior,
                                    move_kind=L.SMC_MOVE_MALA if sp.move == "mala"
                                    else L.SMC_MOVE_RW, sweeps=sp.sweeps)
                buf = ProblemBuffers(cfg, y, S + 1, self.device)
                self.schedules.append(sched)
                bp.schedule = sched.data_ptr()
                bp.schedule_len = S + 1
            else:
                raise TypeError("spec must be PfSpec or GmmSpec")
            bp.cfg = cfg
            bp.buf = buf.view
            self.bufs.append(buf)
            probs.append(bp)
        self._probs = probs
        nbytes = L.smc_batch_table_size(probs)
        self.table = torch.zeros(nbytes + 256, dtype=torch.uint8, device=self.device)
        self._table_ptr = self.table.data_ptr() + (-self.table.data_ptr()) % 256
        torch.cuda.synchronize(self.device)  # buffers were filled on torch's stream
        self.handle = L.smc_batch_create(probs, self._table_ptr, nbytes, self.stream.cuda_stream)
        self.steps_done = 0
        self.particles = sum(int(sp.n) for sp in self.specs)

    def close(self):
        if getattr(self, "handle", None):
            L.smc_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------------- calls
    def autotune(self, repeats: int = 5, cache_path: Optional[str] = None):
        L.smc_batch_autotune(self.handle, repeats, cache_path)

    def waves(self, K: int) -> int:
        return L.smc_batch_waves(self.handle, K)

    def schedule(self) -> dict:
        """The step launch's schedule: queue order, tiles per Metropolis
        item, workgroups (per compute unit and in all), items per step."""
        return L.smc_batch_schedule(self.handle)

    def set_schedule(self, order: int, per_item: int, wgs_per_cu: int):
        L.smc_batch_set_schedule(self.handle, order, per_item, wgs_per_cu)

    def queue(self, order: int = 0, per_item: int = 1) -> np.ndarray:
        """The step's work queue for these problems (host only)."""
        return L.smc_batch_plan_queue(self._probs, order, per_item)

    def init(self):
        L.smc_batch_init(self.handle)
        self.steps_done = 0

    def step(self):
        L.smc_batch_step(self.handle)
        self.steps_done += 1

    def capture(self):
        L.smc_batch_capture(self.handle)

    def replay(self):
        L.smc_batch_replay(self.handle)
        self.steps_done += 1

    def run(self, steps: int, graph: bool = True, latencies: bool = False, adapt: bool = False):
        """init, then `steps` steps (graph replays when graph=True).  With
        latencies=True returns the per-step times in ms (events around
        every step on the batch stream).  With adapt, every mixture
        sampler's block scales follow its acceptance rates (BlockAdapter:
        after each step the host reads the step's acceptance counts and
        rewrites the next step's schedule row)."""
        self.init()
        if graph:
            self.capture()
        go = self.replay if graph else self.step
        if adapt:
            ad = {i: BlockAdapter(self.specs[i].move) for i in self._base_scales}
            for k in range(steps):
                go()
                if k + 1 < steps:
                    acc = self.accept_counts(k + 1)
                    for i, a in ad.items():
                        f = a.update(acc[i], self.specs[i].n)
                        self.set_block_scales(i, k + 2, self._base_scales[i][k + 2] * f)
            return []
        times = []
        if latencies:
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
            with torch.cuda.stream(self.stream):
                ev[0].record(self.stream)
                for k in range(steps):
                    go()
                    ev[k + 1].record(self.stream)
            self.stream.synchronize()
            times = [ev[k].elapsed_time(ev[k + 1]) for k in range(steps)]
        else:
            for _ in range(steps):
                go()
        return times

    def check(self):
        st, bad = L.smc_batch_check(self.handle)
        if st != L.SMC_OK:
            msg = L.load().smc_batch_last_error(self.handle)
            raise L.SmcError(st, "smc_batch_check", (msg.decode() if msg else "") +
                             " (problem %d)" % bad)

    # -------------------------------------------------------------- results
    def state(self, i: int) -> torch.Tensor:
        """State of problem i after the last step (state of step t lives in
        buffer t mod 2)."""
        self.stream.synchronize()
        b = self.bufs[i]
        return b.state_a if self.steps_done % 2 == 0 else b.state_b

    def accept_counts(self, t: int) -> np.ndarray:
        """Accepted proposals per Metropolis block at step t, [problems][3]
        (zeros for tracking filters)."""
        self.stream.synchronize()
        return np.stack([b.history[t, L.SMC_H_ACC0:L.SMC_H_ACC0 + 3].cpu().numpy()
                         for b in self.bufs])

    def schedule_host(self, i: int) -> np.ndarray:
        """Rows [alpha_t, s_mu, s_eta, s_z] mixture sampler i runs with (after
        an adaptive run: the scales it used)."""
        self.stream.synchronize()
        return self.schedules[i].cpu().numpy()

    def set_block_scales(self, i: int, t: int, scales) -> None:
        """Overwrites the block scales of problem i at step t (its schedule
        row), in stream order: steps enqueued later read the new row."""
        row = torch.as_tensor(np.asarray(scales, dtype=np.float64).reshape(3))
        with torch.cuda.stream(self.stream):
            self.schedules[i][t, 1:4].copy_(row)
        self.stream.synchronize()

    def history_host(self, i: int) -> np.ndarray:
        self.stream.synchronize()
        return self.bufs[i].history.cpu().numpy()

    def log_z_path(self, i: int) -> float:
        """Path-sampling estimate of log Z of mixture sampler i (Section 5.2:
        the trapezoid over the schedule of U_t = sum_i W_i l(theta_i))."""
        self.stream.synchronize()
        return float(self.bufs[i].scalars[L.SMC_S_PS_LOGZ].item())

    def log_z(self, i: int) -> float:
        self.stream.synchronize()
        return float(self.bufs[i].scalars[L.SMC_S_LOGZ].item())
