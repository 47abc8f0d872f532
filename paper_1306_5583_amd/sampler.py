"""Drivers that own torch device buffers and call the C ABI in the order of
the paper's algorithms.  Host logic only: every numeric step is a HIP kernel
behind include/smc.h.
"""
from __future__ import annotations

import math
from typing import Optional

import numpy as np
import torch

from . import _lib as L


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else t.data_ptr()


class ProblemBuffers:
    """Device buffers of one problem: state ping-pong pair, log-weights,
    ancestors, data, history, workspace and the scalar block, with the
    smc_buffers view the C ABI takes."""

    def __init__(self, cfg, data: torch.Tensor, history_len: int, device):
        self.cfg = cfg
        self.device = torch.device(device)
        rows, eb = L.smc_state_rows(cfg)
        dt = torch.float32 if eb == 4 else torch.float64
        n = int(cfg.n)
        self.n = n
        self.rows = rows
        self.state_a = torch.zeros((rows, n), dtype=dt, device=self.device)
        self.state_b = torch.zeros((rows, n), dtype=dt, device=self.device)
        self.log_weight = torch.zeros(n, dtype=torch.float64, device=self.device)
        self.ancestors = torch.zeros(n, dtype=torch.int32, device=self.device)
        self.data = data.to(self.device, torch.float64).contiguous()
        self.history = torch.zeros((max(history_len, 1), L.SMC_HIST_COLS), dtype=torch.float64,
                                   device=self.device)
        ws = L.smc_workspace_size(cfg)
        self.workspace = torch.zeros(ws + 256, dtype=torch.uint8, device=self.device)
        off = (-self.workspace.data_ptr()) % 256
        self.ws_ptr = self.workspace.data_ptr() + off
        self.ws_bytes = ws
        self.scalars = torch.zeros(L.SMC_SCALARS_LEN, dtype=torch.float64, device=self.device)
        b = L.smc_buffers()
        b.state = self.state_a.data_ptr()
        b.state_alt = self.state_b.data_ptr()
        b.log_weight = self.log_weight.data_ptr()
        b.ancestors = self.ancestors.data_ptr()
        b.data = self.data.data_ptr()
        b.history = self.history.data_ptr()
        b.history_len = history_len
        b.workspace = self.ws_ptr
        b.workspace_bytes = ws
        b.scalars = self.scalars.data_ptr()
        self.view = b


class _Base(ProblemBuffers):
    """A problem's buffers plus its single-problem context."""

    def __init__(self, cfg, data: torch.Tensor, history_len: int, device, stream):
        super().__init__(cfg, data, history_len, device)
        self._bufs = self.view
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.ctx = L.smc_create(cfg, self.view, self.stream.cuda_stream)

    def close(self):
        if getattr(self, "ctx", None):
            L.smc_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def state(self) -> torch.Tensor:
        """The buffer currently holding the state ([rows][n])."""
        p = L.smc_current_state(self.ctx)
        return self.state_a if p == self.state_a.data_ptr() else self.state_b

    def scalars_host(self):
        return L.smc_read_scalars(self.ctx)

    def log_z(self) -> float:
        return self.scalars_host()[L.SMC_S_LOGZ]

    def copy_from(self) -> torch.Tensor:
        """In-place parent layout (Section 4.1, copy(N, copy_from)) of the
        last resample: survivors keep their index, the extra copies fill the
        indices without offspring in ascending order."""
        out = torch.empty(self.n, dtype=torch.int32, device=self.device)
        L.smc_copy_from(self.ctx, out.data_ptr())
        return out

    def check(self):
        L.smc_check(self.ctx)

    def capture(self, body):
        """Records the launches that body() enqueues on this problem into a
        HIP graph without running them, and returns the graph; its replay()
        runs the same launches on the current stream.  body must read nothing
        back to the host.  The capture runs on a side stream (the default
        stream cannot be captured); the problem's own stream is restored
        afterwards."""
        side = torch.cuda.Stream(self.device)
        side.wait_stream(self.stream)
        g = torch.cuda.CUDAGraph()
        L.smc_set_stream(self.ctx, side.cuda_stream)
        try:
            with torch.cuda.graph(g, stream=side):
                body()
        finally:
            L.smc_set_stream(self.ctx, self.stream.cuda_stream)
        self.stream.wait_stream(side)
        return g


class ParticleFilter(_Base):
    """Bootstrap filter of the almost-constant-velocity model (Section 5.1,
    Algorithm 'pf') over observations y[T][2]."""

    def __init__(self, n: int, y, *, seed: int = 1, scheme: str = "systematic",
                 threshold: float = 0.5, fp32_state: bool = False, obs_nu: float = 10.0,
                 obs_scale: float = 0.1, dt: float = 0.1, sd_pos: float = 0.02,
                 sd_vel: float = 0.5, init_sd=(1.0, 1.0, 1.0, 1.0), paper_compatible=False,
                 problem_id: int = 0, device="cuda", stream=None):
        y = torch.as_tensor(np.ascontiguousarray(y, dtype=np.float64))
        T = int(y.shape[0])
        cfg = L.make_config(L.SMC_MODEL_CV_TRACK, n, seed=seed, problem_id=problem_id,
                            scheme=scheme, threshold=threshold,
                            precision=L.SMC_F32_STATE if fp32_state else L.SMC_F64,
                            paper_compatible=paper_compatible, dt=dt, sd_pos=sd_pos,
                            sd_vel=sd_vel, obs_scale=obs_scale, obs_nu=obs_nu, init_sd=init_sd,
                            n_obs=T)
        self.T = T
        super().__init__(cfg, y, T, device, stream)
        self._margs = L.smc_move_args()
        self._margs.fuse_reweight = 1
        self._mon_pending = -1

    def init(self, monitor: bool = True):
        L.smc_init(self.ctx)
        L.smc_ess(self.ctx, 0)
        L.smc_resample(self.ctx, 0)
        self._mon_pending = 0 if monitor else -1

    def step(self, t: int, monitor: bool = True):
        """One iteration: move + weight (fused, also completing the monitor
        of the previous step from the same pass), normalise, resample if
        ESS < threshold N (smc_step: one launch for a one-tile filter).  The
        monitor of step t is carried by the next move; finish() completes
        the last one."""
        m = self._margs
        m.obs_index = t
        m.monitor_step = self._mon_pending
        L.smc_step(self.ctx, t, m)
        self._mon_pending = t if monitor else -1

    def finish(self):
        """Completes a monitor still pending after the last step."""
        if self._mon_pending >= 0:
            L.smc_monitor(self.ctx, self._mon_pending)
            self._mon_pending = -1

    def _steps(self, monitor: bool = True):
        self.init(monitor)
        for t in range(1, self.T):
            self.step(t, monitor)
        self.finish()

    def run(self, monitor: bool = True) -> float:
        self._steps(monitor)
        return self.log_z()

    def capture_run(self, monitor: bool = True):
        """The whole run (prior draws, every step, the last monitor) as one
        HIP graph: every decision of the run is taken on the device (the
        resampling kernels read the normalisation's flag), so one capture
        replays the filter from its prior draws; log_z() and the history
        read the replay's results."""
        return self.capture(lambda: self._steps(monitor))

    def history_host(self) -> np.ndarray:
        torch.cuda.synchronize(self.device)
        return self.history.cpu().numpy()


def rw_scales(alpha: float, base: float = 0.15):
    """Per-block random-walk standard deviations of the paper's sampler
    (Section 5.2.3, the scales chosen each iteration from alpha):
    mean 0.15/a, log-precision 0.15 (1 + sqrt(1/a)), logit 0.2 (1 + sqrt(1/a)),
    a = max(alpha, 0.02).  `base` rescales all three."""
    a = max(alpha, 0.02)
    f = base / 0.15
    return (f * 0.15 / a, f * (1.0 + math.sqrt(1.0 / a)) * 0.15,
            f * (1.0 + math.sqrt(1.0 / a)) * 0.2)


def mala_scales(alpha: float, step: float = 0.05):
    """MALA step sizes per block: `step` times the random-walk multipliers
    normalised by the random-walk base 0.15."""
    return tuple(step * s / 0.15 for s in rw_scales(alpha))


# Acceptance rates the adaptive step sizes steer towards: the asymptotically
# optimal rates of Langevin (Roberts & Rosenthal 1998) and random-walk
# (Roberts, Gelman & Gilks 1997) proposals.
TARGET_ACCEPT = {"mala": 0.574, "rw": 0.234}


class BlockAdapter:
    """Per-block step sizes adapted to the population's acceptance rates:
    the scales of step t + 1 are the base scales of that step times factors
    f_b <- clip(f_b exp(a_b - target), 0.05, 20), a_b the fraction of
    proposals of block b accepted at step t (all particles).  The factors
    depend only on past steps of the run, so the target distributions and
    the estimators are unchanged (an adaptive SMC sampler); the scales used
    are recorded, and a run can be replayed with them."""

    def __init__(self, move: str, blocks: int = 3):
        self.target = TARGET_ACCEPT[move]
        self.f = np.ones(blocks)

    def update(self, accepted, n: int) -> np.ndarray:
        rate = np.asarray(accepted, dtype=np.float64) / float(n)
        self.f = np.clip(self.f * np.exp(rate - self.target), 0.05, 20.0)
        return self.f


class GmmSampler(_Base):
    """Tempered SMC sampler for the Bayesian Gaussian mixture (Section 5.2,
    Algorithm 'gmm'): reweight by the tempering increment, normalise,
    resample when ESS < threshold N, then the three Metropolis blocks."""

    def __init__(self, n: int, y, K: int, T: int, *, seed: int = 1, scheme: str = "systematic",
                 threshold: float = 0.5, move: str = "rw", sweeps: int = 1,
                 prior=(0.0, 10.0, 1.0, 1.0, 1.0), problem_id: int = 0, device="cuda",
                 stream=None):
        y = torch.as_tensor(np.ascontiguousarray(y, dtype=np.float64))
        cfg = L.make_config(L.SMC_MODEL_GMM_TEMPERED, n, seed=seed, problem_id=problem_id,
                            scheme=scheme, threshold=threshold, K=K, n_data=int(y.numel()),
                            prior=prior,
                            move_kind=L.SMC_MOVE_MALA if move == "mala" else L.SMC_MOVE_RW,
                            sweeps=sweeps)
        self.K = K
        self.D = 3 * K - 1
        self.T = T
        self.move = move
        super().__init__(cfg, y, T + 1, device, stream)
        self._margs = L.smc_move_args()
        self._rargs = L.smc_reweight_args()
        self.alpha_prev = 0.0
        self.monitor_out = torch.zeros(self.D + 1, dtype=torch.float64, device=self.device)

    def init(self, monitor: bool = True):
        """Prior draws (alpha = 0).  With `monitor` the initial population is
        normalised and monitored as step 0, the first point of the
        path-sampling estimate."""
        L.smc_init(self.ctx)
        self.alpha_prev = 0.0
        if monitor:
            L.smc_ess(self.ctx, 0)
            L.smc_monitor(self.ctx, 0, self.monitor_out.data_ptr())

    def step(self, t: int, alpha: float, scales=None, monitor: bool = True):
        """Iteration t of Algorithm 'gmm' at tempering exponent alpha."""
        a = min(max(alpha, 0.0), 1.0)
        dalpha = 0.0 if a == 0.0 else a - self.alpha_prev
        self.alpha_prev = a
        if scales is None:
            scales = rw_scales(a) if self.move == "rw" else mala_scales(a)
        self._rargs.dalpha = dalpha
        L.smc_reweight(self.ctx, t, self._rargs)
        L.smc_ess(self.ctx, t)
        L.smc_resample(self.ctx, t)
        m = self._margs
        m.alpha = a
        for b in range(3):
            m.scale[b] = scales[b]
        L.smc_move(self.ctx, t, m)
        if monitor:
            L.smc_monitor(self.ctx, t, self.monitor_out.data_ptr())

    def run(self, alphas, scales=None, monitor: bool = True, adapt: bool = False) -> float:
        """alphas[0..T] with alphas[0] = 0; scales[t] per block or None for
        the default schedule.  With adapt, each step's scales are the base
        scales times the BlockAdapter factors (the host reads the previous
        step's acceptance counts, one synchronisation per step); the scales
        used are kept in self.scales_used[T + 1][3]."""
        self._steps(alphas, scales, monitor, adapt)
        return self.log_z()

    def _steps(self, alphas, scales=None, monitor: bool = True, adapt: bool = False):
        self.init(monitor)
        T = len(alphas) - 1
        base = np.array([(rw_scales if self.move == "rw" else mala_scales)(
            min(max(float(a), 0.0), 1.0)) for a in alphas]) if scales is None \
            else np.asarray(scales, dtype=np.float64).reshape(T + 1, 3)
        used = base.copy()
        ad = BlockAdapter(self.move) if adapt else None
        for t in range(1, T + 1):
            self.step(t, float(alphas[t]), used[t], monitor)
            if ad is not None and t < T:
                acc = self.history_host()[t, L.SMC_H_ACC0:L.SMC_H_ACC0 + 3]
                used[t + 1] = base[t + 1] * ad.update(acc, self.n)
        self.scales_used = used

    def capture_run(self, alphas, scales=None, monitor: bool = True):
        """The whole run at the given block scales as one HIP graph (the
        acceptance-rate adaptation reads the acceptance counts on the host
        between steps, so it cannot be captured): the resampling decisions
        are taken on the device, so one capture replays the sampler from its
        prior draws; log_z(), log_z_path() and the history read the
        replay's results."""
        return self.capture(lambda: self._steps(alphas, scales, monitor, False))

    def log_z_path(self) -> float:
        """Path-sampling estimate of log Z (Section 5.2): the trapezoid over
        the monitored tempering exponents of U_t = sum_i W_i l(theta_i),
        accumulated on the device by each monitor call."""
        return self.scalars_host()[L.SMC_S_PS_LOGZ]

    def history_host(self) -> np.ndarray:
        torch.cuda.synchronize(self.device)
        return self.history.cpu().numpy()
