"""torch.autograd.Function over the mixture log-likelihood kernel.

GmmLogLik.apply(mu[K,N], eta[K,N], z[K-1,N], y[n]) returns l[N], the
log-likelihood of N independent parameter vectors of the Gaussian mixture of
Section 5.2.1 (eta = log precision, z = log(omega_j / omega_K)).  The forward
pass runs the library's likelihood-and-adjoint kernel once and keeps the
gradient rows; backward scales them by the incoming gradient.  Double
precision on the GPU only.
"""
from __future__ import annotations

import torch

from . import _lib as L


def loglik_and_grad(mu: torch.Tensor, eta: torch.Tensor, z: torch.Tensor, y: torch.Tensor,
                    with_grad: bool = True):
    """(l[N], dl/dphi[3K-1][N]) from one kernel launch (grad None if not asked)."""
    K, n = mu.shape
    for t in (mu, eta, z, y):
        if t.dtype != torch.float64 or not t.is_cuda:
            raise TypeError("GmmLogLik needs float64 CUDA tensors")
    mu = mu.contiguous()
    eta = eta.contiguous()
    z = z.contiguous() if K > 1 else torch.zeros((1, n), dtype=torch.float64, device=mu.device)
    y = y.contiguous()
    ll = torch.empty(n, dtype=torch.float64, device=mu.device)
    grad = torch.empty((3 * K - 1, n), dtype=torch.float64, device=mu.device) if with_grad else None
    stream = torch.cuda.current_stream(mu.device).cuda_stream
    L.smc_gmm_loglik_grad(mu.data_ptr(), eta.data_ptr(), z.data_ptr(), n, K, y.data_ptr(),
                          y.numel(), ll.data_ptr(), None if grad is None else grad.data_ptr(),
                          stream)
    return ll, grad


class GmmLogLik(torch.autograd.Function):
    @staticmethod
    def forward(ctx, mu, eta, z, y):
        need = any(ctx.needs_input_grad[:3])
        ll, grad = loglik_and_grad(mu, eta, z, y, with_grad=need)
        ctx.K = mu.shape[0]
        ctx.save_for_backward(grad if grad is not None else ll)
        ctx.has_grad = grad is not None
        return ll

    @staticmethod
    def backward(ctx, g):
        if not ctx.has_grad:
            return None, None, None, None
        (grad,) = ctx.saved_tensors
        K = ctx.K
        gg = grad * g.unsqueeze(0)
        gz = gg[2 * K:] if K > 1 else None
        return gg[:K], gg[K:2 * K], gz, None


gmm_loglik = GmmLogLik.apply
