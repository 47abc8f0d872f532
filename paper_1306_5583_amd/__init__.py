"""MI355X (gfx950) sequential Monte Carlo sweep: HIP kernels behind the C ABI
of include/smc.h, with a thin ctypes binding and drivers for the paper's two
examples (the tracking particle filter and the tempered Gaussian-mixture
sampler).  Importing the package loads libsmc.so and fails if it is absent.
"""
from . import _lib
from ._lib import SmcError

_lib.load()

from .sampler import (BlockAdapter, GmmSampler, ParticleFilter, mala_scales,  # noqa: E402
                      rw_scales)

from .autograd import GmmLogLik, gmm_loglik  # noqa: E402

from .batch import BatchRunner, GmmSpec, PfSpec  # noqa: E402

__all__ = ["ParticleFilter", "GmmSampler", "GmmLogLik", "gmm_loglik", "rw_scales",
           "mala_scales", "BlockAdapter", "SmcError", "BatchRunner", "PfSpec", "GmmSpec"]
