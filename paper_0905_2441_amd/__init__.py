"""MI355X-native hot path of tempered Gaussian-mixture SMC samplers and
population MCMC (Lee, Yau, Giles, Doucet & Holmes).

Every step runs in the HIP kernels of ``libsmcgpu.so`` behind the C ABI in
``include/smc.h``; this package only marshals torch tensors (device memory) and
streams into those calls. Importing it fails if the library was not built.
"""

from ._lib import SmcError, load  # noqa: F401
from .api import (  # noqa: F401
    Context,
    Gmm,
    fsv_init,
    fsv_step,
    fsv_steps,
    PREC,
    pt_exchange,
    pt_iteration,
    pt_iterations,
    pt_record,
    smc_ess,
    smc_loglik,
    smc_prior_init,
    smc_resample,
    smc_resample_systematic,
    smc_reweight,
    smc_rng_normals,
    smc_rng_words,
    smc_rwmh_move,
    smc_sort_data,
    smc_step,
    smc_steps,
    smc_step_batched,
)
from .samplers import (BatchSampler, FSVFilter, PTSampler, SMCSampler,  # noqa: F401
                       mode_census, traversal_time)

load()
