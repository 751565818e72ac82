"""FP64 CPU oracle for the tempered Gaussian-mixture SMC / population-MCMC hot path.

TEST INFRASTRUCTURE ONLY. This package is the plain, slow and obviously
correct statement of what the GPU path computes. It is imported only by
``tests/``, by ``__graft_entry__.smoke()`` (to check one GPU invocation) and by
the ``cpu_baseline`` leg of ``bench.py``. The product path (the HIP library
and its Python binding) never imports, calls or links anything here, and this
package imports nothing from the product package.

Modules
-------
philox    Philox4x32-10 counter-based generator (Salmon, Moraes, Dror & Shaw,
          SC'11), exact u32 -> uniform maps and Box-Muller normals.
gmm       Mixture log-likelihood (Mixture Modelling section) and log-priors.
smc       SMC-sampler and population-MCMC steps: RW-MH move, incremental
          reweight, log-sum-exp normalisation, ESS, systematic resampling,
          exchange move, whole-run drivers.
evidence  Exact and quadrature log-evidence used to pin the sampler.

Everything is FP64 unless stated. Pins (tests that tie each function to
something other than itself) live in ``tests/test_oracle_*.py``; the only
unpinned result is the FP32 sample path after the first flipped accept
decision, which is compared statistically.
"""

from . import philox, gmm, smc, evidence  # noqa: F401
