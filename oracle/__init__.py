"""CPU reference for parity testing (test infrastructure, not part of the product).

Plain, slow, float64 numpy implementations of what the SRTM filter and smoother
compute, written from Yaghoobi & Sarkka, "Parallel state estimation for systems
with integrated measurements" (arXiv 2410.00627):

  srtm_oracle  -- the sequential route: slow-rate IMKF (Sec. III-A), dense
                  window fast-rate filter (Sec. III-B) and the proposed
                  sequential SRTM smoother (Sec. III-C).
  scan_form    -- the parallel formulation of Sec. IV: filter and smoother
                  elements, the two associative operators, and folds of them.

Only the tests, the package smoke check and the benchmark's CPU-baseline leg may
import this package. The GPU library never calls it, and the two share no code:
only the seeded input generators (paper_2410_00627_amd.workloads) feed both.
"""
from .srtm_oracle import (  # noqa: F401
    slow_rate_model, batch_model, imkf, fast_filter_window, srtm_filter,
    srtm_smoother, slow_rate_smoother, loglik_grad_fd, imkf_tv, srtm_filter_tv, srtm_smoother_tv,
)
from . import scan_form  # noqa: F401
