"""FP64 CPU oracle for the acoustic RTM hot path.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package; the product library never does.  It shares no code with the HIP path.
"""
from .rtm import (  # noqa: F401
    fd_coefficients,
    stability_limit,
    stable_dt,
    sponge_profile,
    ricker,
    kappa_field,
    injection_weight,
    laplacian,
    step,
    adjoint_step,
    forward,
    migrate,
    adjoint_sources,
    gradient_kappa,
    misfit,
    pack_faces,
    snapshot_encode,
    snapshot_decode,
    bf16_rne,
    bf16_to_f32,
    rel_l2,
)
