"""Plain FP64 CPU oracle of the messenger-field Wiener-posterior Gibbs sampler.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and
its Python binding) may import, call or link anything in this package; only
the test suite, the smoke check and the benchmark's CPU-baseline leg use it.
It shares no code with the HIP path: the two meet only through the seeded
input generators (``paper_1402_1763_amd.workloads``) and through the
counter-based random-number contract, which each side implements on its own
from the published Philox4x32-10 definition.

Modules
  philox    Philox4x32-10 counter-based generator, uniform/normal/gamma draws
  shells    |k|-shell binning with exact integer thresholds, mode counts
  sampler   one Gibbs sweep: messenger draw, FFT, signal draw, shell power,
            inverse-gamma P(k) draw, inverse FFT (paper Sec. 3, Algs. 1-2)
  wiener    dense closed-form Wiener filter used to pin the sampler on tiny
            grids (paper Eq. target_wiener_post)

Parity status of each function is stated in its module docstring; every
function that has no independent pin says "parity unpinned".
"""
