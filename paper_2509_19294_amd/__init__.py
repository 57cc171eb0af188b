"""MI355X-native direct-summation N-body: softened all-pairs accelerations and
potentials, kick-drift-kick leapfrog and diagnostics, behind the C ABI of
``libnbody.so`` (hand-written HIP kernels for gfx950).

``paper_2509_19294_amd.nbody`` is the thin binding over that library; the
library is loaded on first use, and every call fails loudly if it is missing.
``paper_2509_19294_amd.ics`` draws seeded synthetic initial conditions.
"""
__all__ = ["ics", "nbody"]
