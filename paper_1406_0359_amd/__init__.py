"""MI355X-native SDMM radio-interferometric imaging hot path (PURIFY, Carrillo, McEwen & Wiaux).

The measurement operator Phi = G F Z S and its adjoint, the SARA dictionary Psi / Psi^dagger,
the proximal steps and the SDMM solver (Section 3, Algorithm 1) run as hand-written HIP
kernels for gfx950 inside ``libpurify.so``.  This package only marshals arguments:

* :mod:`paper_1406_0359_amd.purify` -- ctypes binding over the C ABI declared in
  ``include/purify.h`` (``purify_phi``, ``purify_phi_adj``, ``purify_psi``,
  ``purify_psi_adj``, ``purify_sdmm_solve``).
* :mod:`paper_1406_0359_amd.synth` -- seeded synthetic inputs (images, uv coverages, noise
  draws).  It holds none of the method's arithmetic.

Importing the package does not load the HIP library; the binding loads it on first use and
raises if it is missing.
"""

__all__ = ["purify", "synth"]
