"""FP64 CPU oracle for the PURIFY SDMM imaging hot path (Carrillo, McEwen & Wiaux).

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously correct NumPy/SciPy
restatement of what the GPU library computes, used to check it.  Only the test suite, the
smoke check and the benchmark's CPU-baseline leg may import it.  It shares no code with the
HIP library (``paper_1406_0359_amd``) and never imports it; the only module both sides use
is the seeded input generator ``paper_1406_0359_amd.synth``, which holds no method
arithmetic.

Modules
-------
kaiser_bessel   Kaiser-Bessel interpolation kernel, its Fourier transform, deapodisation.
nufft           Measurement operator Phi = G F Z S and its adjoint (Section 4, NUFFT).
daubechies      Extremal-phase Daubechies filters by spectral factorisation (Section 2.2).
sara            Periodised multi-level 2D DWT and the SARA dictionary Psi, Psi^dagger.
prox            Proximity operators of eq. (7) for the functions of eq. (6).
sdmm            Operator norm, conjugate gradient and SDMM (Algorithm 1).

Every function is FP64.  Where the paper leaves a choice open, the reading taken is stated
in the function's docstring.
"""
