"""FP64 CPU oracle for the discrete-DtN absorbing boundary time stepper.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, deliberately
unoptimised restatement of Wu & Li, "Absorbing boundary conditions for the
time-dependent Schroedinger-type equations in R^3" (arXiv:1908.02456), written
in NumPy/SciPy at float64.  It exists to check the HIP implementation and is
imported only by the test-suite, the package's smoke check and the benchmark's
CPU-baseline leg.  It shares no code with the HIP path; the only common module
is the seeded input generator (``paper_1908_02456_amd.workloads``), which holds
none of the method's arithmetic.

Modules
-------
stencil     finite-difference weights, the box Hamiltonian H_{I,I} and the
            boundary sets Gamma / Sigma with their coupling H_{Gamma,Sigma}
            (Sec. 2).
greens      lattice Green's functions: 3D by the Brillouin-zone Fourier
            integral (App. D), 1D characteristic roots (App. B) and the
            half-line DtN symbol of one face.
dtn         the DtN map K(s) by the discrete boundary-element formula (App. A),
            its zeroth/first-order rational approximations (Sec. 3) in the
            paper's dense box form, and the per-face (half-space) form.
integrate   the 4th-order Taylor propagator (Sec. 4) applied to the dynamics
            with the zeroth/first-order conditions, diagnostics and the
            density-dependent mean field.
adjoint     the exact discrete adjoint of the stepping map.

Every function names the passage it follows.  Where the paper is garbled or
silent the reading taken is stated in the docstring.
"""
