"""Plain FP64 CPU oracle of the Generalized Source Method (GSM) solve.

TEST INFRASTRUCTURE ONLY.  Nothing in the product library imports, links or
calls this package; only the test-suite, the smoke check and the CPU-baseline
leg of the benchmark do.  It is slow on purpose: every function writes the
method out from its definition in the paper (Shcherbakov & Tishchenko,
"3D periodic dielectric composite homogenization based on the Generalized
Source Method", arXiv 1501.01752), using NumPy/SciPy library primitives
(dense LU, FFT, GMRES) as single steps.

Modules
-------
gsm      Eq.(4) of the paper: Fourier images of a voxel body, the per-harmonic
         dyadic Green tensor, the dense truncated system (route O1, LU), the
         same operator applied by FFT (route O2, GMRES), the field-averaged
         effective tensor and its Schur-complement form, the 1D stack reduction.
grad     dense forward-mode derivative of the effective tensor with respect to
         voxel permittivities (tangent route) and central finite differences.
"""
