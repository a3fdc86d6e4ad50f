"""MI355X-native Generalized Source Method (GSM) solve for 3D periodic
dielectric composites (Shcherbakov & Tishchenko, arXiv 1501.01752).

The compute path lives in the HIP library ``libgsm.so`` built from ``csrc/``;
``paper_1501_01752_amd.gsm`` is a thin ctypes binding with the same entry
points (gsm_plan, gsm_solve, gsm_solve_adjoint, gsm_eff_tensor, ...).
Importing this package does not load the library; ``gsm`` loads it on first
use and raises if it has not been built.
"""
__all__ = ["inputs", "gsm"]
