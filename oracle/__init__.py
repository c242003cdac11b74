"""Plain FP64 CPU oracle of the digital shearlet filter-bank transform.

TEST INFRASTRUCTURE ONLY. Nothing in the product path may import, call or
execute anything in this package: only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` use it. It shares no code,
tables or constants with the HIP library; the two meet only through the
seeded generators in ``synth``.

Contents
  filters    -- the shearlet system (Section 2.1 construction, Section 3.4.1
                defaults): low-pass design, a-trous chains, fan filter, digitally
                sheared wedges, band-passes, low-pass, dual-frame weight, RMS.
  transform  -- Fourier shifts (Section 3.3), Algorithm 1 (decomposition),
                Algorithm 2 (reconstruction), the adjoint, and shift-free and
                brute-force forms used to pin them.
  apps       -- hard thresholding, PSNR, denoising and inpainting (Section 4.2,
                4.3, Algorithm 3).

Parity status: the filter values the paper used come from MATLAB design
commands whose outputs are not printed, so agreement with those exact values
is "parity unpinned"; every function here is pinned instead against
closed-form identities, a spatial re-construction and brute force in
``tests/test_oracle_*.py``.
"""
