"""FP64 CPU oracle for the PM-FEM effective field (arXiv 2409.13958).

TEST INFRASTRUCTURE ONLY. Nothing in the product path may import this
package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it. It shares no code with the
library under ``paper_2409_13958_amd/csrc`` (no kernels, headers, helpers,
tables or constants); the two only meet in the seeded input generators.

The oracle is plain, slow and written to be read against the paper:

* ``periodic``  -- PBC pairs, union-find LCA, unknown numbering (Sec. 2.2),
  protruding-cell remap (Sec. 3.2.2, Eq. shift_hms).
* ``fem``       -- P1 tetrahedral operators: exchange Laplacian (Sec. 3.1,
  Eqs. hex, lapl, lapl_1, lapl_2), nodal charges and gradient (Eq. hms_d).
* ``pgf``       -- periodic Green's functions for 1D/2D/3D periodicity
  (Eq. 2 with k0 = 0), Ewald-regularised, plus brute-force lattice sums.
* ``elem``      -- element-exact near-field potentials by quadrature
  (the correction matrix of Eq. hms_d2b).
* ``aim``       -- the four-step box-AIM (Sec. 3.2.2: project, FFT-convolve
  with the grid PGF, interpolate, precorrect with G0 only).
* ``model``     -- the assembled H_eff (Eq. heff), energies and RK4 LLG (Eq. llg).

Readings of points where the paper is silent or garbled (charge signs,
units, grid spacing, self term, precorrection form) are listed in the
module docstrings where they are used.
"""
