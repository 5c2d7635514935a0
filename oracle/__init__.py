"""Plain, slow FP64 CPU oracle for the FFT-accelerated VIE matrix-vector product.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or call anything in this package.
It shares no code with the HIP library (``paper_2105_08627_amd``) and never
imports it; the two meet only through the seeded input generators in
``workloads/``, which hold none of the method's arithmetic.

Modules
-------
green     voxel-pair Green integrals (Sec. II.A eq. 1 kernel, App. A eqs. 19-21,
          App. B eqs. 24-27) by tensor Gauss-Legendre quadrature of the exact
          tent-weighted 3D form, with Duffy pyramids at the singular corner.
operator  two-fluid material (eq. 3, eqs. 22-23), the Galerkin blocks of eq. 8,
          dense O(N^2) matvec, circulant embedding and FFT convolution (eq. 9).
tucker    Algorithm 1 (Tucker-SVD / HOSVD) and the mode products of eqs. 10-11.

Every function cites the passage of the paper it follows.  Where the paper is
silent the reading taken is stated in the docstring.  Functions with no
independent pin say "parity unpinned" in their docstring.
"""
