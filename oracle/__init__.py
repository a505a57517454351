"""CPU FP64 oracle for the MLFMA characteristic-mode hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product library imports, links or
runs this package; only the tests, the smoke check and the benchmark's CPU
baseline leg do.  It shares no code with the GPU library: the only shared
module is ``workloads`` (mesh and random-vector generation, no method
arithmetic).

What it computes, each by its plain definition:

* ``rwg``          RWG basis functions on a triangle mesh (eq. (4)).
* ``quadrature``   the 7-point degree-5 triangle rule used for every
                   Galerkin integral.
* ``potentials``   analytic integrals of 1/R and (rho'-rho)/R over a flat
                   triangle (singularity extraction).
* ``efie``         the Galerkin EFIE impedance matrix Z = R + iX of eq. (5)
                   (dense, or row by row), its k-derivative, and Z x.
* ``planewave``    R by its plane-wave (far-field) representation, a second,
                   independent route to R = Re Z (eqs. (19)-(22)).
* ``modes``        characteristic values by dense QZ of X J = lambda R J
                   (eq. (6)) and the closed-form PEC-sphere values.
* ``translators``  the truncated translator series of eqs. (10), (16), (20)
                   with the truncation rule of eq. (30), and the point test of
                   the numerical-results section.
* ``cmp``          the Calderon multiplicative preconditioner of eqs.
                   (25)-(27): barycentric refinement, Buffa-Christiansen
                   functions, the mixed Gram matrix, Z~ and Z~ G^-1 Z (dense).
* ``sai``          the sparse approximate inverse of the near-field matrix
                   (section IV), column by column by least squares.
                   Parity unpinned: the paper does not define its thresholds.

Sign convention: the public impedance matrix is
Z = ik*eta <f, [I - grad grad'/k^2] exp(-ikR)/R, f>, so that R = Re Z is
positive semidefinite and the characteristic values carry the signs printed in
Table II (electric-energy modes negative).  This is the complex conjugate of
eq. (5) written with eq. (3), times -1.
"""
