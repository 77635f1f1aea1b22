"""CPU FP64 oracle for the Burton-Miller collocation BEM (arXiv 2312.00005).

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
bench's CPU-baseline leg may import anything from this package.  The HIP
library never calls it, and it shares no code, tables or constants with the
library: every rule (Gauss nodes, sub-triangle patterns, sphere grids, the
cluster tree) is computed here independently from the paper's prose.

What it computes (each module cites the passage it follows):

* ``geometry``  -- flat-triangle centroid, unit normal and area (Sec. 2.2-2.3).
* ``kernels``   -- G, H = dG/dn_y, H' = dG/dn_x, E = d2G/dn_x dn_y (Sec. 2.1, 2.5).
* ``rules``     -- Gauss-Legendre, Gauss-Jacobi, the conical triangle rule,
                   the six-triangle Duffy rule, the edge rule (Sec. 3.1).
* ``integrals`` -- singular, hypersingular, quasi-singular and regular element
                   integrals (Sec. 3.1.1-3.1.4).
* ``operator``  -- the dense Burton-Miller matrix of Eq. (SystemI) and its
                   right-hand sides (Sec. 2.4-2.5), dense LU solve (Sec. 3.2).
* ``sphere``    -- analytic rigid / impedance sphere series and the modal
                   eigenvalues of the continuous operators.
* ``fmm``       -- the cluster tree (Sec. 3.3.2-3.3.4), the expansion of
                   Eq. (FMMBase) and a multilevel FMM matvec in plain steps.
* ``field``     -- exterior field points from the representation formula.
* ``adjoint``   -- dense adjoint gradient of field-point energy with respect
                   to per-element admittance.

Parity status of each function is listed in its module header.
"""
