"""FP64 CPU oracle for adaptive multigrid on the Shamir domain-wall operator.

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow, obviously correct
reference that the GPU library is checked against.  Only the test suite, the
smoke check of the entry module and the CPU-baseline leg of the benchmark may
import it; the product library never does, and it shares no code with it.

Contents, each following the paper (Cohen, Brower, Clark, Osborn, "Multigrid
Algorithms for Domain-Wall Fermions", Lattice 2011):

* ``dwf``       -- the 5D Shamir operator D and its adjoint (Sec. 2, last
                   paragraph: fifth dimension; Sec. 4: one site plus ten unit
                   neighbours).  The paper never writes D; the standard Shamir
                   form used here is a stated reading.
* ``transfer``  -- chirality-split, block-orthonormalised near-null basis,
                   restrictor R and prolongator P with R P = 1 (Sec. 1, R/P
                   definition; Sec. 2, blocks spanning the fifth dimension).
* ``coarse``    -- Galerkin coarse operator D_c = R D P as a 9-point stencil of
                   dense blocks (Sec. 2, V-cycle step 3; Sec. 4, coarsening of
                   the unsquared operator).
* ``solvers``   -- minimal-residual smoother, GCR / flexible GCR, CG on the
                   normal equations, the five-step V-cycle (Sec. 2 and Sec. 3).
* ``setup``     -- adaptive near-null vector search (Sec. 2, adaptive setup).
* ``squared``   -- the multigrid on the squared operator D^+D that the paper
                   ran (Sec. 3 first paragraph, Sec. 4): basis of D^+D's
                   near-null vectors, A_c = P^+ D^+D P (33-offset stencil),
                   MR smoothing on D^+D, CG on A_c.
* ``threelevel`` -- a third level under the squared two-level method: near-null
                   vectors of A_c, their block basis, A_cc = R2 A_c P2, the
                   level-2 cycle, V- and W-cycles (Sec. 2, recursion).
* ``lowmodes``  -- lowest eigenpairs of D^+D from a dense eigensolver and the
                   fraction |P R e|^2 / |e|^2 of a field in the coarse space
                   (Sec. 2, Fig. 1 right).
* ``u1_2d``     -- the paper's 2D U(1) test problem (Sec. 3, Fig. 2): the 2D
                   domain-wall operator, its chirality-split block basis and
                   transfer, A_c = P^+ D^+D P as a 9-offset stencil, the
                   squared V-cycle and setup.
* ``nullnet``   -- forward/backward of the gauge-covariant proposal network.

Every function works in complex128.
"""
