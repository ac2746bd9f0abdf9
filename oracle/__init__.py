"""CPU FP64 oracle for GSE-TDVP1 -- TEST INFRASTRUCTURE ONLY.

A plain, slow, dense (no symmetry) NumPy/SciPy implementation of what the GPU
path computes, written from the paper (Yang & White, "Time dependent
variational principle with ancillary Krylov subspace"):

* ``ed``         exact diagonalisation from term lists (independent of MPOs)
* ``mpo``        finite-state-automaton MPO for c0*1 + c1*H (section I.C, step 1)
* ``mps``        MPS utilities, canonical forms (eq. (1))
* ``tdvp``       environments, one-site/zero-site effective Hamiltonians,
                 Lanczos exponential, one-site TDVP sweep (section I.C, step 3)
* ``krylov``     global Krylov vectors (1 - i tau H)^l |psi> by the density
                 matrix MPO application (eq. (10), section I.B)
* ``extension``  state-averaged basis extension (eqs. (5)-(7), section I.A)
* ``gse``        one GSE-TDVP1 time step (section I.C)
* ``observables`` energy, <S^z_i>, fidelity, OAT moments (eqs. (13)-(15))

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product path (the HIP library and
its Python binding) never imports, calls or links anything in here, and this
package imports nothing from the product path.

Every floating-point computation is complex128 / float64.
"""
