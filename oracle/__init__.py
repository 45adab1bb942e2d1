"""CPU oracle for the generalized MBE-FCI hot path -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import or execute anything in this package.  The product
path (the HIP library and its Python binding) never touches it, and this
package imports nothing from the product package.

What it computes, in the paper's order and notation (arXiv:1910.03527):

* ``fci``  -- f(T): the lowest eigenvalue of the full-space Hamiltonian
  restricted to the determinant space of the CASCI in R u T (Eq. 1 calls these
  the constituent CASCI calculations), built element by element with the
  Slater-Condon rules (``sc.c``) over *full-space* determinants, frozen
  doubly occupied orbitals and deleted virtuals included explicitly.  Dense
  ``eigh`` for small spaces, SciPy Lanczos (``eigsh``) above.
* ``mbe``  -- the increments of Eq. 2 by the recursion exactly as written
  (sum over all proper sub-tuples), the order sums E^(n) and the total of
  Eq. 1 (Eq. 3 for an empty reference space), plus the Moebius closed form as
  an independent second evaluation.
* ``screen`` -- the screened order-by-order expansion: the thresholds of
  Eq. 4, child spawning from the computed parent tuples, and Eq. 2 over the
  computed sub-tuples.
* ``rdm``  -- full-space spin-summed 1- and 2-RDMs by applying every operator
  string a+ a+ a a to every determinant; gradients dE/dh and dE/d(pq|rs) of
  f(T) and, through the adjoint of the Eq. 2 recursion, of E_MBE; central
  finite differences.

Where the paper is silent the oracle takes these readings: eps_T = f(T) - E_ref
(Eq. 1 adds E_ref separately); a CASCI in the active set A = R u T holds
2|O n A| electrons with O \\ A frozen doubly occupied and every other orbital
deleted; the solved state is the lowest eigenvalue of the S_z = 0 sector.

Parity status: every function here is pinned by ``tests/test_oracle_*.py``
against closed forms, invariants, brute force or dense diagonalisation.
"""
