"""Plain FP64 CPU oracle for the fast-multipole BEM operator (TEST INFRASTRUCTURE).

Only `tests/`, the smoke check in `__graft_entry__.py` and the `cpu_baseline`
leg of `bench.py` may import, call or build anything in this package.  The
GPU library and its Python binding never do; they share no code with it.

Contents (each module cites the passage of the paper it follows):
  kernel.py       g and grad'g (eq. 2.4)
  direct.py       direct O(N^2) Nystrom sum of one wavenumber's operator (eqs. 2.5, 2.8, 2.12)
  direct_sum.c    the same sum as a plain C / OpenMP loop (native.py builds and loads it)
  corrections.py  self-triangle integrals (Appendix B) and their node blocks
  tree.py         reference octree, Morton order and box lists (Sec. 2.2, Appendix C)
  bem.py          the 6N system for one scatterer and the block preconditioner (eqs. 2.6-2.13, 3.1-3.2)
  gmres.py        right-preconditioned flexible GMRES (Sec. 3.1)
  mie.py          Mie series for a sphere (the external check of Sec. 3.2)
  shape.py        shape derivatives of the point sum; the two forms of C_sca (eq. 4.2)

Every function is pinned by tests/test_oracle_*.py against closed forms,
brute force, identities or textbook results.
"""
