"""CPU FP64 oracle for cell-wise matrix-free Q_k finite elements.

TEST INFRASTRUCTURE ONLY.  Nothing in the product package imports this
package; only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline``
leg of ``bench.py`` may use it.  It is written from the definitions in the
paper "Coalesced Matrix-Free Geometric Multigrid on Persistent Cell-Wise
Storage" (Wichrowski): it assembles sparse global matrices and dense local
patch matrices and inverts them directly, so that every fast route taken by
the HIP library (sum factorization, DSS cascades, fast diagonalization,
cell-wise transfers, primal-dual CG) can be checked against a plain
definition.  It shares no code with the HIP path.

Modules
-------
basis      1D Gauss-Lobatto Lagrange basis, 1D mass/stiffness, 1D transfers
mesh       structured mesh indexing, the gather operator G, valence
operators  element matrices, CSR assembly of A_CG, cell-wise apply, DSS
patch      vertex patches, dense patch matrices and their inverses
geometry   deformed Q_k geometry, coefficient field, general element matrices
kron       Kronecker form of the Cartesian operator and its exact solver
multigrid  assembled hierarchy, classical smoothers, V-cycle, PCG
sepfit     averaged-geometry separable factors and the separable patch inverse
learned    patch features, best-fit targets, reference MLP forward / manual backward / Adam step
adaptive   refinement tree, level spaces, hanging-node constraints, classical local V-cycle
multiblock multi-block atlas, its global numbering and inter-block DSS
rhs        load vectors of the manufactured solution
c_oracle   the Cartesian cell-wise apply and vertex-patch inverse as plain C (csrc/fe_oracle.c,
           OpenMP over independent outputs), for the CPU baseline at full benchmark sizes
"""
