"""Plain FP64 CPU oracle for the hp-multigrid preconditioned H(div)-HDG solve.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import or call
this package: only the test-suite, the smoke check and the CPU-baseline leg
of the benchmark use it.  It shares no code with the HIP library.

Layout (sections, equations and algorithms of Fu & Kuang, arXiv 2303.06762):
  quad    data quadrature rule and facet Gauss rule
  mesh    nested red-refined triangulations T_1..T_J (Sec. 3.4.2)
  hdg     element local solver + static condensation of scheme (stWeak),
          condensed operators A, B (stOptForm), direct solve, recovery
  cr      closed-form lowest-order operator (Thm 3.1, k0-stOptForm),
          interpolations Pi^RT / Pi^CR (CR_2RT0, RT0N1_2CR), and an
          independent pressure-robust CR solve (equivCRstWeak)
  mg      vertex-patch block Gauss-Seidel, averaging + harmonic-extension
          transfers (avgOpt, div-transfer, harmonic-ex), MG_h (Alg. 1),
          MG_hp (Alg. 2)
  krylov  flexible CG and AL-Uzawa (stOpEq-ALU)
  solver  end-to-end drivers R1 (direct) and R2 (the method)
Tetrahedral meshes (the same scheme and method in three dimensions):
  mesh3d    nested Kuhn / Bey-refined tetrahedral meshes, faces, edges,
            edge patches and their colouring
  hdg3d     local solver + static condensation on tetrahedra (face basis,
            tangential components in the face frame), R1, uncondensed solve
  cr3d      closed-form lowest-order block on tetrahedra (Thm 3.1)
  mg3d      edge-patch block Gauss-Seidel, averaging + harmonic-extension
            transfers at face centroids, MG_h (Alg. 1), MG_hp (Alg. 2)
  solver3d  end-to-end drivers R1 and R2 on tetrahedra

Parity status of each function is stated in its docstring; every function
is pinned by a CPU test unless it says "parity unpinned".
"""
