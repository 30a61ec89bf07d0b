"""FP64 CPU oracle for the He-Luo MRT lattice Boltzmann step and its strain-rate formulas.

TEST INFRASTRUCTURE ONLY. Nothing in the product path (the HIP library and its Python
binding) may import, call or link anything in this package. Only the test suite, the smoke
check and the CPU-baseline leg of the benchmark use it.

The oracle is written from the paper (Zhang, Huang, Wang, Shi, "The computation of strain
rate tensor in multiple-relaxation-time lattice Boltzmann model", arXiv 1704.07559), plain
and dense: the 19x19 transformation matrix is applied as a dense matrix product, the
strain by the Chai formula is the literal T^-1 diag(s) T contraction, streaming is
``np.roll``. It shares no code, tables or constants with the GPU path; each side holds its
own transcription of the paper.

Modules
-------
d3q19        the D3Q19 model (Section 2), the Yu formula (Eq. LuoS), the Chai formula
             (Eq. ChaiS), the viscosity models, Guo forcing, bounce-back walls, the step
d2q9         the D2Q9 variant (Section 5.3/5.4 generality; lattice from outside the paper)
d3q15        the D3Q15 variant (Section 5.3/5.4 generality; basis from outside the paper)
adjoint      discrete adjoint of the D3Q19 step and of the strain-squared loss (constant
             viscosity)
adjoint_visc the same for strain-dependent viscosities (lagged Smagorinsky and power law,
             implicit Smagorinsky)
storage      round-to-nearest-even into binary16 / bfloat16 (the reduced-precision storage)
closed_forms exact Navier-Stokes solutions used as expected values (Taylor-Green,
             power-law Poiseuille, start-up Poiseuille series)
naive        a per-node pure-Python loop of the step for brute-force checks on tiny grids
naive_other  the same per-node loop for D2Q9 and D3Q15 (closed-form Yu-type formulas)
"""
