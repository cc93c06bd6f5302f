"""CPU oracle for the Rosenbrock-Krylov (ROK) hot path.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, float64 statement of
what the GPU library computes, written from the paper (Sarshar et al., "A
numerical investigation of matrix-free implicit time-stepping methods for large
CFD simulations", Computers & Fluids 159, 2017).  It exists to check the GPU
path, and only the test-suite, the smoke check and the CPU-baseline leg of the
benchmark may import it.  It shares no code with the GPU library and imports
nothing from it; the product path never routes through it.

Modules
-------
fv          finite-volume right-hand side f(y) (Sec. 3.2, eq. 11) and its
            Jacobian-vector products (Sec. 2.3, eq. 10 and the exact product)
krylov      modified Arnoldi (Sec. 2.2.2) and the reduced M x M solve
rok         one ROK step (Sec. 2.2.2, eq. 9) and trajectories
rk          explicit Runge-Kutta (Sec. 2.1, eq. 2), used as an independent check,
            and the Lorenz-96 test problem of the Appendix
conditions  order conditions used to derive and check ROK coefficient tables
derive_rok4 the script that derives the ROK4 table from those conditions
adaptive    step-size control by step doubling (Sec. 4.2 reading)
eigen       eigenvalues of the dense Jacobian (the stiffness diagnostic of Sec. 4)
rok_ad      reverse- and forward-mode gradients of ROK trajectories
"""
