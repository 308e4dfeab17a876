"""FP64 CPU oracle for the pole-shifted TEM solves.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call,
link or execute anything in this package: only the test-suite, the smoke
check and the CPU-baseline leg of the benchmark use it.  It shares no code
with the GPU library; the two meet only in the seeded inputs of
``tem_inputs``.

Every function is a plain, slow, obviously correct transcription of what
the paper computes:

* ``fem``       edge-element operators K and M on a uniform hex mesh
                (section "Spatial discretization", semi-discrete system);
* ``ordering``  nested-dissection ordering and supernodal symbolic
                structure of the shifted matrices (the structure one
                factorisation of each shifted matrix needs, shared by all
                poles);
* ``tet``       the same operators with lowest-order edge elements on
                tetrahedra, and the RT0 smoothness operator with a lumped
                (diagonal) mass (section "Regularization");
* ``tem``       shifted solves g_i = (K - xi_i M)^{-1} f (Algorithm 1),
                time assembly u(t_j) = 2 Re sum_i alpha_i^[j] g_i, data
                d_j = Q u(t_j), Jv and J^T w (section "Jacobian
                computation"), LSQR on the augmented Gauss-Newton system
                (section "Optimization").

Parity status of each function is stated in its module header.
"""
