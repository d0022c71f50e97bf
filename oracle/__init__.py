"""Plain FP64 CPU oracle for the EREM / phi1 heat-transport path.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
baseline leg of the benchmark may import this package.  The product path (the
HIP library and its Python binding) never imports, links or calls it, and it
shares no code with that path: everything here is written directly from the
paper (Tambue, Berre, Nordbotten, "Efficient simulation of geothermal
processes in heterogeneous porous media based on the exponential
Rosenbrock-Euler and Rosenbrock-type methods") and from textbook definitions.

Modules
-------
physics : water laws, TPFA transmissibilities, steady pressure, face fluxes,
          upwind heat operator, G(T) and its Jacobian J (Sec. 2, Sec. 3.1).
phi     : phi1 scalar, dense exponential by Taylor scaling-and-squaring,
          phi1 action by the augmented-matrix exponential (tier A) and by a
          substepped Taylor action (tier B) (Sec. 3.2.2, Sec. 4); phi2 and
          the non-autonomous increment in the same two tiers (Sec. 3.2.3).
erem    : the EREM step and the coupled sequential step (Eq. EERM, Sec. 3.2.2);
          the non-autonomous EREM step (Eq. nEERMg, Sec. 3.2.3).
adjoint : dense reverse-mode sensitivities of the EREM step map.
compressible : the transient pressure ODE (Eq. masscon4, Eq. spaceheat3)
          and its EREM step (Eq. EERM1); the sequential temperature and
          pressure step (Sec. 3.2.2).
rosenbrock : the comparison schemes: ROSM(gamma), ROS2(1), ROS3p (Eq. ROS,
          Eq. ROSMh, Tables ros2 and ros3) and theta-Euler with Newton
          (Eq. temscheme), all with exact sparse solves.

Parity status of each function is stated in its docstring; none is unpinned
unless it says "parity unpinned".
"""
