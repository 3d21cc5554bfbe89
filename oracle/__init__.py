"""Plain FP64 CPU oracle for the differentiable particle-mesh method.

This package is TEST INFRASTRUCTURE. Only the test-suite, the smoke check and
the CPU-baseline leg of the benchmark may import it. The GPU library never
imports, links or calls it, and it shares no code, table or helper with the
GPU path.

Every function follows a passage of Li et al., "Differentiable Cosmological
Simulation with the Adjoint Method" (arXiv:2211.09815), cited by section and
equation label.  Everything is numpy/scipy in float64, written for clarity and
not for speed.

Units (reading of the paper, which does not fix them): lengths inside the force
and integrator are in mesh cells, time in 1/H0 (so H0 = 1 and the Poisson
coefficient is 1.5*Omega_m); the initial-condition power spectrum uses k in
h/Mpc and box lengths in Mpc/h.

Modules:
  cosmology  background, growth ODEs (Appendix A), FastPM factors (eq. G_eval),
             KDK step coefficients (Sec. 2.3), EH no-wiggle transfer function,
             sigma8 normalisation (eq. Plin)
  pm         CIC paint / readout (eq. cic), spectral Poisson gradient (Sec. 2.2),
             force and force VJP
  lpt        2LPT initial conditions (eq. lpt and Sec. 2.1) and their VJP/JVP
  integrate  KDK leapfrog (eq. KDFK), stored-trajectory discrete adjoint and the
             reverse-time adjoint (eqs. KDFKO_adj, KDFKO_grad)
  objective  final-density MSE objective and its VJP; power-spectrum estimator
  simulate   end-to-end J(omega, theta) and its gradients
"""
