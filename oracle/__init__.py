"""FP64 CPU oracle for the KSA-XL-BOMD electronic hot path.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, deliberately
unoptimised NumPy implementation of what the hot path computes, written from
the paper's equations (Kulichenko et al., "Semi-Empirical Shadow Molecular
Dynamics: A PyTorch implementation", arXiv:2303.00689).  Only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import it.  It shares no code with the HIP path (no kernels, headers, helpers,
tables or constants) and never imports it; the two meet only in the seeded
inputs of the ``synth`` package.

Conventions (shared with the C ABI as a contract, not as code):
  * orbital index 4*atom + {0: s, 1: px, 2: py, 3: pz};
  * density matrices at the interface are spin-summed, Tr P = N_e; the paper's
    one-spin D is P / 2;
  * atom pairs (A < B) are enumerated row-major; a packed orbital pair (mu nu)
    of one atom runs over the row-major upper triangle of its 4 x 4 block.

Readings of silent or ambiguous points of the paper (entropy factor, X-Verlet
form and coefficients, Krylov recipe, the synthetic Hamiltonian) are stated in
the docstrings of the functions that take them.

Parity status per function:
  model.hcore, model.two_electron, model.nuclear_repulsion   pinned (tests/test_oracle_model.py)
  density.density_matrix, density.entropy                    pinned (tests/test_oracle_density.py)
  density.response                                           pinned (finite differences, closed forms)
  krylov.krylov_kernel                                       pinned (full rank = exact inverse Jacobian)
  dynamics.energy_forces                                     pinned (finite differences of U)
  dynamics.md_step / dynamics.scf                            pinned (dt^2 scaling, reversibility, residual)
  dynamics.evaluate with m = 0 (K = -c I)                    pinned (closed form; equals the full-rank
                                                             kernel when J = -I; unstable where KSA is not)
  dynamics.ou_coefficients / dynamics.langevin_step          pinned (Maxwell-Boltzmann variance; gamma = 0
                                                             is md_step; thermalisation to the bath T)
  overlap.overlap, overlap.overlap_derivative_blocks         pinned (symmetry, rotation covariance, finite
                                                             differences)
  overlap.lowdin, overlap.density_matrix, overlap.response   pinned (Z^T S Z = I; the generalized
                                                             eigenproblem; another Z of eq. 21; finite
                                                             differences)
  overlap.pulay_forces                                       pinned (finite differences of the grand
                                                             potential through S at fixed F)
"""

from . import model, density, krylov, dynamics, overlap  # noqa: F401
