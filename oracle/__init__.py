"""Plain CPU FP64 oracle of the IOBM scattering-state solve.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: it exists so that tests, the smoke check and the
benchmark's CPU baseline can check the GPU library against an independent,
slow, obviously correct implementation written from the paper.  It shares no
code with the library (no kernels, tables, helpers or pre/post-processing);
only the seeded input generators of the `workloads` package feed both.

Method (Egami, Hirose, Ono, Sec. II and appendix):
  fd.py      FD coefficients from their defining Taylor conditions (Eq. (1))
  lead.py    lateral modes and generalized Bloch states of the jellium leads,
             retarded self-energies (Eqs. (9)-(13), generalised to N_f planes),
             real-space Sigma by explicit DFT sums (Eq. (11))
  system.py  sparse assembly of E - H_T - Htilde (Eqs. (4), (6), (8)), the
             right-hand side of Eq. (6), sparse direct LU, current-based
             transmission / reflection and eigenchannel transmissions
  adjoint.py dT/dV by the transposed solve on the same LU factors
  precond.py the two preconditioners by their definitions (Eq. (17); the
             flat-wire inverse by a direct solve)

Every floating-point step is FP64 / complex128.
"""
from .fd import fd_coefficients, fd_coefficients_exact
from .lead import (AtThreshold, LeadMode, lateral_energy, lead_modes, open_channels,
                   sigma_realspace, mode_numbers, bloch_current, transfer_matrix)
from .system import Problem, kinetic, lead_coupling, solve_workload
from .adjoint import total_transmission_and_gradient, total_transmission
from . import precond
