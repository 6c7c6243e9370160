"""Seeded synthetic workloads shared by the CPU oracle and the GPU library's
tests and benchmark.  Input generation only: no part of the method."""
from .synth import (Grid, Nonlocal, Workload, flat, barrier, chain, wide, adjoint,
                    make, random_field, CONFIGS, CONFIG4_ENERGIES, na_wire, jellium_fermi_energy)
