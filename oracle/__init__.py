"""FP64 CPU oracle of the 2D hybrid lattice-Boltzmann / immersed-boundary step.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously correct
NumPy implementation of what one time step computes, written from the
paper's equations.  It exists to check the HIP library; only the test
suite, the smoke entry point and the benchmark's CPU-baseline leg may
import it.  The product path never calls it and shares no code with it.

Modules:
  lattice    D2Q9 BGK collide-and-stream with Guo forcing (Sec. 2.1, 2.2)
  ib         Roma 3-point delta kernel, interpolation and spreading (Sec. 2.2)
  membrane   strain, bending and enclosed-area forces (Sec. 2.2)
  philox     Philox4x32-10 counter-based generator (Salmon et al., SC'11)
  adhesion   ligand-receptor bond kinetics and spring force (Sec. 2.2)
  particles  probe stresses and dynamic-IB particle motion (Sec. 2.2, 2.3)
  sim        the time step in order, state, set-up (Sec. 2.3, 3)
"""
from . import lattice, ib, membrane, philox, adhesion, particles, sim  # noqa: F401
from .sim import Sim  # noqa: F401
