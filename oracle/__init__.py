"""FP64 CPU oracle for the dynamic-bonding Langevin MD step.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it, as the slow and obviously correct
reference that the HIP library is checked against.

It shares no code with the HIP library.  The only thing both sides agree on
by construction is the counter-based generator (Philox4x32-10, Salmon et al.
2011), which each side implements separately from its published definition.

Modules
-------
philox  : Philox4x32-10 and the conversions of its words to uniforms,
          Gaussians and a random permutation.
dybond  : the system (forces, BAOAB integrator, bonding sweep, observables).
"""

from .philox import (  # noqa: F401
    philox4x32_10, stream_key, u53, box_muller3, reaction_order,
    KIND_THERMO, KIND_ORDER, KIND_MATCH, KIND_ON, KIND_OFF,
)
from .dybond import OracleSystem, Reaction, BOND_HARMONIC, BOND_FENE  # noqa: F401
