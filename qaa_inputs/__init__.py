"""Seeded synthetic inputs shared by the oracle side and the HIP side.

This module holds no arithmetic of the evolution itself: it draws random
numbers and builds 3-SAT clause lists.  Both sides receive the same clause
list and compute energies, phases and amplitudes on their own.

Random numbers come from SplitMix64 (G. Steele, D. Lea, C. Flood, "Fast
splittable pseudorandom number generators", OOPSLA 2014), written here from
its published definition.

Instances are *planted, unique-solution* 3-SAT formulas (Sec. 2.2 defines
K-SAT; Sec. 4.3 uses hard 3-SAT instances; the workloads ask for a unique
planted solution):

1. draw the planted assignment z* uniformly from [0, 2^n);
2. repeat: draw 3 distinct variables uniformly (rejection), draw a sign
   pattern uniformly from the 8 patterns and redraw while it is the one
   pattern z* violates; append the clause;
3. stop at the first clause after which z* is the only assignment that
   satisfies every clause (checked exhaustively over 2^n).

Step 3 keeps a bitset of the still-satisfying assignments (one bit per z)
and clears, per clause, the assignments that violate it; once few survive it
switches to an explicit candidate list.
"""
from .planted import (  # noqa: F401
    SplitMix64,
    Instance,
    planted_unique_3sat,
    batch_workload,
    serving_workload,
    load_instance,
    save_instance,
)
