"""Seeded synthetic protein-family inputs.

This package only draws random inputs: protein sequences grouped into families
(plus unrelated singletons) with the length mixes of the workloads the paper
evaluates on (Metaclust50 subsets and SCOPe families, Section VI), which are not
available here.  It holds none of the search method's arithmetic: no k-mers, no
alignment, no scoring.  Both the CPU oracle tests and the GPU path consume its
output, and neither is imported from here.
"""

from .families import (  # noqa: F401
    ALPHABET20,
    WORKLOADS,
    FamilySet,
    background_frequencies,
    make_family_set,
    pair_list,
    workload,
)
