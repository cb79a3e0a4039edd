"""gfx950 (MI355X) hot path of many-to-many protein similarity search.

Candidate discovery by sparse products over k-mers and batched pairwise
alignment with identity/coverage filtering (PASTIS, Selvitopi et al., SC20),
implemented as hand-written HIP kernels behind the C ABI of include/pastis.h.
This package is the thin Python binding; it needs the built library.
"""

from ._binding import (  # noqa: F401
    EDGE_DTYPE,
    MLP_FEATURES,
    MLP_PARAMS,
    RECORD_DTYPE,
    Context,
    Params,
    PastisError,
    exported_names,
    lib,
    records_to_numpy,
)
