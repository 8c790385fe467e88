"""MI355X-native per-timestep constraint solver.

Newton (ILVES-M style) or chord (ILVES-F style) iterations on the sparse
constraint Jacobian, with a sparse LU whose ordering and symbolic
factorisation are planned once per topology, all in hand-written HIP
kernels for gfx950 behind the C ABI in include/ilves.h.  ``synth`` builds
seeded synthetic workloads; ``_lib`` is the ctypes binding.
"""
from ._lib import (ERR_ARG, ERR_HIP, ERR_NOMEM, ERR_NONFINITE, ERR_NOT_CONVERGED, ERR_SINGULAR, ERR_TIMEOUT,
                   ERR_TOPOLOGY, ERR_UNSUPPORTED, OK, PREC_FP64, PREC_MIXED, VARIANT_CHORD, VARIANT_NEWTON,
                   WARM_CALLER, WARM_DECOUPLED, WARM_MLP, WARM_ZERO, IlvesError, Plan)

__all__ = ["Plan", "IlvesError", "OK", "ERR_ARG", "ERR_TOPOLOGY", "ERR_HIP", "ERR_NOMEM", "ERR_SINGULAR",
           "ERR_NOT_CONVERGED", "ERR_NONFINITE", "ERR_UNSUPPORTED", "ERR_TIMEOUT", "PREC_FP64", "PREC_MIXED",
           "VARIANT_NEWTON", "VARIANT_CHORD", "WARM_ZERO", "WARM_MLP", "WARM_CALLER", "WARM_DECOUPLED"]
