"""MI355X-native per-barrier-interval SIMT data-race checker.

The work is done by librv.so (hand-written HIP for gfx950, C ABI in
include/rv.h); this package is its Python binding.  Importing it does not
touch the GPU; the first call that needs the library loads it and raises if
it is missing.
"""

from .rv import (EXPORTED, STAGES, STATUS, Batch, Context, JobResult, Kernel, Marshalled, Result, RVError, Server,
                 Side, Witness, lib, plan, selftest, validate)

__all__ = ["EXPORTED", "STAGES", "STATUS", "Batch", "Context", "JobResult", "Kernel", "Marshalled", "Result", "RVError",
           "Server", "Side", "Witness", "lib", "plan", "selftest", "validate"]
