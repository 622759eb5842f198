"""MI355X-native barrier-hoisted normalize (arXiv 2207.00257, Fig. 1).

out[i] = in[i] / sum(in) computed by the HIP kernels of libnrm.so (C ABI in
include/nrm.h). The compute entry points live in `api`; importing this
package does not load the library, calling them does (and fails loudly if it
is not built).
"""


def __getattr__(name):
    if name in ("normalize", "normalize_batched", "normalize_rows", "device_error", "Context"):
        from . import api

        return getattr(api, name)
    raise AttributeError(name)
