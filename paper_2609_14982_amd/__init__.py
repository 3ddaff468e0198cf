"""Python binding of libfmbtf: the frozen full-metric tangent transport J, J^T
applied through the SCC condensation graph on an MI355X.

The binding only marshals arguments: host arrays are numpy, device buffers and
the stream come from torch; every step of the transport runs in the native
library (host setup in C++, applies in HIP kernels).  Importing fails loudly
when the library is not built; nothing falls back to another implementation.
"""
from .binding import (  # noqa: F401
    FM_DS_BROADCAST,
    FM_DS_PER_PAIR,
    FM_FP32,
    FM_FP64,
    FM_JT_PER_SOURCE,
    FM_JT_SUMMED,
    FM_OUT_NODES,
    FM_OUT_RECEIVERS,
    FM_W_NODES,
    FM_W_RECEIVERS,
    Batch,
    Cgls,
    Eikonal,
    apply_J_static,
    autotune,
    FmError,
    Lsqr,
    ModelMap,
    State,
    build_frozen_state,
    build_frozen_states,
    build_frozen_states_gpu,
    build_frozen_states_pt,
    set_iterative_block_min,
    exported_symbols,
    lib_path,
    load,
)
