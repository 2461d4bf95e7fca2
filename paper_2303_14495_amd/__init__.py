"""MI355X (gfx950) preconditioned DCA for the graph Ginzburg-Landau model.

The solver is the HIP library ``libgl_dca.so`` (C ABI in include/gl_dca.h);
this package holds its sources, its build script and a thin ctypes binding.
"""

from .gl import (  # noqa: F401
    GLError,
    Operator,
    Server,
    assign_labels,
    knn,
    knn_fallback_rows,
    knn_graph,
    load_library,
    split_stats,
    stats_length,
    time_stream,
    time_sweeps,
    version,
    DTYPES,
    PRECONDS,
    TORCH_DTYPES,
)
