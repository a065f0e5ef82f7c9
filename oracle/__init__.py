"""FP64 CPU oracle of the PonD finite-volume step (test infrastructure only).

Only the tests, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline
leg use this package.  The product library never imports, links or calls it.
"""
from .pondref import Oracle, OracleConfig, lattice, transform_matrix, transform_matrix_full, \
    cfl_dt, set_threads, get_threads, load_library, qe_half_step, ms_matrix, F_D2Q16, F_D2Q9, \
    F_MULTISCALE, F_D2Q25, MS_THRESHOLD

__all__ = ["Oracle", "OracleConfig", "lattice", "transform_matrix", "transform_matrix_full",
           "cfl_dt", "set_threads", "get_threads", "load_library", "qe_half_step", "ms_matrix",
           "F_D2Q16", "F_D2Q9", "F_MULTISCALE", "F_D2Q25", "MS_THRESHOLD"]
