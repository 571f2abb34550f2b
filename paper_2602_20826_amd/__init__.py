"""libdagbound: batched exact evaluation of the makespan bound of DAG-structured
GPU tasks (Zhang et al., DAC 2026) on AMD Instinct MI355X.

The C-ABI library (``libdagbound.so``, HIP kernels for gfx950) does the work;
``dagbound`` is its thin Python binding with the same call names.
"""
from .dagbound import (  # noqa: F401
    OK, E_ARG, E_CYCLE, E_RANGE, E_DUP_EDGE, E_OOM, E_DEVICE, E_STATE, E_OVERFLOW, E_UNSUPPORTED, E_IO,
    ALLOC_EXPLICIT, ALLOC_SEEDED, PARA_SPATIAL, PARA_TEMPORAL, PTR_DEVICE, PTR_HOST, SEARCH_EXHAUSTIVE,
    SEARCH_SURROGATE, set_para_launch,
    Batch, DagboundError, best_allocation, best_allocation_static, create_batch, destroy_batch, eval_bounds, eval_conditional, eval_listed, shutdown,
    baselines, get_division, get_schedule, last_error, load_library, run_schedule, set_allocations, set_tuning,
    version,
    Model, model_forward, model_select, model_train_step,
)
