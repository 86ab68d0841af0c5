"""MI355X-native (gfx950) many-body DPD timestep.

The hot path runs in hand-written HIP kernels behind the C ABI of
``include/mdpd.h`` (``libmdpd.so``); this package is its thin Python binding
(``mdpd_*`` functions with the C names, plus an owning ``System`` wrapper) and
the seeded synthetic workloads (``workloads``).  The native library is loaded
on first use and its absence is an error: there is no CPU fallback.
"""
from ._native import (FP32_FORCES, FP64, KERNELS, MEM_DEVICE, MEM_HOST, WALL_BVF, WALL_OFF, Batch,
                      MdpdError, Params, System, lib, make_params, mdpd_autotune, mdpd_backward, mdpd_checkpoint_size, mdpd_create,
                      mdpd_create_batch,
                      mdpd_debug_forces, mdpd_debug_neighbors, mdpd_destroy, mdpd_forward_record,
                      mdpd_get_state,
                      mdpd_last_error, mdpd_load_checkpoint, mdpd_read_kernel_timing,
                      mdpd_read_list_builds, mdpd_read_observables, mdpd_read_profile,
                      mdpd_read_replica_observables,
                      mdpd_read_stress, mdpd_read_stress_noalloc,
                      mdpd_save_checkpoint,
                      mdpd_set_graph, mdpd_set_kernel_timing, mdpd_set_lanes, mdpd_step)

__all__ = ["FP32_FORCES", "FP64", "KERNELS", "MEM_DEVICE", "MEM_HOST", "WALL_BVF", "WALL_OFF", "Batch",
           "MdpdError", "Params", "System", "lib", "make_params", "mdpd_autotune", "mdpd_backward", "mdpd_checkpoint_size", "mdpd_create",
           "mdpd_create_batch",
           "mdpd_debug_forces", "mdpd_debug_neighbors", "mdpd_destroy", "mdpd_forward_record",
           "mdpd_get_state",
           "mdpd_last_error", "mdpd_load_checkpoint", "mdpd_read_kernel_timing",
           "mdpd_read_list_builds", "mdpd_read_observables", "mdpd_read_profile",
           "mdpd_read_replica_observables",
           "mdpd_read_stress", "mdpd_read_stress_noalloc",
           "mdpd_save_checkpoint",
           "mdpd_set_graph", "mdpd_set_kernel_timing", "mdpd_set_lanes", "mdpd_step"]
