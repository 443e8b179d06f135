"""MI355X-native k-bisimulation partition refinement.

Python binding of the C ABI in ``include/kbisim.h`` (``libkbisim.so``, HIP
kernels for gfx950). Arguments are marshalled here; every step of the
refinement runs in the library's kernels. PyTorch supplies device memory and
the stream.
"""
from ._binding import (KbisimError, Graph, refine, kbisim_create, kbisim_refine, kbisim_result,
                       kbisim_result_round, kbisim_update, kbisim_update_stats, kbisim_refine_static, kbisim_stream_stats,
                       kbisim_profile, kbisim_work, kbisim_round_profile, kbisim_release_cached, kbisim_destroy,
                       kbisim_status_str, kbisim_last_error,
                       lib_path, load_library, PROF_CLASSES, WORK_BUCKETS, kbisim_batch_create, kbisim_batch_refine,
                       kbisim_batch_result, kbisim_batch_destroy, refine_batch, Server)

__all__ = ["KbisimError", "Graph", "refine", "kbisim_create", "kbisim_refine", "kbisim_result",
           "kbisim_result_round", "kbisim_update", "kbisim_update_stats", "kbisim_refine_static", "kbisim_stream_stats",
           "kbisim_profile", "kbisim_work", "kbisim_round_profile", "kbisim_release_cached", "kbisim_destroy",
           "kbisim_status_str", "kbisim_last_error",
           "lib_path", "load_library", "PROF_CLASSES", "WORK_BUCKETS", "kbisim_batch_create", "kbisim_batch_refine",
           "kbisim_batch_result", "kbisim_batch_destroy", "refine_batch", "Server"]
