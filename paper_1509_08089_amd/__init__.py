"""MI355X-native Moss: sample-and-classify estimation of 4- and 5-node graphlet counts.

The hot path (table build, MOSS-4 / T-5 / Path-5 sampling, classification, histograms,
batched persistent launches, the serving loop) is in libmoss.so (HIP, gfx950), behind
the C ABI of include/moss.h.  This package is its ctypes binding.
"""
from . import moss
from .moss import (Graph, MossError, moss_estimate, moss_estimate_batch, moss_finals,
                   moss_graph_create, moss_graph_create_device, moss_graph_destroy, moss_build_tables,
                   moss_graph_get_info, moss_table_read, moss_sample_range, moss_sample_nodes,
                   moss_class_lut, moss_status_string, moss_set_tuning, moss_get_tuning, moss_autotune,
                   moss_server_create, moss_server_add_graph, moss_server_submit, moss_server_wait,
                   moss_server_cancel, moss_server_stats_get, moss_server_destroy)

__all__ = [n for n in dir(moss) if n.startswith("moss_") or n in ("Graph", "MossError")]
