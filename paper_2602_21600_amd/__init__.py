"""MI355X-native AQR-HNSW query path: 8-bit density-aware codes for the graph
search, then asymmetric distances, early termination and exact FP32 re-rank.

The compute path is the HIP library libaqr.so (C-ABI in include/aqr.h); the
Python binding in `aqr` only marshals arguments.  `workloads` holds the
seeded synthetic inputs, `presets` the recommended settings per target
recall (Table 3).
"""
__all__ = ["aqr", "workloads", "presets"]
