"""MI355X-native annealer for the UAV coverage-path QUBO (arxiv 2608.25376).

The hot path lives in the C-ABI library ``libuavq.so`` (HIP kernels for
gfx950); ``paper_2608_25376_amd.uavq`` is the thin Python binding over it.
Importing this package loads nothing; the binding loads the library on first use.
"""
