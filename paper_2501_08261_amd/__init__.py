"""MI355X-native time-domain LISA likelihood (arXiv:2501.08261 hot path).

The compute lives in the C-ABI library ``liblisatd.so`` (hand-written HIP
kernels for gfx950); ``paper_2501_08261_amd.lib`` is its thin ctypes binding.
"""
