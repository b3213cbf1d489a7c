"""MI355X-native docking hot path: HIP kernels behind the C ABI of include/exs.h.

``paper_2110_11644_amd.binding`` is the thin ctypes binding of ``libexs.so``;
``paper_2110_11644_amd.build`` compiles it for gfx950.
"""
