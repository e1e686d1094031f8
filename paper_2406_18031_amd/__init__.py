"""MI355X-native structure-flow filter (Adarve & Mahony, arXiv 2406.18031).

The filter runs in the HIP library libsflow.so (sources in csrc/, C ABI in
include/sflow.h); `paper_2406_18031_amd.sflow` is its Python binding and
`paper_2406_18031_amd.build` compiles it for gfx950.
"""
