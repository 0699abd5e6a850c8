"""MI355X-native D3Q19 TRT lattice Boltzmann sweeps (hand-written HIP for gfx950).

The GPU library is loaded lazily by :mod:`paper_1711_11468_amd.lbm`; importing
this package alone loads nothing, so :mod:`paper_1711_11468_amd.inputs` can be
used without a GPU.
"""
