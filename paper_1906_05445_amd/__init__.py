"""MI355X-native lattice Boltzmann hot path (IBB and direct-forcing IBM).

The GPU library is loaded lazily by :mod:`paper_1906_05445_amd.lbm`; importing
the package itself loads nothing, so the seeded input generators in
:mod:`paper_1906_05445_amd.workloads` can be used without a GPU.
"""
