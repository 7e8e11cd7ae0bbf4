"""MI355X-native coupled lattice-Boltzmann / particulate-IBM / DEM step.

``paper_1407_6704_amd.pibm`` is the ctypes binding of the HIP library
(``libpibm.so``, C ABI in ``include/pibm.h``); ``workloads`` draws seeded
synthetic inputs.  Importing the package loads neither.
"""
