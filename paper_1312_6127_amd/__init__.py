"""MI355X (gfx950) implementation of one GRRMHD time step of the HARMRAD
method: hand-written HIP kernels behind the C ABI of include/grrmhd.h, with
a thin ctypes binding in :mod:`paper_1312_6127_amd.grrmhd`."""
