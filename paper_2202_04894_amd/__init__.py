"""defmm on MI355X: the directional equispaced-interpolation FMM matvec as
hand-written HIP kernels behind a C ABI (``libdefmm.so``).

Import :mod:`paper_2202_04894_amd.defmm` for the binding; importing the package
itself loads nothing native.
"""
