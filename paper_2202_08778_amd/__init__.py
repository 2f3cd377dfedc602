"""MI355X-native implicit VET radiation step (VETTAM's implicit update, arXiv:2202.08778).

The compute path is the HIP library libvettam_rad.so (C ABI: include/vettam_rad.h);
``paper_2202_08778_amd.rad`` is its ctypes binding and ``workloads`` draws seeded inputs.
"""
__all__ = ["rad", "workloads", "build"]
