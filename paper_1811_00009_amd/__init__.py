"""Block-based restarted narrow-band fast marching method (Yang 2018) on MI355X.

``fmm``     Python binding of the HIP library's C ABI (include/fmm.h).
``inputs``  seeded synthetic workloads.
``stride``  learned-stride data preparation and training driver.
"""
