"""MI355X-native fixed-radius neighbour search for SPH (relative-coordinate link list).

The search runs in HIP kernels compiled into libnnps.so (C ABI: include/nnps.h);
`nnps` is the Python binding and `workloads` draws seeded synthetic inputs.
"""
