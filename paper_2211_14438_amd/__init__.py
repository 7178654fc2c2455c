"""MI355X (gfx950) implementation of BERN-NN bound propagation.

``bernnn``    ctypes binding of the HIP library ``libbernnn.so`` (C ABI in include/bernnn.h)
``workloads`` seeded synthetic networks, boxes and degree draws
``build``     in-tree hipcc build of the library
"""
