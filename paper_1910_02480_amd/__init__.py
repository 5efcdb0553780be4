"""MI355X (gfx950) radiance-cache autoencoder of Deep Radiance Caching.

``binding`` is the ctypes face of libdrc_cae.so (the C ABI in
include/drc_cae.h); ``cae`` wraps it for PyTorch tensors; ``synth`` draws the
seeded synthetic workloads. Importing the package does not load the library;
the first call into ``binding`` does, and raises if it has not been built.
"""
