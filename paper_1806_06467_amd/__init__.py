"""MI355X-native Fresnel + matrix-Fourier-transform propagation (Douglas & Perrin 2018).

The compute path is the HIP library libfresnel.so (C ABI declared in include/fresnel.h);
this package is its thin ctypes binding plus seeded input generators. Importing the package
does not load the library; the first call into it does, and fails loudly if it is not built.
"""
