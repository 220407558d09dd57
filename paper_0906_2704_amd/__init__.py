"""MI355X-native spectral Tikhonov deblurring under high-order boundary conditions.

The compute path lives in libht.so (HIP, gfx950) behind the C ABI of include/ht.h;
``paper_0906_2704_amd.ht`` is its Python binding and ``paper_0906_2704_amd.synth`` the
seeded synthetic workload generator.  Importing the package loads nothing.
"""
