"""MI355X-native matrix-free spectral/hp elemental operators (hex, prism, tet).

The compute path is the HIP library ``libnir.so`` behind the C ABI declared in
``include/nir.h``; ``paper_2606_20917_amd.nir`` is its thin Python binding and
``paper_2606_20917_amd.inputs`` generates seeded synthetic meshes.  Importing
the package loads nothing: the binding loads the library on first use.
"""
