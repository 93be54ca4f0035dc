"""MI355X-native kernel-weighted auto/cross-correlation for irregularly sampled
series (HIP library ``libncf.so`` behind the C ABI of ``include/ncf.h``).

``paper_2609_03866_amd.ncf`` is the ctypes binding; ``synth`` generates the
seeded synthetic inputs; ``build`` compiles the library.
"""
