"""MI355X-native ray tracer for the uniaxial-dielectric cylindrical cloaks of
Halimeh & Wegener (radial and azimuthal optic axis, mu = 1).

The compute path is the HIP library ``librt_cloak.so`` (C ABI in
``include/rt.h``); ``paper_1209_6038_amd.rt`` is its thin ctypes binding and
``paper_1209_6038_amd.workloads`` builds seeded synthetic inputs.
"""
