"""MI355X-native SU(2) two-site DMRG H.psi library (HIP, gfx950).

The compute path lives in libdmrg_hpsi.so (C ABI in include/dmrg.h);
``binding`` and ``hpsi`` only marshal arguments.  ``synth`` draws seeded
synthetic inputs.
"""
