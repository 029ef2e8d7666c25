"""MI355X-native in situ particle data binning (HIP/gfx950 behind a C ABI).

``binding`` loads ``libbinning.so`` (built in-tree by ``build.py``) and fails
loudly if it is missing; ``synth`` draws seeded synthetic workloads.
"""
