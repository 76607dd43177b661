"""MI355X-native EDGE edge-detection pipeline (fork-join stencils plus a max
reduction) behind a small C ABI, libhx.so.

``paper_2503_10855_amd.hx`` is the ctypes binding of that ABI; importing it
loads the HIP library and fails loudly if it has not been built.
``paper_2503_10855_amd.synth`` draws the seeded synthetic workloads.
"""
