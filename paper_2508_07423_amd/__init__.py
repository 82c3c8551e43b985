"""MI355X-native GNN track finding (ETX4VELO hot path) behind a C ABI.

``etx`` is the ctypes binding of ``libetx.so`` (HIP kernels for gfx950);
``synth`` produces seeded synthetic events and weights; ``evaluate`` computes
the tracking metrics of the thesis (ch. 7) from labels and generator truth.
"""
