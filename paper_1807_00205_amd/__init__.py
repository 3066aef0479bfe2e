"""MI355X-native seed filter for segmental-duplication search (SEDEF, Section 3.1).

``sdf`` binds the C ABI of ``libsdf.so`` (HIP kernels for gfx950);
``synth`` draws seeded synthetic workloads.
"""
__all__ = ["sdf", "synth"]
