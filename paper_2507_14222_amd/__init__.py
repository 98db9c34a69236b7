"""IG hot path on MI355X: bit-packed pairwise intersection, coherence filter,
support weights and scoring in hand-written HIP kernels behind a C ABI.

``paper_2507_14222_amd.ig`` is the Python binding (imports libig lazily);
``paper_2507_14222_amd.synth`` holds the seeded synthetic workloads.
"""
__all__ = ["ig", "synth"]
