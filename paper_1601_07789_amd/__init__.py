"""Multibyte ("flyte") floating point for AMD Instinct MI355X (gfx950).

Values are stored as the top k bytes of an IEEE-754 binary32 or binary64 bit
pattern (Anderson & Gregg, "Vectorization of Multibyte Floating Point Data
Formats", PACT 2016).  The compute path is the HIP library ``libflyte.so``
behind the C-ABI of ``include/flyte.h``; ``paper_1601_07789_amd.flyte`` is its
thin Python binding, and ``paper_1601_07789_amd.workloads`` draws the seeded
synthetic inputs.
"""
